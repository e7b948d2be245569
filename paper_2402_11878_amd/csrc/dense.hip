// Dense k-qubit window by MFMA: psi' = U psi on the qubits of one window,
// with U a dense 2^k x 2^k complex unitary (k = kDenseK).
//
// Per coset (the 2^k amplitudes that differ only in the window bits) this is
// a complex matrix-vector product; over the cosets, a complex matrix product
// U . [2^k x cosets].  It runs as the real product
//   [Re psi'; Im psi'] = [[Re U, -Im U], [Im U, Re U]] . [Re psi; Im psi]
// (64 x 64 times 64 x cosets for k = 5) on the matrix cores: one wave takes a
// tile of 16 consecutive cosets through 4 x 16 MFMA 16x16x4 steps (4 output
// row blocks of 16, 16 steps of 4 over the 64 input rows), FP32 MFMA for a
// complex64 state and FP64 MFMA for complex128.
//
// Operand layout of the 16x16x4 MFMA for lane l = 16 g + j (g < 4, j < 16):
// A element (row j, k-index g), B element (k-index g, column j); result
// register v holds column j of row 4 g + v (FP32 form) or of row g + 4 v
// (FP64 form; both checked on the device).  Column j is coset 16 t + j of the
// tile; lane (g, j) therefore loads patterns g + 4 m (m < 8) of its coset,
// real parts for steps m and imaginary parts for steps 8 + m, and stores
// patterns row(g, v) and 16 + row(g, v).  All window qubits are >= 4, so the
// 16 cosets of a tile are 16 consecutive amplitudes per pattern.
#include "vqe_internal.h"

namespace vqe {
namespace {

template <typename T> struct DenseVec;
template <> struct DenseVec<float> { using type = float2; };
template <> struct DenseVec<double> { using type = double2; };

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static constexpr __device__ int row(int g, int v) { return 4 * g + v; }  // result row of register v
};
template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static constexpr __device__ int row(int g, int v) { return g + 4 * v; }
};

constexpr int kDenseWaves = 4;        // waves (tiles of 16 cosets) per block
constexpr uint32_t kDenseBlocks = 2048;  // persistent grid: U stays in registers over a run of tiles

// Unit of iteration it of block b (grid * cpt = 2^m units, grid a multiple of
// 8 when m >= 3): each block a contiguous run inside the eighth b & 7.
__device__ __forceinline__ uint64_t dense_unit(uint64_t b, uint32_t it, uint32_t cpt, uint32_t m) {
    if (m < 3) return b * cpt + it;
    return ((b & 7ull) << (m - 3)) | ((b >> 3) * cpt + it);
}

template <typename T>
__global__ void __launch_bounds__(64 * kDenseWaves)
dense_kernel(const DenseArgs a, const T* __restrict__ ur, const typename DenseVec<T>::type* in,
             typename DenseVec<T>::type* out, uint32_t cpt, uint32_t mlog) {
    using V = typename DenseVec<T>::type;
    using acc_t = typename Mfma<T>::acc_t;
    constexpr int RR = 2 << kDenseK;  // 64 real rows
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, j = lane & 15;
    // A operands of this lane for the 4 row blocks and 16 steps
    T ua[4][RR / 4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int s = 0; s < RR / 4; ++s) ua[b][s] = ur[(16 * b + j) * RR + 4 * s + g];
    auto offset = [&](int p) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < kDenseK; ++i)
            if ((p >> i) & 1) o += 1ull << a.q[i];
        return o;
    };
    for (uint32_t it = 0; it < cpt; ++it) {
        const uint64_t tile = dense_unit(blockIdx.x, it, cpt, mlog) * kDenseWaves + (threadIdx.x >> 6);
        if (tile >= a.n_tiles) break;
        uint64_t base = tile * 16 + (uint64_t)j;
#pragma unroll
        for (int i = 0; i < kDenseK; ++i) {  // insert a zero at each window position, ascending
            const uint64_t low = base & ((1ull << a.sorted[i]) - 1);
            base = ((base ^ low) << 1) | low;
        }
        V v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = in[base + offset(g + 4 * m)];
        acc_t acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < RR / 4; ++s) {
            const T bs = s < 8 ? v[s].x : v[s - 8].y;
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[b] = Mfma<T>::step(ua[b][s], bs, acc[b]);
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int p = Mfma<T>::row(g, w);
            V o;
            o.x = acc[0][w];
            o.y = acc[2][w];
            out[base + offset(p)] = o;
            o.x = acc[1][w];
            o.y = acc[3][w];
            out[base + offset(16 + p)] = o;
        }
    }
}

}  // namespace

template <typename T>
hipError_t launch_dense(const DenseArgs& a, const T* ur, const void* in, void* out, hipStream_t st) {
    using V = typename DenseVec<T>::type;
    if (a.n_tiles == 0) return hipSuccess;
    const uint64_t units = (a.n_tiles + kDenseWaves - 1) / kDenseWaves;
    const uint32_t grid = (uint32_t)(units < kDenseBlocks ? units : kDenseBlocks);
    const uint64_t cpt = (units + grid - 1) / grid;
    if (cpt > 0xffffffffull) return hipErrorInvalidValue;
    uint32_t mlog = 0;  // log2 of units when units is a power of two (then grid * cpt = units), else 0
    if ((units & (units - 1)) == 0)
        while ((1ull << mlog) < units) ++mlog;
    hipLaunchKernelGGL(dense_kernel<T>, dim3(grid), dim3(64 * kDenseWaves), 0, st, a, ur, (const V*)in, (V*)out,
                       (uint32_t)cpt, mlog);
    return hipGetLastError();
}

template hipError_t launch_dense<float>(const DenseArgs&, const float*, const void*, void*, hipStream_t);
template hipError_t launch_dense<double>(const DenseArgs&, const double*, const void*, void*, hipStream_t);

}  // namespace vqe
