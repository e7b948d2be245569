// HIP kernels of the VQE hot path, written for gfx950 (CDNA4, wave64).
//
//  * window_kernel   : one fused pass of the ansatz (eq. 6).  Each thread owns
//                      the 2^K amplitudes of one coset of a K-qubit window,
//                      found by inserting zero bits at the window positions
//                      into the thread's linear index (index-bit insertion),
//                      so consecutive lanes read consecutive addresses.  All
//                      gates of the pass are applied in registers; the state
//                      is read and written once.  The reverse variant carries
//                      (psi, lam), un-applies the gates in reverse order and
//                      accumulates the adjoint gradient Im<lam|G|psi>.
//  * hpsi_kernel     : (H psi)[b] = sum_x psi[b^x] D_x(b) with
//                      D_x(b) = sum_{z in group x} c_z (-1)^popcount(z&b):
//                      terms grouped by X mask, one read of the partner tile
//                      serves every Z pattern of the group (eq. 7 energy from
//                      the same pass).
//  * expect_term_kernel : one sweep per Pauli term, the paper's evaluation
//                      order (Sec. III-D), used as the baseline form.
//  * reduce_kernel   : fixed-order FP64 sum of per-block partials (no atomics,
//                      deterministic bits).
#include <type_traits>

#include "vqe_internal.h"

namespace vqe {
namespace {

// XCD-aware order of work units.  Workgroups are dispatched round-robin over
// the 8 XCDs (block b runs on XCD b mod 8), each XCD with its own L2.  For a
// power-of-two count of 2^m units, rotating the 3 lowest unit bits to the top
// gives XCD x the contiguous range [x 2^(m-3), (x+1) 2^(m-3)), so every XCD
// streams its own eighth of the state.  Measured on MI355X: forward passes
// whose window spans address bits that otherwise collide (e.g. qubits 20-23
// of a complex128 state) go from 3.9 to 5.4 TB/s; other windows are unchanged.
__device__ __forceinline__ uint64_t xcd_order(uint64_t u, uint32_t m) {
    if (m < 3) return u;
    return (u >> 3) | ((u & 7ull) << (m - 3));
}

// Work unit of iteration it of block b in a grid whose blocks walk runs of
// cpt units (grid * cpt = 2^m units, grid a multiple of 8): block b stays in
// the eighth b & 7 of the units (the XCD it is dispatched to) and walks a
// contiguous run there.  For cpt = 1 this is xcd_order(b, m).  Measured on
// the H psi window passes: complex64 36 -> 28 ms per pass against
// xcd_order(b cpt + it, m); the gate window passes keep the latter (their
// complex128 reverse pass measured 59 ms with it, 63 ms with this order).
__device__ __forceinline__ uint64_t xcd_unit(uint64_t b, uint32_t it, uint32_t cpt, uint32_t m) {
    if (m < 3) return b * cpt + it;
    return ((b & 7ull) << (m - 3)) | ((b >> 3) * cpt + it);
}

__host__ __device__ inline uint32_t log2_pow2(uint64_t v) {
    // exact log2 for a power of two; 0 (no reordering) otherwise
    if (v == 0 || (v & (v - 1))) return 0;
    uint32_t m = 0;
    while ((1ull << m) < v) ++m;
    return m;
}

template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = float2; };
template <> struct VecOf<double> { using type = double2; };

// ---------------------------------------------------------------- register ops
template <int K, int B, int NV, typename T>
__device__ __forceinline__ void op_u2(T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    const T m0r = m[0], m0i = m[1], m1r = m[2], m1i = m[3];
    const T m2r = m[4], m2i = m[5], m3r = m[6], m3i = m[7];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            if (i & (1 << B)) continue;
            const int j = i | (1 << B);
            const T ar = re[v][i], ai = im[v][i], br = re[v][j], bi = im[v][j];
            re[v][i] = m0r * ar - m0i * ai + m1r * br - m1i * bi;
            im[v][i] = m0r * ai + m0i * ar + m1r * bi + m1i * br;
            re[v][j] = m2r * ar - m2i * ai + m3r * br - m3i * bi;
            im[v][j] = m2r * ai + m2i * ar + m3r * bi + m3i * br;
        }
    }
}

template <int K, int B, int NV, typename T>
__device__ __forceinline__ void op_r2(T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    const T a = m[0], b = m[2], c = m[4], d = m[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            if (i & (1 << B)) continue;
            const int j = i | (1 << B);
            const T ar = re[v][i], ai = im[v][i], br = re[v][j], bi = im[v][j];
            re[v][i] = a * ar + b * br;
            im[v][i] = a * ai + b * bi;
            re[v][j] = c * ar + d * br;
            im[v][j] = c * ai + d * bi;
        }
    }
}

template <int K, int B, int NV, typename T>
__device__ __forceinline__ void op_diag(T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    const T p0r = m[0], p0i = m[1], p1r = m[6], p1i = m[7];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            const T pr = (i & (1 << B)) ? p1r : p0r;
            const T pi = (i & (1 << B)) ? p1i : p0i;
            const T ar = re[v][i], ai = im[v][i];
            re[v][i] = pr * ar - pi * ai;
            im[v][i] = pr * ai + pi * ar;
        }
    }
}

template <int K, int C, int Tg, int NV, typename T>
__device__ __forceinline__ void op_cnot(T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            if (!(i & (1 << C)) || (i & (1 << Tg))) continue;
            const int j = i | (1 << Tg);
            const T tr = re[v][i], ti = im[v][i];
            re[v][i] = re[v][j];
            im[v][i] = im[v][j];
            re[v][j] = tr;
            im[v][j] = ti;
        }
    }
}

template <int K, int A, int B, int NV, typename T>
__device__ __forceinline__ void op_cz(T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            if ((i & (1 << A)) && (i & (1 << B))) {
                re[v][i] = -re[v][i];
                im[v][i] = -im[v][i];
            }
        }
    }
}

template <int K, int B, int NV, typename T>
__device__ __forceinline__ void op_xflip(T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            if (i & (1 << B)) continue;
            const int j = i | (1 << B);
            const T tr = re[v][i], ti = im[v][i];
            re[v][i] = re[v][j];
            im[v][i] = im[v][j];
            re[v][j] = tr;
            im[v][j] = ti;
        }
    }
}

// Im<lam| G_B |psi> over the thread's coset; vector 0 = psi, vector 1 = lam.
template <int K, int B, int G, typename T>
__device__ __forceinline__ T op_grad(T (&re)[2][1 << K], T (&im)[2][1 << K]) {
    T acc = 0;
#pragma unroll
    for (int i = 0; i < (1 << K); ++i) {
        if (i & (1 << B)) continue;
        const int j = i | (1 << B);
        const T p0r = re[0][i], p0i = im[0][i], p1r = re[0][j], p1i = im[0][j];
        const T l0r = re[1][i], l0i = im[1][i], l1r = re[1][j], l1i = im[1][j];
        if constexpr (G == OP_GZ) {
            // Z psi = (psi0, -psi1):  Im(conj(l0) p0) - Im(conj(l1) p1)
            acc += (l0r * p0i - l0i * p0r) - (l1r * p1i - l1i * p1r);
        } else if constexpr (G == OP_GY) {
            // Y psi = (-i psi1, i psi0)
            acc += (l1r * p0r + l1i * p0i) - (l0r * p1r + l0i * p1i);
        } else {
            // X psi = (psi1, psi0)
            acc += (l0r * p1i - l0i * p1r) + (l1r * p0i - l1i * p0r);
        }
    }
    return acc;
}

// Explicit switch dispatch from a uniform runtime bit to the template
// instantiation, so that every register index is a compile-time constant.
#define VQE_BIT_CASES(CALL)                                       \
    case 0: if constexpr (K > 0) { constexpr int B = 0; CALL; } break; \
    case 1: if constexpr (K > 1) { constexpr int B = 1; CALL; } break; \
    case 2: if constexpr (K > 2) { constexpr int B = 2; CALL; } break; \
    case 3: if constexpr (K > 3) { constexpr int B = 3; CALL; } break; \
    case 4: if constexpr (K > 4) { constexpr int B = 4; CALL; } break; \
    default: break;

template <int K, int NV, typename T>
__device__ __forceinline__ void d_u2(int b, T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    switch (b) { VQE_BIT_CASES((op_u2<K, B, NV, T>(re, im, m))) }
}
template <int K, int NV, typename T>
__device__ __forceinline__ void d_r2(int b, T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    switch (b) { VQE_BIT_CASES((op_r2<K, B, NV, T>(re, im, m))) }
}
template <int K, int NV, typename T>
__device__ __forceinline__ void d_diag(int b, T (&re)[NV][1 << K], T (&im)[NV][1 << K], const T* m) {
    switch (b) { VQE_BIT_CASES((op_diag<K, B, NV, T>(re, im, m))) }
}
template <int K, int NV, typename T>
__device__ __forceinline__ void d_xflip(int b, T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
    switch (b) { VQE_BIT_CASES((op_xflip<K, B, NV, T>(re, im))) }
}
template <int K, int C, int NV, typename T>
__device__ __forceinline__ void d_cnot_t(int t, T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
    switch (t) { VQE_BIT_CASES(if constexpr (B != C) (op_cnot<K, C, B, NV, T>(re, im))) }
}
template <int K, int NV, typename T>
__device__ __forceinline__ void d_cnot(int c, int t, T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
    switch (c) { VQE_BIT_CASES((d_cnot_t<K, B, NV, T>(t, re, im))) }
}
template <int K, int A, int NV, typename T>
__device__ __forceinline__ void d_cz_b(int b2, T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
    switch (b2) { VQE_BIT_CASES(if constexpr (B != A) (op_cz<K, A, B, NV, T>(re, im))) }
}
template <int K, int NV, typename T>
__device__ __forceinline__ void d_cz(int a, int b2, T (&re)[NV][1 << K], T (&im)[NV][1 << K]) {
    switch (a) { VQE_BIT_CASES((d_cz_b<K, B, NV, T>(b2, re, im))) }
}
template <int K, int G, typename T>
__device__ __forceinline__ T d_grad(int b, T (&re)[2][1 << K], T (&im)[2][1 << K]) {
    T g = 0;
    switch (b) { VQE_BIT_CASES(g = (op_grad<K, B, G, T>(re, im))) }
    return g;
}

template <int K, int NV, typename T>
__device__ __forceinline__ void run_ops(const PassArgs<T>& a, T (&re)[NV][1 << K],
                                        T (&im)[NV][1 << K], double* gacc, int tid) {
    for (uint32_t o = 0; o < a.n_ops; ++o) {
        const KOp op = a.ops[o];
        const T* m = a.mats[op.slot].v;
        switch (op.type) {
            case OP_U2: d_u2<K, NV, T>(op.a, re, im, m); break;
            case OP_R2: d_r2<K, NV, T>(op.a, re, im, m); break;
            case OP_DIAG: d_diag<K, NV, T>(op.a, re, im, m); break;
            case OP_XFLIP: d_xflip<K, NV, T>(op.a, re, im); break;
            case OP_CNOT: d_cnot<K, NV, T>(op.a, op.b, re, im); break;
            case OP_CZ: d_cz<K, NV, T>(op.a, op.b, re, im); break;
            case OP_GX:
                if constexpr (NV == 2) gacc[op.slot * kBlock + tid] += (double)d_grad<K, OP_GX, T>(op.a, re, im);
                break;
            case OP_GY:
                if constexpr (NV == 2) gacc[op.slot * kBlock + tid] += (double)d_grad<K, OP_GY, T>(op.a, re, im);
                break;
            case OP_GZ:
                if constexpr (NV == 2) gacc[op.slot * kBlock + tid] += (double)d_grad<K, OP_GZ, T>(op.a, re, im);
                break;
            default:
                break;
        }
    }
}

// ---------------------------------------------------------------- lane-split ops
// In the lane-split layout a wave holds 64 >> S cosets and S of the K window
// bits live in lane bits: lane slot 0 is lane bit 5 (S = 1) or 4 (S = 2),
// lane slot 1 is lane bit 5.  Which window bit sits in which register bit or
// lane slot is planned on the host per pass (pos_in / pos_out give the qubit
// of every slot at load and store).  Diagonal ops (phases, CZ, Z gradients)
// act on a lane-resident bit per lane; any other op first gets its bits into
// registers with OP_TPOSE: for each pair of register entries (i, i + 2^r),
// v_permlane{32,16}_swap(a, b) turns (a, b) into (a_lo | b_lo, a_hi | b_hi)
// (lanes with the lane bit 0 | 1), which swaps the roles of register bit r
// and the lane bit, one instruction per dword and no copies.

template <int LB>
__device__ __forceinline__ void tpose32(unsigned& a, unsigned& b) {
    if constexpr (LB == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int LB>
__device__ __forceinline__ void tpose(float& a, float& b) {
    unsigned x = __float_as_uint(a), y = __float_as_uint(b);
    tpose32<LB>(x, y);
    a = __uint_as_float(x);
    b = __uint_as_float(y);
}

template <int LB>
__device__ __forceinline__ void tpose(double& a, double& b) {
    const unsigned long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    unsigned xl = (unsigned)x, xh = (unsigned)(x >> 32), yl = (unsigned)y, yh = (unsigned)(y >> 32);
    tpose32<LB>(xl, yl);
    tpose32<LB>(xh, yh);
    a = __longlong_as_double((long long)(((unsigned long long)xh << 32) | xl));
    b = __longlong_as_double((long long)(((unsigned long long)yh << 32) | yl));
}

template <int LB, int KL, int R, int NV, typename T>
__device__ __forceinline__ void xop_tpose(T (&re)[NV][1 << KL], T (&im)[NV][1 << KL]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << KL); ++i) {
            if (i & (1 << R)) continue;
            const int j = i | (1 << R);
            tpose<LB>(re[v][i], re[v][j]);
            tpose<LB>(im[v][i], im[v][j]);
        }
    }
}

// Phase diag(d0, d1) on a lane-resident bit (hb = this lane's value of it).
template <int KL, int NV, typename T>
__device__ __forceinline__ void xop_diag(T (&re)[NV][1 << KL], T (&im)[NV][1 << KL], const T* m, bool hb) {
    const T pr = hb ? m[6] : m[0], pi = hb ? m[7] : m[1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << KL); ++i) {
            const T ar = re[v][i], ai = im[v][i];
            re[v][i] = pr * ar - pi * ai;
            im[v][i] = pr * ai + pi * ar;
        }
    }
}

// Sign flip of the register entries with (i & MASK) == MASK where `neg` holds (CZ with a lane bit).
template <int KL, int MASK, int NV, typename T>
__device__ __forceinline__ void xop_neg(T (&re)[NV][1 << KL], T (&im)[NV][1 << KL], bool neg) {
    const T sg = neg ? T(-1) : T(1);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int i = 0; i < (1 << KL); ++i) {
            if ((i & MASK) != MASK) continue;
            re[v][i] *= sg;
            im[v][i] *= sg;
        }
    }
}

// Im<lam|Z|psi> for Z on a lane-resident bit: the lanes with the bit set count negatively.
template <int KL, typename T>
__device__ __forceinline__ T xop_gz(T (&re)[2][1 << KL], T (&im)[2][1 << KL], bool hb) {
    T acc = 0;
#pragma unroll
    for (int i = 0; i < (1 << KL); ++i) acc += re[1][i] * im[0][i] - im[1][i] * re[0][i];
    return hb ? -acc : acc;
}

#define VQE_LBIT_CASES(CALL)                                              \
    case 0: if constexpr (KL > 0) { constexpr int B = 0; CALL; } break;   \
    case 1: if constexpr (KL > 1) { constexpr int B = 1; CALL; } break;   \
    case 2: if constexpr (KL > 2) { constexpr int B = 2; CALL; } break;   \
    case 3: if constexpr (KL > 3) { constexpr int B = 3; CALL; } break;   \
    default: break;

// Op loop of the lane-split layout (ops already lowered to physical slots).
template <int KL, int S, int NV, typename T>
__device__ __forceinline__ void run_ops_split(const PassArgs<T>& a, T (&re)[NV][1 << KL], T (&im)[NV][1 << KL],
                                              double* gacc, int tid, int lane) {
    constexpr int LB0 = (S == 1) ? 5 : 4;
    const bool h0 = (lane >> LB0) & 1;
    const bool h1 = (lane >> 5) & 1;
    for (uint32_t o = 0; o < a.n_ops; ++o) {
        const KOp op = a.ops[o];
        const T* m = a.mats[op.slot].v;
        const bool la = op.a >= KL, lb = op.b >= KL;
        const bool ha = (op.a - KL) == 0 ? h0 : h1;
        const bool hbb = (op.b - KL) == 0 ? h0 : h1;
        switch (op.type) {
            case OP_U2: d_u2<KL, NV, T>(op.a, re, im, m); break;
            case OP_R2: d_r2<KL, NV, T>(op.a, re, im, m); break;
            case OP_XFLIP: d_xflip<KL, NV, T>(op.a, re, im); break;
            case OP_CNOT: d_cnot<KL, NV, T>(op.a, op.b, re, im); break;
            case OP_DIAG:
                if (la) xop_diag<KL, NV, T>(re, im, m, ha);
                else d_diag<KL, NV, T>(op.a, re, im, m);
                break;
            case OP_CZ:
                if (la && lb) xop_neg<KL, 0, NV, T>(re, im, ha && hbb);
                else if (la) { switch (op.b) { VQE_LBIT_CASES((xop_neg<KL, (1 << B), NV, T>(re, im, ha))) } }
                else if (lb) { switch (op.a) { VQE_LBIT_CASES((xop_neg<KL, (1 << B), NV, T>(re, im, hbb))) } }
                else d_cz<KL, NV, T>(op.a, op.b, re, im);
                break;
            case OP_TPOSE:
                if (op.b == 0) { switch (op.a) { VQE_LBIT_CASES((xop_tpose<LB0, KL, B, NV, T>(re, im))) } }
                else { if constexpr (S == 2) { switch (op.a) { VQE_LBIT_CASES((xop_tpose<5, KL, B, NV, T>(re, im))) } } }
                break;
            case OP_GX:
                if constexpr (NV == 2) gacc[op.slot * kBlock + tid] += (double)d_grad<KL, OP_GX, T>(op.a, re, im);
                break;
            case OP_GY:
                if constexpr (NV == 2) gacc[op.slot * kBlock + tid] += (double)d_grad<KL, OP_GY, T>(op.a, re, im);
                break;
            case OP_GZ:
                if constexpr (NV == 2)
                    gacc[op.slot * kBlock + tid] +=
                        (double)(la ? xop_gz<KL, T>(re, im, ha) : d_grad<KL, OP_GZ, T>(op.a, re, im));
                break;
            default:
                break;
        }
    }
}

// ---------------------------------------------------------------- window pass
// Loads / stores of one coset (the 2^K amplitudes of a window) to / from
// registers.  `base` is the coset's lowest index; offsets are wave-uniform.
template <typename T, int K, int NV>
struct Coset {
    using V = typename VecOf<T>::type;
    T re[NV][1 << K], im[NV][1 << K];
};

template <typename T, int K>
__device__ __forceinline__ uint64_t pattern_offset(const uint64_t (&bitval)[K], int p) {
    uint64_t off = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (p & (1 << j)) off += bitval[j];
    return off;
}

// Direct mode: every window qubit is >= 6, so consecutive lanes hold
// consecutive cosets at consecutive addresses.  Each thread handles cpt
// cosets: one for one-shot grids (forward passes), a block-contiguous run for
// persistent grids (reverse passes, whose per-block gradient reduction is
// amortised over many cosets).
template <typename T, int K, int NV>
__global__ void __launch_bounds__(kBlock)
window_kernel(const PassArgs<T> a, uint32_t cpt, uint32_t mlog,
              const typename VecOf<T>::type* __restrict__ in0,
              typename VecOf<T>::type* __restrict__ out0,
              const typename VecOf<T>::type* __restrict__ in1,
              typename VecOf<T>::type* __restrict__ out1, double* __restrict__ gpart) {
    using V = typename VecOf<T>::type;
    constexpr int N = 1 << K;
    __shared__ double gacc[NV == 2 ? kInterpGradSlots * kBlock : 1];
    const int tid = threadIdx.x;
    if constexpr (NV == 2) {
        for (uint32_t s = 0; s < a.n_gslots; ++s) gacc[s * kBlock + tid] = 0.0;
    }
    uint64_t bitval[K];
#pragma unroll
    for (int j = 0; j < K; ++j) bitval[j] = 1ull << a.pos[j];
    for (uint32_t it = 0; it < cpt; ++it) {
        // block-contiguous units, then XCD-aware (mlog = log2 of the number
        // of kBlock-coset units)
        const uint64_t blk = xcd_order((uint64_t)blockIdx.x * cpt + it, mlog);
        const uint64_t c = blk * kBlock + tid;
        if (c >= a.n_cosets) break;
        uint64_t base = c;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t low = base & (bitval[j] - 1);
            base = ((base ^ low) << 1) | low;
        }
        T re[NV][N], im[NV][N];
        // Only the coset base lives in VGPRs; the empty asm keeps the store
        // base opaque so the 2^K load addresses are not held across the ops.
        uint64_t sbase = base;
#pragma unroll
        for (int p = 0; p < N; ++p) {
            const uint64_t idx = base + pattern_offset<T, K>(bitval, p);
            const V v0 = in0[idx];
            re[0][p] = v0.x;
            im[0][p] = v0.y;
            if constexpr (NV == 2) {
                const V v1 = in1[idx];
                re[NV - 1][p] = v1.x;
                im[NV - 1][p] = v1.y;
            }
        }
        run_ops<K, NV, T>(a, re, im, gacc, tid);
        asm volatile("" : "+v"(sbase));
#pragma unroll
        for (int p = 0; p < N; ++p) {
            const uint64_t idx = sbase + pattern_offset<T, K>(bitval, p);
            V v0;
            v0.x = re[0][p];
            v0.y = im[0][p];
            out0[idx] = v0;
            if constexpr (NV == 2) {
                V v1;
                v1.x = re[NV - 1][p];
                v1.y = im[NV - 1][p];
                out1[idx] = v1;
            }
        }
    }
    if constexpr (NV == 2) {
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (tid < w)
                for (uint32_t s = 0; s < a.n_gslots; ++s)
                    gacc[s * kBlock + tid] += gacc[s * kBlock + tid + w];
            __syncthreads();
        }
        if (tid < (int)a.n_gslots) gpart[(uint64_t)blockIdx.x * a.n_gslots + tid] = gacc[tid * kBlock];
    }
}

// Lane-split direct mode: a wave holds 64 >> S cosets, the S top window bits
// of each coset spread over lane bits (see run_ops_split).  2^S times fewer
// registers per thread than the plain direct mode, for windows whose full
// coset would not fit the register budget (the reverse pass holds psi and lam).
template <typename T, int K, int S, int NV>
__global__ void __launch_bounds__(kBlock)
window_split_kernel(const PassArgs<T> a, uint32_t cpt, uint32_t mlog,
                    const typename VecOf<T>::type* __restrict__ in0, typename VecOf<T>::type* __restrict__ out0,
                    const typename VecOf<T>::type* __restrict__ in1, typename VecOf<T>::type* __restrict__ out1,
                    double* __restrict__ gpart) {
    using V = typename VecOf<T>::type;
    constexpr int KL = K - S;
    constexpr int N = 1 << KL;
    constexpr int CPW = 64 >> S;               // cosets per wave
    constexpr int PER_BLOCK = kBlock >> S;     // cosets per block and iteration
    __shared__ double gacc[NV == 2 ? kInterpGradSlots * kBlock : 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int sub = (tid >> 6) * CPW + (lane & (CPW - 1));
    if constexpr (NV == 2) {
        for (uint32_t s = 0; s < a.n_gslots; ++s) gacc[s * kBlock + tid] = 0.0;
    }
    uint64_t bitval[K], bv_in[K], bv_out[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bitval[j] = 1ull << a.pos[j];
        bv_in[j] = 1ull << a.pos_in[j];
        bv_out[j] = 1ull << a.pos_out[j];
    }
    // this lane's values of the lane slots, at load and at store
    uint64_t half_in = 0, half_out = 0;
    if constexpr (S == 1) {
        if ((lane >> 5) & 1) half_in += bv_in[KL], half_out += bv_out[KL];
    } else {
        if ((lane >> 4) & 1) half_in += bv_in[KL], half_out += bv_out[KL];
        if ((lane >> 5) & 1) half_in += bv_in[KL + 1], half_out += bv_out[KL + 1];
    }
    for (uint32_t it = 0; it < cpt; ++it) {
        const uint64_t blk = xcd_order((uint64_t)blockIdx.x * cpt + it, mlog);
        const uint64_t c = blk * PER_BLOCK + sub;
        if (c >= a.n_cosets) break;
        uint64_t base = c;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t low = base & (bitval[j] - 1);
            base = ((base ^ low) << 1) | low;
        }
        T re[NV][N], im[NV][N];
        uint64_t sbase = base + half_out;
        base += half_in;
#pragma unroll
        for (int p = 0; p < N; ++p) {
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < KL; ++j)
                if (p & (1 << j)) off += bv_in[j];
            const V v0 = in0[base + off];
            re[0][p] = v0.x;
            im[0][p] = v0.y;
            if constexpr (NV == 2) {
                const V v1 = in1[base + off];
                re[NV - 1][p] = v1.x;
                im[NV - 1][p] = v1.y;
            }
        }
        run_ops_split<KL, S, NV, T>(a, re, im, gacc, tid, lane);
        asm volatile("" : "+v"(sbase));
#pragma unroll
        for (int p = 0; p < N; ++p) {
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < KL; ++j)
                if (p & (1 << j)) off += bv_out[j];
            V v0;
            v0.x = re[0][p];
            v0.y = im[0][p];
            out0[sbase + off] = v0;
            if constexpr (NV == 2) {
                V v1;
                v1.x = re[NV - 1][p];
                v1.y = im[NV - 1][p];
                out1[sbase + off] = v1;
            }
        }
    }
    if constexpr (NV == 2) {
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (tid < w)
                for (uint32_t s = 0; s < a.n_gslots; ++s)
                    gacc[s * kBlock + tid] += gacc[s * kBlock + tid + w];
            __syncthreads();
        }
        if (tid < (int)a.n_gslots) gpart[(uint64_t)blockIdx.x * a.n_gslots + tid] = gacc[tid * kBlock];
    }
}

// LDS-staged mode, for windows that include lane qubits (< 6).  The union U of
// the window bits and the 6 lowest non-window bits always contains bits 0..5,
// so the 2^(K+6) amplitudes of one U-chunk are read with fully coalesced
// wave loads (64 consecutive amplitudes per instruction) into LDS; each lane
// then gathers its coset (its lane bits fixed, window bits varying), runs the
// ops in registers, scatters back and the chunk is stored coalesced.  One
// chunk per wave, one-shot grid.  LDS slots are XOR-swizzled,
// slot(u) = u ^ ((u >> 5) & 31), to spread strided gathers over the banks.
struct LdsMap {
    uint64_t n_chunks;          // 2^(n - K - 6)
    uint32_t upos[kMaxWindow + 6];  // U positions, ascending (upos[j] = j for j < 6)
    uint32_t rank_lane[6];      // rank in U of the j-th lowest non-window bit
    uint32_t rank_win[kMaxWindow];  // rank in U of window bit j
};

__device__ __forceinline__ uint32_t lds_slot(uint32_t u) { return u ^ ((u >> 5) & 31u); }

template <typename T, int K, int NV>
__global__ void __launch_bounds__(kBlock)
window_lds_kernel(const PassArgs<T> a, const LdsMap m, uint32_t cpt, uint32_t mlog,
                  const typename VecOf<T>::type* __restrict__ in0,
                  typename VecOf<T>::type* __restrict__ out0,
                  const typename VecOf<T>::type* __restrict__ in1,
                  typename VecOf<T>::type* __restrict__ out1, double* __restrict__ gpart) {
    using V = typename VecOf<T>::type;
    constexpr int N = 1 << K;
    constexpr int NU = K + 6;
    constexpr int CH = 1 << NU;       // amplitudes per chunk
    constexpr int WAVES = kBlock / 64;
    __shared__ V chunk[WAVES][CH];
    __shared__ double gacc[NV == 2 ? kInterpGradSlots * kBlock : 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    if constexpr (NV == 2) {
        for (uint32_t s = 0; s < a.n_gslots; ++s) gacc[s * kBlock + tid] = 0.0;
    }
    // per-lane union index of the lane's coset (its lane bits placed at their U ranks)
    uint32_t ul = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) ul |= (uint32_t)((lane >> j) & 1) << m.rank_lane[j];
    // Every wave of the block runs the same cpt iterations (uniform barriers).
    for (uint32_t it = 0; it < cpt; ++it) {
        const uint64_t blk = xcd_order((uint64_t)blockIdx.x * cpt + it, mlog);
        const uint64_t ch = blk * WAVES + wv;
        const bool live = ch < m.n_chunks;
        // chunk base: insert zeros at the U positions
        uint64_t cbase = live ? ch : 0;
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const uint64_t low = cbase & ((1ull << m.upos[j]) - 1);
            cbase = ((cbase ^ low) << 1) | low;
        }
        T re[NV][N], im[NV][N];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const V* src = v == 0 ? in0 : in1;
            if (live) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    uint64_t off = 0;
#pragma unroll
                    for (int j = 6; j < NU; ++j)
                        if (i & (1 << (j - 6))) off += 1ull << m.upos[j];
                    chunk[wv][lds_slot((uint32_t)(i * 64 + lane))] = src[cbase + off + lane];
                }
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < N; ++p) {
                uint32_t up = 0;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (p & (1 << k)) up |= 1u << m.rank_win[k];
                const V x = chunk[wv][lds_slot(ul | up)];
                re[v][p] = x.x;
                im[v][p] = x.y;
            }
            __syncthreads();
        }
        if (live) run_ops<K, NV, T>(a, re, im, gacc, tid);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            V* dst = v == 0 ? out0 : out1;
#pragma unroll
            for (int p = 0; p < N; ++p) {
                uint32_t up = 0;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (p & (1 << k)) up |= 1u << m.rank_win[k];
                V x;
                x.x = re[v][p];
                x.y = im[v][p];
                chunk[wv][lds_slot(ul | up)] = x;
            }
            __syncthreads();
            if (live) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    uint64_t off = 0;
#pragma unroll
                    for (int j = 6; j < NU; ++j)
                        if (i & (1 << (j - 6))) off += 1ull << m.upos[j];
                    dst[cbase + off + lane] = chunk[wv][lds_slot((uint32_t)(i * 64 + lane))];
                }
            }
            __syncthreads();
        }
    }
    if constexpr (NV == 2) {
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (tid < w)
                for (uint32_t s = 0; s < a.n_gslots; ++s)
                    gacc[s * kBlock + tid] += gacc[s * kBlock + tid + w];
            __syncthreads();
        }
        if (tid < (int)a.n_gslots) gpart[(uint64_t)blockIdx.x * a.n_gslots + tid] = gacc[tid * kBlock];
    }
}

// Sums a and b over a block of NT threads in a fixed order: butterflies
// within each wave (every lane ends with the same bits, addition being
// commutative), then thread 0 adds the wave totals in wave order.  wsum holds
// 2 NT / 64 doubles of LDS that no thread reads any more; the totals are
// valid in thread 0 only.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* wsum) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int t = threadIdx.x;
    if ((t & 63) == 0) {
        wsum[t >> 6] = a;
        wsum[NT / 64 + (t >> 6)] = b;
    }
    __syncthreads();
    if (t == 0) {
        a = wsum[0];
        b = wsum[NT / 64];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            a += wsum[w];
            b += wsum[NT / 64 + w];
        }
    }
}

// ---------------------------------------------------------------- H psi
// Block = one tile of 2^tb amplitudes at a time (grid-stride over tiles);
// thread t owns local indices r*TPT + t, r < R.
template <typename T, int R, int MODE>
__global__ void __launch_bounds__(kBlock)
hpsi_kernel(int n, int tb, uint32_t tpb, const typename VecOf<T>::type* __restrict__ psi,
            typename VecOf<T>::type* __restrict__ lam, const GroupDesc* __restrict__ groups,
            uint32_t n_groups, const TermDesc<T>* __restrict__ terms, double* __restrict__ part) {
    using V = typename VecOf<T>::type;
    __shared__ double red[2 * kBlock / 64];
    const int tid = threadIdx.x;
    const int tpt = (1 << tb) / R;  // threads per tile
    const uint64_t n_tiles = 1ull << (n - tb);
    double e_acc = 0.0, n_acc = 0.0;
    if (tid < tpt) {
        // block b owns tiles [b'*tpb, (b'+1)*tpb), b' the XCD-aware order of b
        const uint64_t bo = xcd_order(blockIdx.x, log2_pow2(gridDim.x));
        const uint64_t t_end = (bo + 1) * tpb < n_tiles ? (bo + 1) * tpb : n_tiles;
        for (uint64_t tile = bo * tpb; tile < t_end; ++tile) {
            const uint64_t tbase = tile << tb;
            uint32_t loc[R];
            V own[R];
            T ar[R], ai[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                loc[r] = (uint32_t)(r * tpt + tid);
                own[r] = psi[tbase | loc[r]];
                ar[r] = 0;
                ai[r] = 0;
            }
            for (uint32_t g = 0; g < n_groups; ++g) {
                const GroupDesc G = groups[g];
                T wgt = 1;
                if (MODE == 1 && G.x != 0 && G.hbit >= (uint32_t)tb) {
                    if ((tbase >> G.hbit) & 1) continue;
                    wgt = 2;
                }
                T dr[R], di[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    dr[r] = 0;
                    di[r] = 0;
                }
                for (uint32_t t = G.begin; t < G.end; ++t) {
                    const TermDesc<T> tm = terms[t];
                    const uint32_t phi = __popcll(tm.z & tbase) & 1u;
                    const uint32_t zl = (uint32_t)tm.z;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const uint32_t par = (__popc(zl & loc[r]) & 1u) ^ phi;
                        dr[r] += par ? -tm.cre : tm.cre;
                        di[r] += par ? -tm.cim : tm.cim;
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const V pv = (G.x == 0) ? own[r] : psi[(tbase | loc[r]) ^ G.x];
                    const T pr = pv.x, pi = pv.y;
                    ar[r] += wgt * (dr[r] * pr - di[r] * pi);
                    ai[r] += wgt * (dr[r] * pi + di[r] * pr);
                }
            }
            T e_t = 0, n_t = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                e_t += own[r].x * ar[r] + own[r].y * ai[r];
                n_t += own[r].x * own[r].x + own[r].y * own[r].y;
                if (MODE == 0) {
                    V o;
                    o.x = ar[r];
                    o.y = ai[r];
                    lam[tbase | loc[r]] = o;
                }
            }
            e_acc += (double)e_t;
            n_acc += (double)n_t;
        }
    }
    block_sum2<kBlock>(e_acc, n_acc, red);
    if (tid == 0) {
        part[2 * blockIdx.x + 0] = e_acc;
        part[2 * blockIdx.x + 1] = n_acc;
    }
}

// ---------------------------------------------------------------- H psi window pass
// One block per coset at a time (persistent grid, block-contiguous runs of
// cosets in XCD-aware order).  Thread t of kHwThreads holds the window
// patterns j = t + kHwThreads r (r < R): the coset of psi is staged in LDS,
// the lam accumulators stay in registers.  For a group with x inside the
// window the partner psi[b ^ x] is psi_coset[j ^ xl] from LDS.  Per coset the
// block first computes every class coefficient A (its terms' coefficients
// signed by the outside z bits against the coset base) into LDS; per group a
// thread then sums its classes' A, signed by the thread part of their z
// bits, into one bucket per register part, and a Walsh-Hadamard transform of
// the R bucket sums gives D_x for its R patterns.
constexpr int kHwThreads = 1 << kHwThreadBits;  // 16 waves per CU at one block

// (-1)^cnt as a floating-point factor: the sign bit set from the low bit of
// cnt on the bit pattern of 1.0.
__device__ __forceinline__ void parity_sign(uint32_t cnt, double& s) {
    s = __hiloint2double((int)((cnt << 31) | 0x3ff00000u), 0);
}
__device__ __forceinline__ void parity_sign(uint32_t cnt, float& s) { s = __uint_as_float((cnt << 31) | 0x3f800000u); }

// One group of a window pass for the patterns t + kHwThreads r of thread t:
// bucket sums E_u over the classes (A and zt staged in LDS at local index
// j - cbase), D_r = sum_{u in M} (-1)^{popcount(u & r)} E_u (a transform over
// the register bits in M only: buckets outside M are empty, so D_r = D_{r & M}),
// returned in dr (and di); hw_apply then adds D_r psi[(t + kHwThreads r) ^ xl].
// REAL: every folded coefficient is real (a real symmetric H: each term holds
// an even number of Y, so w (-i)^popcount(x&z) = +-w); D is then real and the
// imaginary halves of the class sums, the transform and the update vanish.
template <typename T, int M, bool REAL>
__device__ __forceinline__ void hw_group(const HwGroup& G, uint32_t cbase, uint32_t t,
                                         const typename VecOf<T>::type* A, const uint32_t* zt, T* dr, T* di) {
    using V = typename VecOf<T>::type;
    constexpr int R = 1 << kHwRegBits;
    T er[R], ei[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        if (u & ~M) continue;
        T sr = 0, si = 0;
        uint32_t j = G.cb[u] - cbase;
        const uint32_t e = G.cb[u + 1] - cbase;
        // The class index is uniform; holding a copy in a vector register lets
        // the unrolled LDS reads share one address with immediate offsets.
        uint32_t jv = j;
        asm volatile("" : "+v"(jv));
        for (; j + 4 <= e; j += 4, jv += 4) {
            uint32_t z[4];
            V a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                z[q] = zt[jv + q];
                a[q] = A[jv + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T sg;
                parity_sign((uint32_t)__popc(z[q] & t), sg);
                sr = fma(sg, a[q].x, sr);
                if (!REAL) si = fma(sg, a[q].y, si);
            }
        }
        for (; j < e; ++j, ++jv) {
            T sg;
            parity_sign((uint32_t)__popc(zt[jv] & t), sg);
            const V a = A[jv];
            sr = fma(sg, a.x, sr);
            if (!REAL) si = fma(sg, a.y, si);
        }
        er[u] = sr;
        ei[u] = si;
    }
#pragma unroll
    for (int bit = 1; bit < R; bit <<= 1) {
        if (!(M & bit)) continue;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (!(i & ~M) && !(i & bit)) {
                const T r0 = er[i], r1 = er[i | bit];
                er[i] = r0 + r1;
                er[i | bit] = r0 - r1;
                if (!REAL) {
                    const T i0 = ei[i], i1 = ei[i | bit];
                    ei[i] = i0 + i1;
                    ei[i | bit] = i0 - i1;
                }
            }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        dr[r] = er[r & M];
        if (!REAL) di[r] = ei[r & M];
    }
}

// lam_r += D_r psi[(t + kHwThreads r) ^ xl] for the R patterns of thread t
// (one code path for every register-bit subset of the group's classes).
template <typename T, bool REAL>
__device__ __forceinline__ void hw_apply(const HwGroup& G, uint32_t t, const typename VecOf<T>::type* sp,
                                         const T* dr, const T* di, T* lr, T* li) {
    using V = typename VecOf<T>::type;
    constexpr int R = 1 << kHwRegBits;
    // partner of pattern t + kHwThreads r: byte offset a0 + (r ^ xr) kHwThreads sizeof(V)
    const uint32_t a0 = (t ^ (G.xl & (kHwThreads - 1))) * (uint32_t)sizeof(V);
    const uint32_t xr = G.xl >> kHwThreadBits;
    const char* spb = reinterpret_cast<const char*>(sp);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const V pv = *reinterpret_cast<const V*>(spb + a0 + (r ^ xr) * (uint32_t)(kHwThreads * sizeof(V)));
        lr[r] = fma(dr[r], pv.x, lr[r]);
        li[r] = fma(dr[r], pv.y, li[r]);
        if (!REAL) {
            lr[r] = fma(-di[r], pv.y, lr[r]);
            li[r] = fma(di[r], pv.x, li[r]);
        }
    }
}

// EONLY: the energy-only form of the grouped expectation (eq. 7).  No lam is
// read or written: each pass adds Re sum_b conj(psi_b) (H_w psi)_b over its
// own groups H_w to per-block partials, the first pass also <psi|psi>.
// The pass for one block: cosets unit(0), ..., unit(count - 1) while below n_cosets;
// after the last pass (or every energy-only pass) the block's energy and
// norm partials go to *e_out and *n_out.
template <typename T, bool EONLY, bool REAL, typename Unit>
__device__ __forceinline__ void hwin_body(const HwDesc& w, uint64_t n_cosets, uint32_t count, Unit unit,
                                          const typename VecOf<T>::type* __restrict__ psi,
                                          typename VecOf<T>::type* __restrict__ lam,
                                          const HwGroup* __restrict__ groups, const HwClass* __restrict__ classes,
                                          const HwTerm<T>* __restrict__ terms, int first, int last,
                                          double* e_out, double* n_out) {
    using V = typename VecOf<T>::type;
    constexpr int R = 1 << kHwRegBits;
    constexpr int TB = kHwThreadBits;
    // One LDS block, the small tables first so that their addresses fit the
    // immediate offsets of LDS reads: the class coefficients of the current
    // coset (after the last coset, the block reduction), their thread-part z
    // bits, then the psi coset.
    constexpr size_t kTabBytes = kHwMaxClasses * sizeof(V) > 2 * (kHwThreads / 64) * sizeof(double)
                                     ? kHwMaxClasses * sizeof(V)
                                     : 2 * (kHwThreads / 64) * sizeof(double);
    constexpr size_t kZtOff = kTabBytes, kSpOff = kTabBytes + kHwMaxClasses * sizeof(uint32_t);
    static_assert(kSpOff % 16 == 0, "psi coset alignment");
    __shared__ __align__(16) unsigned char lds[kSpOff + (1 << kHwBits) * sizeof(V)];
    V* A = reinterpret_cast<V*>(lds);
    double* red = reinterpret_cast<double*>(lds);
    uint32_t* zt = reinterpret_cast<uint32_t*>(lds + kZtOff);
    V* sp = reinterpret_cast<V*>(lds + kSpOff);
    const int t = threadIdx.x;
    const uint32_t nc = w.c_end - w.c_begin;
    uint64_t bitval[kHwBits];
#pragma unroll
    for (int k = 0; k < kHwBits; ++k) bitval[k] = 1ull << w.pos[k];
    uint64_t off_t = 0;
#pragma unroll
    for (int k = 0; k < TB; ++k)
        if ((t >> k) & 1) off_t += bitval[k];
    double e_acc = 0.0, n_acc = 0.0;
    for (uint32_t it = 0; it < count; ++it) {
        const uint64_t c = unit(it);
        if (c >= n_cosets) break;
        uint64_t base = c;
#pragma unroll
        for (int k = 0; k < kHwBits; ++k) {
            const uint64_t low = base & (bitval[k] - 1);
            base = ((base ^ low) << 1) | low;
        }
        auto addr = [&](int r) {
            uint64_t idx = base + off_t;
#pragma unroll
            for (int k = 0; k < kHwRegBits; ++k)
                if ((r >> k) & 1) idx += bitval[TB + k];
            return idx;
        };
        // All loads of the coset are issued before the first use waits.
        V ps[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ps[r] = psi[addr(r)];
        T lr[R], li[R];
        if (first || EONLY) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                lr[r] = 0;
                li[r] = 0;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const V l = lam[addr(r)];
                lr[r] = l.x;
                li[r] = l.y;
            }
        }
        if ((uint32_t)t < nc) {
            const HwClass C = classes[w.c_begin + t];
            T ar = 0, ai = 0;
            for (uint32_t k = C.k_begin; k < C.k_end; ++k) {
                const HwTerm<T> tm = terms[k];
                T sg;
                parity_sign((uint32_t)__popcll(tm.zo & base), sg);
                ar = fma(sg, tm.cre, ar);
                if (!REAL) ai = fma(sg, tm.cim, ai);
            }
            V a;
            a.x = ar;
            a.y = ai;
            A[t] = a;
            zt[t] = C.zt;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) sp[t + kHwThreads * r] = ps[r];
        __syncthreads();
        for (uint32_t g = w.g_begin; g < w.g_end; ++g) {
            const HwGroup& G = groups[g];
            static_assert(kHwRegBits == 3, "one case per register-bit subset");
            T dr[R], di[R];
            switch (G.zrm) {
                case 0: hw_group<T, 0, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 1: hw_group<T, 1, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 2: hw_group<T, 2, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 3: hw_group<T, 3, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 4: hw_group<T, 4, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 5: hw_group<T, 5, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                case 6: hw_group<T, 6, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
                default: hw_group<T, 7, REAL>(G, w.c_begin, t, A, zt, dr, di); break;
            }
            hw_apply<T, REAL>(G, t, sp, dr, di, lr, li);
        }
        T e_t = 0, n_t = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!EONLY) {
                V o;
                o.x = lr[r];
                o.y = li[r];
                lam[addr(r)] = o;
            }
            const V pv = sp[t + kHwThreads * r];
            e_t += pv.x * lr[r] + pv.y * li[r];
            n_t += pv.x * pv.x + pv.y * pv.y;
        }
        if (EONLY || last) e_acc += (double)e_t;
        if (EONLY ? first : last) n_acc += (double)n_t;
        __syncthreads();  // the next coset overwrites both LDS tables
    }
    if (!EONLY && !last) return;
    block_sum2<kHwThreads>(e_acc, n_acc, red);  // the loop's last barrier freed the class table
    if (t == 0) {
        *e_out = e_acc;
        *n_out = n_acc;
    }
}

template <typename T, bool EONLY, bool REAL>
__global__ void __launch_bounds__(kHwThreads)
hwin_kernel(const HwDesc w, uint64_t n_cosets, uint32_t cpt, uint32_t mlog,
            const typename VecOf<T>::type* __restrict__ psi, typename VecOf<T>::type* __restrict__ lam,
            const HwGroup* __restrict__ groups, const HwClass* __restrict__ classes,
            const HwTerm<T>* __restrict__ terms, int first, int last, double* __restrict__ part) {
    const uint64_t b = blockIdx.x;
    hwin_body<T, EONLY, REAL>(
        w, n_cosets, cpt, [=](uint32_t it) { return xcd_unit(b, it, cpt, mlog); }, psi, lam, groups, classes, terms,
        first, last, part + 2 * b, part + 2 * b + 1);
}

// One window pass of lam = H psi for every item of a batch: descriptor i
// owns blocks [blk_begin, blk_begin + n_blk), block blk takes cosets blk,
// blk + n_blk, ... of its item.
template <typename T, bool REAL>
__global__ void __launch_bounds__(kHwThreads)
hwin_batch_kernel(const HwItem* __restrict__ d, uint32_t n_desc, double* __restrict__ part) {
    using V = typename VecOf<T>::type;
    uint32_t lo = 0, hi = n_desc;
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (d[m].blk_begin <= blockIdx.x) lo = m;
        else hi = m;
    }
    const HwItem& x = d[lo];
    const uint64_t blk = blockIdx.x - x.blk_begin, nb = x.n_blk;
    const uint32_t count = (uint32_t)((x.n_cosets - blk + nb - 1) / nb);
    hwin_body<T, false, REAL>(
        x.w, x.n_cosets, count, [=](uint32_t it) { return blk + (uint64_t)it * nb; }, (const V*)x.psi, (V*)x.lam,
        x.groups,
        x.classes, (const HwTerm<T>*)x.terms, (int)x.first, (int)x.last, part + x.part_off + blk,
        part + x.part_off + nb + blk);
}

// ---------------------------------------------------------------- one term
// x != 0: visit each pair (b, b^x) once (bit h of b clear) and add
// 2 Re(conj(psi_b) c (-1)^{z.b} psi_{b^x}); x = 0: sum (-1)^{z.b} |psi_b|^2.
// c = (-i)^popcount(x&z).
template <typename T>
__global__ void __launch_bounds__(kBlock)
expect_term_kernel(int n, uint32_t cpt, const typename VecOf<T>::type* __restrict__ psi, uint64_t x, uint64_t z,
                   uint32_t hbit, T cre, T cim, double* __restrict__ part) {
    using V = typename VecOf<T>::type;
    __shared__ double red[2 * kBlock / 64];
    const int tid = threadIdx.x;
    const uint64_t count = (x == 0) ? (1ull << n) : (1ull << (n - 1));
    const uint64_t hmask = (x == 0) ? 0 : ((1ull << hbit) - 1);
    double v_acc = 0.0, n_acc = 0.0;
    const uint64_t i0 = xcd_order(blockIdx.x, log2_pow2(gridDim.x)) * kBlock * cpt + tid;
    for (uint32_t it = 0; it < cpt; ++it) {
        const uint64_t i = i0 + (uint64_t)it * kBlock;
        if (i >= count) break;
        uint64_t b = i;
        if (x != 0) {
            const uint64_t low = i & hmask;
            b = ((i ^ low) << 1) | low;
        }
        const V p = psi[b];
        const T sgn = (__popcll(z & b) & 1) ? T(-1) : T(1);
        if (x == 0) {
            const T m = p.x * p.x + p.y * p.y;
            v_acc += (double)(sgn * m);
            n_acc += (double)m;
        } else {
            const V q = psi[b ^ x];
            // conj(p) * (cre + i cim) * q
            const T qr = cre * q.x - cim * q.y, qi = cre * q.y + cim * q.x;
            v_acc += 2.0 * (double)(sgn * (p.x * qr + p.y * qi));
            n_acc += (double)(p.x * p.x + p.y * p.y + q.x * q.x + q.y * q.y);
        }
    }
    block_sum2<kBlock>(v_acc, n_acc, red);
    if (tid == 0) {
        part[2 * blockIdx.x + 0] = v_acc;
        part[2 * blockIdx.x + 1] = n_acc;
    }
}

// ---------------------------------------------------------------- misc
template <typename V>
__global__ void __launch_bounds__(kBlock) set_basis_kernel(V* __restrict__ psi, uint64_t dim, uint64_t b) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += stride) {
        V v;
        v.x = (i == b) ? 1 : 0;
        v.y = 0;
        psi[i] = v;
    }
}

__global__ void __launch_bounds__(kBlock) zero_kernel(double* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

template <typename V>
__global__ void __launch_bounds__(kBlock) copy_kernel(const V* __restrict__ src, V* __restrict__ dst, uint64_t dim) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < dim; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(kBlock)
reduce_kernel(const double* __restrict__ part, uint32_t nblocks, uint32_t nslots,
              const int32_t* __restrict__ map, double* __restrict__ out, int accumulate) {
    __shared__ double red[2 * kBlock / 64];
    const int tid = threadIdx.x;
    const uint32_t s = blockIdx.x;
    double acc = 0.0, unused = 0.0;
    for (uint32_t i = tid; i < nblocks; i += kBlock) acc += part[(uint64_t)i * nslots + s];
    block_sum2<kBlock>(acc, unused, red);
    if (tid == 0) {
        const int idx = map ? map[s] : (int)s;
        out[idx] = accumulate > 0 ? out[idx] + acc : accumulate < 0 ? out[idx] - acc : acc;
    }
}

// out[0] = sums[0] / sums[1] (the energy of eq. 7), out[1] = sums[1] (the norm).
__global__ void energy_ratio_kernel(const double* __restrict__ sums, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        const double e = sums[0], nrm = sums[1];
        out[0] = e / nrm;
        out[1] = nrm;
    }
}

uint32_t grid_for(uint64_t items) {
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (uint64_t)kMaxBlocks) b = kMaxBlocks;
    return (uint32_t)b;
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_set_basis(int dtype, void* psi, uint64_t dim, uint64_t b, hipStream_t st) {
    const uint32_t g = grid_for(dim);
    if (dtype == VQE_C64)
        hipLaunchKernelGGL(set_basis_kernel<float2>, dim3(g), dim3(kBlock), 0, st, (float2*)psi, dim, b);
    else
        hipLaunchKernelGGL(set_basis_kernel<double2>, dim3(g), dim3(kBlock), 0, st, (double2*)psi, dim, b);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_copy(int dtype, const void* src, void* dst, uint64_t dim, hipStream_t st) {
    const uint32_t g = grid_for(dim);
    if (dtype == VQE_C64)
        hipLaunchKernelGGL(copy_kernel<float2>, dim3(g), dim3(kBlock), 0, st, (const float2*)src, (float2*)dst, dim);
    else
        hipLaunchKernelGGL(copy_kernel<double2>, dim3(g), dim3(kBlock), 0, st, (const double2*)src, (double2*)dst, dim);
    return hipGetLastError();
}

// Launch shape of a window pass.  LDS mode for forward passes whose window
// includes a lane qubit (< 6), when the state has at least K + 6 qubits.
struct WinShape {
    bool lds;
    int split;  // lane-split bits S (0: plain direct or LDS mode)
    LdsMap m;
    uint32_t cpt, grid, mlog;
};



// Reverse passes (with per-block gradient partials) use a persistent grid of
// at most kRevBlocks blocks; forward passes a one-shot grid.
constexpr uint64_t kRevBlocks = 2048;

void grid_for_units(uint64_t units, bool persistent, WinShape& w) {
    w.mlog = log2_pow2(units);
    if (persistent) {
        const uint64_t g = units < kRevBlocks ? units : kRevBlocks;
        w.grid = (uint32_t)(g ? g : 1);
        w.cpt = (uint32_t)((units + w.grid - 1) / w.grid);
    } else {
        w.grid = (uint32_t)(units ? units : 1);
        w.cpt = 1;
    }
}

template <typename T>
WinShape window_shape(const PassArgs<T>& a, int n, bool with_partials) {
    WinShape w{};
    const int K = (int)a.K;
    w.split = (int)a.split;
    bool low = false;
    for (int j = 0; j < K; ++j) low |= a.pos[j] < 6;
    // Measured on MI355X: staging pays for forward passes (one vector) but
    // not for reverse passes, whose two-vector chunks and barriers cost more
    // than the partly coalesced direct loads they replace.
    if (low && n >= K + 6 && !with_partials && !w.split) {
        w.lds = true;
        uint64_t wmask = 0;
        for (int j = 0; j < K; ++j) wmask |= 1ull << a.pos[j];
        uint64_t umask = wmask;
        int got = 0;
        for (int q = 0; q < n && got < 6; ++q)
            if (!((wmask >> q) & 1)) {
                umask |= 1ull << q;
                ++got;
            }
        int r = 0, lj = 0;
        for (int q = 0; q < n; ++q) {
            if (!((umask >> q) & 1)) continue;
            w.m.upos[r] = (uint32_t)q;
            if ((wmask >> q) & 1) {
                for (int j = 0; j < K; ++j)
                    if ((int)a.pos[j] == q) w.m.rank_win[j] = (uint32_t)r;
            } else {
                w.m.rank_lane[lj++] = (uint32_t)r;
            }
            ++r;
        }
        w.m.n_chunks = 1ull << (n - K - 6);
        const uint64_t per_block = kBlock / 64;
        grid_for_units((w.m.n_chunks + per_block - 1) / per_block, with_partials, w);
        return w;
    }
    w.lds = false;
    const uint64_t per_unit = (uint64_t)kBlock >> w.split;
    grid_for_units((a.n_cosets + per_unit - 1) / per_unit, with_partials, w);
    return w;
}

template <typename T>
uint32_t window_blocks(const PassArgs<T>& a, int n, bool with_partials) {
    return window_shape<T>(a, n, with_partials).grid;
}

template <typename T, int NV>
hipError_t launch_window(const PassArgs<T>& a, int n, const void* in0, void* out0, const void* in1, void* out1,
                         double* gpart, hipStream_t st) {
    using V = typename VecOf<T>::type;
    const WinShape w = window_shape<T>(a, n, NV == 2);
    const V* i0 = (const V*)in0;
    V* o0 = (V*)out0;
    const V* i1 = (const V*)in1;
    V* o1 = (V*)out1;
#define VQE_WIN(KK)                                                                                      \
    case KK:                                                                                             \
        if (w.split == 1) {                                                                              \
            if constexpr (KK == 5)                                                                       \
                hipLaunchKernelGGL((window_split_kernel<T, KK, 1, NV>), dim3(w.grid), dim3(kBlock), 0, st, \
                                   a, w.cpt, w.mlog, i0, o0, i1, o1, gpart);               \
        } else if (w.split == 2) {                                                                       \
            if constexpr (KK == 5)                                                                       \
                hipLaunchKernelGGL((window_split_kernel<T, KK, 2, NV>), dim3(w.grid), dim3(kBlock), 0, st, \
                                   a, w.cpt, w.mlog, i0, o0, i1, o1, gpart);               \
        } else if (w.lds)                                                                                \
            hipLaunchKernelGGL((window_lds_kernel<T, KK, NV>), dim3(w.grid), dim3(kBlock), 0, st, a, w.m, \
                               w.cpt, w.mlog, i0, o0, i1, o1, gpart);                      \
        else                                                                                             \
            hipLaunchKernelGGL((window_kernel<T, KK, NV>), dim3(w.grid), dim3(kBlock), 0, st, a, w.cpt, \
                               w.mlog, i0, o0, i1, o1, gpart);                             \
        break;
    switch (a.K) {
        VQE_WIN(1)
        VQE_WIN(2)
        VQE_WIN(3)
        VQE_WIN(4)
        VQE_WIN(5)
        default:
            return hipErrorInvalidValue;
    }
#undef VQE_WIN
    return hipGetLastError();
}

template <typename T>
hipError_t launch_window_fwd(const PassArgs<T>& a, int n, const void* in, void* out, hipStream_t st) {
    return launch_window<T, 1>(a, n, in, out, nullptr, nullptr, nullptr, st);
}

template <typename T>
hipError_t launch_window_rev(const PassArgs<T>& a, int n, const void* psi_in, void* psi_out, const void* lam_in,
                             void* lam_out, double* gpart, uint32_t* nblocks, hipStream_t st) {
    *nblocks = window_blocks<T>(a, n, true);
    return launch_window<T, 2>(a, n, psi_in, psi_out, lam_in, lam_out, gpart, st);
}

hipError_t launch_window_jit(void* fn, const JitArgs& a, int S, const void* mats, bool reverse, const void* in0,
                             void* out0, const void* in1, void* out1, double* gpart, uint32_t* nblocks,
                             hipStream_t st) {
    WinShape w{};
    const uint64_t per_unit = (uint64_t)kBlock >> S;
    grid_for_units((a.n_cosets + per_unit - 1) / per_unit, reverse, w);
    if (nblocks) *nblocks = w.grid;
    JitArgs ka = a;
    uint32_t cpt = w.cpt, mlog = w.mlog;
    void* params[] = {&ka, (void*)&mats, &cpt, &mlog, (void*)&in0, (void*)&out0,
                      (void*)&in1, (void*)&out1, (void*)&gpart};
    return hipModuleLaunchKernel((hipFunction_t)fn, w.grid, 1, 1, kBlock, 1, 1, 0, st, params, nullptr);
}


template <typename T>
hipError_t launch_hwin(int n, const HwDesc& w, const void* psi, void* lam, const HwGroup* groups,
                       const HwClass* classes, const HwTerm<T>* terms, bool real, bool first, bool last,
                       double* part, uint32_t* nblocks, hipStream_t st) {
    using V = typename VecOf<T>::type;
    if (n < kHwBits || w.c_end < w.c_begin || w.c_end - w.c_begin > (uint32_t)kHwMaxClasses)
        return hipErrorInvalidValue;
    WinShape ws{};
    grid_for_units(1ull << (n - kHwBits), true, ws);
    *nblocks = ws.grid;
#define VQE_HWIN(EO, RE)                                                                                      \
    hipLaunchKernelGGL((hwin_kernel<T, EO, RE>), dim3(ws.grid), dim3(kHwThreads), 0, st, w, 1ull << (n - kHwBits), \
                       ws.cpt, ws.mlog, (const V*)psi, (V*)lam, groups, classes, terms, first ? 1 : 0, last ? 1 : 0, \
                       part)
    if (lam) {
        if (real) VQE_HWIN(false, true); else VQE_HWIN(false, false);
    } else {
        if (real) VQE_HWIN(true, true); else VQE_HWIN(true, false);
    }
#undef VQE_HWIN
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hwin_batch(const HwItem* d, uint32_t n_desc, uint32_t grid, bool real, double* part,
                             hipStream_t st) {
    if (real)
        hipLaunchKernelGGL((hwin_batch_kernel<T, true>), dim3(grid), dim3(kHwThreads), 0, st, d, n_desc, part);
    else
        hipLaunchKernelGGL((hwin_batch_kernel<T, false>), dim3(grid), dim3(kHwThreads), 0, st, d, n_desc, part);
    return hipGetLastError();
}

uint32_t hpsi_blocks(int n, uint32_t max_blocks) {
    const int tb = n < kTileBits ? n : kTileBits;
    const uint64_t n_tiles = 1ull << (n - tb);
    uint32_t tpb = 1;
    while ((n_tiles + tpb - 1) / tpb > (uint64_t)max_blocks) tpb *= 2;
    return (uint32_t)((n_tiles + tpb - 1) / tpb);
}

template <typename T>
hipError_t launch_hpsi(int n, const void* psi, void* lam, const GroupDesc* groups, uint32_t n_groups,
                       const TermDesc<T>* terms, int mode, uint32_t max_blocks, double* part, uint32_t* nblocks,
                       hipStream_t st) {
    using V = typename VecOf<T>::type;
    const int tb = n < kTileBits ? n : kTileBits;
    const uint64_t n_tiles = 1ull << (n - tb);
    if (max_blocks < 1) return hipErrorInvalidValue;
    uint32_t tpb = 1;
    while ((n_tiles + tpb - 1) / tpb > (uint64_t)max_blocks) tpb *= 2;
    const uint32_t g = (uint32_t)((n_tiles + tpb - 1) / tpb);
    *nblocks = g;
    const int tile = 1 << tb;
    const int R = tile >= 4 * kBlock ? 4 : (tile >= 2 * kBlock ? 2 : 1);
    const V* p = (const V*)psi;
    V* l = (V*)lam;
#define VQE_HPSI(RR, MM) \
    hipLaunchKernelGGL((hpsi_kernel<T, RR, MM>), dim3(g), dim3(kBlock), 0, st, n, tb, tpb, p, l, groups, n_groups, terms, part)
    if (mode == 0) {
        if (R == 4) VQE_HPSI(4, 0); else if (R == 2) VQE_HPSI(2, 0); else VQE_HPSI(1, 0);
    } else {
        if (R == 4) VQE_HPSI(4, 1); else if (R == 2) VQE_HPSI(2, 1); else VQE_HPSI(1, 1);
    }
#undef VQE_HPSI
    return hipGetLastError();
}

template <typename T>
hipError_t launch_expect_term(int n, const void* psi, uint64_t x, uint64_t z, double* part,
                              uint32_t* nblocks, hipStream_t st) {
    using V = typename VecOf<T>::type;
    const uint64_t count = (x == 0) ? (1ull << n) : (1ull << (n - 1));
    uint32_t cpt = 1;
    while ((count + (uint64_t)kBlock * cpt - 1) / ((uint64_t)kBlock * cpt) > (uint64_t)kMaxPartBlocks) cpt *= 2;
    const uint32_t g = (uint32_t)((count + (uint64_t)kBlock * cpt - 1) / ((uint64_t)kBlock * cpt));
    *nblocks = g;
    uint32_t hbit = 0;
    if (x != 0) hbit = 63 - __builtin_clzll(x);
    const int y = __builtin_popcountll(x & z) & 3;
    // (-i)^y
    const T cre = (y == 0) ? T(1) : (y == 2 ? T(-1) : T(0));
    const T cim = (y == 1) ? T(-1) : (y == 3 ? T(1) : T(0));
    hipLaunchKernelGGL(expect_term_kernel<T>, dim3(g), dim3(kBlock), 0, st, n, cpt, (const V*)psi, x, z, hbit, cre, cim, part);
    return hipGetLastError();
}

uint32_t hwin_blocks(int n) {
    WinShape ws{};
    grid_for_units(n >= kHwBits ? 1ull << (n - kHwBits) : 1, true, ws);
    return ws.grid;
}

hipError_t launch_energy_ratio(const double* sums, double* out, hipStream_t st) {
    hipLaunchKernelGGL(energy_ratio_kernel, dim3(1), dim3(64), 0, st, sums, out);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* part, uint32_t nblocks, uint32_t nslots, const int32_t* map, double* out,
                         int accumulate, hipStream_t st) {
    if (nslots == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(nslots), dim3(kBlock), 0, st, part, nblocks, nslots, map, out, accumulate);
    return hipGetLastError();
}

template hipError_t launch_window_fwd<float>(const PassArgs<float>&, int, const void*, void*, hipStream_t);
template hipError_t launch_window_fwd<double>(const PassArgs<double>&, int, const void*, void*, hipStream_t);
template hipError_t launch_window_rev<float>(const PassArgs<float>&, int, const void*, void*, const void*, void*, double*, uint32_t*, hipStream_t);
template hipError_t launch_window_rev<double>(const PassArgs<double>&, int, const void*, void*, const void*, void*, double*, uint32_t*, hipStream_t);
template hipError_t launch_hwin<float>(int, const HwDesc&, const void*, void*, const HwGroup*, const HwClass*,
                                       const HwTerm<float>*, bool, bool, bool, double*, uint32_t*, hipStream_t);
template hipError_t launch_hwin<double>(int, const HwDesc&, const void*, void*, const HwGroup*, const HwClass*,
                                        const HwTerm<double>*, bool, bool, bool, double*, uint32_t*, hipStream_t);
template hipError_t launch_hwin_batch<float>(const HwItem*, uint32_t, uint32_t, bool, double*, hipStream_t);
template hipError_t launch_hwin_batch<double>(const HwItem*, uint32_t, uint32_t, bool, double*, hipStream_t);
template hipError_t launch_hpsi<float>(int, const void*, void*, const GroupDesc*, uint32_t, const TermDesc<float>*, int, uint32_t, double*, uint32_t*, hipStream_t);
template hipError_t launch_hpsi<double>(int, const void*, void*, const GroupDesc*, uint32_t, const TermDesc<double>*, int, uint32_t, double*, uint32_t*, hipStream_t);
template hipError_t launch_expect_term<float>(int, const void*, uint64_t, uint64_t, double*, uint32_t*, hipStream_t);
template hipError_t launch_expect_term<double>(int, const void*, uint64_t, uint64_t, double*, uint32_t*, hipStream_t);

}  // namespace vqe
