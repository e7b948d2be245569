// Batched evaluations of many independent requests.
//
// Small states: one workgroup evaluates one request (energy and
// adjoint gradient of psi(theta) = U(theta)|0...0>, eqs. 6-7) with the whole
// state held in LDS.  psi and lam = H psi both live in LDS (2 x 2^n
// amplitudes, n <= 13 for complex64, n <= 12 for complex128), so a request
// touches HBM only for its gate table, matrices and results.  Many requests
// of different circuits and Hamiltonians share one launch (grid = requests).
//
// Per request, in order: psi = |0>; every gate applied in turn (one LDS sweep
// and barrier per gate; excitation gates as rotations between two basis
// patterns); lam[b] = sum_x psi[b^x] sum_z c_z (-1)^popcount(z&b)
// with the energy and norm reduced over the block in a fixed tree; then the
// gates in reverse: for a parameterised gate, g += Im<lam|G|psi> reduced in
// the same fixed tree, followed by un-applying the gate (U^dagger = conj
// transpose, exact) from psi and lam.  The thread -> amplitude map and the
// reduction order depend only on n, so a request's bits do not depend on the
// other requests of the batch.
#include "vqe_internal.h"

namespace vqe {
namespace {

template <typename T> struct VecB;
template <> struct VecB<float> { using type = float2; };
template <> struct VecB<double> { using type = double2; };

constexpr int kBT = 1024;  // threads per request

__device__ __forceinline__ uint32_t ins0(uint32_t k, uint32_t q) {
    const uint32_t low = k & ((1u << q) - 1);
    return ((k ^ low) << 1) | low;
}

// Block sum of NT threads in a fixed order: butterflies within each wave
// (every lane ends with the same bits, addition being commutative), then the
// wave totals in wave order; every thread gets the total.  red holds NT / 64
// doubles of LDS.
template <int NT>
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int t = threadIdx.x;
    __syncthreads();  // earlier readers of red are done
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r += red[w];
    return r;
}

// Applies gate g (or its adjoint) to the 2^n amplitudes s[] in LDS with NT
// threads, then waits at a block barrier.
template <int NT, typename T>
__device__ void apply_gate(typename VecB<T>::type* s, int n, const BatchGate& g, const T* m, bool dag) {
    using V = typename VecB<T>::type;
    const int t = threadIdx.x;
    if (g.type == OP_CNOT || g.type == OP_CZ) {
        const uint32_t a = g.q0, b = g.q1;
        const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        const uint32_t cnt = 1u << (n - 2);
        for (uint32_t k = t; k < cnt; k += NT) {
            const uint32_t i = ins0(ins0(k, lo), hi) | (1u << a);  // control (or first) bit set
            if (g.type == OP_CNOT) {
                const uint32_t j = i | (1u << b);
                const V x = s[i];
                s[i] = s[j];
                s[j] = x;
            } else {
                const uint32_t j = i | (1u << b);
                V x = s[j];
                x.x = -x.x;
                x.y = -x.y;
                s[j] = x;
            }
        }
    } else if (g.type == OP_PAIR2) {
        // rotation between the basis patterns A = pa and B = pb on the bits pa | pb
        T u0r = m[0], u1r = m[2], u2r = m[4], u3r = m[6];
        if (dag) {
            const T t = u1r;
            u1r = u2r;
            u2r = t;
        }
        const uint32_t M = (uint32_t)g.pa | g.pb, X = (uint32_t)g.pa ^ g.pb;
        for (uint32_t i = t; i < (1u << n); i += NT) {
            if ((i & M) != g.pa) continue;
            const uint32_t j = i ^ X;
            const V x = s[i], y = s[j];
            V o0, o1;
            o0.x = u0r * x.x + u1r * y.x;
            o0.y = u0r * x.y + u1r * y.y;
            o1.x = u2r * x.x + u3r * y.x;
            o1.y = u2r * x.y + u3r * y.y;
            s[i] = o0;
            s[j] = o1;
        }
    } else if (g.type == OP_XFLIP) {
        const uint32_t cnt = 1u << (n - 1);
        for (uint32_t k = t; k < cnt; k += NT) {
            const uint32_t i = ins0(k, g.q0), j = i | (1u << g.q0);
            const V x = s[i];
            s[i] = s[j];
            s[j] = x;
        }
    } else {
        // general 2x2 (U or, for dag, conj(U)^T)
        T u0r = m[0], u0i = m[1], u1r = m[2], u1i = m[3], u2r = m[4], u2i = m[5], u3r = m[6], u3i = m[7];
        if (dag) {
            const T a0r = u0r, a0i = -u0i, a1r = u2r, a1i = -u2i, a2r = u1r, a2i = -u1i, a3r = u3r, a3i = -u3i;
            u0r = a0r; u0i = a0i; u1r = a1r; u1i = a1i; u2r = a2r; u2i = a2i; u3r = a3r; u3i = a3i;
        }
        const uint32_t cnt = 1u << (n - 1);
        for (uint32_t k = t; k < cnt; k += NT) {
            const uint32_t i = ins0(k, g.q0), j = i | (1u << g.q0);
            const V x = s[i], y = s[j];
            V o0, o1;
            o0.x = u0r * x.x - u0i * x.y + u1r * y.x - u1i * y.y;
            o0.y = u0r * x.y + u0i * x.x + u1r * y.y + u1i * y.x;
            o1.x = u2r * x.x - u2i * x.y + u3r * y.x - u3i * y.y;
            o1.y = u2r * x.y + u2i * x.x + u3r * y.y + u3i * y.x;
            s[i] = o0;
            s[j] = o1;
        }
    }
    __syncthreads();
}

// This thread's share of the gradient term of parameterised gate g over the
// 2^n amplitudes of psi and lam in LDS (g.gen: OP_GX / OP_GY / OP_GZ give
// Im<lam| P |psi>-type sums on bit q0, OP_GPAIR2 the pair form
// Re(conj(lam_B) psi_A) - Re(conj(lam_A) psi_B) over the pattern pairs).
template <int NT, typename T>
__device__ T grad_part(const typename VecB<T>::type* psi, const typename VecB<T>::type* lam, int n,
                       const BatchGate& g) {
    using V = typename VecB<T>::type;
    const int t = threadIdx.x;
    T acc = 0;
    if (g.gen == OP_GPAIR2) {
        const uint32_t M = (uint32_t)g.pa | g.pb, X = (uint32_t)g.pa ^ g.pb;
        for (uint32_t i = t; i < (1u << n); i += NT) {
            if ((i & M) != g.pa) continue;
            const uint32_t j = i ^ X;
            const V pa = psi[i], pb = psi[j], la = lam[i], lb = lam[j];
            acc += (lb.x * pa.x + lb.y * pa.y) - (la.x * pb.x + la.y * pb.y);
        }
        return acc;
    }
    const uint32_t q = g.q0;
    const uint32_t cnt = 1u << (n - 1);
    for (uint32_t k = t; k < cnt; k += NT) {
        const uint32_t i = ins0(k, q), j = i | (1u << q);
        const V p0 = psi[i], p1 = psi[j], l0 = lam[i], l1 = lam[j];
        if (g.gen == OP_GZ)
            acc += (l0.x * p0.y - l0.y * p0.x) - (l1.x * p1.y - l1.y * p1.x);
        else if (g.gen == OP_GY)
            acc += (l1.x * p0.x + l1.y * p0.y) - (l0.x * p1.x + l0.y * p1.y);
        else
            acc += (l0.x * p1.y - l0.y * p1.x) + (l1.x * p0.y - l1.y * p0.x);
    }
    return acc;
}

template <typename T>
__global__ void __launch_bounds__(kBT)
batch_kernel(const BatchDesc<T>* __restrict__ items, const BatchGate* __restrict__ gates,
             const Mat2<T>* __restrict__ mats, double* __restrict__ out) {
    using V = typename VecB<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kBT / 64];
    const BatchDesc<T> d = items[blockIdx.x];
    const int n = d.n;
    const uint32_t dim = 1u << n;
    V* psi = reinterpret_cast<V*>(smem);
    V* lam = psi + dim;
    const int t = threadIdx.x;
    double* o = out + d.out_off;
    for (uint32_t b = t; b < dim; b += kBT) {
        V v;
        v.x = (b == 0) ? T(1) : T(0);
        v.y = 0;
        psi[b] = v;
    }
    __syncthreads();
    // forward
    for (uint32_t gi = 0; gi < d.n_gates; ++gi) {
        const BatchGate g = gates[d.gate_off + gi];
        apply_gate<kBT, T>(psi, n, g, mats[d.mat_off + g.mat].v, false);
    }
    // lam = H psi, energy and norm
    double e_acc = 0.0, n_acc = 0.0;
    for (uint32_t b = t; b < dim; b += kBT) {
        T ar = 0, ai = 0;
        for (uint32_t gq = 0; gq < d.n_groups; ++gq) {
            const GroupDesc G = d.groups[gq];
            T dr = 0, di = 0;
            for (uint32_t k = G.begin; k < G.end; ++k) {
                const TermDesc<T> tm = d.terms[k];
                const bool neg = __popcll(tm.z & (uint64_t)b) & 1;
                dr += neg ? -tm.cre : tm.cre;
                di += neg ? -tm.cim : tm.cim;
            }
            const V p = psi[b ^ (uint32_t)G.x];
            ar += dr * p.x - di * p.y;
            ai += dr * p.y + di * p.x;
        }
        V l;
        l.x = ar;
        l.y = ai;
        lam[b] = l;
        const V p = psi[b];
        e_acc += (double)(p.x * ar + p.y * ai);
        n_acc += (double)(p.x * p.x + p.y * p.y);
    }
    __syncthreads();
    const double E = block_sum<kBT>(e_acc, red);
    const double nrm = block_sum<kBT>(n_acc, red);
    if (t == 0) o[0] = E / nrm;
    for (uint32_t k = t; k < d.n_params; k += kBT) o[1 + k] = 0.0;
    __syncthreads();
    // reverse sweep
    for (uint32_t gi = d.n_gates; gi-- > 0;) {
        const BatchGate g = gates[d.gate_off + gi];
        if (g.pidx >= 0) {
            const double gsum = block_sum<kBT>((double)grad_part<kBT, T>(psi, lam, n, g), red);
            if (t == 0) o[1 + g.pidx] += gsum / nrm;
        }
        const T* m = mats[d.mat_off + g.mat].v;
        apply_gate<kBT, T>(psi, n, g, m, true);
        apply_gate<kBT, T>(lam, n, g, m, true);
    }
}

// ------------------------------------------------------------------ mid-size items
// Cache-resident tiles: psi and lam of an item stay in device memory; each
// launch applies one fused pass (a window of kMidWin qubits) of every item.
// A block stages a coset of the window (2^kMidWin amplitudes) in LDS, runs
// the pass's gates there with the same per-gate code as the small-state
// kernel, and writes the coset back.  Reverse passes carry lam along and
// add each parameterised gate's term, reduced over the block in a fixed
// order, to a per-block slot; the slots are summed over blocks by
// mid_reduce_kernel, again in a fixed order.  An item's blocks, cosets and
// reduction order depend only on the item, so its bits do not depend on the
// rest of the batch.
constexpr int kMT = 256;                       // threads per block
constexpr int kMidTile = 1 << kMidWin;         // amplitudes per coset
constexpr int kMidPer = kMidTile / kMT;        // ... per thread
static_assert(kMidPer == 4, "two register bits per thread");

// Index of the descriptor that owns block b: the last one with blk_begin <= b.
template <typename D>
__device__ uint32_t owner(const D* d, uint32_t n, uint32_t b) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (d[m].blk_begin <= b) lo = m;
        else hi = m;
    }
    return lo;
}

template <typename T, bool REV>
__global__ void __launch_bounds__(kMT)
mid_pass_kernel(const MidPass* __restrict__ descs, uint32_t n_desc, const BatchGate* __restrict__ gates,
                const Mat2<T>* __restrict__ mats, double* __restrict__ part) {
    using V = typename VecB<T>::type;
    __shared__ V sp[kMidTile];
    __shared__ V sl[REV ? kMidTile : 1];
    __shared__ double red[kMT / 64];
    __shared__ double acc[kMidMaxSlots];
    const MidPass& d = descs[owner(descs, n_desc, blockIdx.x)];
    const uint32_t blk = blockIdx.x - d.blk_begin;
    const int t = threadIdx.x;
    V* psi = reinterpret_cast<V*>(d.psi);
    V* lam = reinterpret_cast<V*>(d.lam);
    uint64_t off[kMidPer];
    {
        uint64_t o = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((t >> k) & 1) o += 1ull << d.pos[k];
#pragma unroll
        for (int r = 0; r < kMidPer; ++r)
            off[r] = o + ((r & 1) ? 1ull << d.pos[8] : 0) + ((r & 2) ? 1ull << d.pos[9] : 0);
    }
    if (REV && t < (int)d.n_slots) acc[t] = 0.0;
    for (uint64_t c = blk; c < d.n_cosets; c += d.n_blk) {
        uint64_t base = c;
#pragma unroll
        for (int k = 0; k < kMidWin; ++k) {
            const uint64_t low = base & ((1ull << d.pos[k]) - 1);
            base = ((base ^ low) << 1) | low;
        }
#pragma unroll
        for (int r = 0; r < kMidPer; ++r) {
            const uint64_t idx = base + off[r];
            if (!REV && d.first) {
                V v;
                v.x = idx == 0 ? T(1) : T(0);
                v.y = 0;
                sp[t + kMT * r] = v;
            } else {
                sp[t + kMT * r] = psi[idx];
            }
            if (REV) sl[t + kMT * r] = lam[idx];
        }
        __syncthreads();
        if (!REV) {
            for (uint32_t gi = 0; gi < d.n_gates; ++gi) {
                const BatchGate g = gates[d.gate_off + gi];
                apply_gate<kMT, T>(sp, kMidWin, g, mats[d.mat_off + g.mat].v, false);
            }
        } else {
            uint32_t s = 0;
            for (uint32_t gi = d.n_gates; gi-- > 0;) {
                const BatchGate g = gates[d.gate_off + gi];
                if (g.pidx >= 0) {
                    const double v = block_sum<kMT>((double)grad_part<kMT, T>(sp, sl, kMidWin, g), red);
                    if (t == 0) acc[s] += v;
                    ++s;
                }
                const T* m = mats[d.mat_off + g.mat].v;
                apply_gate<kMT, T>(sp, kMidWin, g, m, true);
                apply_gate<kMT, T>(sl, kMidWin, g, m, true);
            }
        }
#pragma unroll
        for (int r = 0; r < kMidPer; ++r) {
            const uint64_t idx = base + off[r];
            psi[idx] = sp[t + kMT * r];
            if (REV) lam[idx] = sl[t + kMT * r];
        }
        __syncthreads();  // the next coset restages the tiles
    }
    if (!REV) return;
    __syncthreads();
    if (t < (int)d.n_slots) part[d.part_off + (uint64_t)t * d.n_blk + blk] = acc[t];
}

template <typename T>
__global__ void __launch_bounds__(kMT)
mid_hpsi_kernel(const MidHam* __restrict__ descs, uint32_t n_desc, double* __restrict__ part) {
    using V = typename VecB<T>::type;
    __shared__ double red[kMT / 64];
    const MidHam& d = descs[owner(descs, n_desc, blockIdx.x)];
    const uint32_t blk = blockIdx.x - d.blk_begin;
    const int t = threadIdx.x;
    const V* psi = reinterpret_cast<const V*>(d.psi);
    V* lam = reinterpret_cast<V*>(d.lam);
    const TermDesc<T>* terms = reinterpret_cast<const TermDesc<T>*>(d.terms);
    double e_acc = 0.0, n_acc = 0.0;
    for (uint64_t c = blk; c < d.n_tiles; c += d.n_blk) {
#pragma unroll
        for (int r = 0; r < kMidPer; ++r) {
            const uint64_t b = c * kMidTile + t + kMT * r;
            T ar = 0, ai = 0;
            for (uint32_t gq = 0; gq < d.n_groups; ++gq) {
                const GroupDesc G = d.groups[gq];
                T dr = 0, di = 0;
                for (uint32_t k = G.begin; k < G.end; ++k) {
                    const TermDesc<T> tm = terms[k];
                    const bool neg = __popcll(tm.z & b) & 1;
                    dr += neg ? -tm.cre : tm.cre;
                    di += neg ? -tm.cim : tm.cim;
                }
                const V p = psi[b ^ G.x];
                ar += dr * p.x - di * p.y;
                ai += dr * p.y + di * p.x;
            }
            V l;
            l.x = ar;
            l.y = ai;
            lam[b] = l;
            const V p = psi[b];
            e_acc += (double)(p.x * ar + p.y * ai);
            n_acc += (double)(p.x * p.x + p.y * p.y);
        }
    }
    const double e = block_sum<kMT>(e_acc, red);
    const double nn = block_sum<kMT>(n_acc, red);
    if (t == 0) {
        part[d.part_off + blk] = e;
        part[d.part_off + d.n_blk + blk] = nn;
    }
}

__global__ void __launch_bounds__(kMT)
mid_reduce_kernel(const MidRed* __restrict__ r, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[kMT / 64];
    const MidRed d = r[blockIdx.x];
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < d.count; i += kMT) s += part[d.part_off + i];
    const double tot = block_sum<kMT>(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

}  // namespace

template <typename T>
hipError_t launch_batch(const BatchDesc<T>* items, uint32_t n_items, const BatchGate* gates, const Mat2<T>* mats,
                        double* out, int max_n, hipStream_t st) {
    using V = typename VecB<T>::type;
    const size_t lds = 2 * ((size_t)1 << max_n) * sizeof(V);
    hipLaunchKernelGGL(batch_kernel<T>, dim3(n_items), dim3(kBT), lds, st, items, gates, mats, out);
    return hipGetLastError();
}

hipError_t batch_set_lds_limit() {
    hipError_t e = hipFuncSetAttribute((const void*)batch_kernel<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLdsBytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)batch_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kBatchLdsBytes);
}

template <typename T>
hipError_t launch_mid_pass(const MidPass* d, uint32_t n_desc, uint32_t grid, bool rev, const BatchGate* gates,
                           const Mat2<T>* mats, double* part, hipStream_t st) {
    if (rev)
        hipLaunchKernelGGL((mid_pass_kernel<T, true>), dim3(grid), dim3(kMT), 0, st, d, n_desc, gates, mats, part);
    else
        hipLaunchKernelGGL((mid_pass_kernel<T, false>), dim3(grid), dim3(kMT), 0, st, d, n_desc, gates, mats, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mid_hpsi(const MidHam* d, uint32_t n_desc, uint32_t grid, double* part, hipStream_t st) {
    hipLaunchKernelGGL(mid_hpsi_kernel<T>, dim3(grid), dim3(kMT), 0, st, d, n_desc, part);
    return hipGetLastError();
}

hipError_t launch_mid_reduce(const MidRed* r, uint32_t n, const double* part, double* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mid_reduce_kernel, dim3(n), dim3(kMT), 0, st, r, part, out);
    return hipGetLastError();
}

template hipError_t launch_mid_pass<float>(const MidPass*, uint32_t, uint32_t, bool, const BatchGate*,
                                           const Mat2<float>*, double*, hipStream_t);
template hipError_t launch_mid_pass<double>(const MidPass*, uint32_t, uint32_t, bool, const BatchGate*,
                                            const Mat2<double>*, double*, hipStream_t);
template hipError_t launch_mid_hpsi<float>(const MidHam*, uint32_t, uint32_t, double*, hipStream_t);
template hipError_t launch_mid_hpsi<double>(const MidHam*, uint32_t, uint32_t, double*, hipStream_t);

template hipError_t launch_batch<float>(const BatchDesc<float>*, uint32_t, const BatchGate*, const Mat2<float>*,
                                        double*, int, hipStream_t);
template hipError_t launch_batch<double>(const BatchDesc<double>*, uint32_t, const BatchGate*,
                                         const Mat2<double>*, double*, int, hipStream_t);

}  // namespace vqe
