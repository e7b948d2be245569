// Specialised window pass kernels, generated per op list and compiled at run
// time with hiprtc for gfx950.
//
// The interpreted window kernels (kernels.hip) read each op from the pass
// arguments and branch on its type and bits.  Every branch writes the whole
// register-resident coset, so the compiler merges the branches through copies
// of the full coset: on complex128 reverse passes about two thirds of the
// vector instructions are such moves and the pass is VALU-bound.  A generated
// kernel instead spells out the pass as straight-line code with every bit a
// constant:
//   * permutation ops (CNOT, Pauli X) only rename registers at generation
//     time and cost no instruction;
//   * 2x2 ops, phases and gradient terms are written per register pair with
//     the pair indices known;
//   * lane-split transposes are permlane swaps (lane bits 4, 5) or DPP moves
//     with a select (lane bits 2, 3) on named registers.
// Window positions stay kernel arguments and matrices come from a device
// table filled per evaluation, so passes with equal op lists share a kernel.
// Windows of up to 7 qubits are split over lane bits 2..5 (see split_bits_for).
// The load/store addressing, work order and grid follow the interpreted
// kernels, so both forms give the same results up to the rounding of fused
// multiply-adds and of the gradient sums.
#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>

#include "vqe_internal.h"

namespace vqe {
namespace {

std::atomic<int> g_mode{VQE_SPECIALIZE_AUTO};

struct Entry {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};
std::mutex g_mu;
std::map<std::pair<int, std::string>, Entry> g_cache;  // (device, source) -> loaded kernel

// Text of the kernel argument types; must match JitArgs / Mat2.
std::string prelude(bool dbl) {
    const char* T = dbl ? "double" : "float";
    std::ostringstream o;
    o << "typedef unsigned long long u64;\ntypedef unsigned int u32;\n"
      << "typedef " << T << " T;\n"
      << "struct Mat2 { T v[8]; };\n"
      << "struct JitArgs { u64 n_cosets; u32 pos[" << kMaxWindow << "]; u32 pos_in[" << kMaxWindow
      << "]; u32 pos_out[" << kMaxWindow << "]; };\n"
      << "struct __attribute__((aligned(" << (dbl ? 16 : 8) << "))) V { T x, y; };\n"
      << "__device__ __forceinline__ u64 xcd_order(u64 u, u32 m) {\n"
      << "  if (m < 3) return u;\n  return (u >> 3) | ((u & 7ull) << (m - 3));\n}\n";
    // Lane transpose over lane bit LB (mask m = 2^LB) of the register pair
    // (a, b): a' = a on lanes with the bit clear, b(lane - m) on lanes with it
    // set; b' = a(lane + m) on lanes with the bit clear, b on lanes with it set.
    // Lane bits 5 and 4: one v_permlane{32,16}_swap per dword.  Lane bits 3
    // and 2: DPP row_ror:8 (lane ^ 8) or row_shr:4 / row_shl:4 (lane - 4 /
    // lane + 4 within a row of 16) and a per-lane select.
    o << "template <int LB> __device__ __forceinline__ void tp32(u32& a, u32& b) {\n"
      << "  if constexpr (LB == 5) { const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false); a = r[0]; "
         "b = r[1]; }\n"
      << "  else if constexpr (LB == 4) { const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false); a = "
         "r[0]; b = r[1]; }\n"
      << "  else {\n"
      << "    constexpr int DN = LB == 3 ? 0x128 : 0x114;\n"
      << "    constexpr int UP = LB == 3 ? 0x128 : 0x104;\n"
      << "    const bool hb = (threadIdx.x >> LB) & 1;\n"
      << "    const u32 bd = (u32)__builtin_amdgcn_update_dpp(0, (int)b, DN, 0xF, 0xF, false);\n"
      << "    const u32 au = (u32)__builtin_amdgcn_update_dpp(0, (int)a, UP, 0xF, 0xF, false);\n"
      << "    const u32 na = hb ? bd : a;\n"
      << "    b = hb ? b : au;\n"
      << "    a = na;\n"
      << "  }\n}\n";
    if (dbl)
        o << "template <int LB> __device__ __forceinline__ void tp(T& a, T& b) {\n"
          << "  u64 x = __builtin_bit_cast(u64, a), y = __builtin_bit_cast(u64, b);\n"
          << "  u32 xl = (u32)x, xh = (u32)(x >> 32), yl = (u32)y, yh = (u32)(y >> 32);\n"
          << "  tp32<LB>(xl, yl); tp32<LB>(xh, yh);\n"
          << "  a = __builtin_bit_cast(T, ((u64)xh << 32) | xl); b = __builtin_bit_cast(T, ((u64)yh << 32) | yl);\n}\n";
    else
        o << "template <int LB> __device__ __forceinline__ void tp(T& a, T& b) {\n"
          << "  u32 x = __builtin_bit_cast(u32, a), y = __builtin_bit_cast(u32, b);\n"
          << "  tp32<LB>(x, y);\n  a = __builtin_bit_cast(T, x); b = __builtin_bit_cast(T, y);\n}\n";
    return o.str();
}

// Straight-line body generator.  loc[p] = variable holding register entry p.
struct Gen {
    int K, S, NV, KL, N;
    std::vector<int> loc;
    std::ostringstream o;
    std::string R(int v, int p) const { return "r" + std::to_string(v) + "_" + std::to_string(loc[p]); }
    std::string I(int v, int p) const { return "i" + std::to_string(v) + "_" + std::to_string(loc[p]); }
    std::string H(int lane_slot) const { return "h" + std::to_string(lane_slot); }
    int lane_bit(int lane_slot) const { return 6 - S + lane_slot; }

    void mats(int s, bool all) {
        o << "  { const T* m = mats[" << s << "].v;\n";
        if (all)
            o << "    const T m0r = m[0], m0i = m[1], m1r = m[2], m1i = m[3], m2r = m[4], m2i = m[5], m3r = m[6], "
                 "m3i = m[7];\n";
    }

    void op(const KOp& k) {
        const int A = k.a, B = k.b;
        const bool la = A >= KL, lb = B >= KL;
        switch (k.type) {
            case OP_U2:
                mats(k.slot, true);
                for (int p = 0; p < N; ++p) {
                    if (p & (1 << A)) continue;
                    const int q = p | (1 << A);
                    for (int v = 0; v < NV; ++v) {
                        o << "    { const T ar = " << R(v, p) << ", ai = " << I(v, p) << ", br = " << R(v, q)
                          << ", bi = " << I(v, q) << ";\n"
                          << "      " << R(v, p) << " = m0r * ar - m0i * ai + m1r * br - m1i * bi;\n"
                          << "      " << I(v, p) << " = m0r * ai + m0i * ar + m1r * bi + m1i * br;\n"
                          << "      " << R(v, q) << " = m2r * ar - m2i * ai + m3r * br - m3i * bi;\n"
                          << "      " << I(v, q) << " = m2r * ai + m2i * ar + m3r * bi + m3i * br; }\n";
                    }
                }
                o << "  }\n";
                break;
            case OP_R2:
                mats(k.slot, false);
                if (NV == 2 && k.c == 1) {
                    // un-applied rotation as three shears of each (a_p, a_q) plane,
                    // coefficients k1 = m[0], k2 = m[1] (shear_coefficients)
                    o << "    const T k1 = m[0], k2 = m[1];\n";
                    for (int p = 0; p < N; ++p) {
                        if (p & (1 << A)) continue;
                        const int q = p | (1 << A);
                        for (int v = 0; v < NV; ++v)
                            o << "    { T xr = " << R(v, p) << ", yr = " << R(v, q) << ", xi = " << I(v, p)
                              << ", yi = " << I(v, q) << ";\n"
                              << "      xr += k1 * yr; xi += k1 * yi; yr += k2 * xr; yi += k2 * xi; xr += k1 * yr; "
                                 "xi += k1 * yi;\n"
                              << "      " << R(v, p) << " = xr; " << I(v, p) << " = xi; " << R(v, q) << " = yr; "
                              << I(v, q) << " = yi; }\n";
                    }
                    o << "  }\n";
                    break;
                }
                o << "    const T ca = m[0], cb = m[2], cc = m[4], cd = m[6];\n";
                for (int p = 0; p < N; ++p) {
                    if (p & (1 << A)) continue;
                    const int q = p | (1 << A);
                    for (int v = 0; v < NV; ++v) {
                        o << "    { const T ar = " << R(v, p) << ", ai = " << I(v, p) << ", br = " << R(v, q)
                          << ", bi = " << I(v, q) << ";\n"
                          << "      " << R(v, p) << " = ca * ar + cb * br; " << I(v, p) << " = ca * ai + cb * bi;\n"
                          << "      " << R(v, q) << " = cc * ar + cd * br; " << I(v, q) << " = cc * ai + cd * bi; }\n";
                    }
                }
                o << "  }\n";
                break;
            case OP_DIAG:
                mats(k.slot, false);
                if (NV == 2 && k.c == 1) {
                    // un-applied phase rotation of (Re, Im) as three shears: k1 = m[0],
                    // k2 = m[1] for bit 0, the opposite angle (-k1, -k2) for bit 1
                    if (la)
                        o << "    const T k1 = " << H(A - KL) << " ? -m[0] : m[0], k2 = " << H(A - KL)
                          << " ? -m[1] : m[1];\n";
                    else
                        o << "    const T k1 = m[0], k2 = m[1], n1 = -m[0], n2 = -m[1];\n";
                    for (int p = 0; p < N; ++p) {
                        const char* s1 = (!la && (p & (1 << A))) ? "n1" : "k1";
                        const char* s2 = (!la && (p & (1 << A))) ? "n2" : "k2";
                        for (int v = 0; v < NV; ++v)
                            o << "    { T xr = " << R(v, p) << ", xi = " << I(v, p) << "; xr += " << s1
                              << " * xi; xi += " << s2 << " * xr; xr += " << s1 << " * xi; " << R(v, p) << " = xr; "
                              << I(v, p) << " = xi; }\n";
                    }
                    o << "  }\n";
                    break;
                }
                if (la)
                    o << "    const T p0r = " << H(A - KL) << " ? m[6] : m[0], p0i = " << H(A - KL)
                      << " ? m[7] : m[1];\n";
                else
                    o << "    const T p0r = m[0], p0i = m[1], p1r = m[6], p1i = m[7];\n";
                for (int p = 0; p < N; ++p) {
                    const char* pr = (!la && (p & (1 << A))) ? "p1r" : "p0r";
                    const char* pi = (!la && (p & (1 << A))) ? "p1i" : "p0i";
                    for (int v = 0; v < NV; ++v)
                        o << "    { const T ar = " << R(v, p) << ", ai = " << I(v, p) << "; " << R(v, p) << " = "
                          << pr << " * ar - " << pi << " * ai; " << I(v, p) << " = " << pr << " * ai + " << pi
                          << " * ar; }\n";
                }
                o << "  }\n";
                break;
            case OP_CNOT:
                // control A, target B, both register bits: rename
                for (int p = 0; p < N; ++p)
                    if ((p & (1 << A)) && !(p & (1 << B))) std::swap(loc[p], loc[p | (1 << B)]);
                break;
            case OP_XFLIP:
                for (int p = 0; p < N; ++p)
                    if (!(p & (1 << A))) std::swap(loc[p], loc[p | (1 << A)]);
                break;
            case OP_CZ: {
                if (la && lb) {
                    o << "  { const T sg = (" << H(A - KL) << " && " << H(B - KL) << ") ? T(-1) : T(1);\n";
                    for (int p = 0; p < N; ++p)
                        for (int v = 0; v < NV; ++v)
                            o << "    " << R(v, p) << " *= sg; " << I(v, p) << " *= sg;\n";
                    o << "  }\n";
                } else if (la || lb) {
                    const int rb = la ? B : A;
                    const int ls = la ? A - KL : B - KL;
                    o << "  { const T sg = " << H(ls) << " ? T(-1) : T(1);\n";
                    for (int p = 0; p < N; ++p)
                        if (p & (1 << rb))
                            for (int v = 0; v < NV; ++v)
                                o << "    " << R(v, p) << " *= sg; " << I(v, p) << " *= sg;\n";
                    o << "  }\n";
                } else {
                    for (int p = 0; p < N; ++p)
                        if ((p & (1 << A)) && (p & (1 << B)))
                            for (int v = 0; v < NV; ++v)
                                o << "  " << R(v, p) << " = -" << R(v, p) << "; " << I(v, p) << " = -" << I(v, p)
                                  << ";\n";
                }
                break;
            }
            case OP_TPOSE: {
                const int lb_ = lane_bit(B);
                for (int p = 0; p < N; ++p) {
                    if (p & (1 << A)) continue;
                    const int q = p | (1 << A);
                    for (int v = 0; v < NV; ++v)
                        o << "  tp<" << lb_ << ">(" << R(v, p) << ", " << R(v, q) << "); tp<" << lb_ << ">(" << I(v, p)
                          << ", " << I(v, q) << ");\n";
                }
                break;
            }
            case OP_PAIR2:
            case OP_PAIR4: {
                uint32_t mask, PA, PB;
                pair_patterns(k, mask, PA, PB);
                mats(k.slot, false);
                o << "    const T ca = m[0], cb = m[2], cc = m[4], cd = m[6];\n";
                for (int p = 0; p < N; ++p) {
                    if ((p & (int)mask) != (int)PA) continue;
                    const int q = p ^ (int)PA ^ (int)PB;
                    for (int v = 0; v < NV; ++v)
                        o << "    { const T ar = " << R(v, p) << ", ai = " << I(v, p) << ", br = " << R(v, q)
                          << ", bi = " << I(v, q) << ";\n"
                          << "      " << R(v, p) << " = ca * ar + cb * br; " << I(v, p) << " = ca * ai + cb * bi;\n"
                          << "      " << R(v, q) << " = cc * ar + cd * br; " << I(v, q) << " = cc * ai + cd * bi; }\n";
                }
                o << "  }\n";
                break;
            }
            case OP_GPAIR2:
            case OP_GPAIR4: {
                if (NV != 2) break;
                uint32_t mask, PA, PB;
                pair_patterns(k, mask, PA, PB);
                // Re<lam|K|psi>, K = |B><A| - |A><B|: Re(conj(lam_B) psi_A) - Re(conj(lam_A) psi_B)
                o << "  { T acc = 0;\n";
                for (int p = 0; p < N; ++p) {
                    if ((p & (int)mask) != (int)PA) continue;
                    const int q = p ^ (int)PA ^ (int)PB;
                    o << "    acc += " << R(1, q) << " * " << R(0, p) << "; acc += " << I(1, q) << " * " << I(0, p)
                      << "; acc -= " << R(1, p) << " * " << R(0, q) << "; acc -= " << I(1, p) << " * " << I(0, q)
                      << ";\n";
                }
                o << "    g" << (int)k.slot << " += (double)acc; }\n";
                break;
            }
            case OP_GX:
            case OP_GY:
            case OP_GZ: {
                if (NV != 2) break;
                o << "  { T acc = 0;\n";
                if (k.type == OP_GZ && la) {
                    for (int p = 0; p < N; ++p)
                        o << "    acc += " << R(1, p) << " * " << I(0, p) << "; acc -= " << I(1, p) << " * " << R(0, p)
                          << ";\n";
                    o << "    g" << (int)k.slot << " += (double)(" << H(A - KL) << " ? -acc : acc); }\n";
                    break;
                }
                for (int p = 0; p < N; ++p) {
                    if (p & (1 << A)) continue;
                    const int q = p | (1 << A);
                    const std::string p0r = R(0, p), p0i = I(0, p), p1r = R(0, q), p1i = I(0, q);
                    const std::string l0r = R(1, p), l0i = I(1, p), l1r = R(1, q), l1i = I(1, q);
                    // one fused multiply-add per product (the sum of the pair's four
                    // products, accumulated term by term)
                    if (k.type == OP_GZ)
                        o << "    acc += " << l0r << " * " << p0i << "; acc -= " << l0i << " * " << p0r << "; acc -= "
                          << l1r << " * " << p1i << "; acc += " << l1i << " * " << p1r << ";\n";
                    else if (k.type == OP_GY)
                        o << "    acc += " << l1r << " * " << p0r << "; acc += " << l1i << " * " << p0i << "; acc -= "
                          << l0r << " * " << p1r << "; acc -= " << l0i << " * " << p1i << ";\n";
                    else
                        o << "    acc += " << l0r << " * " << p1i << "; acc -= " << l0i << " * " << p1r << "; acc += "
                          << l1r << " * " << p0i << "; acc -= " << l1i << " * " << p0r << ";\n";
                }
                o << "    g" << (int)k.slot << " += (double)acc; }\n";
                break;
            }
            default:
                break;
        }
    }
};

std::string offset_expr(const char* arr, int p, int KL) {
    std::string e;
    for (int j = 0; j < KL; ++j)
        if (p & (1 << j)) e += (e.empty() ? "" : " + ") + std::string(arr) + "[" + std::to_string(j) + "]";
    return e.empty() ? "0" : e;
}

bool compile(const std::string& src, std::vector<char>& code, std::string& log) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "vqe_window.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return false;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=fast",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    log.assign(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    bool ok = r == HIPRTC_SUCCESS;
    if (ok) {
        size_t cs = 0;
        ok = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
        if (ok) {
            code.resize(cs);
            ok = hiprtcGetCode(prog, code.data()) == HIPRTC_SUCCESS;
        }
    }
    hiprtcDestroyProgram(&prog);
    return ok;
}

}  // namespace

const char* jit_kernel_name(int NV, bool dbl) {
    return NV == 2 ? (dbl ? "vqe_window_rev_c128" : "vqe_window_rev_c64")
                   : (dbl ? "vqe_window_fwd_c128" : "vqe_window_fwd_c64");
}

int jit_mode() { return g_mode.load(); }

int jit_set_mode(int mode) { return g_mode.exchange(mode); }

std::string jit_source(bool dbl, int K, int S, int NV, const std::vector<KOp>& ops, uint32_t n_gslots) {
    Gen g;
    g.K = K;
    g.S = S;
    g.NV = NV;
    g.KL = K - S;
    g.N = 1 << g.KL;
    g.loc.resize(g.N);
    for (int p = 0; p < g.N; ++p) g.loc[p] = p;
    const int CPW = 64 >> S, PER_BLOCK = kBlock >> S;
    std::ostringstream& o = g.o;
    o << prelude(dbl);
    // Reverse kernels ask for two blocks per CU: unconstrained they take 256 VGPRs plus a few
    // AGPRs, one wave per SIMD; at two waves the compiler spills a few dwords (complex64
    // reverse pass 37.9 -> 36.4 ms at 32 qubits, complex128 unchanged).
    o << "extern \"C\" __global__ void __launch_bounds__(" << kBlock << (NV == 2 ? ", 2" : "") << ")\n"
      << jit_kernel_name(NV, dbl) << "(const JitArgs a, const Mat2* __restrict__ mats, u32 cpt, u32 mlog, "
         "const V* __restrict__ in0, V* __restrict__ out0, const V* __restrict__ in1, V* __restrict__ out1, "
         "double* __restrict__ gpart) {\n"
      << "  const int tid = threadIdx.x;\n  const int lane = tid & 63;\n"
      << "  const int sub = (tid >> 6) * " << CPW << " + (lane & " << (CPW - 1) << ");\n"
      << "  u64 bitval[" << K << "], bv_in[" << K << "], bv_out[" << K << "];\n"
      << "#pragma unroll\n  for (int j = 0; j < " << K
      << "; ++j) { bitval[j] = 1ull << a.pos[j]; bv_in[j] = 1ull << a.pos_in[j]; bv_out[j] = 1ull << a.pos_out[j]; }\n"
      << "  u64 half_in = 0, half_out = 0;\n";
    for (int j = 0; j < S; ++j)
        o << "  const bool h" << j << " = (lane >> " << g.lane_bit(j) << ") & 1;\n"
          << "  if (h" << j << ") { half_in += bv_in[" << g.KL + j << "]; half_out += bv_out[" << g.KL + j << "]; }\n";
    for (uint32_t s = 0; s < n_gslots; ++s) o << "  double g" << s << " = 0.0;\n";
    o << "  for (u32 it = 0; it < cpt; ++it) {\n"
      << "    const u64 blk = xcd_order((u64)blockIdx.x * cpt + it, mlog);\n"
      << "    const u64 c = blk * " << PER_BLOCK << " + sub;\n"
      << "    if (c >= a.n_cosets) break;\n"
      << "    u64 base = c;\n"
      << "#pragma unroll\n    for (int j = 0; j < " << K
      << "; ++j) { const u64 low = base & (bitval[j] - 1); base = ((base ^ low) << 1) | low; }\n"
      << "    u64 sbase = base + half_out;\n    base += half_in;\n";
    for (int p = 0; p < g.N; ++p) {
        for (int v = 0; v < NV; ++v)
            o << "    const V l" << v << "_" << p << " = in" << v << "[base + " << offset_expr("bv_in", p, g.KL)
              << "];\n";
    }
    for (int p = 0; p < g.N; ++p)
        for (int v = 0; v < NV; ++v)
            o << "    T r" << v << "_" << p << " = l" << v << "_" << p << ".x, i" << v << "_" << p << " = l" << v << "_"
              << p << ".y;\n";
    for (const KOp& k : ops) g.op(k);
    o << "    asm volatile(\"\" : \"+v\"(sbase));\n";
    for (int p = 0; p < g.N; ++p)
        for (int v = 0; v < NV; ++v)
            o << "    out" << v << "[sbase + " << offset_expr("bv_out", p, g.KL) << "] = V{" << g.R(v, p) << ", "
              << g.I(v, p) << "};\n";
    o << "  }\n";
    if (NV == 2 && n_gslots) {
        // block reduction in a fixed order: butterflies within each wave (every
        // lane ends with the same bits), then thread s adds slot s's wave totals
        // in wave order
        constexpr int W = kBlock / 64;
        o << "  __shared__ double red[" << W * n_gslots << "];\n"
          << "  double gv[" << n_gslots << "] = {";
        for (uint32_t s = 0; s < n_gslots; ++s) o << (s ? ", " : "") << "g" << s;
        o << "};\n"
          << "#pragma unroll\n  for (int s = 0; s < " << n_gslots << "; ++s) {\n"
          << "#pragma unroll\n    for (int d = 32; d > 0; d >>= 1) gv[s] += __shfl_xor(gv[s], d);\n"
          << "    if ((tid & 63) == 0) red[s * " << W << " + (tid >> 6)] = gv[s];\n  }\n"
          << "  __syncthreads();\n"
          << "  if (tid < " << n_gslots << ") {\n    double r = red[tid * " << W << "];\n"
          << "#pragma unroll\n    for (int w = 1; w < " << W << "; ++w) r += red[tid * " << W << " + w];\n"
          << "    gpart[(u64)blockIdx.x * " << n_gslots << " + tid] = r;\n  }\n";
    }
    o << "}\n";
    return o.str();
}

int jit_prepare(const std::vector<std::string>& srcs, std::vector<void*>& fns, std::string& err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "no HIP device for specialised kernels";
        return VQE_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    // unique sources not yet loaded on this device
    std::vector<const std::string*> todo;
    {
        std::map<std::string, int> seen;
        for (const auto& s : srcs)
            if (!s.empty() && !g_cache.count({dev, s}) && !seen.count(s)) {
                seen[s] = 1;
                todo.push_back(&s);
            }
    }
    std::vector<std::vector<char>> codes(todo.size());
    std::vector<std::string> logs(todo.size());
    std::vector<char> ok(todo.size(), 0);
    if (!todo.empty()) {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t nt = std::min<size_t>(todo.size(), std::min(16u, hw));
        std::atomic<size_t> next{0};
        auto work = [&]() {
            for (size_t i; (i = next.fetch_add(1)) < todo.size();) ok[i] = compile(*todo[i], codes[i], logs[i]);
        };
        std::vector<std::thread> th;
        for (size_t t = 1; t < nt; ++t) th.emplace_back(work);
        work();
        for (auto& t : th) t.join();
    }
    for (size_t i = 0; i < todo.size(); ++i) {
        if (!ok[i]) {
            err = "specialised pass kernel failed to compile: " + logs[i].substr(0, 2000);
            return VQE_ERR_STATE;
        }
        Entry e;
        const char* name = nullptr;
        for (int nv = 1; nv <= 2 && !name; ++nv)
            for (int dbl = 0; dbl < 2 && !name; ++dbl)
                if (todo[i]->find(std::string(jit_kernel_name(nv, dbl)) + "(") != std::string::npos)
                    name = jit_kernel_name(nv, dbl);
        if (!name) {
            err = "specialised pass kernel without a known symbol (internal error)";
            return VQE_ERR_STATE;
        }
        if (hipModuleLoadData(&e.mod, codes[i].data()) != hipSuccess ||
            hipModuleGetFunction(&e.fn, e.mod, name) != hipSuccess) {
            err = "loading a specialised pass kernel failed";
            return VQE_ERR_DEVICE;
        }
        g_cache[{dev, *todo[i]}] = e;
    }
    fns.assign(srcs.size(), nullptr);
    for (size_t i = 0; i < srcs.size(); ++i)
        if (!srcs[i].empty()) fns[i] = (void*)g_cache[{dev, srcs[i]}].fn;
    return VQE_OK;
}

size_t jit_cached() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_cache.size();
}

}  // namespace vqe
