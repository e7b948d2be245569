// Internal definitions shared by the host side (planner, Hamiltonian tables,
// C ABI) and the HIP kernels of the VQE library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vqe.h"

namespace vqe {

// ---------------------------------------------------------------- limits
constexpr int kMaxWindow = 7;     // qubits fused per pass (specialised kernels)
static_assert(kMaxWindow == VQE_MAX_WINDOW, "public and internal window limits differ");
constexpr int kInterpWindow = 5;  // qubits fused per pass by the interpreted kernels
constexpr int kMaxOps = 64;       // logical kernel ops per pass of an interpreted plan
constexpr int kMaxPhysOps = 160;  // ops per interpreted pass after inserting lane transposes
constexpr int kMaxMats = 32;      // 2x2 matrices per interpreted pass (kernel arguments)
constexpr int kMaxGradSlots = 24; // parameterised gates per pass (any plan)
constexpr int kInterpGradSlots = 16;  // ... of an interpreted pass (LDS accumulators)
constexpr int kBlock = 256;       // threads per block of every streaming kernel
constexpr int kMaxBlocks = 2048;  // grid-stride kernels use at most this many blocks
constexpr int kMaxPartBlocks = 1 << 17;  // blocks writing per-block partial sums
constexpr int kTileBits = 10;     // amplitudes per Hamiltonian tile = 2^kTileBits
constexpr int kMaxPlanWindow = 10;  // largest window the planner forms (mid-size tile passes)

// Per-pass limits of the fusion planner.
struct PlanLimits {
    int kmax;   // window qubits
    int ops;    // logical ops (gates + gradient terms)
    int mats;   // gates carrying a 2x2 matrix
    int slots;  // distinct parameters (gradient slots)
};
// Interpreted kernels: ops and matrices travel as kernel arguments.
constexpr PlanLimits kInterpLimits = {kInterpWindow, kMaxOps, kMaxMats, kInterpGradSlots};
// Specialised kernels: ops are compiled in, matrices read from a device table,
// gradient slots accumulate in registers (2 VGPRs each in FP64).
constexpr PlanLimits kJitLimits = {kMaxWindow, 96, 64, kMaxGradSlots};

// ---------------------------------------------------------------- kernel ops
// A fused pass is a list of ops on the local bits 0..K-1 of a window.
enum OpType : uint8_t {
    OP_U2 = 0,    // general complex 2x2 on bit a, matrix mats[slot]
    OP_R2 = 1,    // real 2x2 on bit a (re parts of mats[slot])
    OP_DIAG = 2,  // diag(m00, m11) on bit a
    OP_CNOT = 3,  // control a, target b
    OP_CZ = 4,    // phase -1 where bits a and b are both set
    OP_XFLIP = 5, // Pauli X on bit a
    OP_GX = 6,    // gradient slot += Im<lam| X_a |psi>
    OP_GY = 7,    // gradient slot += Im<lam| Y_a |psi>
    OP_GZ = 8,    // gradient slot += Im<lam| Z_a |psi>
    OP_TPOSE = 9, // lane-split layout: swap the roles of register bit a and lane slot b
    // Excitation gates: rotation by mats[slot] = [[c, -s], [s, c]] between the
    // patterns A and B of a 2- or 4-bit subset (specialised kernels only).
    OP_PAIR2 = 10,  // A = {a = 1, b = 0}, B = {a = 0, b = 1}
    OP_PAIR4 = 11,  // A = {a = b = 1, c = d = 0}, B = {a = b = 0, c = d = 1}
    OP_GPAIR2 = 12, // gradient slot += Re<lam| K |psi>, K = |B><A| - |A><B| of OP_PAIR2
    OP_GPAIR4 = 13, // ... of OP_PAIR4
};

struct KOp {
    uint8_t type, a, b, slot;
    uint8_t c, d;  // third and fourth bit of OP_PAIR4 / OP_GPAIR4
    uint8_t pad[2];
};

// Bit subset and the A / B patterns of a pair op (over the op's local bits).
inline void pair_patterns(const KOp& k, uint32_t& mask, uint32_t& A, uint32_t& B) {
    if (k.type == OP_PAIR2 || k.type == OP_GPAIR2) {
        A = 1u << k.a;
        B = 1u << k.b;
    } else {
        A = (1u << k.a) | (1u << k.b);
        B = (1u << k.c) | (1u << k.d);
    }
    mask = A | B;
}

// Matrix of a 2x2 op: row-major entries u00 u01 u10 u11, each (re, im).
template <typename T>
struct Mat2 {
    T v[8];
};

template <typename T>
struct PassArgs {
    uint64_t n_cosets;      // 2^(n-K): one coset = the 2^K amplitudes of a window
    uint32_t K;
    uint32_t n_ops;
    uint32_t n_gslots;
    uint32_t split;            // lane-split bits S (0: every window bit in registers)
    uint32_t pos[kMaxWindow];  // window qubits, ascending
    // Lane-split layout: qubit held by physical slot s at load / at store
    // (slots 0..K-S-1 are register bits, K-S.. lane slots).
    uint32_t pos_in[kMaxWindow];
    uint32_t pos_out[kMaxWindow];
    KOp ops[kMaxPhysOps];
    Mat2<T> mats[kMaxMats];
};

// Arguments of a specialised (run-time compiled) window kernel; its ops are
// compiled in and its matrices come from a device table.
struct JitArgs {
    uint64_t n_cosets;
    uint32_t pos[kMaxWindow];      // window qubits, ascending
    uint32_t pos_in[kMaxWindow];   // qubit held by physical slot s at load
    uint32_t pos_out[kMaxWindow];  // ... and at store
};

// Lane-split bits S of a window pass: S of the K window bits live in lane bits
// 6-S .. 5, the other K-S in registers.  Specialised kernels keep
// K-S = 6 (complex64 forward), 5 (complex64 reverse, complex128 forward) or
// 4 (complex128 reverse): 128 VGPRs of state per thread.  Measured at 32
// qubits with 7-qubit windows, one more register bit (and one lane bit less)
// than a 64-VGPR state is 13-15% faster per evaluation: fewer lane
// transposes and longer contiguous runs per load outweigh the lower
// occupancy.  Interpreted kernels split 5-qubit windows only, to
// K-S = 5 / 4 / 4 / 3 (their op dispatch needs the smaller state).
inline int split_bits_for(bool jit, bool is_double, int K, bool two_vectors) {
    const int kl = (jit ? 6 : 5) - (is_double ? 1 : 0) - (two_vectors ? 1 : 0);
    if (!jit && K != kInterpWindow) return 0;
    return K > kl ? K - kl : 0;
}

// ---------------------------------------------------------------- Hamiltonian tables
// Terms grouped by x mask.  For group g, terms [begin, end) carry z masks and
// the coefficient c = w * (-i)^popcount(x&z) split as (cre, cim), so that
// (H psi)[b] = sum_g psi[b ^ x_g] * sum_t c_t (-1)^popcount(z_t & b).
struct GroupDesc {
    uint64_t x;
    uint32_t begin, end;
    uint32_t hbit;     // highest set bit of x (0 for x = 0)
    uint32_t pad;
};

template <typename T>
struct TermDesc {
    uint64_t z;
    T cre, cim;
};

// ---------------------------------------------------------------- batched small states (batch.hip)
constexpr int kBatchLdsBytes = 128 * 1024;  // psi + lam in LDS
constexpr int kBatchMaxQubitsC64 = 13;
constexpr int kBatchMaxQubitsC128 = 12;

struct BatchGate {
    uint8_t type;  // OP_U2, OP_CNOT, OP_CZ, OP_XFLIP, OP_PAIR2 (any pair rotation)
    uint8_t q0, q1;
    uint8_t gen;   // OP_GX / OP_GY / OP_GZ / OP_GPAIR2 for parameterised gates
    int32_t pidx;  // parameter index or -1
    uint32_t mat;  // matrix index within the request
    uint16_t pa, pb;  // pair rotations: basis patterns A and B (n <= 16)
};

template <typename T>
struct BatchDesc {
    int32_t n;
    uint32_t n_gates, gate_off, mat_off, n_groups, n_params;
    uint64_t out_off;  // out[out_off] = energy, out[out_off + 1 + k] = dE/dtheta_k
    const GroupDesc* groups;
    const TermDesc<T>* terms;
};

template <typename T>
hipError_t launch_batch(const BatchDesc<T>* items, uint32_t n_items, const BatchGate* gates, const Mat2<T>* mats,
                        double* out, int max_n, hipStream_t st);
hipError_t batch_set_lds_limit();

// ---------------------------------------------------------------- batched mid-size states (batch.hip)
// Items above the LDS limit, up to kMidMaxQubits: psi and lam stay in device
// memory (up to 256 MiB per state in complex64, held in the last-level cache
// between passes at the small end), and one launch applies one fused pass of
// every item of the batch.  A pass is a window of kMidWin qubits (padded
// with the lowest qubits outside it, so a tile's loads run over consecutive
// amplitudes); a block stages a coset of 2^kMidWin amplitudes in LDS, applies
// the pass's gates there one at a time and writes it back.
constexpr int kMidWin = 10;
constexpr int kMidMaxQubits = 24;
constexpr int kMidMaxSlots = 64;          // parameterised gates per pass
constexpr uint32_t kMidMaxBlocks = 1024;  // blocks per item and launch
constexpr PlanLimits kMidLimits = {kMidWin, 1024, 1024, kMidMaxSlots};
static_assert(kMidWin <= kMaxPlanWindow, "planner window");
static_assert(kMidMaxQubits == VQE_BATCH_MAX_QUBITS_MID, "public and internal mid-size limits differ");

// One item's pass in one launch.  Blocks [blk_begin, blk_begin + n_blk) of
// the launch take cosets blk, blk + n_blk, ...; in a reverse pass block blk
// writes gradient slot s (the pass's parameterised gates, last gate first)
// to part[part_off + s n_blk + blk].
struct MidPass {
    void* psi;
    void* lam;
    uint64_t n_cosets;
    uint64_t part_off;
    uint32_t pos[kMidWin];  // window qubits, ascending
    uint32_t gate_off, n_gates, mat_off, n_slots;
    uint32_t blk_begin, n_blk;
    uint32_t first;         // forward pass 0: stage |0...0> instead of reading psi
    uint32_t pad;
};

// lam = H psi of one item over tiles of 2^kMidWin amplitudes; block blk
// writes its energy and norm partials to part[part_off + blk] and
// part[part_off + n_blk + blk].
struct MidHam {
    const void* psi;
    void* lam;
    const GroupDesc* groups;
    const void* terms;      // TermDesc<T>
    uint64_t n_tiles;
    uint64_t part_off;
    uint32_t n_groups, blk_begin, n_blk, pad;
};

// out[k] = sum of part[part_off .. part_off + count) in a fixed order.
struct MidRed {
    uint64_t part_off;
    uint32_t count, pad;
};

template <typename T>
hipError_t launch_mid_pass(const MidPass* d, uint32_t n_desc, uint32_t grid, bool rev, const BatchGate* gates,
                           const Mat2<T>* mats, double* part, hipStream_t st);
template <typename T>
hipError_t launch_mid_hpsi(const MidHam* d, uint32_t n_desc, uint32_t grid, double* part, hipStream_t st);
hipError_t launch_mid_reduce(const MidRed* r, uint32_t n, const double* part, double* out, hipStream_t st);

// ---------------------------------------------------------------- launchers (kernels.hip)
hipError_t launch_set_basis(int dtype, void* psi, uint64_t dim, uint64_t b, hipStream_t st);
hipError_t launch_zero(double* p, uint64_t n, hipStream_t st);
hipError_t launch_copy(int dtype, const void* src, void* dst, uint64_t dim, hipStream_t st);

// Interpreted window passes (K <= kInterpWindow).  in == out allowed (in
// place).  n = qubits of the state.
template <typename T>
hipError_t launch_window_fwd(const PassArgs<T>& a, int n, const void* in, void* out, hipStream_t st);

// Reverse pass on (psi, lam); writes per-block gradient partials
// [blocks][n_gslots] into gpart.  Returns the block count used via *nblocks.
template <typename T>
hipError_t launch_window_rev(const PassArgs<T>& a, int n, const void* psi_in, void* psi_out,
                             const void* lam_in, void* lam_out, double* gpart,
                             uint32_t* nblocks, hipStream_t st);

// Specialised kernel launch (fn = hipFunction_t of the pass, see jit.cpp):
// S lane-split bits, mats = this pass's matrix table on the device; reverse
// passes use the persistent grid; *nblocks = blocks used.
hipError_t launch_window_jit(void* fn, const JitArgs& a, int S, const void* mats, bool reverse, const void* in0,
                             void* out0, const void* in1, void* out1, double* gpart, uint32_t* nblocks,
                             hipStream_t st);


// ---------------------------------------------------------------- specialised kernels (jit.cpp)
int jit_mode();
int jit_set_mode(int mode);
// Kernel symbol of a generated pass: vqe_window_{fwd,rev}_{c64,c128}.
const char* jit_kernel_name(int NV, bool dbl);
// HIP source of the specialised kernel of one pass: K window bits, S lane-split
// bits, NV = 1 (forward) or 2 (reverse, psi and lam), ops on physical slots.
std::string jit_source(bool dbl, int K, int S, int NV, const std::vector<KOp>& ops, uint32_t n_gslots);
// Compiles (in parallel) and loads on the current device every source not yet
// cached; fns[i] = kernel of srcs[i] (nullptr for an empty source).
int jit_prepare(const std::vector<std::string>& srcs, std::vector<void*>& fns, std::string& err);
size_t jit_cached();

// ---------------------------------------------------------------- H psi by window passes
// lam = H psi as a few passes over qubit windows of kHwBits qubits that all
// contain qubits 0 .. kHwLow-1 (contiguous runs per load): every X group lies
// in one window, a pass stages each coset (the 2^kHwBits amplitudes that
// differ only in the window bits) of psi in LDS and adds the contributions of
// its groups to lam (written by the first pass, read-modify-written by the
// others); the last pass also reduces (Re<psi|lam>, <psi|psi>).
//
// Window-local pattern j = t + 2^kHwThreadBits r: thread t of a block holds
// the patterns of all r < 2^(kHwBits - kHwThreadBits).  For a group x,
//   D_x(b) = sum_z c_z (-1)^{z.b} = sum_{zl} (-1)^{zl.j} A_{x,zl}(coset),
//   A_{x,zl} = sum_{z: z & window = zl} c_z (-1)^{(z & ~window).base},
// so the terms of a group with equal in-window z bits form one class whose
// coefficient A is uniform over a coset (computed once per coset); the sign
// (-1)^{zl.j} splits into a thread part (zl bits below kHwThreadBits) and a
// register part, and the classes of a group are sorted into buckets by the
// register part, whose 2^(kHwBits - kHwThreadBits) bucket sums give D for
// every r through one Walsh-Hadamard transform.
// 13-qubit windows measured faster than 12 on both 32-qubit workloads (Hubbard
// 4 passes instead of 5, molecule-shaped 21 instead of 26) at the same 16 waves
// per CU (one 1024-thread block with a 128 KiB complex128 coset in LDS).
constexpr int kHwBits = 13;
static_assert(kHwBits == VQE_HPSI_WINDOW_QUBITS, "public and internal window sizes differ");
constexpr int kHwLow = 3;
constexpr int kHwThreadBits = 10;       // 1024 threads per block
constexpr int kHwRegBits = kHwBits - kHwThreadBits;
constexpr int kHwMaxClasses = 512;      // classes per pass (their coefficients are staged in LDS)

struct HwDesc {
    uint32_t pos[kHwBits];    // window qubits, ascending
    uint32_t g_begin, g_end;  // this pass's groups in the group table
    uint32_t c_begin, c_end;  // this pass's classes in the class table (at most kHwMaxClasses)
};

struct HwGroup {
    uint32_t xl;                       // x mask in window-local bits
    uint32_t cb[(1 << kHwRegBits) + 1];  // bucket u (register-part z bits = u): classes [cb[u], cb[u + 1])
    uint32_t zrm;                      // OR of the register-part z bits of its classes (empty buckets outside it)
    uint32_t pad;
};

struct HwClass {
    uint32_t zt;              // in-window z bits on the thread part (window-local bits below kHwThreadBits)
    uint32_t k_begin, k_end;  // its terms in the term table
    uint32_t pad;
};

template <typename T>
struct HwTerm {
    uint64_t zo;  // z bits outside the window (parity from the coset base)
    T cre, cim;   // folded coefficient, as in TermDesc
};

// One window pass; returns the block count (partials of the last pass).
// lam == nullptr: energy-only pass (no lam traffic); its partials hold this
// pass's share of Re<psi|H psi> and, for the first pass, <psi|psi>.
// real: every folded coefficient has a zero imaginary part (the real form
// of the pass, half the arithmetic).
template <typename T>
hipError_t launch_hwin(int n, const HwDesc& w, const void* psi, void* lam, const HwGroup* groups,
                       const HwClass* classes, const HwTerm<T>* terms, bool real, bool first, bool last,
                       double* part, uint32_t* nblocks, hipStream_t st);

// One window pass of lam = H psi for one item of a batch of mid-size
// states (one launch covers the pass of every item): blocks [blk_begin,
// blk_begin + n_blk) of the launch; after the item's last pass block blk
// writes its energy and norm partials to part[part_off + blk] and
// part[part_off + n_blk + blk].
struct HwItem {
    HwDesc w;
    const void* psi;
    void* lam;
    const HwGroup* groups;
    const HwClass* classes;
    const void* terms;  // HwTerm<T>
    uint64_t n_cosets, part_off;
    uint32_t blk_begin, n_blk, first, last;
};
template <typename T>
hipError_t launch_hwin_batch(const HwItem* d, uint32_t n_desc, uint32_t grid, bool real, double* part,
                             hipStream_t st);

// ---------------------------------------------------------------- dense window by MFMA
// psi' = U psi on kDenseK qubits, all >= 4 (16 consecutive cosets are 16
// consecutive amplitudes), U given to the kernel as the real 2^(k+1) square
// matrix [[Re U, -Im U], [Im U, Re U]] in row-major order, rows = output
// pattern (bit i of a pattern is qubit q[i]).  In place allowed.
constexpr int kDenseK = 5;

struct DenseArgs {
    uint64_t n_tiles;           // 2^(n - kDenseK) / 16
    uint32_t q[kDenseK];        // window qubits in pattern-bit order
    uint32_t sorted[kDenseK];   // the same, ascending
};

template <typename T>
hipError_t launch_dense(const DenseArgs& a, const T* ur, const void* in, void* out, hipStream_t st);

// H psi tile kernel.  mode 0: lam = H psi and (Re<psi|lam>, <psi|psi>) partials.
// mode 1: energy partials only, off-tile groups visited once per pair.  At
// most max_blocks blocks (each owns a contiguous run of tiles), each writing
// two partials.
template <typename T>
hipError_t launch_hpsi(int n, const void* psi, void* lam, const GroupDesc* groups, uint32_t n_groups,
                       const TermDesc<T>* terms, int mode, uint32_t max_blocks, double* part, uint32_t* nblocks,
                       hipStream_t st);
// Blocks that launch_hpsi uses at n qubits under max_blocks, and that a
// window pass of H psi (launch_hwin) uses at n qubits.
uint32_t hpsi_blocks(int n, uint32_t max_blocks);
uint32_t hwin_blocks(int n);
// Grouped energy-only sweeps (vqe_expect_pauli and its no-allocation form)
// launch at most this many blocks: one block count, hence one reduction
// order, for both.
constexpr uint32_t kEnergyPartBlocks = 4096;

// out[0] = sums[0] / sums[1], out[1] = sums[1] (one thread; device memory).
hipError_t launch_energy_ratio(const double* sums, double* out, hipStream_t st);

// One term: partials of Re<psi|P(x,z)|psi> (pair-halved) and <psi|psi>.
template <typename T>
hipError_t launch_expect_term(int n, const void* psi, uint64_t x, uint64_t z, double* part,
                              uint32_t* nblocks, hipStream_t st);

// out[map ? map[s] : s] = (accumulate 0), += (1) or -= (-1) the sum over blocks
// of part[block][s], fixed order, FP64.
hipError_t launch_reduce(const double* part, uint32_t nblocks, uint32_t nslots,
                         const int32_t* map, double* out, int accumulate, hipStream_t st);

// ---------------------------------------------------------------- planner (plan.cpp)
struct Gate {
    int kind, q0, q1, pidx;
    double angle;
    int q2 = 0, q3 = 0;  // DEXC only
};

// Qubits of a gate (1, 2 or 4); returns the count.
inline int gate_qubits(const Gate& g, int q[4]) {
    q[0] = g.q0;
    switch (g.kind) {
        case VQE_GATE_CNOT:
        case VQE_GATE_CZ:
        case VQE_GATE_SEXC:
            q[1] = g.q1;
            return 2;
        case VQE_GATE_DEXC:
            q[1] = g.q1;
            q[2] = g.q2;
            q[3] = g.q3;
            return 4;
        default:
            return 1;
    }
}

struct PlannedPass {
    int K = 0;
    int pos[kMaxPlanWindow] = {0};
    std::vector<int> gates;      // indices into the circuit's gate list, execution order
};

// Partition gates into fused passes.  Returns false (with msg) on failure.
// lim.kmax = largest window (<= kMaxPlanWindow).
bool plan_passes(int n, const std::vector<Gate>& gates, const PlanLimits& lim, std::vector<PlannedPass>& out,
                 std::string& msg);

// ---------------------------------------------------------------- errors
void set_error(const std::string& m);

}  // namespace vqe
