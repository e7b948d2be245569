/*
 * vqe.h -- C ABI of the MI355X (gfx950) VQE state-vector library.
 *
 * The library evaluates the variational quantum eigensolver objective of
 * Morita et al., "Simulator Demonstration of Large Scale Variational Quantum
 * Algorithm on HPC Cluster" (arXiv 2402.11878):
 *   psi(theta) = U(theta) psi_ref                          (Sec. II-B, eq. 6)
 *   E(theta)   = <psi|H|psi> / <psi|psi>                   (Sec. II-B, eq. 7)
 *   H          = sum_i w_i P_i,  P_i = (x) sigma_k, sigma in {I,X,Y,Z}  (eqs. 2-4)
 * with the Hamiltonian optionally slimmed by dropping terms of small |w|
 * (Sec. II-D, Sec. III-D), the drop being bounded by |<psi|wP|psi>| <= |w|.
 *
 * Conventions used by every entry point
 *   - Qubit j is bit j (value 2^j) of the basis index.  A state of n qubits is
 *     2^n contiguous interleaved complex amplitudes (re, im), index = basis
 *     integer: complex64 (2 x float) or complex128 (2 x double).
 *   - A Pauli string is a pair of bit masks (x, z): (x_j, z_j) = (0,0) I,
 *     (1,0) X, (0,1) Z, (1,1) Y, i.e. P(x,z) = i^popcount(x&z) X^x Z^z.
 *   - RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2), RX(t) = exp(-i t X/2);
 *     CNOT(c -> t) maps |b> to |b xor (b_c << t)>.
 *   - All device work of a call is enqueued on the stream of the state handle
 *     (a hipStream_t given at allocation; NULL = the null stream).  Calls that
 *     return host scalars synchronise that stream before returning.
 *
 * Errors
 *   Every function returns VQE_OK (0) or a negative status.  No C++ exception
 *   crosses the ABI.  On error the outputs are left untouched and
 *   vqe_last_error() returns a message (thread-local, valid until the next
 *   call on the same thread).
 *
 * Ownership
 *   The caller owns every host array passed in; the library copies what it
 *   keeps.  Handles own their device tables and are released by the matching
 *   *_free call.  A handle may not be used from two threads at once.
 */
#ifndef VQE_H_
#define VQE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define VQE_OK               0
#define VQE_ERR_ARG         -1  /* invalid argument (null, size, range, mismatch) */
#define VQE_ERR_OOM         -2  /* device or host allocation failed */
#define VQE_ERR_DEVICE      -3  /* HIP runtime error or no usable device */
#define VQE_ERR_UNSUPPORTED -4  /* valid request the library does not implement */
#define VQE_ERR_STATE       -5  /* handle in the wrong state for this call */

/* ---- amplitude types ---- */
#define VQE_C64   1   /* complex64: float re, float im (8 bytes per amplitude)   */
#define VQE_C128  2   /* complex128: double re, double im (16 bytes per amplitude) */

/* ---- gate kinds ---- */
#define VQE_GATE_RY    0
#define VQE_GATE_RZ    1
#define VQE_GATE_RX    2
#define VQE_GATE_H     3
#define VQE_GATE_X     4
#define VQE_GATE_CNOT  5   /* q0 = control, q1 = target */
#define VQE_GATE_CZ    6
/* Excitation gate sets of the paper's ansatz (eq. 5): particle-conserving
 * rotations by theta/2 inside a two-state subspace, applied as
 *   psi'[a] = c psi[a] - s psi[a'],  psi'[a'] = s psi[a] + c psi[a'],
 *   c = cos(theta/2), s = sin(theta/2),
 * for every basis index a in pattern A and a' = a with the A bits replaced by
 * the B bits; other amplitudes are unchanged (no Jordan-Wigner strings).
 *   SEXC on (q0, q1):          A = {q0 = 1, q1 = 0}, B = {q0 = 0, q1 = 1}
 *   DEXC on (q0, q1, q2, q3):  A = {q0 = q1 = 1, q2 = q3 = 0},
 *                              B = {q0 = q1 = 0, q2 = q3 = 1}
 * Only specialised kernels (vqe_set_specialize) and the batched small-state
 * kernel apply them; interpreted evaluations of a circuit holding one return
 * VQE_ERR_UNSUPPORTED, and the default kernel form runs such circuits
 * specialised at every size. */
#define VQE_GATE_SEXC  7
#define VQE_GATE_DEXC  8

/* ---- expectation modes ---- */
#define VQE_EXPECT_GROUPED   0  /* one sweep per X-mask group serves every Z pattern */
#define VQE_EXPECT_PER_TERM  1  /* one sweep per Pauli term (Sec. III-D evaluation order) */

/* ---- gradient methods ---- */
#define VQE_GRAD_ADJOINT      0  /* reverse sweep un-applying one gate at a time */
#define VQE_GRAD_PARAM_SHIFT  1  /* [E(t + pi/2 e_k) - E(t - pi/2 e_k)] / 2 per parameter;
                                     excitation gates: the four-term rule (see vqe_energy_grad) */

/* ---- slimming modes (Sec. II-D, III-D) ---- */
#define VQE_SLIM_THRESHOLD       0  /* keep iff |w| >= value */
#define VQE_SLIM_REMOVE_PERCENT  1  /* remove floor(N * value / 100) smallest terms */
#define VQE_SLIM_BUDGET          2  /* remove smallest terms while sum |w| <= value */
#define VQE_SLIM_KEEP_TOP        3  /* keep the value most important non-identity terms */

typedef struct vqe_state vqe_state;
typedef struct vqe_circuit vqe_circuit;
typedef struct vqe_hamiltonian vqe_hamiltonian;

/* One gate (24 bytes).  A gate with param_index >= 0 takes its angle from
 * the parameter vector passed at evaluation time, else from `angle`.  RY, RZ,
 * RX, SEXC and DEXC may be parameterised.  q1 is used by CNOT, CZ, SEXC and
 * DEXC, q2 and q3 by DEXC; the qubits of one gate must differ.  Reserved
 * fields are ignored. */
typedef struct vqe_gate {
    uint8_t kind;
    uint8_t q0;
    uint8_t q1;
    uint8_t q2;
    uint8_t q3;
    uint8_t reserved[3];
    int32_t param_index;
    int32_t reserved2;
    double angle;
} vqe_gate;

/* Options of vqe_energy_grad. */
typedef struct vqe_grad_opts {
    int32_t method;        /* VQE_GRAD_ADJOINT or VQE_GRAD_PARAM_SHIFT */
    int32_t expect_mode;   /* energy evaluation used by PARAM_SHIFT: VQE_EXPECT_* */
    int32_t n_ckpt;        /* number of checkpoint states in ckpt (ADJOINT only; may be 0) */
    int32_t chunk_passes;  /* ADJOINT: > 0 waits for the state's stream after every chunk_passes
                              window passes of the forward and reverse sweeps (one ansatz layer
                              is about passes / layers), so that at most that many passes of
                              this evaluation are queued on the device at a time and work that
                              other threads submit on other streams starts within one chunk;
                              0 queues the whole evaluation at once; < 0 is VQE_ERR_ARG.
                              Results do not depend on it. */
    vqe_state* const* ckpt;/* n_ckpt states of the same n and dtype as psi; their
                              contents are overwritten */
} vqe_grad_opts;

/* Message of the last failed call on this thread ("" if none). */
const char* vqe_last_error(void);

/* Library version, e.g. "1.0.0". */
const char* vqe_version(void);

/* Number of HIP devices visible (0 when none); never fails. */
int vqe_device_count(void);

/* ------------------------------------------------------------------ states
 * A state holds 2^n amplitudes (memory 2^(n+3) or 2^(n+4) bytes, Sec. I).
 *   n_qubits   1 .. 40
 *   dtype      VQE_C64 or VQE_C128
 *   device_buf device memory of at least buf_bytes >= 2^n * amplitude size,
 *              BORROWED (it must outlive the handle), or NULL: the library
 *              allocates and owns the memory.
 *   hip_stream hipStream_t on which all work of this state is enqueued.
 * The new state is |0...0>. */
int vqe_state_alloc(int n_qubits, int dtype, void* device_buf, size_t buf_bytes,
                    void* hip_stream, vqe_state** out);
int vqe_state_free(vqe_state* s);

/* psi = |b>, the basis state with index b < 2^n (eq. 6 with psi_ref = |b>). */
int vqe_state_set_basis(vqe_state* s, uint64_t basis_index);

/* Device pointer, qubit count and dtype of a state. */
int vqe_state_info(const vqe_state* s, void** device_ptr, int* n_qubits, int* dtype);

/* Copy `count` amplitudes starting at `offset` to / from host memory
 * (interleaved re, im of the state's dtype).  Synchronous. */
int vqe_state_read(const vqe_state* s, uint64_t offset, uint64_t count, void* host_dst);
int vqe_state_write(vqe_state* s, uint64_t offset, uint64_t count, const void* host_src);

/* ------------------------------------------------------------------ circuits
 * U(theta) as an ordered gate list (applied first to last).  Creating a
 * circuit plans its fused passes: gates are grouped into windows of at most
 * 5 (interpreted kernels) or VQE_MAX_WINDOW (specialised kernels) qubits, one
 * HBM read and write of the state per window, respecting the order of every
 * gate pair that shares a qubit. */
int vqe_circuit_create(int n_qubits, const vqe_gate* gates, size_t n_gates, vqe_circuit** out);
int vqe_circuit_free(vqe_circuit* c);

/* n_params = 1 + the largest param_index used (0 if none); n_passes = fused
 * state sweeps per application under the current kernel form. */
int vqe_circuit_info(const vqe_circuit* c, size_t* n_params, size_t* n_passes);

/* Inspection of the fused plan that an evaluation would use now (it depends
 * on the kernel form, see vqe_set_specialize: windows of at most 5 qubits for
 * interpreted kernels, VQE_MAX_WINDOW for specialised ones; the same plan for
 * both dtypes, which are only checked): pass `pass` has a window of *window
 * qubits (listed ascending in qubits[0..*window-1]; the caller provides
 * VQE_MAX_WINDOW entries) and applies *n_gates gates whose indices into the
 * circuit's gate list, in execution order, are written to gate_index
 * (capacity entries; may be NULL to query the count).  Host only. */
#define VQE_MAX_WINDOW 7
int vqe_circuit_pass(const vqe_circuit* c, int dtype, size_t pass, int* window, int* qubits,
                     size_t* n_gates, int32_t* gate_index, size_t capacity);

/* psi <- U(params) psi  (eq. 6).  params has n_params doubles (host). */
int vqe_apply_circuit(vqe_state* s, const vqe_circuit* c, const double* params, size_t n_params);

/* psi <- U psi for a dense 2^k x 2^k complex unitary U on k = VQE_DENSE_K
 * qubits (one fused window of the ansatz of eq. 6 as a matrix), on the matrix
 * cores: FP32 MFMA for a complex64 state, FP64 MFMA for complex128.  This is
 * the dense alternative to the gate-by-gate window passes of
 * vqe_apply_circuit, kept for comparing the two (it is not used by the other
 * calls).
 *   qubits: k distinct qubits, each in [4, n): bit i of a row or column index
 *           of U is qubit qubits[i]; the four lowest qubits stay outside the
 *           window so that the 16 cosets a wave takes are contiguous.
 *   u:      host, 2^k x 2^k complex row-major (row = output pattern) as
 *           interleaved (re, im) doubles; copied before the call returns.
 *           Unitarity is not checked.
 * Enqueued on the state's stream, no synchronisation.  Errors: VQE_ERR_ARG
 * (null, k != VQE_DENSE_K, a qubit outside [4, n) or repeated),
 * VQE_ERR_DEVICE. */
#define VQE_DENSE_K 5
int vqe_apply_dense(vqe_state* s, const int* qubits, int k, const double* u);

/* ------------------------------------------------------------------ Hamiltonians
 * H = sum_i w_i P(x_i, z_i)  (eqs. 2-4).  Masks must have no bit >= n and the
 * weights must be finite.  Repeated (x, z) pairs are summed.  The terms are
 * grouped by x mask and the phase i^popcount(x&z) is folded into signed real
 * or imaginary coefficients; the tables are uploaded to the current device. */
int vqe_hamiltonian_create(int n_qubits, const uint64_t* x, const uint64_t* z, const double* w,
                           size_t n_terms, vqe_hamiltonian** out);
int vqe_hamiltonian_free(vqe_hamiltonian* h);

/* Number of distinct terms, of X-mask groups (the identity counted with the
 * diagonal group), and the identity coefficient. */
int vqe_hamiltonian_info(const vqe_hamiltonian* h, size_t* n_terms, size_t* n_groups,
                         double* identity_weight);

/* energy = <psi|H|psi> / <psi|psi>  (eq. 7); norm (nullable) = <psi|psi>.
 * mode VQE_EXPECT_GROUPED serves every Z pattern of an X-mask group from one
 * read of the partner amplitudes: either m passes over 13-qubit windows (the
 * window form of vqe_hamiltonian_plan, reading psi once per pass, m S in
 * all), when that reads less than the tile form, or one sweep over tiles of
 * 1024 amplitudes that reads each distinct out-of-tile partner tile once per
 * pair ((1 + D/2) S; D as for vqe_hamiltonian_plan; S = state bytes).
 * VQE_EXPECT_PER_TERM sweeps the state once per term.  Reductions across
 * blocks are FP64 in a fixed order, so repeated calls give identical bits. */
int vqe_expect_pauli(vqe_state* s, const vqe_hamiltonian* h, int mode, double* energy, double* norm);

/* vqe_expect_pauli in VQE_EXPECT_GROUPED mode for callers that cannot
 * allocate memory: code under HIP graph capture, serving loops and harnesses
 * that forbid hipMalloc.  It allocates nothing (no hipMalloc, no pinned host
 * memory) and does not synchronise: its kernels, the same as
 * vqe_expect_pauli's grouped sweep, are enqueued on the state's stream, and
 * the results are written to device memory of the caller:
 *   d_out  device memory of the state's device, 2 doubles:
 *          d_out[0] = <psi|H|psi> / <psi|psi>, d_out[1] = <psi|psi>;
 *          bitwise equal to vqe_expect_pauli's energy and norm.
 * The per-block partial sums and the reduced sums live in a library-owned
 * device array of VQE_NOALLOC_SCRATCH_BYTES per device (held until the process
 * ends), shared by every call on that device and left holding the last
 * call's values: calls on one device that may overlap (other streams, no
 * ordering between them) race and give undefined results.  Tracing
 * (vqe_profile_enable) records nothing on a stream under capture.
 * The Hamiltonian's device tables must already exist: any earlier
 * evaluation with h (vqe_expect_pauli, vqe_apply_hamiltonian,
 * vqe_energy_grad) uploads them.
 * Errors: VQE_ERR_ARG (null, qubit counts differ, d_out not device memory of
 * the state's device), VQE_ERR_STATE (tables not uploaded),
 * VQE_ERR_UNSUPPORTED (a sweep needing more partial sums than the scratch
 * holds), VQE_ERR_DEVICE. */
#define VQE_NOALLOC_SCRATCH_BYTES 65792
int vqe_expect_pauli_noalloc(vqe_state* s, const vqe_hamiltonian* h, double* d_out);

/* lam <- H psi (out of place) and energy = Re<psi|lam>/<psi|psi>. */
int vqe_apply_hamiltonian(vqe_state* psi, vqe_state* lam, const vqe_hamiltonian* h,
                          double* energy, double* norm);

/* Energy of psi(theta) = U(theta)|0...0> and its gradient dE/dtheta_k for all
 * k (grad has n_params doubles).
 *   ADJOINT: forward sweep, lam = H psi, then one reverse sweep un-applying
 *     one gate at a time from psi and lam, with dE/dtheta_k = Im<lam|G_k|psi>
 *     / <psi|psi> just after gate k, R_k = exp(-i theta_k G_k / 2).  lam must
 *     be a distinct state of the same n and dtype.  With n_ckpt > 0 forward
 *     states are kept at evenly spaced pass boundaries and restored during the
 *     reverse sweep, which bounds the drift of the un-applied psi.
 *   PARAM_SHIFT: one circuit run at theta and two per parameter (the
 *     independent circuit runs of Sec. II-C), energies by opts->expect_mode;
 *     for a parameter of an excitation gate four runs and
 *     dE/dt = d1 [E(t + pi/2) - E(t - pi/2)] - d2 [E(t + 3pi/2) - E(t - 3pi/2)],
 *     d1,2 = (sqrt2 +- 1) / (4 sqrt2) (generator eigenvalues 0, +-1; Anselmetti
 *     et al. 2021).  Exact when each parameter drives one gate.  lam is unused
 *     (may be NULL).
 * psi is overwritten; on return it holds U(theta)|0> for PARAM_SHIFT and the
 * reference |0...0> (up to rounding) for ADJOINT, possibly with the sign -1:
 * the specialised reverse kernels un-apply rotations by angles beyond a
 * quarter turn as a half turn (a sign on psi and lam together, which the
 * gradient does not see) and three shears. */
int vqe_energy_grad(vqe_state* psi, vqe_state* lam, const vqe_circuit* c,
                    const double* params, size_t n_params, const vqe_hamiltonian* h,
                    const vqe_grad_opts* opts, double* energy, double* grad);

/* ------------------------------------------------------------------ batched states
 * Many independent energy + gradient evaluations (the independent circuit
 * runs of Sec. II-C, here from many optimiser instances) in few launches.
 * Items may mix circuits, Hamiltonians and qubit counts (n <=
 * VQE_BATCH_MAX_QUBITS_MID).
 *   Small items, n <= VQE_BATCH_MAX_QUBITS_C64 (complex64) or
 *   VQE_BATCH_MAX_QUBITS_C128 (complex128): one launch, one workgroup per
 *   item holding psi and lam = H psi in LDS, running the forward gates, the
 *   energy (eq. 7) and the adjoint reverse sweep.
 *   Mid-size items, above that up to VQE_BATCH_MAX_QUBITS_MID: psi and lam
 *   in device memory owned by the batch handle (2 x 2^n amplitudes per
 *   item); the gates are fused into passes over 10-qubit windows, and one
 *   launch applies pass k of every item that has one, a workgroup staging
 *   one 2^10-amplitude tile of a window in LDS at a time; then lam = H psi
 *   and the energy (the 13-qubit window passes of each Hamiltonian, one
 *   launch per pass index, or one tile launch for Hamiltonians without a
 *   window cover), the reverse passes likewise, and one launch reducing
 *   per-block partial sums.
 * Each item's result depends only on that item (fixed per-item work and
 * reduction order), so it is bitwise the same alone or in any batch.  A
 * batch handle owns device and pinned staging buffers, grown on demand to
 * the largest call and held until vqe_batch_free, and runs on its stream;
 * vqe_batch_energy_grad returns after the results are on the host.  Calls on
 * one handle must not overlap (one handle per thread); handles are
 * independent of each other.
 * Errors: VQE_ERR_ARG (a null field, n above the limit, a Hamiltonian of
 * another size, too few parameters), VQE_ERR_OOM (buffers). */
#define VQE_BATCH_MAX_QUBITS_C64  13
#define VQE_BATCH_MAX_QUBITS_C128 12
#define VQE_BATCH_MAX_QUBITS_MID  24
typedef struct vqe_batch vqe_batch;
typedef struct vqe_batch_item {
    const vqe_circuit* circuit;
    const vqe_hamiltonian* hamiltonian;  /* same n as the circuit */
    const double* params;                /* host, n_params of the circuit */
    size_t n_params;
    double* energy;                      /* host out */
    double* grad;                        /* host out, n_params */
} vqe_batch_item;
int vqe_batch_create(int dtype, void* hip_stream, vqe_batch** out);
int vqe_batch_free(vqe_batch* b);
int vqe_batch_energy_grad(vqe_batch* b, size_t n_items, const vqe_batch_item* items);

/* ------------------------------------------------------------------ streams
 * A HIP stream of the current device for the work of states (vqe_state_alloc's
 * hip_stream), optionally restricted to a subset of the compute units, so
 * that the short kernels of latency-sensitive evaluations (small served
 * requests) do not wait for compute units held by long-running passes of
 * large ones.
 *   cu_mask     bit i of word i / 32 selects compute unit i (hipExtStreamCreateWithCUMask);
 *               NULL with mask_words = 0: an ordinary non-blocking stream
 *   mask_words  32-bit words in cu_mask
 *   stream      out: the hipStream_t; release with vqe_stream_destroy
 * Default priority.  Errors: VQE_ERR_ARG (null, a mask selecting no compute
 * unit of the device), VQE_ERR_DEVICE. */
int vqe_stream_create(const uint32_t* cu_mask, size_t mask_words, void** stream);
int vqe_stream_destroy(void* stream);

/* ------------------------------------------------------------------ tracing
 * Per-kernel timing with HIP events.  While enabled (process-wide), every
 * launch of a state-sweeping kernel is bracketed by two events recorded on
 * the stream it runs on; vqe_profile_read synchronises those events and
 * returns, for one kernel kind, the number of launches, their summed device
 * time in milliseconds and their summed algorithmic bytes (the bytes the
 * method must move: 2 S per forward window pass, 4 S per reverse window
 * pass, (1 + D) S read + S written for H psi where D is the number of
 * distinct partner tiles, or 2 S (first) / 3 S (others) per window pass of H
 * psi, S per per-term sweep; S = state bytes). */
#define VQE_KERNEL_WINDOW_FWD  0
#define VQE_KERNEL_WINDOW_REV  1
#define VQE_KERNEL_HPSI        2
#define VQE_KERNEL_EXPECT_HALF 3   /* grouped energy-only sweep: S per window pass, or (1 + D/2) S */
#define VQE_KERNEL_PER_TERM    4
#define VQE_KERNEL_DENSE       5   /* vqe_apply_dense (2 S) */
#define VQE_KERNEL_KINDS       6
int vqe_profile_enable(int on);
int vqe_profile_reset(void);
int vqe_profile_read(int kind, uint64_t* launches, double* total_ms, double* bytes);

/* Inspection of how lam = H psi (vqe_apply_hamiltonian, the adjoint of
 * vqe_energy_grad) runs for this Hamiltonian.  Host only.
 *   Tile form (*n_windows = 0): one sweep over tiles of 1024 amplitudes that
 *     reads the partner tile of every distinct out-of-tile x: (1 + D) S read,
 *     S written (D = distinct non-zero x >> 10, S = state bytes).
 *   Window form (*n_windows = m > 0): m passes over 13-qubit windows that
 *     all contain qubits 0..2, every X group inside one window; a pass reads
 *     psi and writes lam (the first) or reads and writes it (the others):
 *     (3 m - 1) S.  Chosen when it moves fewer bytes; n >= VQE_HPSI_WINDOW_QUBITS
 *     only.  Terms
 *     of a group with equal z bits inside the window share one coefficient
 *     per coset (a class); a window with more than 512 classes takes several
 *     passes over the same qubits.
 * window_masks (capacity entries, may be NULL) receives each pass's qubit
 * mask in pass order. */
#define VQE_HPSI_WINDOW_QUBITS 13
int vqe_hamiltonian_plan(const vqe_hamiltonian* h, size_t* n_windows, uint64_t* window_masks, size_t capacity);

/* ------------------------------------------------------------------ kernel form
 * Window passes of the ansatz (eq. 6) and of the adjoint sweep run either as
 * interpreted kernels (one compiled kernel per window size that reads the
 * pass's op list at run time) or as specialised kernels: straight-line code
 * generated for each distinct op list and compiled at run time (hiprtc,
 * gfx950) the first time a circuit runs on a device, then cached for the
 * process.  Both compute the same pass; specialised kernels spend no
 * instructions on op dispatch or on permutation gates (CNOT, X), which
 * matters when a pass is bound by vector instructions.
 *   VQE_SPECIALIZE_NEVER   interpreted kernels only
 *   VQE_SPECIALIZE_AUTO    specialised kernels for circuits of at least
 *                          VQE_SPECIALIZE_AUTO_MIN_QUBITS qubits (default)
 *   VQE_SPECIALIZE_ALWAYS  specialised kernels for every circuit
 * Process-wide; takes effect at the next evaluation of a circuit.  Returns
 * the previous mode, or VQE_ERR_ARG for an unknown mode.  A specialised
 * kernel that fails to compile or load makes the evaluation fail with
 * VQE_ERR_STATE / VQE_ERR_DEVICE (message in vqe_last_error). */
#define VQE_SPECIALIZE_NEVER   0
#define VQE_SPECIALIZE_AUTO    1
#define VQE_SPECIALIZE_ALWAYS  2
#define VQE_SPECIALIZE_AUTO_MIN_QUBITS 20
int vqe_set_specialize(int mode);

/* Compiles and loads, on the calling thread's current HIP device, the
 * specialised kernels that an evaluation of `dtype` (VQE_C64 / VQE_C128)
 * would use under the current kernel form; returns VQE_OK at once when that
 * form is interpreted or the kernels are already loaded.  Evaluations do this
 * themselves on first use: call it to keep compilation (about a second per
 * distinct pass, in parallel) out of a latency-sensitive first evaluation,
 * e.g. when a served instance is registered.  Errors as for evaluations. */
int vqe_circuit_prepare(const vqe_circuit* c, int dtype);

/* ------------------------------------------------------------------ slimming
 * Hamiltonian cutoff (Sec. II-D; terms sorted by |w|, small ones dropped).
 * Host only.  The identity term (x = z = 0) is always kept.  The order of
 * importance is (|w| descending, x ascending, z ascending).
 *   THRESHOLD:       keep iff |w| >= value (value >= 0).
 *   REMOVE_PERCENT:  value = integer percentage p in [0, 100]; drop the last
 *                    floor(N p / 100) non-identity terms of that order.
 *   BUDGET:          walk that order from its end adding |w| into an FP64
 *                    running sum; drop while the sum stays <= value.
 *   KEEP_TOP:        value = integer count K >= 0; keep the first K
 *                    non-identity terms of that order (all if K >= N): the
 *                    "top N x ratio terms" of the cutoff-ratio search
 *                    (Algorithm 1), with K = floor(N x ratio).
 * keep[i] (out, n_terms bytes) = 1 to keep term i, else 0; n_kept (nullable)
 * = number kept; dropped_abs_sum (nullable) = sum of the dropped |w|, added in
 * ascending order of importance: a bound on |E_full - E_slim| for any
 * normalised state (Sec. II-D). */
int vqe_slim_hamiltonian(const uint64_t* x, const uint64_t* z, const double* w, size_t n_terms,
                         int mode, double value, uint8_t* keep, size_t* n_kept,
                         double* dropped_abs_sum);

#ifdef __cplusplus
}
#endif

#endif /* VQE_H_ */
