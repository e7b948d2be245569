// C ABI of the VQE library: state handles, circuits (fused pass plans),
// Hamiltonian tables and the energy / gradient drivers.  All device work is
// enqueued on the state's stream; host scalars are returned after one
// synchronisation of that stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "vqe_internal.h"

using namespace vqe;

namespace vqe {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& m) { g_last_error = m; }
}  // namespace vqe

#define VQE_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
            return VQE_ERR_DEVICE;                                                     \
        }                                                                              \
    } while (0)

#define VQE_GUARD_BEGIN try {
#define VQE_GUARD_END                                                                  \
    }                                                                                  \
    catch (const std::bad_alloc&) {                                                    \
        set_error("host allocation failed");                                           \
        return VQE_ERR_OOM;                                                            \
    }                                                                                  \
    catch (const std::exception& ex) {                                                 \
        set_error(std::string("internal error: ") + ex.what());                        \
        return VQE_ERR_STATE;                                                          \
    }

// ---------------------------------------------------------------- handles
struct vqe_state {
    int n = 0;
    int dtype = 0;
    void* data = nullptr;
    size_t bytes = 0;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    double* d_part = nullptr;  // per-block partial sums (allocated on first use)
    double* d_res = nullptr;   // results (energies, gradients), grown on demand
    size_t res_cap = 0;
    double* h_res = nullptr;   // pinned host mirror of d_res
    void* d_mats = nullptr;    // matrix table of the specialised kernels, filled per evaluation
    void* h_mats = nullptr;    // pinned staging of d_mats
    // per pass, whether the shear forms of its reverse rotations flip the sign
    // of psi and lam an odd number of times (filled with the matrix table)
    std::vector<int8_t> rev_flip;
    size_t mats_cap = 0;
    hipEvent_t mats_ev = nullptr;  // completion of the last upload from h_mats
};

// Physical op list of a pass in the lane-split layout with S split bits.
struct SplitOps {
    std::vector<KOp> ops;
    uint8_t map_in[kMaxWindow] = {0}, map_out[kMaxWindow] = {0};  // physical slot -> window local bit
};

struct PassOps {
    std::vector<KOp> fwd, rev;
    std::vector<int> fwd_mat_gate, rev_mat_gate;  // matrix slot -> gate index
    std::vector<int32_t> slot_param;              // reverse gradient slot -> parameter
    // Per dtype (0: complex64, 1: complex128): lane-split bits of the forward
    // and reverse pass and, where S > 0, the ops lowered to physical slots.
    int S_f[2] = {0, 0}, S_r[2] = {0, 0};
    SplitOps fwd_l[2], rev_l[2];
};

// A fused pass plan: interpreted (windows <= kInterpWindow qubits, ops and
// matrices as kernel arguments) or specialised (windows <= kMaxWindow, one
// run-time compiled kernel per pass, matrices from a per-evaluation table).
struct Plan {
    bool jit = false;
    std::vector<PlannedPass> passes;
    std::vector<PassOps> ops;
    std::vector<int32_t> slotmap;   // all passes' gradient slot -> parameter maps
    int32_t* d_slotmap = nullptr;   // uploaded on first use on a device
    std::vector<size_t> slot_off;
    std::vector<size_t> mat_off;    // [2 pass + dir]: first matrix of the pass in the table
    size_t mat_total = 0;
    std::vector<void*> jfn[2][2];   // [dtype][dir] specialised kernels, built on first use
    int jit_dev[2] = {-1, -1};      // device they are loaded on
};

// One pass of the mid-size batched form: a window of kMidWin qubits and its
// gates (window-local qubits) in mid_gates[gate_off, gate_off + n_gates);
// its parameterised gates, last first, own gradient slots
// [slot_off, slot_off + n_slots) of mid_slot_pidx.
struct MidPlanPass {
    uint32_t pos[kMidWin];
    uint32_t gate_off, n_gates, slot_off, n_slots;
};

struct vqe_circuit {
    int n = 0;
    std::vector<Gate> gates;
    size_t n_params = 0;
    std::vector<BatchGate> bgates;  // gate table of the batched small-state kernel
    uint32_t n_mats = 0;            // matrices per evaluation (gates with a 2x2 matrix)
    Plan plan[2];  // [0]: interpreted (not built for circuits with excitation gates), [1]: specialised
    bool has_excitation = false;
    // batched mid-size form (kMidWin < n <= kMidMaxQubits)
    std::vector<MidPlanPass> mid;
    std::vector<BatchGate> mid_gates;
    std::vector<int32_t> mid_slot_pidx;
};

struct vqe_hamiltonian {
    int n = 0;
    std::vector<uint64_t> x, z;  // combined terms, sorted by (x, z)
    std::vector<double> w;
    std::vector<GroupDesc> groups;
    std::vector<TermDesc<float>> t32;
    std::vector<TermDesc<double>> t64;
    double identity = 0.0;
    // every folded coefficient real (each term has an even number of Y, as for
    // any real symmetric H): the window passes of H psi skip imaginary parts
    bool real_coeffs = true;
    // device tables, uploaded on first use on a device (all of them, then d_ready)
    bool d_ready = false;
    GroupDesc* d_groups = nullptr;
    TermDesc<float>* d_t32 = nullptr;
    TermDesc<double>* d_t64 = nullptr;
    // window-pass form of H psi (empty when the tile kernel moves fewer bytes
    // for both uses): hw_lam selects it for lam = H psi, hw_energy for the
    // energy-only sweep
    bool hw_lam = false, hw_energy = false;
    std::vector<HwDesc> hw_wins;
    std::vector<HwGroup> hw_groups;
    std::vector<HwClass> hw_classes;
    std::vector<HwTerm<float>> hw_t32;
    std::vector<HwTerm<double>> hw_t64;
    HwGroup* d_hw_groups = nullptr;
    HwClass* d_hw_classes = nullptr;
    HwTerm<float>* d_hw_t32 = nullptr;
    HwTerm<double>* d_hw_t64 = nullptr;
};

struct vqe_batch {
    int dtype = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    void* d_buf = nullptr;   // items | gates | mats | out, one allocation
    size_t d_cap = 0;
    void* h_buf = nullptr;   // pinned staging of the same layout
    size_t h_cap = 0;
    // mid-size items: tables | out | partial sums | states (device), tables | out (pinned)
    void* md_buf = nullptr;
    size_t md_cap = 0;
    void* mh_buf = nullptr;
    size_t mh_cap = 0;
};

namespace {

size_t amp_bytes(int dtype) { return dtype == VQE_C64 ? 8 : 16; }

std::mutex g_upload_mu;  // lazy device uploads of shared handles

// ---------------------------------------------------------------- tracing
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;
};
struct ProfTotals {
    uint64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
ProfTotals g_prof_tot[VQE_KERNEL_KINDS];

// Brackets one kernel launch with events when tracing is on.
struct ProfScope {
    bool on;
    ProfRec r{};
    hipStream_t st;
    ProfScope(int kind, double bytes, hipStream_t s) : on(false), st(s) {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on) return;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
        if (hipEventCreate(&r.a) != hipSuccess) return;
        if (hipEventCreate(&r.b) != hipSuccess) {
            (void)hipEventDestroy(r.a);
            return;
        }
        r.kind = kind;
        r.bytes = bytes;
        on = hipEventRecord(r.a, st) == hipSuccess;
    }
    void end() {
        if (!on) return;
        on = false;
        (void)hipEventRecord(r.b, st);
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof_pending.push_back(r);
    }
    ~ProfScope() { end(); }
};

void prof_drain() {
    for (auto& r : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof_tot[r.kind].launches += 1;
            g_prof_tot[r.kind].ms += ms;
            g_prof_tot[r.kind].bytes += r.bytes;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
}

int ensure_res(vqe_state* s, size_t count) {
    if (count <= s->res_cap) return VQE_OK;
    size_t cap = std::max<size_t>(count, 1024);
    if (s->d_res) {
        VQE_HIP(hipStreamSynchronize(s->stream));
        VQE_HIP(hipFree(s->d_res));
        s->d_res = nullptr;
    }
    if (s->h_res) {
        VQE_HIP(hipHostFree(s->h_res));
        s->h_res = nullptr;
    }
    s->res_cap = 0;
    if (hipMalloc((void**)&s->d_res, cap * sizeof(double)) != hipSuccess) {
        set_error("hipMalloc of the result buffer failed");
        return VQE_ERR_OOM;
    }
    if (hipHostMalloc((void**)&s->h_res, cap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc of the result buffer failed");
        return VQE_ERR_OOM;
    }
    s->res_cap = cap;
    return VQE_OK;
}

int upload_plan(const Plan& cpl);
bool lower_split(const std::vector<KOp>& ops, int K, int S, size_t cap, SplitOps& out);

// Device copies of a Hamiltonian's tables; the handle publishes them only
// when every one was allocated and copied (d_ready), so a failed upload
// leaves nothing half-built behind.
void free_hamiltonian_tables(vqe_hamiltonian* h) {
    void* ptrs[] = {h->d_groups, h->d_t32, h->d_t64, h->d_hw_groups, h->d_hw_classes, h->d_hw_t32, h->d_hw_t64};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    h->d_groups = nullptr;
    h->d_t32 = nullptr;
    h->d_t64 = nullptr;
    h->d_hw_groups = nullptr;
    h->d_hw_classes = nullptr;
    h->d_hw_t32 = nullptr;
    h->d_hw_t64 = nullptr;
    h->d_ready = false;
}

template <typename E>
int upload_table(E** dst, const std::vector<E>& src) {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(E);
    if (hipMalloc((void**)dst, bytes) != hipSuccess) {
        *dst = nullptr;
        set_error("hipMalloc of a Hamiltonian table failed");
        return VQE_ERR_OOM;
    }
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(E), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hipMemcpy of a Hamiltonian table failed");
        return VQE_ERR_DEVICE;
    }
    return VQE_OK;
}

// Uploads the grouped term tables to the current device (once).
int upload_hamiltonian(const vqe_hamiltonian* ch) {
    vqe_hamiltonian* h = const_cast<vqe_hamiltonian*>(ch);
    std::lock_guard<std::mutex> g(g_upload_mu);
    if (h->d_ready) return VQE_OK;
    free_hamiltonian_tables(h);  // leftovers of an earlier failed attempt
    int rc = upload_table(&h->d_groups, h->groups);
    if (!rc) rc = upload_table(&h->d_t32, h->t32);
    if (!rc) rc = upload_table(&h->d_t64, h->t64);
    if (!rc && !h->hw_wins.empty()) {
        rc = upload_table(&h->d_hw_groups, h->hw_groups);
        if (!rc) rc = upload_table(&h->d_hw_classes, h->hw_classes);
        if (!rc) rc = upload_table(&h->d_hw_t32, h->hw_t32);
        if (!rc) rc = upload_table(&h->d_hw_t64, h->hw_t64);
    }
    if (rc) {
        free_hamiltonian_tables(h);
        return rc;
    }
    h->d_ready = true;
    return VQE_OK;
}

// Greedy cover of the X masks xs (none inside `low`) by windows of kHwBits
// qubits that contain `low`.  A window grows one qubit at a time, taking the
// qubit with the largest sum over the uncovered masks containing it (and
// still fitting) of 1 / outside^p (outside = their bits not yet in the
// window), so that nearly complete masks weigh most; it takes every mask
// inside it.  With rng_state != 0 the scores are perturbed by a factor in
// [1, 1.001) from a splitmix64 stream, which only reorders near-ties.
// Returns the windows (empty if no progress is possible); *work counts the
// inner-loop steps.
std::vector<uint64_t> cover_windows(int n, const std::vector<uint64_t>& xs, uint64_t low, int p, uint64_t rng_state,
                                    size_t* work) {
    auto uniform = [&]() {
        uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
    };
    std::vector<uint64_t> rem = xs, wins;
    while (!rem.empty() || wins.empty()) {
        uint64_t W = low;
        while (__builtin_popcountll(W) < kHwBits) {
            int best = -1;
            double best_score = 0.0;
            const int inside = __builtin_popcountll(W);
            for (int q = 0; q < n; ++q) {
                if ((W >> q) & 1) continue;
                double sc = 0.0;
                for (uint64_t x : rem) {
                    if (!((x >> q) & 1)) continue;
                    const int outside = __builtin_popcountll(x & ~W);
                    if (inside + outside <= kHwBits) sc += 1.0 / std::pow((double)outside, p);
                }
                *work += rem.size();
                if (rng_state && sc > 0.0) sc *= 1.0 + 1e-3 * uniform();
                if (sc > best_score) {
                    best_score = sc;
                    best = q;
                }
            }
            if (best < 0) break;
            W |= 1ull << best;
        }
        for (int q = 0; q < n && __builtin_popcountll(W) < kHwBits; ++q) W |= 1ull << q;  // fill up
        std::vector<uint64_t> left;
        for (uint64_t x : rem)
            if (x & ~W) left.push_back(x);
        if (left.size() == rem.size() && !rem.empty()) return {};  // no progress
        rem.swap(left);
        wins.push_back(W);
    }
    return wins;
}

// Window-pass plan of lam = H psi (see HwDesc): the smallest of several
// greedy covers (cover_windows with p = 1, 2, 3, each deterministic and
// with seeded tie perturbations, as many restarts as a fixed work budget
// allows); the groups spread evenly over the windows holding them.  Used for
// lam = H psi if its (3 m - 1) S of traffic (m passes; psi read per pass, lam
// written once and read-modify-written m - 1 times) is below the tile
// kernel's (D + 2) S, and for the energy-only sweep if its m S (psi read per
// pass) is below the tile kernel's (1 + D / 2) S; kept if either holds.
void plan_hwin(vqe_hamiltonian* h) {
    const int n = h->n;
    if (n < kHwBits) return;
    const uint64_t low = (1ull << kHwLow) - 1;
    const size_t G = h->groups.size();
    std::vector<uint64_t> xs;
    for (size_t g = 0; g < G; ++g) {
        if (__builtin_popcountll(h->groups[g].x | low) > kHwBits) return;  // a mask no window can hold
        if (h->groups[g].x & ~low) xs.push_back(h->groups[g].x);
    }
    if (xs.size() > 4096) return;  // planning cost; such Hamiltonians stay on the tile kernel
    constexpr size_t kWorkBudget = 200000000;  // inner-loop steps over all restarts (well under a second)
    constexpr int kMaxRestarts = 12;
    std::vector<uint64_t> wins;
    size_t work = 0;
    for (int p = 1; p <= 3; ++p) {
        for (int r = 0; r <= kMaxRestarts; ++r) {
            const size_t before = work;
            std::vector<uint64_t> w = cover_windows(n, xs, low, p, r ? 0x5eedull * (uint64_t)(16 * p + r) : 0, &work);
            if (w.empty()) return;
            if (wins.empty() || w.size() < wins.size()) wins.swap(w);
            if (work + 3 * (work - before) > kWorkBudget) break;  // a later restart could overrun the budget
        }
        if (work > kWorkBudget) break;
    }
    // Each group goes to one of the windows holding its X mask.  A pass costs
    // about the larger of its memory time and a fixed amount of arithmetic per
    // group (the per-group bodies dominate; the class count matters little),
    // so the groups are spread evenly: those only one window holds first, then
    // the others, the most constrained first, each to the holding window where
    // it adds the least cost, max(kHwPassGroups x passes, groups) with passes =
    // ceil(classes / kHwMaxClasses); ties go to the window with fewer groups,
    // then fewer classes, then the lower index.
    constexpr size_t kHwPassGroups = 16;  // groups per pass whose arithmetic about matches its memory time
    const size_t Wn = wins.size();
    std::vector<std::vector<std::pair<int, size_t>>> cand(G);  // (window, classes of the group in it)
    std::vector<uint64_t> zw;
    for (size_t g = 0; g < G; ++g)
        for (size_t wi = 0; wi < Wn; ++wi) {
            if (h->groups[g].x & ~wins[wi]) continue;
            zw.clear();
            for (uint32_t t = h->groups[g].begin; t < h->groups[g].end; ++t) zw.push_back(h->t64[t].z & wins[wi]);
            std::sort(zw.begin(), zw.end());
            cand[g].emplace_back((int)wi, (size_t)(std::unique(zw.begin(), zw.end()) - zw.begin()));
        }
    std::vector<size_t> order(G);
    for (size_t g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cand[a].size() < cand[b].size(); });
    std::vector<size_t> w_groups(Wn, 0), w_classes(Wn, 0);
    auto w_cost = [&](size_t groups, size_t classes) {
        const size_t passes = std::max<size_t>(1, (classes + kHwMaxClasses - 1) / kHwMaxClasses);
        return std::max(kHwPassGroups * passes, groups);
    };
    std::vector<int> win_of(G, -1);
    for (size_t g : order) {
        int best = -1;
        size_t best_add = 0, best_cls = 0;
        for (const auto& [wi, cls] : cand[g]) {
            const size_t add = w_cost(w_groups[wi] + 1, w_classes[wi] + cls) - w_cost(w_groups[wi], w_classes[wi]);
            if (best < 0 || add < best_add ||
                (add == best_add && (w_groups[wi] < w_groups[best] ||
                                     (w_groups[wi] == w_groups[best] && w_classes[wi] + cls < w_classes[best] + best_cls)))) {
                best = wi;
                best_add = add;
                best_cls = cls;
            }
        }
        if (best < 0) return;  // cannot happen for a cover; the tile form stays
        win_of[g] = best;
        w_groups[best] += 1;
        w_classes[best] += best_cls;
    }
    // Passes: per window its groups, the terms of a group merged into classes
    // of equal in-window z bits and sorted by them (register part first), at
    // most kHwMaxClasses classes per pass.  A window with more classes takes
    // several passes over the same qubits; lam accumulates over passes, so a
    // group's classes may also be split between two of them.
    std::vector<HwDesc> passes;
    std::vector<HwGroup> hgroups;
    std::vector<HwClass> hclasses;
    std::vector<HwTerm<float>> ht32;
    std::vector<HwTerm<double>> ht64;
    constexpr int kBuckets = 1 << kHwRegBits;
    const uint32_t tmask = (1u << kHwThreadBits) - 1;
    for (size_t wi = 0; wi < wins.size(); ++wi) {
        HwDesc d{};
        int k = 0, local[64];
        for (int q = 0; q < n; ++q)
            if ((wins[wi] >> q) & 1) {
                local[q] = k;
                d.pos[k++] = (uint32_t)q;
            }
        auto compress = [&](uint64_t m) {
            uint32_t r = 0;
            for (int q = 0; q < n; ++q)
                if ((m >> q) & 1) r |= 1u << local[q];
            return r;
        };
        d.g_begin = (uint32_t)hgroups.size();
        d.c_begin = (uint32_t)hclasses.size();
        for (size_t g = 0; g < G; ++g) {
            if (win_of[g] != (int)wi) continue;
            const GroupDesc& gd = h->groups[g];
            std::map<uint32_t, std::vector<uint32_t>> cls;  // in-window z bits -> terms
            for (uint32_t t = gd.begin; t < gd.end; ++t) cls[compress(h->t64[t].z & wins[wi])].push_back(t);
            auto it = cls.begin();
            while (it != cls.end()) {
                if (hclasses.size() - d.c_begin == (size_t)kHwMaxClasses) {  // pass full
                    d.g_end = (uint32_t)hgroups.size();
                    d.c_end = (uint32_t)hclasses.size();
                    passes.push_back(d);
                    d.g_begin = d.g_end;
                    d.c_begin = d.c_end;
                }
                HwGroup hg{};
                hg.xl = compress(gd.x);
                int u = 0;
                hg.cb[0] = (uint32_t)hclasses.size();
                for (; it != cls.end() && hclasses.size() - d.c_begin < (size_t)kHwMaxClasses; ++it) {
                    const int bucket = (int)(it->first >> kHwThreadBits);
                    while (u < bucket) hg.cb[++u] = (uint32_t)hclasses.size();
                    hg.zrm |= (uint32_t)bucket;
                    HwClass hc{};
                    hc.zt = it->first & tmask;
                    hc.k_begin = (uint32_t)ht64.size();
                    for (uint32_t t : it->second) {
                        const uint64_t zo = h->t64[t].z & ~wins[wi];
                        ht64.push_back(HwTerm<double>{zo, h->t64[t].cre, h->t64[t].cim});
                        ht32.push_back(HwTerm<float>{zo, h->t32[t].cre, h->t32[t].cim});
                    }
                    hc.k_end = (uint32_t)ht64.size();
                    hclasses.push_back(hc);
                }
                while (u < kBuckets) hg.cb[++u] = (uint32_t)hclasses.size();
                hgroups.push_back(hg);
            }
        }
        d.g_end = (uint32_t)hgroups.size();
        d.c_end = (uint32_t)hclasses.size();
        passes.push_back(d);
    }
    std::vector<uint64_t> hi;
    for (const auto& g : h->groups)
        if (g.x >> kTileBits) hi.push_back(g.x >> kTileBits);
    std::sort(hi.begin(), hi.end());
    const size_t D = std::unique(hi.begin(), hi.end()) - hi.begin();
    const size_t m = passes.size();
    h->hw_lam = 3 * m - 1 < D + 2;
    h->hw_energy = 2 * m < 2 + D;
    // batched mid-size states use the window passes whenever a cover exists
    // (their states stay in cache, so arithmetic, not bytes, decides)
    if (!h->hw_lam && !h->hw_energy && n > kMidMaxQubits) return;
    h->hw_wins.swap(passes);
    h->hw_groups.swap(hgroups);
    h->hw_classes.swap(hclasses);
    h->hw_t32.swap(ht32);
    h->hw_t64.swap(ht64);
}

// Per-block partial-sum buffer of a state: room for the largest launch
// (kMaxPartBlocks blocks x kMaxGradSlots slots).
int ensure_part(vqe_state* s) {
    if (s->d_part) return VQE_OK;
    const size_t count = std::max((size_t)kMaxPartBlocks * kMaxGradSlots, (size_t)kMaxBlocks * 2);
    if (hipMalloc((void**)&s->d_part, count * sizeof(double)) != hipSuccess) {
        s->d_part = nullptr;
        set_error("hipMalloc of the partial-sum buffer failed");
        return VQE_ERR_OOM;
    }
    return VQE_OK;
}

// Angle of gate g under params.
double angle_of(const Gate& g, const double* params) { return g.pidx >= 0 ? params[g.pidx] : g.angle; }

template <typename T>
void fill_matrix(Mat2<T>& m, const Gate& g, double th, bool inverse) {
    if (inverse) th = -th;
    const double c = std::cos(th / 2), s = std::sin(th / 2);
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    switch (g.kind) {
        case VQE_GATE_RY:  // [[c, -s], [s, c]]
        case VQE_GATE_SEXC:  // the same rotation between the A and B patterns
        case VQE_GATE_DEXC:
            v[0] = c; v[2] = -s; v[4] = s; v[6] = c;
            break;
        case VQE_GATE_RZ:  // diag(e^{-i t/2}, e^{i t/2})
            v[0] = c; v[1] = -s; v[6] = c; v[7] = s;
            break;
        case VQE_GATE_RX:  // [[c, -i s], [-i s, c]]
            v[0] = c; v[3] = -s; v[5] = -s; v[6] = c;
            break;
        case VQE_GATE_H: {
            const double r = 1.0 / std::sqrt(2.0);
            v[0] = r; v[2] = r; v[4] = r; v[6] = -r;
            break;
        }
        default:
            break;
    }
    for (int i = 0; i < 8; ++i) m.v[i] = (T)v[i];
}

uint8_t mat_op(int kind) {
    switch (kind) {
        case VQE_GATE_RY: return OP_R2;
        case VQE_GATE_RZ: return OP_DIAG;
        case VQE_GATE_H: return OP_R2;
        default: return OP_U2;
    }
}

uint8_t grad_op(int kind) {
    switch (kind) {
        case VQE_GATE_RY: return OP_GY;
        case VQE_GATE_RZ: return OP_GZ;
        case VQE_GATE_SEXC: return OP_GPAIR2;
        case VQE_GATE_DEXC: return OP_GPAIR4;
        default: return OP_GX;
    }
}

bool is_excitation(int kind) { return kind == VQE_GATE_SEXC || kind == VQE_GATE_DEXC; }

int local_bit(const PlannedPass& p, int q) {
    for (int j = 0; j < p.K; ++j)
        if (p.pos[j] == q) return j;
    return -1;
}

// Appends the op that applies gate gi (or its inverse) to `ops`.
void emit_gate(const Gate& g, int gi, const PlannedPass& p, std::vector<KOp>& ops,
               std::vector<int>& mat_gate) {
    KOp op{};
    op.a = (uint8_t)local_bit(p, g.q0);
    switch (g.kind) {
        case VQE_GATE_CNOT:
            op.type = OP_CNOT;
            op.b = (uint8_t)local_bit(p, g.q1);
            break;
        case VQE_GATE_CZ:
            op.type = OP_CZ;
            op.b = (uint8_t)local_bit(p, g.q1);
            break;
        case VQE_GATE_X:
            op.type = OP_XFLIP;
            break;
        case VQE_GATE_SEXC:
        case VQE_GATE_DEXC:
            op.type = g.kind == VQE_GATE_SEXC ? OP_PAIR2 : OP_PAIR4;
            op.b = (uint8_t)local_bit(p, g.q1);
            if (g.kind == VQE_GATE_DEXC) {
                op.c = (uint8_t)local_bit(p, g.q2);
                op.d = (uint8_t)local_bit(p, g.q3);
            }
            op.slot = (uint8_t)mat_gate.size();
            mat_gate.push_back(gi);
            break;
        default:
            op.type = mat_op(g.kind);
            op.slot = (uint8_t)mat_gate.size();
            mat_gate.push_back(gi);
            // RY and RZ are plane rotations (of the amplitude pair, of each
            // amplitude's real and imaginary parts): the specialised reverse
            // kernels un-apply them as three shears (shear_coefficients)
            if (g.kind == VQE_GATE_RY || g.kind == VQE_GATE_RZ) op.c = 1;
            break;
    }
    ops.push_back(op);
}

template <typename T>
void build_args(const vqe_circuit* c, const Plan& pl, size_t pi, const double* params, bool reverse,
                PassArgs<T>& a) {
    const PlannedPass& p = pl.passes[pi];
    const PassOps& po = pl.ops[pi];
    std::memset(&a, 0, sizeof(a));
    a.K = (uint32_t)p.K;
    a.n_cosets = 1ull << (c->n - p.K);
    for (int j = 0; j < p.K; ++j) a.pos[j] = (uint32_t)p.pos[j];
    const int d = sizeof(T) == 8 ? 1 : 0;
    const int S = reverse ? po.S_r[d] : po.S_f[d];
    a.split = (uint32_t)S;
    const auto& mg = reverse ? po.rev_mat_gate : po.fwd_mat_gate;
    if (S == 0) {
        const auto& ops = reverse ? po.rev : po.fwd;
        a.n_ops = (uint32_t)ops.size();
        for (size_t i = 0; i < ops.size(); ++i) a.ops[i] = ops[i];
        for (int sl = 0; sl < p.K; ++sl) a.pos_in[sl] = a.pos_out[sl] = (uint32_t)p.pos[sl];
    } else {
        const SplitOps& so = reverse ? po.rev_l[d] : po.fwd_l[d];
        a.n_ops = (uint32_t)so.ops.size();
        for (size_t i = 0; i < so.ops.size(); ++i) a.ops[i] = so.ops[i];
        for (int sl = 0; sl < p.K; ++sl) {
            a.pos_in[sl] = (uint32_t)p.pos[so.map_in[sl]];
            a.pos_out[sl] = (uint32_t)p.pos[so.map_out[sl]];
        }
    }
    for (size_t i = 0; i < mg.size(); ++i) {
        const Gate& g = c->gates[mg[i]];
        fill_matrix(a.mats[i], g, angle_of(g, params), reverse);
    }
    a.n_gslots = reverse ? (uint32_t)po.slot_param.size() : 0;
}

int check_state(const vqe_state* s, const char* fn) {
    if (!s || !s->data) {
        set_error(std::string(fn) + ": null state");
        return VQE_ERR_ARG;
    }
    return VQE_OK;
}

int check_params(const vqe_circuit* c, const double* params, size_t n_params, const char* fn) {
    if (n_params != c->n_params) {
        set_error(std::string(fn) + ": n_params " + std::to_string(n_params) + " does not match the circuit's " +
                  std::to_string(c->n_params));
        return VQE_ERR_ARG;
    }
    if (n_params > 0 && !params) {
        set_error(std::string(fn) + ": null params");
        return VQE_ERR_ARG;
    }
    for (size_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) {
            set_error(std::string(fn) + ": non-finite parameter");
            return VQE_ERR_ARG;
        }
    return VQE_OK;
}

std::mutex g_jit_plan_mu;

// True if evaluations of c run the specialised plan (see vqe_set_specialize).
bool use_specialised(const vqe_circuit* c) {
    const int mode = jit_mode();
    return mode == VQE_SPECIALIZE_ALWAYS ||
           (mode == VQE_SPECIALIZE_AUTO && (c->n >= VQE_SPECIALIZE_AUTO_MIN_QUBITS || c->has_excitation));
}

// VQE_OK if the current kernel form can evaluate c (interpreted kernels have
// no excitation gates).
int check_form(const vqe_circuit* c, const char* fn) {
    if (c->has_excitation && !use_specialised(c)) {
        set_error(std::string(fn) + ": excitation gates need specialised kernels (vqe_set_specialize)");
        return VQE_ERR_UNSUPPORTED;
    }
    return VQE_OK;
}

const Plan& plan_now(const vqe_circuit* c) { return c->plan[use_specialised(c) ? 1 : 0]; }

// Physical ops, lane-split bits and slot positions of one specialised pass.
const std::vector<KOp>& jit_ops(const Plan& pl, size_t pi, int d, bool reverse, int* S, JitArgs* a, int n) {
    const PlannedPass& p = pl.passes[pi];
    const PassOps& po = pl.ops[pi];
    *S = reverse ? po.S_r[d] : po.S_f[d];
    if (a) {
        std::memset(a, 0, sizeof(*a));
        a->n_cosets = 1ull << (n - p.K);
        for (int j = 0; j < p.K; ++j) a->pos[j] = (uint32_t)p.pos[j];
    }
    if (*S == 0) {
        if (a)
            for (int j = 0; j < p.K; ++j) a->pos_in[j] = a->pos_out[j] = (uint32_t)p.pos[j];
        return reverse ? po.rev : po.fwd;
    }
    const SplitOps& so = reverse ? po.rev_l[d] : po.fwd_l[d];
    if (a)
        for (int sl = 0; sl < p.K; ++sl) {
            a->pos_in[sl] = (uint32_t)p.pos[so.map_in[sl]];
            a->pos_out[sl] = (uint32_t)p.pos[so.map_out[sl]];
        }
    return so.ops;
}

// Compiles and loads the specialised kernels of every pass of a specialised
// plan for dtype index d on the current device (once; cached).
int ensure_jit(const vqe_circuit* c, const Plan& cpl, int d) {
    Plan& pl = const_cast<Plan&>(cpl);
    int dev = 0;
    VQE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_jit_plan_mu);
    const size_t P = pl.passes.size();
    if (pl.jit_dev[d] == dev && pl.jfn[d][0].size() == P) return VQE_OK;
    std::vector<std::string> srcs(2 * P);
    for (size_t pi = 0; pi < P; ++pi)
        for (int dir = 0; dir < 2; ++dir) {
            int S = 0;
            const auto& ops = jit_ops(pl, pi, d, dir == 1, &S, nullptr, c->n);
            srcs[2 * pi + dir] = jit_source(d == 1, pl.passes[pi].K, S, dir == 1 ? 2 : 1, ops,
                                            dir == 1 ? (uint32_t)pl.ops[pi].slot_param.size() : 0);
        }
    std::vector<void*> fns;
    std::string err;
    const int rc = jit_prepare(srcs, fns, err);
    if (rc) {
        set_error(err);
        return rc;
    }
    for (int dir = 0; dir < 2; ++dir) {
        pl.jfn[d][dir].assign(P, nullptr);
        for (size_t pi = 0; pi < P; ++pi) pl.jfn[d][dir][pi] = fns[2 * pi + dir];
    }
    pl.jit_dev[d] = dev;
    return VQE_OK;
}

// Fills the matrix table of a specialised plan (every pass, both directions)
// for these parameters and uploads it on the state's stream.  The pinned
// staging buffer is reused only after its previous upload has completed.
// The state's matrix table (device) and its pinned staging copy, at least
// `bytes` long; waits until the previous upload from the staging copy is done.
int stage_mats(vqe_state* s, size_t bytes) {
    if (!s->mats_ev) VQE_HIP(hipEventCreateWithFlags(&s->mats_ev, hipEventDisableTiming));
    if (bytes > s->mats_cap) {
        VQE_HIP(hipStreamSynchronize(s->stream));
        if (s->d_mats) VQE_HIP(hipFree(s->d_mats));
        if (s->h_mats) VQE_HIP(hipHostFree(s->h_mats));
        s->d_mats = s->h_mats = nullptr;
        s->mats_cap = 0;
        if (hipMalloc(&s->d_mats, bytes) != hipSuccess || hipHostMalloc(&s->h_mats, bytes) != hipSuccess) {
            set_error("allocation of the matrix table failed");
            return VQE_ERR_OOM;
        }
        s->mats_cap = bytes;
    } else {
        VQE_HIP(hipEventSynchronize(s->mats_ev));
    }
    return VQE_OK;
}

// A plane rotation by a (x' = x cos a - y sin a, y' = x sin a + y cos a) as
// three shears x += k1 y, y += k2 x, x += k1 y with k1 = -tan(a/2) and
// k2 = sin a (Paeth's decomposition; three fused multiply-adds per plane
// instead of two products and two FMAs).  a is first brought into
// [-pi/2, pi/2] by a half turn, R(a) = -R(a -+ pi), so |k1|, |k2| <= 1;
// returns whether that flipped the sign.
template <typename T>
bool shear_coefficients(double a, Mat2<T>& m) {
    bool flip = false;
    if (a > M_PI / 2) {
        a -= M_PI;
        flip = true;
    } else if (a < -M_PI / 2) {
        a += M_PI;
        flip = true;
    }
    std::memset(&m, 0, sizeof(m));
    m.v[0] = (T)-std::tan(a / 2);
    m.v[1] = (T)std::sin(a);
    return flip;
}

template <typename T>
int upload_mats(vqe_state* s, const vqe_circuit* c, const Plan& pl, const double* params, const Mat2<T>** out) {
    const size_t bytes = std::max<size_t>(pl.mat_total, 1) * sizeof(Mat2<T>);
    if (int rc = stage_mats(s, bytes)) return rc;
    Mat2<T>* h = (Mat2<T>*)s->h_mats;
    s->rev_flip.assign(pl.passes.size(), 0);
    for (size_t pi = 0; pi < pl.passes.size(); ++pi)
        for (int dir = 0; dir < 2; ++dir) {
            const auto& mg = dir ? pl.ops[pi].rev_mat_gate : pl.ops[pi].fwd_mat_gate;
            Mat2<T>* m = h + pl.mat_off[2 * pi + dir];
            for (size_t i = 0; i < mg.size(); ++i) {
                const Gate& g = c->gates[mg[i]];
                if (dir == 1 && (g.kind == VQE_GATE_RY || g.kind == VQE_GATE_RZ)) {
                    // the inverse as a rotation: RY^-1 turns (a_0, a_1), RZ^-1 turns
                    // (Re, Im) of an amplitude with bit 0 (bit 1 by the opposite angle).
                    // Every amplitude takes part, so a half turn is a sign on the whole
                    // state; an excitation turns only its (A, B) patterns, where a half
                    // turn would not be, so excitations keep the matrix form.
                    Mat2<double> u;
                    fill_matrix(u, g, angle_of(g, params), true);
                    const double a = g.kind == VQE_GATE_RY ? std::atan2(u.v[4], u.v[0]) : std::atan2(u.v[1], u.v[0]);
                    s->rev_flip[pi] ^= (int8_t)shear_coefficients(a, m[i]);
                } else {
                    fill_matrix(m[i], g, angle_of(g, params), dir == 1);
                }
            }
        }
    VQE_HIP(hipMemcpyAsync(s->d_mats, s->h_mats, bytes, hipMemcpyHostToDevice, s->stream));
    VQE_HIP(hipEventRecord(s->mats_ev, s->stream));
    *out = (const Mat2<T>*)s->d_mats;
    return VQE_OK;
}

// psi <- U psi on one dense window (see DenseArgs).
template <typename T>
int apply_dense(vqe_state* s, const DenseArgs& a, const double* u) {
    constexpr int P = 1 << kDenseK, RR = 2 * P;
    if (int rc = stage_mats(s, sizeof(T) * RR * RR)) return rc;
    T* h = (T*)s->h_mats;
    for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) {
            const double re = u[2 * (r * P + c)], im = u[2 * (r * P + c) + 1];
            h[r * RR + c] = (T)re;
            h[r * RR + P + c] = (T)-im;
            h[(P + r) * RR + c] = (T)im;
            h[(P + r) * RR + P + c] = (T)re;
        }
    VQE_HIP(hipMemcpyAsync(s->d_mats, s->h_mats, sizeof(T) * RR * RR, hipMemcpyHostToDevice, s->stream));
    VQE_HIP(hipEventRecord(s->mats_ev, s->stream));
    ProfScope ps(VQE_KERNEL_DENSE, 2.0 * (double)s->bytes, s->stream);
    VQE_HIP(launch_dense<T>(a, (const T*)s->d_mats, s->data, s->data, s->stream));
    return VQE_OK;
}

// Forward passes from |b0> (or in place on the current state when reset is false).
// ckpt_ptr[k] receives the state at boundary bounds[k] (pass index + 1).
template <typename T>
int forward(vqe_state* s, const vqe_circuit* c, const Plan& pl, const double* params,
            const std::vector<size_t>& bounds, const std::vector<void*>& ckpt_ptr, int chunk = 0) {
    void* cur = s->data;
    const int d = sizeof(T) == 8 ? 1 : 0;
    const Mat2<T>* mats = nullptr;
    if (pl.jit) {
        int rc = ensure_jit(c, pl, d);
        if (!rc) rc = upload_mats<T>(s, c, pl, params, &mats);
        if (rc) return rc;
    }
    PassArgs<T> a;
    JitArgs ja;
    for (size_t pi = 0; pi < pl.passes.size(); ++pi) {
        void* out = s->data;
        for (size_t k = 0; k < bounds.size(); ++k)
            if (bounds[k] == pi + 1) out = ckpt_ptr[k];
        ProfScope ps(VQE_KERNEL_WINDOW_FWD, 2.0 * (double)s->bytes, s->stream);
        if (pl.jit) {
            int S = 0;
            jit_ops(pl, pi, d, false, &S, &ja, s->n);
            VQE_HIP(launch_window_jit(pl.jfn[d][0][pi], ja, S, mats + pl.mat_off[2 * pi], false, cur, out, nullptr,
                                      nullptr, nullptr, nullptr, s->stream));
        } else {
            build_args<T>(c, pl, pi, params, false, a);
            VQE_HIP(launch_window_fwd<T>(a, s->n, cur, out, s->stream));
        }
        ps.end();
        cur = out;
        if (chunk > 0 && (pi + 1) % (size_t)chunk == 0 && pi + 1 < pl.passes.size())
            VQE_HIP(hipStreamSynchronize(s->stream));
    }
    return VQE_OK;
}

template <typename T>
const TermDesc<T>* terms_of(const vqe_hamiltonian* h);
template <>
const TermDesc<float>* terms_of<float>(const vqe_hamiltonian* h) { return h->d_t32; }
template <>
const TermDesc<double>* terms_of<double>(const vqe_hamiltonian* h) { return h->d_t64; }

template <typename T>
const HwTerm<T>* hw_terms_of(const vqe_hamiltonian* h);
template <>
const HwTerm<float>* hw_terms_of<float>(const vqe_hamiltonian* h) { return h->d_hw_t32; }
template <>
const HwTerm<double>* hw_terms_of<double>(const vqe_hamiltonian* h) { return h->d_hw_t64; }

double hpsi_bytes(const vqe_hamiltonian* h, const vqe_state* s, bool write);

// lam = H psi with the energy partials reduced into d_out[0..1]
// (Re<psi|lam>, <psi|psi>): window passes when planned, else the tile kernel.
template <typename T>
int apply_h(vqe_state* psi, void* lam, const vqe_hamiltonian* h, double* d_out) {
    hipStream_t st = psi->stream;
    uint32_t nb = 0;
    if (h->hw_lam) {
        const size_t m = h->hw_wins.size();
        for (size_t wi = 0; wi < m; ++wi) {
            ProfScope ps(VQE_KERNEL_HPSI, (wi ? 3.0 : 2.0) * (double)psi->bytes, st);
            VQE_HIP(launch_hwin<T>(psi->n, h->hw_wins[wi], psi->data, lam, h->d_hw_groups, h->d_hw_classes,
                                   hw_terms_of<T>(h), h->real_coeffs,
                                   wi == 0, wi + 1 == m, psi->d_part, &nb, st));
        }
    } else {
        ProfScope ps(VQE_KERNEL_HPSI, hpsi_bytes(h, psi, true), st);
        VQE_HIP(launch_hpsi<T>(psi->n, psi->data, lam, h->d_groups, (uint32_t)h->groups.size(), terms_of<T>(h), 0,
                               (uint32_t)kMaxPartBlocks, psi->d_part, &nb, st));
    }
    VQE_HIP(launch_reduce(psi->d_part, nb, 2, nullptr, d_out, 0, st));
    return VQE_OK;
}

// Algorithmic bytes of one H psi sweep: own tile + one partner tile per
// distinct out-of-tile partner offset (x >> tile bits), plus the write of lam.
// The energy-only sweep visits each out-of-tile pair once (half the partners).
double hpsi_bytes(const vqe_hamiltonian* h, const vqe_state* s, bool write) {
    const int tb = s->n < kTileBits ? s->n : kTileBits;
    std::vector<uint64_t> hi;
    for (const auto& g : h->groups) {
        const uint64_t xh = g.x >> tb;
        if (xh && (hi.empty() || hi.back() != xh)) hi.push_back(xh);
    }
    std::sort(hi.begin(), hi.end());
    const size_t D = std::unique(hi.begin(), hi.end()) - hi.begin();
    const double S = (double)s->bytes;
    return write ? (1.0 + (double)D) * S + S : (1.0 + 0.5 * (double)D) * S;
}

// Grouped energy sums (Re<psi|H|psi>, <psi|psi>) reduced into sums[0..1]
// on the device, with per-block partials in part (at most
// energy_part_blocks() blocks of 2): m energy-only window passes (m S read;
// per pass, its partials reduced and added in pass order) or one tile sweep
// that visits each out-of-tile pair once ((1 + D/2) S read).
uint32_t energy_part_blocks(const vqe_hamiltonian* h, int n) {
    return h->hw_energy ? hwin_blocks(n) : hpsi_blocks(n, kEnergyPartBlocks);
}

template <typename T>
int energy_grouped(vqe_state* s, const vqe_hamiltonian* h, double* part, double* sums) {
    uint32_t nb = 0;
    if (h->hw_energy) {
        const size_t m = h->hw_wins.size();
        for (size_t wi = 0; wi < m; ++wi) {
            ProfScope ps(VQE_KERNEL_EXPECT_HALF, (double)s->bytes, s->stream);
            VQE_HIP(launch_hwin<T>(s->n, h->hw_wins[wi], s->data, nullptr, h->d_hw_groups, h->d_hw_classes,
                                   hw_terms_of<T>(h), h->real_coeffs, wi == 0, wi + 1 == m, part, &nb, s->stream));
            ps.end();
            VQE_HIP(launch_reduce(part, nb, 2, nullptr, sums, wi ? 1 : 0, s->stream));
        }
        return VQE_OK;
    }
    {
        ProfScope ps(VQE_KERNEL_EXPECT_HALF, hpsi_bytes(h, s, false), s->stream);
        VQE_HIP(launch_hpsi<T>(s->n, s->data, nullptr, h->d_groups, (uint32_t)h->groups.size(), terms_of<T>(h), 1,
                               kEnergyPartBlocks, part, &nb, s->stream));
    }
    VQE_HIP(launch_reduce(part, nb, 2, nullptr, sums, 0, s->stream));
    return VQE_OK;
}

// Per-term partials: d_res[off + 2t] = <P_t>, d_res[off + 2t + 1] = norm.
template <typename T>
int energy_per_term(vqe_state* s, const vqe_hamiltonian* h, size_t off) {
    for (size_t t = 0; t < h->w.size(); ++t) {
        uint32_t nb = 0;
        ProfScope ps(VQE_KERNEL_PER_TERM, (double)s->bytes, s->stream);
        VQE_HIP(launch_expect_term<T>(s->n, s->data, h->x[t], h->z[t], s->d_part, &nb, s->stream));
        ps.end();
        VQE_HIP(launch_reduce(s->d_part, nb, 2, nullptr, s->d_res + off + 2 * t, 0, s->stream));
    }
    return VQE_OK;
}

double combine_per_term(const vqe_hamiltonian* h, const double* r, double* norm) {
    double e = 0.0;
    for (size_t t = 0; t < h->w.size(); ++t) e += h->w[t] * r[2 * t];
    *norm = h->w.empty() ? 0.0 : r[1];
    return e;
}

template <typename T>
int expect_impl(vqe_state* s, const vqe_hamiltonian* h, int mode, double* energy, double* norm) {
    const size_t need = mode == VQE_EXPECT_PER_TERM ? 2 * h->w.size() + 2 : 2;
    int rc = ensure_res(s, need);
    if (rc) return rc;
    if (mode == VQE_EXPECT_PER_TERM) {
        if (h->w.empty()) {
            set_error("vqe_expect_pauli: empty Hamiltonian");
            return VQE_ERR_ARG;
        }
        rc = energy_per_term<T>(s, h, 0);
        if (rc) return rc;
        VQE_HIP(hipMemcpyAsync(s->h_res, s->d_res, 2 * h->w.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        VQE_HIP(hipStreamSynchronize(s->stream));
        double nrm = 0.0;
        const double e = combine_per_term(h, s->h_res, &nrm);
        *energy = e / nrm;
        if (norm) *norm = nrm;
    } else {
        rc = energy_grouped<T>(s, h, s->d_part, s->d_res);
        if (rc) return rc;
        VQE_HIP(hipMemcpyAsync(s->h_res, s->d_res, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        VQE_HIP(hipStreamSynchronize(s->stream));
        *energy = s->h_res[0] / s->h_res[1];
        if (norm) *norm = s->h_res[1];
    }
    return VQE_OK;
}

template <typename T>
int adjoint_impl(vqe_state* psi, vqe_state* lam, const vqe_circuit* c, const double* params,
                 const vqe_hamiltonian* h, const vqe_grad_opts* o, double* energy, double* grad) {
    const Plan& pl = plan_now(c);
    if (int rc0 = upload_plan(pl)) return rc0;
    const size_t P = pl.passes.size();
    std::vector<size_t> bounds;
    std::vector<void*> ck;
    const int nck = o ? o->n_ckpt : 0;
    for (int k = 0; k < nck; ++k) {
        size_t b = (size_t)std::llround((double)(k + 1) * (double)P / (double)(nck + 1));
        if (b < 1 || b >= P) continue;
        if (std::find(bounds.begin(), bounds.end(), b) != bounds.end()) continue;
        bounds.push_back(b);
        ck.push_back(o->ckpt[k]->data);
    }
    int rc = ensure_res(psi, 2 + c->n_params);
    if (rc) return rc;
    double* d_e = psi->d_res;
    double* d_g = psi->d_res + 2;
    hipStream_t st = psi->stream;
    const int chunk = o && o->chunk_passes > 0 ? o->chunk_passes : 0;
    VQE_HIP(launch_set_basis(psi->dtype, psi->data, 1ull << psi->n, 0, st));
    rc = forward<T>(psi, c, pl, params, bounds, ck, chunk);
    if (rc) return rc;
    rc = apply_h<T>(psi, lam->data, h, d_e);
    if (rc) return rc;
    VQE_HIP(launch_zero(d_g, c->n_params, st));
    const int d = sizeof(T) == 8 ? 1 : 0;
    const Mat2<T>* mats = (const Mat2<T>*)psi->d_mats;  // uploaded by forward()
    PassArgs<T> a;
    JitArgs ja;
    // Half turns of the sheared rotations flip psi and lam together, so the
    // gradient terms (bilinear in them) keep their sign until psi is restored
    // from a checkpoint; from there on they carry the flips made before it.
    bool flipped = false, grad_neg = false;
    for (size_t pi = P; pi-- > 0;) {
        const void* pin = psi->data;
        for (size_t k = 0; k < bounds.size(); ++k)
            if (bounds[k] == pi + 1) pin = ck[k];
        if (pl.jit && pin != psi->data) grad_neg = flipped;
        uint32_t gb = 0;
        const uint32_t n_gslots = (uint32_t)pl.ops[pi].slot_param.size();
        ProfScope ps(VQE_KERNEL_WINDOW_REV, 4.0 * (double)psi->bytes, st);
        if (pl.jit) {
            int S = 0;
            jit_ops(pl, pi, d, true, &S, &ja, psi->n);
            VQE_HIP(launch_window_jit(pl.jfn[d][1][pi], ja, S, mats + pl.mat_off[2 * pi + 1], true, pin, psi->data,
                                      lam->data, lam->data, psi->d_part, &gb, st));
        } else {
            build_args<T>(c, pl, pi, params, true, a);
            VQE_HIP(launch_window_rev<T>(a, psi->n, pin, psi->data, lam->data, lam->data, psi->d_part, &gb, st));
        }
        ps.end();
        if (n_gslots)
            VQE_HIP(launch_reduce(psi->d_part, gb, n_gslots, pl.d_slotmap + pl.slot_off[pi], d_g, grad_neg ? -1 : 1,
                                  st));
        if (pl.jit && psi->rev_flip[pi]) flipped = !flipped;
        if (chunk > 0 && (P - pi) % (size_t)chunk == 0 && pi > 0) VQE_HIP(hipStreamSynchronize(st));
    }
    VQE_HIP(hipMemcpyAsync(psi->h_res, psi->d_res, (2 + c->n_params) * sizeof(double), hipMemcpyDeviceToHost, st));
    VQE_HIP(hipStreamSynchronize(st));
    const double nrm = psi->h_res[1];
    *energy = psi->h_res[0] / nrm;
    for (size_t k = 0; k < c->n_params; ++k) grad[k] = psi->h_res[2 + k] / nrm;
    return VQE_OK;
}

template <typename T>
int param_shift_impl(vqe_state* psi, const vqe_circuit* c, const double* params, const vqe_hamiltonian* h,
                     int mode, double* energy, double* grad) {
    // Shift rule per parameter: two runs at +-pi/2 for the rotations (their
    // generators square to one); four runs at +-pi/2 and +-3pi/2 for the
    // excitation gates, whose generators have eigenvalues 0 and +-1 (the
    // four-term rule of Anselmetti et al. 2021).
    const size_t P = c->n_params;
    std::vector<char> exc(P, 0);
    for (const Gate& g : c->gates)
        if (g.pidx >= 0 && is_excitation(g.kind)) exc[g.pidx] = 1;
    std::vector<std::pair<size_t, double>> shifts;  // evaluation e >= 1: (parameter, shift)
    for (size_t k = 0; k < P; ++k) {
        shifts.push_back({k, M_PI / 2});
        shifts.push_back({k, -M_PI / 2});
        if (exc[k]) {
            shifts.push_back({k, 3 * M_PI / 2});
            shifts.push_back({k, -3 * M_PI / 2});
        }
    }
    const size_t per = mode == VQE_EXPECT_PER_TERM ? 2 * h->w.size() : 2;
    const size_t n_eval = 1 + shifts.size();
    int rc = ensure_res(psi, per * n_eval);
    if (rc) return rc;
    std::vector<double> th(params, params + P);
    const std::vector<size_t> nob;
    const std::vector<void*> nock;
    // Evaluation 0 last so that psi ends in U(theta)|0>.
    for (size_t e = n_eval; e-- > 0;) {
        std::copy(params, params + P, th.begin());
        if (e > 0) th[shifts[e - 1].first] += shifts[e - 1].second;
        VQE_HIP(launch_set_basis(psi->dtype, psi->data, 1ull << psi->n, 0, psi->stream));
        rc = forward<T>(psi, c, plan_now(c), th.data(), nob, nock);
        if (rc) return rc;
        rc = mode == VQE_EXPECT_PER_TERM ? energy_per_term<T>(psi, h, e * per)
                                         : energy_grouped<T>(psi, h, psi->d_part, psi->d_res + e * per);
        if (rc) return rc;
    }
    VQE_HIP(hipMemcpyAsync(psi->h_res, psi->d_res, per * n_eval * sizeof(double), hipMemcpyDeviceToHost, psi->stream));
    VQE_HIP(hipStreamSynchronize(psi->stream));
    std::vector<double> E(n_eval);
    for (size_t e = 0; e < n_eval; ++e) {
        const double* r = psi->h_res + e * per;
        if (mode == VQE_EXPECT_PER_TERM) {
            double nrm = 0.0;
            const double v = combine_per_term(h, r, &nrm);
            E[e] = v / nrm;
        } else {
            E[e] = r[0] / r[1];
        }
    }
    *energy = E[0];
    const double d1 = (std::sqrt(2.0) + 1) / (4 * std::sqrt(2.0)), d2 = (std::sqrt(2.0) - 1) / (4 * std::sqrt(2.0));
    size_t e = 1;
    for (size_t k = 0; k < P; ++k) {
        if (exc[k]) {
            grad[k] = d1 * (E[e] - E[e + 1]) - d2 * (E[e + 2] - E[e + 3]);
            e += 4;
        } else {
            grad[k] = 0.5 * (E[e] - E[e + 1]);
            e += 2;
        }
    }
    return VQE_OK;
}


void free_circuit(vqe_circuit* c) {
    if (!c) return;
    for (auto& pl : c->plan)
        if (pl.d_slotmap) (void)hipFree(pl.d_slotmap);
    delete c;
}

// Tile passes of the batched mid-size form: the planner's windows of at most
// kMidWin qubits, each padded to kMidWin with the lowest qubits outside it,
// and the pass's gates rewritten to window-local qubits and patterns.
int build_mid_plan(vqe_circuit* c) {
    if (c->n <= kMidWin || c->n > kMidMaxQubits) return VQE_OK;
    std::vector<PlannedPass> passes;
    std::string msg;
    if (!plan_passes(c->n, c->gates, kMidLimits, passes, msg)) {
        set_error("vqe_circuit_create: " + msg);
        return VQE_ERR_STATE;
    }
    if (passes.empty()) passes.emplace_back();  // no gates: one pass that only prepares |0...0>
    for (const PlannedPass& p : passes) {
        uint64_t w = 0;
        for (int j = 0; j < p.K; ++j) w |= 1ull << p.pos[j];
        for (int q = 0; __builtin_popcountll(w) < kMidWin; ++q) w |= 1ull << q;
        MidPlanPass mp{};
        int local[64] = {0};
        int k = 0;
        for (int q = 0; q < c->n; ++q)
            if ((w >> q) & 1) {
                local[q] = k;
                mp.pos[k++] = (uint32_t)q;
            }
        mp.gate_off = (uint32_t)c->mid_gates.size();
        mp.n_gates = (uint32_t)p.gates.size();
        mp.slot_off = (uint32_t)c->mid_slot_pidx.size();
        for (int gi : p.gates) {
            const Gate& g = c->gates[gi];
            BatchGate bg = c->bgates[gi];
            bg.q0 = (uint8_t)local[g.q0];
            bg.q1 = (uint8_t)local[g.q1];
            if (is_excitation(g.kind)) {
                const bool dbl = g.kind == VQE_GATE_DEXC;
                bg.pa = (uint16_t)(dbl ? (1u << local[g.q0]) | (1u << local[g.q1]) : (1u << local[g.q0]));
                bg.pb = (uint16_t)(dbl ? (1u << local[g.q2]) | (1u << local[g.q3]) : (1u << local[g.q1]));
            }
            c->mid_gates.push_back(bg);
        }
        for (size_t j = p.gates.size(); j-- > 0;)
            if (c->gates[p.gates[j]].pidx >= 0) c->mid_slot_pidx.push_back(c->gates[p.gates[j]].pidx);
        mp.n_slots = (uint32_t)c->mid_slot_pidx.size() - mp.slot_off;
        c->mid.push_back(mp);
    }
    return VQE_OK;
}

// Plans fused passes within the given limits and lowers them to kernel op
// lists (forward, and reverse with gradient ops), per dtype also to the
// lane-split layout.
int build_plan(vqe_circuit* c, const PlanLimits& lim, bool jit, Plan& pl) {
    std::string msg;
    pl.jit = jit;
    if (!plan_passes(c->n, c->gates, lim, pl.passes, msg)) {
        set_error("vqe_circuit_create: " + msg);
        return VQE_ERR_STATE;
    }
    std::vector<int32_t>& slotmap = pl.slotmap;
    pl.ops.resize(pl.passes.size());
    for (size_t pi = 0; pi < pl.passes.size(); ++pi) {
        const PlannedPass& p = pl.passes[pi];
        PassOps& po = pl.ops[pi];
        for (int gi : p.gates) emit_gate(c->gates[gi], gi, p, po.fwd, po.fwd_mat_gate);
        std::map<int, int> pslot;
        for (auto it = p.gates.rbegin(); it != p.gates.rend(); ++it) {
            const Gate& g = c->gates[*it];
            if (g.pidx >= 0) {
                auto f = pslot.find(g.pidx);
                int slot;
                if (f == pslot.end()) {
                    slot = (int)po.slot_param.size();
                    pslot[g.pidx] = slot;
                    po.slot_param.push_back(g.pidx);
                } else {
                    slot = f->second;
                }
                KOp gop{};
                gop.type = grad_op(g.kind);
                gop.a = (uint8_t)local_bit(p, g.q0);
                if (is_excitation(g.kind)) gop.b = (uint8_t)local_bit(p, g.q1);
                if (g.kind == VQE_GATE_DEXC) {
                    gop.c = (uint8_t)local_bit(p, g.q2);
                    gop.d = (uint8_t)local_bit(p, g.q3);
                }
                gop.slot = (uint8_t)slot;
                po.rev.push_back(gop);
            }
            emit_gate(g, *it, p, po.rev, po.rev_mat_gate);
        }
        pl.slot_off.push_back(slotmap.size());
        slotmap.insert(slotmap.end(), po.slot_param.begin(), po.slot_param.end());
        pl.mat_off.push_back(pl.mat_total);
        pl.mat_total += po.fwd_mat_gate.size();
        pl.mat_off.push_back(pl.mat_total);
        pl.mat_total += po.rev_mat_gate.size();
        // interpreted kernels hold the lowered ops in their arguments
        const size_t cap = jit ? (size_t)-1 : (size_t)kMaxPhysOps;
        for (int d = 0; d < 2; ++d) {
            po.S_f[d] = split_bits_for(jit, d == 1, p.K, false);
            po.S_r[d] = split_bits_for(jit, d == 1, p.K, true);
            if ((po.S_f[d] && !lower_split(po.fwd, p.K, po.S_f[d], cap, po.fwd_l[d])) ||
                (po.S_r[d] && !lower_split(po.rev, p.K, po.S_r[d], cap, po.rev_l[d]))) {
                set_error("vqe_circuit_create: too many ops in a pass after lane transposes (internal limit)");
                return VQE_ERR_STATE;
            }
        }
    }
    return VQE_OK;
}


// Window bits an op needs in registers (the others it can apply per lane).
uint32_t reg_needs(const KOp& op) {
    switch (op.type) {
        case OP_U2:
        case OP_R2:
        case OP_XFLIP:
        case OP_GX:
        case OP_GY:
            return 1u << op.a;
        case OP_CNOT:
        case OP_PAIR2:
        case OP_GPAIR2:
            return (1u << op.a) | (1u << op.b);
        case OP_PAIR4:
        case OP_GPAIR4:
            return (1u << op.a) | (1u << op.b) | (1u << op.c) | (1u << op.d);
        default:  // OP_DIAG, OP_CZ, OP_GZ act per lane on a lane-resident bit
            return 0;
    }
}

// Lowers a logical op list (window local bits 0..K-1) to the lane-split layout
// with S of the K bits in lane slots.  The S bits needed in registers least
// often start in the lanes; before an op that needs a lane-resident bit in
// registers, a TPOSE swaps it with the register bit whose next use is
// furthest away.  Returns false if the op capacity would be exceeded.
bool lower_split(const std::vector<KOp>& ops, int K, int S, size_t cap, SplitOps& out) {
    const int KL = K - S;
    int cost[kMaxWindow] = {0};
    for (const auto& op : ops)
        for (int w = 0; w < K; ++w)
            if (reg_needs(op) >> w & 1) cost[w]++;
    int order[kMaxWindow];
    for (int w = 0; w < K; ++w) order[w] = w;
    std::sort(order, order + K, [&](int x, int y) { return cost[x] != cost[y] ? cost[x] < cost[y] : x > y; });
    int bit_at[kMaxWindow], slot_of[kMaxWindow];
    std::vector<int> regs;
    for (int j = 0; j < S; ++j) bit_at[KL + j] = order[j];
    for (int j = S; j < K; ++j) regs.push_back(order[j]);
    std::sort(regs.begin(), regs.end());
    for (int r = 0; r < KL; ++r) bit_at[r] = regs[r];
    for (int sl = 0; sl < K; ++sl) slot_of[bit_at[sl]] = sl;
    for (int sl = 0; sl < K; ++sl) out.map_in[sl] = (uint8_t)bit_at[sl];
    out.ops.clear();
    for (size_t i = 0; i < ops.size(); ++i) {
        const KOp& op = ops[i];
        const uint32_t need = reg_needs(op);
        for (int w = 0; w < K; ++w) {
            if (!(need >> w & 1) || slot_of[w] < KL) continue;
            // evict the register bit (not needed by this op) used furthest in the future
            int best_r = -1;
            size_t best_next = 0;
            for (int r = 0; r < KL; ++r) {
                const int wb = bit_at[r];
                if (need >> wb & 1) continue;
                size_t nxt = ops.size();
                for (size_t k = i + 1; k < ops.size(); ++k)
                    if (reg_needs(ops[k]) >> wb & 1) {
                        nxt = k;
                        break;
                    }
                if (best_r < 0 || nxt > best_next) {
                    best_r = r;
                    best_next = nxt;
                }
            }
            const int lane_slot = slot_of[w];
            KOp t{};
            t.type = OP_TPOSE;
            t.a = (uint8_t)best_r;
            t.b = (uint8_t)(lane_slot - KL);
            out.ops.push_back(t);
            const int wr = bit_at[best_r];
            bit_at[best_r] = w;
            bit_at[lane_slot] = wr;
            slot_of[w] = best_r;
            slot_of[wr] = lane_slot;
        }
        KOp ph = op;
        ph.a = (uint8_t)slot_of[op.a];
        if (op.type == OP_CNOT || op.type == OP_CZ || op.type == OP_PAIR2 || op.type == OP_GPAIR2 ||
            op.type == OP_PAIR4 || op.type == OP_GPAIR4)
            ph.b = (uint8_t)slot_of[op.b];
        if (op.type == OP_PAIR4 || op.type == OP_GPAIR4) {
            ph.c = (uint8_t)slot_of[op.c];
            ph.d = (uint8_t)slot_of[op.d];
        }
        out.ops.push_back(ph);
    }
    for (int sl = 0; sl < K; ++sl) out.map_out[sl] = (uint8_t)bit_at[sl];
    return out.ops.size() <= cap;
}

// Uploads the gradient slot maps of a plan to the current device (once).
int upload_plan(const Plan& cpl) {
    Plan& pl = const_cast<Plan&>(cpl);
    std::lock_guard<std::mutex> g(g_upload_mu);
    if (pl.d_slotmap || pl.slotmap.empty()) return VQE_OK;
    if (hipMalloc((void**)&pl.d_slotmap, pl.slotmap.size() * sizeof(int32_t)) != hipSuccess) {
        set_error("hipMalloc of the gradient slot map failed");
        return VQE_ERR_OOM;
    }
    VQE_HIP(hipMemcpy(pl.d_slotmap, pl.slotmap.data(), pl.slotmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return VQE_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <typename T>
int batch_impl(vqe_batch* b, size_t n_items, const vqe_batch_item* items) {
    const int max_q = b->dtype == VQE_C64 ? kBatchMaxQubitsC64 : kBatchMaxQubitsC128;
    size_t n_gates = 0, n_mats = 1, n_out = 0;
    int max_n = 1;
    for (size_t i = 0; i < n_items; ++i) {
        const vqe_batch_item& it = items[i];
        if (!it.circuit || !it.hamiltonian || !it.energy || (it.n_params && (!it.params || !it.grad))) {
            set_error("vqe_batch_energy_grad: item " + std::to_string(i) + " has a null field");
            return VQE_ERR_ARG;
        }
        const vqe_circuit* c = it.circuit;
        if (c->n > max_q || it.hamiltonian->n != c->n) {
            set_error("vqe_batch_energy_grad: item " + std::to_string(i) + " has " + std::to_string(c->n) +
                      " qubits (limit " + std::to_string(max_q) + ") or a Hamiltonian of another size");
            return VQE_ERR_ARG;
        }
        if (int rc = check_params(c, it.params, it.n_params, "vqe_batch_energy_grad")) return rc;
        if (int rc = upload_hamiltonian(it.hamiltonian)) return rc;
        n_gates += c->bgates.size();
        n_mats += c->n_mats;
        n_out += 1 + c->n_params;
        max_n = std::max(max_n, c->n);
    }
    const size_t o_items = 0;
    const size_t o_gates = align_up(o_items + n_items * sizeof(BatchDesc<T>), 256);
    const size_t o_mats = align_up(o_gates + std::max<size_t>(n_gates, 1) * sizeof(BatchGate), 256);
    const size_t o_out = align_up(o_mats + n_mats * sizeof(Mat2<T>), 256);
    const size_t total = align_up(o_out + n_out * sizeof(double), 256);
    if (total > b->d_cap) {
        VQE_HIP(hipStreamSynchronize(b->stream));
        if (b->d_buf) VQE_HIP(hipFree(b->d_buf));
        if (b->h_buf) VQE_HIP(hipHostFree(b->h_buf));
        b->d_buf = b->h_buf = nullptr;
        b->d_cap = b->h_cap = 0;
        const size_t cap = std::max(total * 2, (size_t)1 << 20);
        if (hipMalloc(&b->d_buf, cap) != hipSuccess || hipHostMalloc(&b->h_buf, cap, hipHostMallocDefault) != hipSuccess) {
            set_error("vqe_batch_energy_grad: staging allocation failed");
            return VQE_ERR_OOM;
        }
        b->d_cap = b->h_cap = cap;
    }
    char* h = (char*)b->h_buf;
    char* d = (char*)b->d_buf;
    auto* hi = (BatchDesc<T>*)(h + o_items);
    auto* hg = (BatchGate*)(h + o_gates);
    auto* hm = (Mat2<T>*)(h + o_mats);
    size_t g_off = 0, m_off = 0, out_off = 0;
    for (size_t i = 0; i < n_items; ++i) {
        const vqe_circuit* c = items[i].circuit;
        const vqe_hamiltonian* hh = items[i].hamiltonian;
        BatchDesc<T> bd{};
        bd.n = c->n;
        bd.n_gates = (uint32_t)c->bgates.size();
        bd.gate_off = (uint32_t)g_off;
        bd.mat_off = (uint32_t)m_off;
        bd.n_groups = (uint32_t)hh->groups.size();
        bd.n_params = (uint32_t)c->n_params;
        bd.out_off = out_off;
        bd.groups = hh->d_groups;
        bd.terms = terms_of<T>(hh);
        hi[i] = bd;
        for (size_t k = 0; k < c->bgates.size(); ++k) {
            hg[g_off + k] = c->bgates[k];
            const Gate& gt = c->gates[k];
            if (c->bgates[k].type == OP_U2 || c->bgates[k].type == OP_PAIR2)
                fill_matrix(hm[m_off + c->bgates[k].mat], gt, angle_of(gt, items[i].params), false);
        }
        g_off += c->bgates.size();
        m_off += c->n_mats;
        out_off += 1 + c->n_params;
    }
    std::memset(&hm[m_off], 0, sizeof(Mat2<T>));
    VQE_HIP(hipMemcpyAsync(d, h, o_out, hipMemcpyHostToDevice, b->stream));
    VQE_HIP(launch_batch<T>((const BatchDesc<T>*)(d + o_items), (uint32_t)n_items, (const BatchGate*)(d + o_gates),
                            (const Mat2<T>*)(d + o_mats), (double*)(d + o_out), max_n, b->stream));
    VQE_HIP(hipMemcpyAsync(h + o_out, d + o_out, n_out * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    VQE_HIP(hipStreamSynchronize(b->stream));
    const double* r = (const double*)(h + o_out);
    out_off = 0;
    for (size_t i = 0; i < n_items; ++i) {
        const vqe_circuit* c = items[i].circuit;
        *items[i].energy = r[out_off];
        for (size_t k = 0; k < c->n_params; ++k) items[i].grad[k] = r[out_off + 1 + k];
        out_off += 1 + c->n_params;
    }
    return VQE_OK;
}
// Bytes of one state of n qubits in the mid-size buffer (256-byte aligned).
size_t st_bytes_half(int n, size_t amp) { return align_up(((size_t)1 << n) * amp, 256); }

// Grows a batch's mid-size buffers to at least dev / host bytes.
int mid_reserve(vqe_batch* b, size_t dev, size_t host) {
    if (dev <= b->md_cap && host <= b->mh_cap) return VQE_OK;
    VQE_HIP(hipStreamSynchronize(b->stream));
    if (dev > b->md_cap) {
        if (b->md_buf) VQE_HIP(hipFree(b->md_buf));
        b->md_buf = nullptr;
        b->md_cap = 0;
        const size_t cap = dev + dev / 4;
        if (hipMalloc(&b->md_buf, cap) != hipSuccess) {
            b->md_buf = nullptr;
            set_error("vqe_batch_energy_grad: device allocation of " + std::to_string(cap) +
                      " bytes for mid-size items failed");
            return VQE_ERR_OOM;
        }
        b->md_cap = cap;
    }
    if (host > b->mh_cap) {
        if (b->mh_buf) VQE_HIP(hipHostFree(b->mh_buf));
        b->mh_buf = nullptr;
        b->mh_cap = 0;
        const size_t cap = std::max(host + host / 4, (size_t)1 << 20);
        if (hipHostMalloc(&b->mh_buf, cap, hipHostMallocDefault) != hipSuccess) {
            b->mh_buf = nullptr;
            set_error("vqe_batch_energy_grad: pinned staging allocation failed");
            return VQE_ERR_OOM;
        }
        b->mh_cap = cap;
    }
    return VQE_OK;
}

// Mid-size items (LDS limit < n <= kMidMaxQubits): forward tile passes, one
// launch per pass index over every item that has that pass; lam = H psi over
// tiles; reverse tile passes likewise; one reduction launch; results to the
// host.  Per item: psi and lam in the batch's device buffer, n_blk =
// min(2^(n - kMidWin), kMidMaxBlocks) blocks per launch.
template <typename T>
int mid_impl(vqe_batch* b, const vqe_batch_item* items, const std::vector<size_t>& idx) {
    const size_t m = idx.size();
    const size_t amp = 2 * sizeof(T);
    // lam = H psi: window passes (hwin_batch_kernel, one launch per pass index
    // and coefficient form) where the Hamiltonian has a window cover, else the
    // tile kernel (mid_hpsi_kernel)
    std::vector<uint32_t> nblk(m), nblk_e(m);
    std::vector<uint64_t> ncos(m), part_base(m), part_s(m), red_base(m), st_off(m), m_off(m);
    std::vector<char> use_hw(m);
    size_t n_gates = 0, n_mats = 1, n_fwd = 0, n_part = 0, n_red = 0, st_bytes = 0, n_hw = 0, n_tile = 0;
    size_t pmax = 0, hmax = 0;
    for (size_t k = 0; k < m; ++k) {
        const vqe_circuit* c = items[idx[k]].circuit;
        const vqe_hamiltonian* hh = items[idx[k]].hamiltonian;
        ncos[k] = 1ull << (c->n - kMidWin);
        nblk[k] = (uint32_t)std::min<uint64_t>(ncos[k], kMidMaxBlocks);
        use_hw[k] = !hh->hw_wins.empty();
        nblk_e[k] = use_hw[k] ? (uint32_t)std::min<uint64_t>(1ull << (c->n - kHwBits), kMidMaxBlocks) : nblk[k];
        if (use_hw[k]) {
            n_hw += hh->hw_wins.size();
            hmax = std::max(hmax, hh->hw_wins.size());
        } else {
            ++n_tile;
        }
        part_base[k] = n_part;
        part_s[k] = n_part + 2 * (size_t)nblk_e[k];
        n_part += 2 * (size_t)nblk_e[k] + c->mid_slot_pidx.size() * (size_t)nblk[k];
        red_base[k] = n_red;
        n_red += 2 + c->mid_slot_pidx.size();
        st_off[k] = st_bytes;
        st_bytes += 2 * align_up(((size_t)1 << c->n) * amp, 256);
        m_off[k] = n_mats;
        n_gates += c->mid_gates.size();
        n_mats += c->n_mats;
        n_fwd += c->mid.size();
        pmax = std::max(pmax, c->mid.size());
        if (int rc = upload_hamiltonian(items[idx[k]].hamiltonian)) return rc;
    }
    // host-written tables | out, then (device only) partial sums | states
    const size_t o_fwd = 0;
    const size_t o_rev = align_up(o_fwd + n_fwd * sizeof(MidPass), 256);
    const size_t o_ham = align_up(o_rev + n_fwd * sizeof(MidPass), 256);
    const size_t o_hw = align_up(o_ham + std::max<size_t>(n_tile, 1) * sizeof(MidHam), 256);
    const size_t o_red = align_up(o_hw + std::max<size_t>(n_hw, 1) * sizeof(HwItem), 256);
    const size_t o_gates = align_up(o_red + n_red * sizeof(MidRed), 256);
    const size_t o_mats = align_up(o_gates + std::max<size_t>(n_gates, 1) * sizeof(BatchGate), 256);
    const size_t o_out = align_up(o_mats + (n_mats + 1) * sizeof(Mat2<T>), 256);  // + a zero matrix at the end
    const size_t o_part = align_up(o_out + n_red * sizeof(double), 256);
    const size_t o_st = align_up(o_part + n_part * sizeof(double), 256);
    if (int rc = mid_reserve(b, o_st + st_bytes, o_part)) return rc;
    char* h = (char*)b->mh_buf;
    char* d = (char*)b->md_buf;
    auto* hf = (MidPass*)(h + o_fwd);
    auto* hr = (MidPass*)(h + o_rev);
    auto* hh = (MidHam*)(h + o_ham);
    auto* hred = (MidRed*)(h + o_red);
    auto* hg = (BatchGate*)(h + o_gates);
    auto* hm = (Mat2<T>*)(h + o_mats);
    std::memset(&hm[0], 0, sizeof(Mat2<T>));
    std::memset(&hm[n_mats], 0, sizeof(Mat2<T>));
    double* part = (double*)(d + o_part);
    // gates, matrices, tile-form H psi and reduction descriptors per item
    auto* hw = (HwItem*)(h + o_hw);
    size_t g_off = 0, n_th = 0;
    uint32_t hblk = 0;
    for (size_t k = 0; k < m; ++k) {
        const vqe_batch_item& it = items[idx[k]];
        const vqe_circuit* c = it.circuit;
        std::copy(c->mid_gates.begin(), c->mid_gates.end(), hg + g_off);
        for (size_t i = 0; i < c->gates.size(); ++i)
            if (c->bgates[i].type == OP_U2 || c->bgates[i].type == OP_PAIR2)
                fill_matrix(hm[m_off[k] + c->bgates[i].mat], c->gates[i], angle_of(c->gates[i], it.params), false);
        if (!use_hw[k]) {
            MidHam mh{};
            mh.psi = d + o_st + st_off[k];
            mh.lam = d + o_st + st_off[k] + st_bytes_half(c->n, amp);
            mh.groups = it.hamiltonian->d_groups;
            mh.terms = terms_of<T>(it.hamiltonian);
            mh.n_tiles = ncos[k];
            mh.part_off = part_base[k];
            mh.n_groups = (uint32_t)it.hamiltonian->groups.size();
            mh.blk_begin = hblk;
            mh.n_blk = nblk[k];
            hh[n_th++] = mh;
            hblk += nblk[k];
        }
        hred[red_base[k]] = MidRed{part_base[k], nblk_e[k], 0};
        hred[red_base[k] + 1] = MidRed{part_base[k] + nblk_e[k], nblk_e[k], 0};
        for (size_t sl = 0; sl < c->mid_slot_pidx.size(); ++sl)
            hred[red_base[k] + 2 + sl] = MidRed{part_s[k] + sl * (uint64_t)nblk[k], nblk[k], 0};
        g_off += c->mid_gates.size();
    }
    // window-form H psi descriptors, grouped by launch: pass index, then real
    // coefficients or not
    struct HwLaunch {
        size_t off, cnt;
        uint32_t grid;
        bool real;
    };
    std::vector<HwLaunch> hw_launch;
    {
        size_t e = 0;
        for (size_t p = 0; p < hmax; ++p)
            for (int real = 1; real >= 0; --real) {
                HwLaunch L{e, 0, 0, real == 1};
                for (size_t k = 0; k < m; ++k) {
                    const vqe_hamiltonian* H = items[idx[k]].hamiltonian;
                    if (!use_hw[k] || p >= H->hw_wins.size() || H->real_coeffs != (real == 1)) continue;
                    const vqe_circuit* c = items[idx[k]].circuit;
                    HwItem x{};
                    x.w = H->hw_wins[p];
                    x.psi = d + o_st + st_off[k];
                    x.lam = d + o_st + st_off[k] + st_bytes_half(c->n, amp);
                    x.groups = H->d_hw_groups;
                    x.classes = H->d_hw_classes;
                    x.terms = hw_terms_of<T>(H);
                    x.n_cosets = 1ull << (c->n - kHwBits);
                    x.part_off = part_base[k];
                    x.blk_begin = L.grid;
                    x.n_blk = nblk_e[k];
                    x.first = p == 0 ? 1u : 0u;
                    x.last = p + 1 == H->hw_wins.size() ? 1u : 0u;
                    hw[e++] = x;
                    L.grid += nblk_e[k];
                    ++L.cnt;
                }
                if (L.cnt) hw_launch.push_back(L);
            }
    }
    // pass descriptors, grouped by launch
    std::vector<size_t> l_off(pmax), l_cnt(pmax);
    std::vector<uint32_t> l_grid(pmax);
    size_t e = 0;
    for (size_t p = 0; p < pmax; ++p) {
        l_off[p] = e;
        uint32_t blk = 0;
        size_t gbase = 0;
        for (size_t k = 0; k < m; ++k) {
            const vqe_circuit* c = items[idx[k]].circuit;
            const size_t P = c->mid.size();
            if (p < P) {
                for (int dir = 0; dir < 2; ++dir) {
                    const MidPlanPass& mp = c->mid[dir ? P - 1 - p : p];
                    MidPass x{};
                    x.psi = d + o_st + st_off[k];
                    x.lam = d + o_st + st_off[k] + st_bytes_half(c->n, amp);
                    x.n_cosets = ncos[k];
                    x.part_off = part_s[k] + (uint64_t)mp.slot_off * nblk[k];
                    for (int j = 0; j < kMidWin; ++j) x.pos[j] = mp.pos[j];
                    x.gate_off = (uint32_t)(gbase + mp.gate_off);
                    x.n_gates = mp.n_gates;
                    x.mat_off = (uint32_t)m_off[k];
                    x.n_slots = mp.n_slots;
                    x.blk_begin = blk;
                    x.n_blk = nblk[k];
                    x.first = (dir == 0 && p == 0) ? 1u : 0u;
                    (dir ? hr : hf)[e] = x;
                }
                blk += nblk[k];
                ++e;
            }
            gbase += c->mid_gates.size();
        }
        l_cnt[p] = e - l_off[p];
        l_grid[p] = blk;
    }
    VQE_HIP(hipMemcpyAsync(d, h, o_out, hipMemcpyHostToDevice, b->stream));
    const auto* dg = (const BatchGate*)(d + o_gates);
    const auto* dm = (const Mat2<T>*)(d + o_mats);
    for (size_t p = 0; p < pmax; ++p)
        VQE_HIP(launch_mid_pass<T>((const MidPass*)(d + o_fwd) + l_off[p], (uint32_t)l_cnt[p], l_grid[p], false, dg,
                                   dm, part, b->stream));
    if (n_th) VQE_HIP(launch_mid_hpsi<T>((const MidHam*)(d + o_ham), (uint32_t)n_th, hblk, part, b->stream));
    for (const HwLaunch& L : hw_launch)
        VQE_HIP(launch_hwin_batch<T>((const HwItem*)(d + o_hw) + L.off, (uint32_t)L.cnt, L.grid, L.real, part,
                                     b->stream));
    for (size_t p = 0; p < pmax; ++p)
        VQE_HIP(launch_mid_pass<T>((const MidPass*)(d + o_rev) + l_off[p], (uint32_t)l_cnt[p], l_grid[p], true, dg,
                                   dm, part, b->stream));
    VQE_HIP(launch_mid_reduce((const MidRed*)(d + o_red), (uint32_t)n_red, part, (double*)(d + o_out), b->stream));
    VQE_HIP(hipMemcpyAsync(h + o_out, d + o_out, n_red * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    VQE_HIP(hipStreamSynchronize(b->stream));
    const double* r = (const double*)(h + o_out);
    for (size_t k = 0; k < m; ++k) {
        const vqe_batch_item& it = items[idx[k]];
        const vqe_circuit* c = it.circuit;
        const double* o = r + red_base[k];
        const double nrm = o[1];
        *it.energy = o[0] / nrm;
        for (size_t q = 0; q < c->n_params; ++q) it.grad[q] = 0.0;
        for (size_t sl = 0; sl < c->mid_slot_pidx.size(); ++sl) it.grad[c->mid_slot_pidx[sl]] += o[2 + sl] / nrm;
    }
    return VQE_OK;
}
}  // namespace

// ================================================================ exported
extern "C" {

const char* vqe_last_error(void) { return g_last_error.c_str(); }

const char* vqe_version(void) { return "1.0.0"; }

int vqe_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

int vqe_state_alloc(int n_qubits, int dtype, void* device_buf, size_t buf_bytes, void* hip_stream, vqe_state** out) {
    VQE_GUARD_BEGIN
    if (!out) {
        set_error("vqe_state_alloc: null out");
        return VQE_ERR_ARG;
    }
    if (n_qubits < 1 || n_qubits > 40) {
        set_error("vqe_state_alloc: n_qubits must be in [1, 40]");
        return VQE_ERR_ARG;
    }
    if (dtype != VQE_C64 && dtype != VQE_C128) {
        set_error("vqe_state_alloc: dtype must be VQE_C64 or VQE_C128");
        return VQE_ERR_ARG;
    }
    const size_t need = (size_t(1) << n_qubits) * amp_bytes(dtype);
    if (device_buf && buf_bytes < need) {
        set_error("vqe_state_alloc: device buffer of " + std::to_string(buf_bytes) + " bytes is smaller than the " +
                  std::to_string(need) + " bytes the state needs");
        return VQE_ERR_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        set_error("vqe_state_alloc: no HIP device");
        return VQE_ERR_DEVICE;
    }
    auto* s = new vqe_state();
    s->n = n_qubits;
    s->dtype = dtype;
    s->bytes = need;
    s->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        set_error("vqe_state_alloc: hipGetDevice failed");
        return VQE_ERR_DEVICE;
    }
    if (device_buf) {
        s->data = device_buf;
    } else {
        if (hipMalloc(&s->data, need) != hipSuccess) {
            delete s;
            set_error("vqe_state_alloc: hipMalloc of " + std::to_string(need) + " bytes failed");
            return VQE_ERR_OOM;
        }
        s->owned = true;
    }
    int rc = ensure_res(s, 1024);
    if (rc) {
        if (s->owned) (void)hipFree(s->data);
        delete s;
        return rc;
    }
    if (launch_set_basis(dtype, s->data, 1ull << n_qubits, 0, s->stream) != hipSuccess) {
        set_error("vqe_state_alloc: initialisation kernel failed");
        (void)hipFree(s->d_res);
        (void)hipHostFree(s->h_res);
        if (s->owned) (void)hipFree(s->data);
        delete s;
        return VQE_ERR_DEVICE;
    }
    *out = s;
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_state_free(vqe_state* s) {
    if (!s) return VQE_OK;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->owned && s->data) (void)hipFree(s->data);
    if (s->d_part) (void)hipFree(s->d_part);
    if (s->d_res) (void)hipFree(s->d_res);
    if (s->h_res) (void)hipHostFree(s->h_res);
    if (s->d_mats) (void)hipFree(s->d_mats);
    if (s->h_mats) (void)hipHostFree(s->h_mats);
    if (s->mats_ev) (void)hipEventDestroy(s->mats_ev);
    delete s;
    return VQE_OK;
}

int vqe_state_set_basis(vqe_state* s, uint64_t b) {
    if (int rc = check_state(s, "vqe_state_set_basis")) return rc;
    if (b >= (1ull << s->n)) {
        set_error("vqe_state_set_basis: basis index out of range");
        return VQE_ERR_ARG;
    }
    VQE_HIP(hipSetDevice(s->device));
    VQE_HIP(launch_set_basis(s->dtype, s->data, 1ull << s->n, b, s->stream));
    return VQE_OK;
}

int vqe_state_info(const vqe_state* s, void** device_ptr, int* n_qubits, int* dtype) {
    if (int rc = check_state(s, "vqe_state_info")) return rc;
    if (device_ptr) *device_ptr = s->data;
    if (n_qubits) *n_qubits = s->n;
    if (dtype) *dtype = s->dtype;
    return VQE_OK;
}

int vqe_state_read(const vqe_state* s, uint64_t offset, uint64_t count, void* host_dst) {
    if (int rc = check_state(s, "vqe_state_read")) return rc;
    if (!host_dst && count) {
        set_error("vqe_state_read: null destination");
        return VQE_ERR_ARG;
    }
    if (offset > (1ull << s->n) || count > (1ull << s->n) - offset) {
        set_error("vqe_state_read: range out of bounds");
        return VQE_ERR_ARG;
    }
    const size_t ab = amp_bytes(s->dtype);
    VQE_HIP(hipSetDevice(s->device));
    VQE_HIP(hipMemcpyAsync(host_dst, (const char*)s->data + offset * ab, count * ab, hipMemcpyDeviceToHost, s->stream));
    VQE_HIP(hipStreamSynchronize(s->stream));
    return VQE_OK;
}

int vqe_state_write(vqe_state* s, uint64_t offset, uint64_t count, const void* host_src) {
    if (int rc = check_state(s, "vqe_state_write")) return rc;
    if (!host_src && count) {
        set_error("vqe_state_write: null source");
        return VQE_ERR_ARG;
    }
    if (offset > (1ull << s->n) || count > (1ull << s->n) - offset) {
        set_error("vqe_state_write: range out of bounds");
        return VQE_ERR_ARG;
    }
    const size_t ab = amp_bytes(s->dtype);
    VQE_HIP(hipSetDevice(s->device));
    VQE_HIP(hipMemcpyAsync((char*)s->data + offset * ab, host_src, count * ab, hipMemcpyHostToDevice, s->stream));
    VQE_HIP(hipStreamSynchronize(s->stream));
    return VQE_OK;
}

int vqe_circuit_create(int n_qubits, const vqe_gate* gates, size_t n_gates, vqe_circuit** out) {
    VQE_GUARD_BEGIN
    if (!out || (n_gates && !gates)) {
        set_error("vqe_circuit_create: null argument");
        return VQE_ERR_ARG;
    }
    if (n_qubits < 1 || n_qubits > 40) {
        set_error("vqe_circuit_create: n_qubits must be in [1, 40]");
        return VQE_ERR_ARG;
    }
    std::vector<Gate> gs(n_gates);
    size_t n_params = 0;
    for (size_t i = 0; i < n_gates; ++i) {
        const vqe_gate& g = gates[i];
        if (g.kind > VQE_GATE_DEXC) {
            set_error("vqe_circuit_create: gate " + std::to_string(i) + " has an unknown kind");
            return VQE_ERR_ARG;
        }
        Gate ig{g.kind, g.q0, g.q1, g.param_index, g.angle};
        ig.q2 = g.q2;
        ig.q3 = g.q3;
        int gq[4];
        const int nqg = gate_qubits(ig, gq);
        bool ok = true;
        for (int a = 0; a < nqg; ++a) {
            ok = ok && gq[a] < n_qubits;
            for (int b = 0; b < a; ++b) ok = ok && gq[a] != gq[b];
        }
        if (!ok) {
            set_error("vqe_circuit_create: gate " + std::to_string(i) + " has an invalid or repeated qubit");
            return VQE_ERR_ARG;
        }
        if (g.param_index >= 0 && !(g.kind == VQE_GATE_RY || g.kind == VQE_GATE_RZ || g.kind == VQE_GATE_RX ||
                                    is_excitation(g.kind))) {
            set_error("vqe_circuit_create: gate " + std::to_string(i) + " cannot take a parameter");
            return VQE_ERR_ARG;
        }
        if (g.param_index < -1) {
            set_error("vqe_circuit_create: gate " + std::to_string(i) + " has param_index < -1");
            return VQE_ERR_ARG;
        }
        if (g.param_index < 0 && !std::isfinite(g.angle)) {
            set_error("vqe_circuit_create: gate " + std::to_string(i) + " has a non-finite angle");
            return VQE_ERR_ARG;
        }
        if (nqg == 1) ig.q1 = ig.q0;
        if (nqg < 4) ig.q2 = ig.q3 = 0;
        gs[i] = ig;
        if (g.param_index >= 0) n_params = std::max(n_params, (size_t)g.param_index + 1);
    }
    auto* c = new vqe_circuit();
    c->n = n_qubits;
    c->gates = std::move(gs);
    c->n_params = n_params;
    for (size_t i = 0; i < c->gates.size(); ++i) {
        const Gate& g = c->gates[i];
        BatchGate bg{};
        bg.q0 = (uint8_t)g.q0;
        bg.q1 = (uint8_t)g.q1;
        bg.pidx = g.pidx;
        bg.gen = grad_op(g.kind);
        if (g.kind == VQE_GATE_CNOT) bg.type = OP_CNOT;
        else if (g.kind == VQE_GATE_CZ) bg.type = OP_CZ;
        else if (g.kind == VQE_GATE_X) bg.type = OP_XFLIP;
        else if (is_excitation(g.kind)) {
            // pair rotation on the basis patterns A, B (batched states have n <= 13)
            bg.type = OP_PAIR2;
            bg.gen = OP_GPAIR2;
            const bool dbl = g.kind == VQE_GATE_DEXC;
            if (n_qubits <= 16) {
                bg.pa = (uint16_t)(dbl ? (1u << g.q0) | (1u << g.q1) : (1u << g.q0));
                bg.pb = (uint16_t)(dbl ? (1u << g.q2) | (1u << g.q3) : (1u << g.q1));
            }
            bg.mat = c->n_mats++;
            c->has_excitation = true;
        } else {
            bg.type = OP_U2;
            bg.mat = c->n_mats++;
        }
        c->bgates.push_back(bg);
    }
    for (int v = 0; v < 2; ++v) {
        if (v == 0 && c->has_excitation) continue;  // interpreted kernels have no pair ops
        int rc = build_plan(c, v ? kJitLimits : kInterpLimits, v == 1, c->plan[v]);
        if (rc) {
            free_circuit(c);
            return rc;
        }
    }
    if (int rc = build_mid_plan(c)) {
        free_circuit(c);
        return rc;
    }
    *out = c;
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_circuit_free(vqe_circuit* c) {
    free_circuit(c);
    return VQE_OK;
}

int vqe_circuit_info(const vqe_circuit* c, size_t* n_params, size_t* n_passes) {
    if (!c) {
        set_error("vqe_circuit_info: null circuit");
        return VQE_ERR_ARG;
    }
    if (n_params) *n_params = c->n_params;
    if (n_passes) *n_passes = plan_now(c).passes.size();
    return VQE_OK;
}

int vqe_circuit_pass(const vqe_circuit* c, int dtype, size_t pass, int* window, int* qubits, size_t* n_gates,
                     int32_t* gate_index, size_t capacity) {
    if (!c || (dtype != VQE_C64 && dtype != VQE_C128)) {
        set_error("vqe_circuit_pass: null circuit or bad dtype");
        return VQE_ERR_ARG;
    }
    if (int rc = check_form(c, "vqe_circuit_pass")) return rc;
    const Plan& pl = plan_now(c);
    if (pass >= pl.passes.size()) {
        set_error("vqe_circuit_pass: pass index out of range");
        return VQE_ERR_ARG;
    }
    const PlannedPass& p = pl.passes[pass];
    if (window) *window = p.K;
    if (qubits)
        for (int j = 0; j < p.K; ++j) qubits[j] = p.pos[j];
    if (n_gates) *n_gates = p.gates.size();
    if (gate_index) {
        if (capacity < p.gates.size()) {
            set_error("vqe_circuit_pass: gate_index capacity too small");
            return VQE_ERR_ARG;
        }
        for (size_t i = 0; i < p.gates.size(); ++i) gate_index[i] = p.gates[i];
    }
    return VQE_OK;
}

int vqe_apply_circuit(vqe_state* s, const vqe_circuit* c, const double* params, size_t n_params) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(s, "vqe_apply_circuit")) return rc;
    if (!c || c->n != s->n) {
        set_error("vqe_apply_circuit: circuit missing or of a different qubit count");
        return VQE_ERR_ARG;
    }
    if (int rc = check_params(c, params, n_params, "vqe_apply_circuit")) return rc;
    if (int rc = check_form(c, "vqe_apply_circuit")) return rc;
    VQE_HIP(hipSetDevice(s->device));
    const std::vector<size_t> nob;
    const std::vector<void*> nock;
    const Plan& pl = plan_now(c);
    return s->dtype == VQE_C64 ? forward<float>(s, c, pl, params, nob, nock) : forward<double>(s, c, pl, params, nob, nock);
    VQE_GUARD_END
}

int vqe_apply_dense(vqe_state* s, const int* qubits, int k, const double* u) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(s, "vqe_apply_dense")) return rc;
    if (!qubits || !u) {
        set_error("vqe_apply_dense: null argument");
        return VQE_ERR_ARG;
    }
    if (k != kDenseK) {
        set_error("vqe_apply_dense: k must be " + std::to_string(kDenseK));
        return VQE_ERR_ARG;
    }
    DenseArgs a{};
    uint64_t seen = 0;
    for (int i = 0; i < k; ++i) {
        if (qubits[i] < 4 || qubits[i] >= s->n || ((seen >> qubits[i]) & 1)) {
            set_error("vqe_apply_dense: qubits must be distinct and in [4, n)");
            return VQE_ERR_ARG;
        }
        seen |= 1ull << qubits[i];
        a.q[i] = (uint32_t)qubits[i];
    }
    for (int i = 0, q = 0; q < s->n; ++q)
        if ((seen >> q) & 1) a.sorted[i++] = (uint32_t)q;
    a.n_tiles = 1ull << (s->n - kDenseK - 4);
    VQE_HIP(hipSetDevice(s->device));
    return s->dtype == VQE_C64 ? apply_dense<float>(s, a, u) : apply_dense<double>(s, a, u);
    VQE_GUARD_END
}

int vqe_hamiltonian_create(int n_qubits, const uint64_t* x, const uint64_t* z, const double* w, size_t n_terms,
                           vqe_hamiltonian** out) {
    VQE_GUARD_BEGIN
    if (!out || (n_terms && (!x || !z || !w))) {
        set_error("vqe_hamiltonian_create: null argument");
        return VQE_ERR_ARG;
    }
    if (n_qubits < 1 || n_qubits > 40) {
        set_error("vqe_hamiltonian_create: n_qubits must be in [1, 40]");
        return VQE_ERR_ARG;
    }
    if (n_terms == 0) {
        set_error("vqe_hamiltonian_create: no terms");
        return VQE_ERR_ARG;
    }
    const uint64_t lim = 1ull << n_qubits;
    for (size_t i = 0; i < n_terms; ++i) {
        if (x[i] >= lim || z[i] >= lim) {
            set_error("vqe_hamiltonian_create: term " + std::to_string(i) + " has a mask bit >= n_qubits");
            return VQE_ERR_ARG;
        }
        if (!std::isfinite(w[i])) {
            set_error("vqe_hamiltonian_create: term " + std::to_string(i) + " has a non-finite weight");
            return VQE_ERR_ARG;
        }
    }
    std::vector<size_t> idx(n_terms);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        return x[a] != x[b] ? x[a] < x[b] : z[a] < z[b];
    });
    auto* h = new vqe_hamiltonian();
    h->n = n_qubits;
    for (size_t k = 0; k < n_terms; ++k) {
        const size_t i = idx[k];
        if (!h->x.empty() && h->x.back() == x[i] && h->z.back() == z[i]) {
            h->w.back() += w[i];
        } else {
            h->x.push_back(x[i]);
            h->z.push_back(z[i]);
            h->w.push_back(w[i]);
        }
    }
    std::vector<TermDesc<float>>& t32 = h->t32;
    std::vector<TermDesc<double>>& t64 = h->t64;
    t32.resize(h->w.size());
    t64.resize(h->w.size());
    for (size_t t = 0; t < h->w.size(); ++t) {
        if (h->x[t] == 0 && h->z[t] == 0) h->identity += h->w[t];
        if (h->groups.empty() || h->groups.back().x != h->x[t]) {
            GroupDesc g{};
            g.x = h->x[t];
            g.begin = (uint32_t)t;
            g.hbit = h->x[t] ? 63 - __builtin_clzll(h->x[t]) : 0;
            h->groups.push_back(g);
        }
        h->groups.back().end = (uint32_t)t + 1;
        // c = w (-i)^y with y = popcount(x & z) mod 4
        const int y = __builtin_popcountll(h->x[t] & h->z[t]) & 3;
        const double wv = h->w[t];
        const double cre = (y == 0) ? wv : (y == 2 ? -wv : 0.0);
        const double cim = (y == 1) ? -wv : (y == 3 ? wv : 0.0);
        t64[t] = TermDesc<double>{h->z[t], cre, cim};
        t32[t] = TermDesc<float>{h->z[t], (float)cre, (float)cim};
        if (y & 1) h->real_coeffs = false;
    }
    plan_hwin(h);
    *out = h;
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_hamiltonian_free(vqe_hamiltonian* h) {
    if (!h) return VQE_OK;
    free_hamiltonian_tables(h);
    delete h;
    return VQE_OK;
}

int vqe_hamiltonian_plan(const vqe_hamiltonian* h, size_t* n_windows, uint64_t* window_masks, size_t capacity) {
    if (!h || !n_windows) {
        set_error("vqe_hamiltonian_plan: null argument");
        return VQE_ERR_ARG;
    }
    const size_t m = h->hw_lam ? h->hw_wins.size() : 0;
    *n_windows = m;
    if (window_masks) {
        if (capacity < m) {
            set_error("vqe_hamiltonian_plan: window_masks capacity too small");
            return VQE_ERR_ARG;
        }
        for (size_t i = 0; i < m; ++i) {
            uint64_t wm = 0;
            for (int k = 0; k < kHwBits; ++k) wm |= 1ull << h->hw_wins[i].pos[k];
            window_masks[i] = wm;
        }
    }
    return VQE_OK;
}

int vqe_hamiltonian_info(const vqe_hamiltonian* h, size_t* n_terms, size_t* n_groups, double* identity_weight) {
    if (!h) {
        set_error("vqe_hamiltonian_info: null Hamiltonian");
        return VQE_ERR_ARG;
    }
    if (n_terms) *n_terms = h->w.size();
    if (n_groups) *n_groups = h->groups.size();
    if (identity_weight) *identity_weight = h->identity;
    return VQE_OK;
}

int vqe_expect_pauli(vqe_state* s, const vqe_hamiltonian* h, int mode, double* energy, double* norm) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(s, "vqe_expect_pauli")) return rc;
    if (!h || h->n != s->n || !energy) {
        set_error("vqe_expect_pauli: Hamiltonian missing, of a different qubit count, or null energy");
        return VQE_ERR_ARG;
    }
    if (mode != VQE_EXPECT_GROUPED && mode != VQE_EXPECT_PER_TERM) {
        set_error("vqe_expect_pauli: unknown mode");
        return VQE_ERR_ARG;
    }
    VQE_HIP(hipSetDevice(s->device));
    if (int rc = upload_hamiltonian(h)) return rc;
    if (int rc = ensure_part(s)) return rc;
    return s->dtype == VQE_C64 ? expect_impl<float>(s, h, mode, energy, norm)
                               : expect_impl<double>(s, h, mode, energy, norm);
    VQE_GUARD_END
}

int vqe_apply_hamiltonian(vqe_state* psi, vqe_state* lam, const vqe_hamiltonian* h, double* energy, double* norm) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(psi, "vqe_apply_hamiltonian")) return rc;
    if (int rc = check_state(lam, "vqe_apply_hamiltonian")) return rc;
    if (psi == lam || psi->data == lam->data || lam->n != psi->n || lam->dtype != psi->dtype || !h ||
        h->n != psi->n) {
        set_error("vqe_apply_hamiltonian: lam must be a distinct state of the same n and dtype as psi");
        return VQE_ERR_ARG;
    }
    VQE_HIP(hipSetDevice(psi->device));
    int rc = upload_hamiltonian(h);
    if (rc) return rc;
    if ((rc = ensure_part(psi))) return rc;
    rc = ensure_res(psi, 2);
    if (rc) return rc;
    rc = psi->dtype == VQE_C64 ? apply_h<float>(psi, lam->data, h, psi->d_res)
                               : apply_h<double>(psi, lam->data, h, psi->d_res);
    if (rc) return rc;
    VQE_HIP(hipMemcpyAsync(psi->h_res, psi->d_res, 2 * sizeof(double), hipMemcpyDeviceToHost, psi->stream));
    VQE_HIP(hipStreamSynchronize(psi->stream));
    if (energy) *energy = psi->h_res[0] / psi->h_res[1];
    if (norm) *norm = psi->h_res[1];
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_energy_grad(vqe_state* psi, vqe_state* lam, const vqe_circuit* c, const double* params, size_t n_params,
                    const vqe_hamiltonian* h, const vqe_grad_opts* opts, double* energy, double* grad) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(psi, "vqe_energy_grad")) return rc;
    if (!c || c->n != psi->n || !h || h->n != psi->n || !energy || (n_params && !grad)) {
        set_error("vqe_energy_grad: circuit / Hamiltonian missing or of a different qubit count, or null output");
        return VQE_ERR_ARG;
    }
    if (int rc = check_params(c, params, n_params, "vqe_energy_grad")) return rc;
    if (int rc = check_form(c, "vqe_energy_grad")) return rc;
    const int method = opts ? opts->method : VQE_GRAD_ADJOINT;
    VQE_HIP(hipSetDevice(psi->device));
    if (int rc = upload_hamiltonian(h)) return rc;
    if (int rc = ensure_part(psi)) return rc;
    if (method == VQE_GRAD_PARAM_SHIFT) {
        const int mode = opts ? opts->expect_mode : VQE_EXPECT_GROUPED;
        if (mode != VQE_EXPECT_GROUPED && mode != VQE_EXPECT_PER_TERM) {
            set_error("vqe_energy_grad: unknown expect_mode");
            return VQE_ERR_ARG;
        }
        return psi->dtype == VQE_C64 ? param_shift_impl<float>(psi, c, params, h, mode, energy, grad)
                                     : param_shift_impl<double>(psi, c, params, h, mode, energy, grad);
    }
    if (method != VQE_GRAD_ADJOINT) {
        set_error("vqe_energy_grad: unknown method");
        return VQE_ERR_ARG;
    }
    if (int rc = check_state(lam, "vqe_energy_grad")) return rc;
    if (lam == psi || lam->data == psi->data || lam->n != psi->n || lam->dtype != psi->dtype) {
        set_error("vqe_energy_grad: lam must be a distinct state of the same n and dtype as psi");
        return VQE_ERR_ARG;
    }
    if (opts && opts->chunk_passes < 0) {
        set_error("vqe_energy_grad: chunk_passes must be >= 0");
        return VQE_ERR_ARG;
    }
    if (opts && opts->n_ckpt > 0) {
        if (!opts->ckpt) {
            set_error("vqe_energy_grad: n_ckpt > 0 with a null ckpt array");
            return VQE_ERR_ARG;
        }
        for (int k = 0; k < opts->n_ckpt; ++k) {
            const vqe_state* ck = opts->ckpt[k];
            if (!ck || !ck->data || ck->n != psi->n || ck->dtype != psi->dtype || ck->data == psi->data ||
                ck->data == lam->data) {
                set_error("vqe_energy_grad: checkpoint " + std::to_string(k) +
                          " must be a distinct state of the same n and dtype as psi");
                return VQE_ERR_ARG;
            }
            for (int j = 0; j < k; ++j)
                if (opts->ckpt[j]->data == ck->data) {
                    set_error("vqe_energy_grad: checkpoint states must be distinct");
                    return VQE_ERR_ARG;
                }
        }
    }
    return psi->dtype == VQE_C64 ? adjoint_impl<float>(psi, lam, c, params, h, opts, energy, grad)
                                 : adjoint_impl<double>(psi, lam, c, params, h, opts, energy, grad);
    VQE_GUARD_END
}

int vqe_batch_create(int dtype, void* hip_stream, vqe_batch** out) {
    VQE_GUARD_BEGIN
    if (!out || (dtype != VQE_C64 && dtype != VQE_C128)) {
        set_error("vqe_batch_create: null out or bad dtype");
        return VQE_ERR_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        set_error("vqe_batch_create: no HIP device");
        return VQE_ERR_DEVICE;
    }
    {
        static std::once_flag once;
        static hipError_t lds_rc = hipSuccess;
        std::call_once(once, [] { lds_rc = batch_set_lds_limit(); });
        if (lds_rc != hipSuccess) {
            set_error(std::string("vqe_batch_create: cannot raise the LDS limit: ") + hipGetErrorString(lds_rc));
            return VQE_ERR_DEVICE;
        }
    }
    auto* b = new vqe_batch();
    b->dtype = dtype;
    b->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        set_error("vqe_batch_create: hipGetDevice failed");
        return VQE_ERR_DEVICE;
    }
    *out = b;
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_batch_free(vqe_batch* b) {
    if (!b) return VQE_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    if (b->d_buf) (void)hipFree(b->d_buf);
    if (b->h_buf) (void)hipHostFree(b->h_buf);
    if (b->md_buf) (void)hipFree(b->md_buf);
    if (b->mh_buf) (void)hipHostFree(b->mh_buf);
    delete b;
    return VQE_OK;
}

int vqe_batch_energy_grad(vqe_batch* b, size_t n_items, const vqe_batch_item* items) {
    VQE_GUARD_BEGIN
    if (!b || (n_items && !items)) {
        set_error("vqe_batch_energy_grad: null batch or items");
        return VQE_ERR_ARG;
    }
    if (n_items == 0) return VQE_OK;
    if (n_items > (1u << 20)) {
        set_error("vqe_batch_energy_grad: too many items in one batch (limit 2^20)");
        return VQE_ERR_ARG;
    }
    VQE_HIP(hipSetDevice(b->device));
    // Items up to the LDS limit go to the small-state kernel, larger ones up
    // to kMidMaxQubits to the tile passes; every item is checked first.
    const int max_small = b->dtype == VQE_C64 ? kBatchMaxQubitsC64 : kBatchMaxQubitsC128;
    std::vector<vqe_batch_item> small;
    std::vector<size_t> mid;
    for (size_t i = 0; i < n_items; ++i) {
        const vqe_batch_item& it = items[i];
        if (!it.circuit || !it.hamiltonian || !it.energy || (it.n_params && (!it.params || !it.grad))) {
            set_error("vqe_batch_energy_grad: item " + std::to_string(i) + " has a null field");
            return VQE_ERR_ARG;
        }
        const int n = it.circuit->n;
        if (n > kMidMaxQubits || it.hamiltonian->n != n) {
            set_error("vqe_batch_energy_grad: item " + std::to_string(i) + " has " + std::to_string(n) +
                      " qubits (limit " + std::to_string(kMidMaxQubits) + ") or a Hamiltonian of another size");
            return VQE_ERR_ARG;
        }
        if (int rc = check_params(it.circuit, it.params, it.n_params, "vqe_batch_energy_grad")) return rc;
        if (n <= max_small) small.push_back(it);
        else mid.push_back(i);
    }
    if (!small.empty()) {
        const int rc = b->dtype == VQE_C64 ? batch_impl<float>(b, small.size(), small.data())
                                           : batch_impl<double>(b, small.size(), small.data());
        if (rc) return rc;
    }
    if (!mid.empty()) return b->dtype == VQE_C64 ? mid_impl<float>(b, items, mid) : mid_impl<double>(b, items, mid);
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_circuit_prepare(const vqe_circuit* c, int dtype) {
    VQE_GUARD_BEGIN
    if (!c || (dtype != VQE_C64 && dtype != VQE_C128)) {
        set_error("vqe_circuit_prepare: null circuit or bad dtype");
        return VQE_ERR_ARG;
    }
    if (int rc = check_form(c, "vqe_circuit_prepare")) return rc;
    const Plan& pl = plan_now(c);
    if (!pl.jit) return VQE_OK;
    return ensure_jit(c, pl, dtype == VQE_C128 ? 1 : 0);
    VQE_GUARD_END
}

int vqe_set_specialize(int mode) {
    if (mode != VQE_SPECIALIZE_NEVER && mode != VQE_SPECIALIZE_AUTO && mode != VQE_SPECIALIZE_ALWAYS) {
        vqe::set_error("vqe_set_specialize: unknown mode");
        return VQE_ERR_ARG;
    }
    return vqe::jit_set_mode(mode);
}

int vqe_stream_create(const uint32_t* cu_mask, size_t mask_words, void** stream) {
    VQE_GUARD_BEGIN
    if (!stream || (mask_words && !cu_mask)) {
        set_error("vqe_stream_create: null argument");
        return VQE_ERR_ARG;
    }
    hipStream_t st = nullptr;
    if (mask_words == 0) {
        VQE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    } else {
        int dev = 0, ncu = 0;
        VQE_HIP(hipGetDevice(&dev));
        VQE_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        size_t on = 0;
        for (size_t i = 0; i < mask_words; ++i)
            for (int b = 0; b < 32; ++b)
                if (((cu_mask[i] >> b) & 1) && (int)(32 * i + b) < ncu) ++on;
        if (on == 0) {
            set_error("vqe_stream_create: the CU mask selects no compute unit of the device");
            return VQE_ERR_ARG;
        }
        VQE_HIP(hipExtStreamCreateWithCUMask(&st, (uint32_t)mask_words, cu_mask));
    }
    *stream = st;
    return VQE_OK;
    VQE_GUARD_END
}

int vqe_stream_destroy(void* stream) {
    if (!stream) return VQE_OK;
    VQE_HIP(hipStreamDestroy((hipStream_t)stream));
    return VQE_OK;
}

int vqe_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return VQE_OK;
}

int vqe_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_drain();
    for (auto& t : g_prof_tot) t = ProfTotals{};
    return VQE_OK;
}

int vqe_profile_read(int kind, uint64_t* launches, double* total_ms, double* bytes) {
    if (kind < 0 || kind >= VQE_KERNEL_KINDS) {
        set_error("vqe_profile_read: unknown kernel kind");
        return VQE_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_drain();
    if (launches) *launches = g_prof_tot[kind].launches;
    if (total_ms) *total_ms = g_prof_tot[kind].ms;
    if (bytes) *bytes = g_prof_tot[kind].bytes;
    return VQE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- grouped energy without allocation
// Scratch memory of vqe_expect_pauli_noalloc: the per-block partial sums of
// the energy sweep (kEnergyPartBlocks blocks x 2) and the two reduced sums,
// in a fixed device array.  Each device that runs the call holds its own
// copy until the process ends.  Host code never passes the array's name to a
// kernel: it uses the address hipGetSymbolAddress returns on each device.
namespace {
constexpr size_t kScratchPart = 2 * (size_t)kEnergyPartBlocks;
constexpr size_t kScratchDoubles = kScratchPart + 32;  // partials | sums[2] | pad
static_assert(kScratchDoubles * sizeof(double) == VQE_NOALLOC_SCRATCH_BYTES, "scratch size and its public limit differ");
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
// Address of this device's scratch array, looked up once per device with that
// device current.
int scratch_of_device(int dev, double** out) {
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("vqe_expect_pauli_noalloc: device index beyond the scratch table");
        return VQE_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double* p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("vqe_expect_pauli_noalloc: hipGetSymbolAddress of the scratch array: ") +
                      hipGetErrorString(e));
            return VQE_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VQE_OK;
}
}  // namespace

extern "C" {

int vqe_expect_pauli_noalloc(vqe_state* s, const vqe_hamiltonian* h, double* d_out) {
    VQE_GUARD_BEGIN
    if (int rc = check_state(s, "vqe_expect_pauli_noalloc")) return rc;
    if (!h || h->n != s->n || !d_out) {
        set_error("vqe_expect_pauli_noalloc: Hamiltonian missing, of a different qubit count, or null d_out");
        return VQE_ERR_ARG;
    }
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, d_out) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != s->device) {
        (void)hipGetLastError();
        set_error("vqe_expect_pauli_noalloc: d_out is not device memory of the state's device");
        return VQE_ERR_ARG;
    }
    if (!h->d_ready) {
        set_error("vqe_expect_pauli_noalloc: the Hamiltonian's tables are not on the device yet (any evaluation "
                  "with it, e.g. vqe_expect_pauli, uploads them)");
        return VQE_ERR_STATE;
    }
    const uint32_t blocks = energy_part_blocks(h, s->n);
    if ((size_t)blocks * 2 > kScratchPart) {
        set_error("vqe_expect_pauli_noalloc: the sweep needs " + std::to_string(blocks) +
                  " blocks of partial sums, more than the scratch holds (" + std::to_string(kEnergyPartBlocks) + ")");
        return VQE_ERR_UNSUPPORTED;
    }
    VQE_HIP(hipSetDevice(s->device));
    double* sc = nullptr;
    if (int rc = scratch_of_device(s->device, &sc)) return rc;
    double* sums = sc + kScratchPart;
    int rc = s->dtype == VQE_C64 ? energy_grouped<float>(s, h, sc, sums) : energy_grouped<double>(s, h, sc, sums);
    if (rc) return rc;
    VQE_HIP(launch_energy_ratio(sums, d_out, s->stream));
    return VQE_OK;
    VQE_GUARD_END
}

}  // extern "C"
