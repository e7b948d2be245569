// Fusion planner: partitions a gate list into passes, each pass a window of at
// most lim.kmax qubits whose gates are applied with one read and one write
// of the state (one HBM sweep instead of one per gate).
//
// Gates on disjoint qubits commute, so a gate may run before any earlier gate
// it shares no qubit with; the order of every pair of gates sharing a qubit is
// kept.  Per qubit the gates form a chain; a gate is ready when it heads the
// chain of each of its qubits.  A pass takes a window W and schedules, to a
// fixed point, every ready gate whose qubits lie in W (its closure).  Windows
// are chosen greedily: candidates are every run of consecutive qubits and a
// window grown qubit by qubit from the earliest unscheduled gate; the
// candidate with the largest closure wins (ties: first found).  For the
// layered RY/RZ + CNOT-ladder ansatz this yields overlapping ladder windows
// that pipeline across layers.
#include <algorithm>
#include <set>

#include "vqe_internal.h"

namespace vqe {
namespace {

struct PlanState {
    int n;
    const PlanLimits* lim;
    const std::vector<Gate>* gates;
    std::vector<std::vector<int>> chain;  // per qubit, gate indices in order
    std::vector<size_t> head;             // per qubit, position of next unscheduled gate
};

bool is_param(const Gate& g) { return g.pidx >= 0; }

bool uses_matrix(const Gate& g) {
    return g.kind == VQE_GATE_RY || g.kind == VQE_GATE_RZ || g.kind == VQE_GATE_RX ||
           g.kind == VQE_GATE_H || g.kind == VQE_GATE_SEXC || g.kind == VQE_GATE_DEXC;
}

uint64_t gate_mask(const Gate& g) {
    int q[4];
    const int k = gate_qubits(g, q);
    uint64_t m = 0;
    for (int i = 0; i < k; ++i) m |= 1ull << q[i];
    return m;
}

// Closure of window W (bit mask over qubits) starting from `head`; appends the
// scheduled gates to `out` (if non-null) and advances `head`.  Respects the
// per-pass op / matrix / gradient-slot limits (a repeated parameter within a
// pass shares its slot, counted here once per gate: a safe overestimate).
int closure(const PlanState& ps, uint64_t W, std::vector<size_t>& head, std::vector<int>* out) {
    const PlanLimits& L = *ps.lim;
    const auto& G = *ps.gates;
    int count = 0, ops_rev = 0, mats = 0, slots = 0;
    bool changed = true;
    while (changed) {
        changed = false;
        for (int q = 0; q < ps.n; ++q) {
            if (!((W >> q) & 1)) continue;
            while (head[q] < ps.chain[q].size()) {
                int gi = ps.chain[q][head[q]];
                const Gate& g = G[gi];
                int gq[4];
                const int nqg = gate_qubits(g, gq);
                bool ready = true;
                for (int i = 0; i < nqg && ready; ++i)
                    ready = ((W >> gq[i]) & 1) && ps.chain[gq[i]][head[gq[i]]] == gi;
                if (!ready) break;
                int add_ops = 1 + (is_param(g) ? 1 : 0);
                int add_mats = uses_matrix(g) ? 1 : 0;
                int add_slots = is_param(g) ? 1 : 0;
                if (ops_rev + add_ops > L.ops || mats + add_mats > L.mats || slots + add_slots > L.slots)
                    return count;
                ops_rev += add_ops;
                mats += add_mats;
                slots += add_slots;
                for (int i = 0; i < nqg; ++i) head[gq[i]]++;
                if (out) out->push_back(gi);
                ++count;
                changed = true;
            }
        }
    }
    return count;
}

int popcount64(uint64_t v) { return __builtin_popcountll(v); }

}  // namespace

bool plan_passes(int n, const std::vector<Gate>& gates, const PlanLimits& lim, std::vector<PlannedPass>& out,
                 std::string& msg) {
    out.clear();
    const int K = std::min(n, std::min(lim.kmax, kMaxPlanWindow));
    PlanState ps;
    ps.n = n;
    ps.lim = &lim;
    ps.gates = &gates;
    ps.chain.assign(n, {});
    ps.head.assign(n, 0);
    for (size_t i = 0; i < gates.size(); ++i) {
        int gq[4];
        const int nqg = gate_qubits(gates[i], gq);
        for (int k = 0; k < nqg; ++k) ps.chain[gq[k]].push_back((int)i);
    }
    size_t scheduled = 0;
    std::vector<char> done(gates.size(), 0);
    size_t earliest = 0;
    while (scheduled < gates.size()) {
        while (done[earliest]) ++earliest;
        // Candidate windows.
        std::vector<uint64_t> cands;
        for (int a = 0; a + K <= n; ++a) cands.push_back(((K == 64 ? ~0ull : ((1ull << K) - 1))) << a);
        {
            uint64_t W = gate_mask(gates[earliest]);
            while (popcount64(W) < K) {
                int best_q = -1, best_c = -1;
                for (int q = 0; q < n; ++q) {
                    if ((W >> q) & 1) continue;
                    std::vector<size_t> h = ps.head;
                    int c = closure(ps, W | (1ull << q), h, nullptr);
                    if (c > best_c) {
                        best_c = c;
                        best_q = q;
                    }
                }
                if (best_q < 0) break;
                W |= 1ull << best_q;
            }
            cands.push_back(W);
        }
        uint64_t bestW = 0;
        int bestC = 0;
        for (uint64_t W : cands) {
            std::vector<size_t> h = ps.head;
            int c = closure(ps, W, h, nullptr);
            if (c > bestC) {
                bestC = c;
                bestW = W;
            }
        }
        if (bestC == 0) {
            msg = "planner made no progress (internal error)";
            return false;
        }
        PlannedPass p;
        closure(ps, bestW, ps.head, &p.gates);
        // Shrink the window to the qubits actually touched.
        uint64_t used = 0;
        for (int gi : p.gates) used |= gate_mask(gates[gi]);
        p.K = 0;
        for (int q = 0; q < n; ++q)
            if ((used >> q) & 1) p.pos[p.K++] = q;
        for (int gi : p.gates) done[gi] = 1;
        scheduled += p.gates.size();
        out.push_back(std::move(p));
    }
    return true;
}

}  // namespace vqe
