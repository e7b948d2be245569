// Hamiltonian cutoff ("slimming"), Sec. II-D and Sec. III-D of the paper:
// the Jordan-Wigner terms are sorted by |w| and the small ones dropped.  For a
// normalised state -|w| <= <psi|wP|psi> <= |w|, so the dropped sum of |w|
// bounds the energy change.  Host-only: selection is a sort over at most a
// few hundred thousand terms.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "vqe_internal.h"

using namespace vqe;

extern "C" int vqe_slim_hamiltonian(const uint64_t* x, const uint64_t* z, const double* w,
                                    size_t n_terms, int mode, double value, uint8_t* keep,
                                    size_t* n_kept, double* dropped_abs_sum) {
    if (n_terms > 0 && (!x || !z || !w || !keep)) {
        set_error("vqe_slim_hamiltonian: null array");
        return VQE_ERR_ARG;
    }
    if (!std::isfinite(value) || value < 0.0) {
        set_error("vqe_slim_hamiltonian: value must be finite and >= 0");
        return VQE_ERR_ARG;
    }
    if (mode == VQE_SLIM_REMOVE_PERCENT && (value > 100.0 || value != std::floor(value))) {
        set_error("vqe_slim_hamiltonian: percentage must be an integer in [0, 100]");
        return VQE_ERR_ARG;
    }
    if (mode == VQE_SLIM_KEEP_TOP && (value != std::floor(value) || value > 1e18)) {
        set_error("vqe_slim_hamiltonian: the kept count must be a non-negative integer");
        return VQE_ERR_ARG;
    }
    if (mode != VQE_SLIM_THRESHOLD && mode != VQE_SLIM_REMOVE_PERCENT && mode != VQE_SLIM_BUDGET &&
        mode != VQE_SLIM_KEEP_TOP) {
        set_error("vqe_slim_hamiltonian: unknown mode");
        return VQE_ERR_ARG;
    }
    for (size_t i = 0; i < n_terms; ++i) {
        if (!std::isfinite(w[i])) {
            set_error("vqe_slim_hamiltonian: non-finite weight");
            return VQE_ERR_ARG;
        }
    }
    // Order of importance over the non-identity terms.
    std::vector<size_t> order;
    order.reserve(n_terms);
    for (size_t i = 0; i < n_terms; ++i)
        if (x[i] != 0 || z[i] != 0) order.push_back(i);
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        double wa = std::fabs(w[a]), wb = std::fabs(w[b]);
        if (wa != wb) return wa > wb;
        if (x[a] != x[b]) return x[a] < x[b];
        return z[a] < z[b];
    });
    std::vector<uint8_t> k(n_terms, 1);
    double dropped = 0.0;
    if (mode == VQE_SLIM_THRESHOLD) {
        for (auto it = order.rbegin(); it != order.rend(); ++it) {
            if (std::fabs(w[*it]) < value) {
                k[*it] = 0;
                dropped += std::fabs(w[*it]);
            }
        }
    } else if (mode == VQE_SLIM_REMOVE_PERCENT || mode == VQE_SLIM_KEEP_TOP) {
        const size_t n_keep = (size_t)value;
        const size_t n_drop = mode == VQE_SLIM_REMOVE_PERCENT ? (order.size() * (size_t)value) / 100
                              : (n_keep < order.size() ? order.size() - n_keep : 0);
        for (size_t j = 0; j < n_drop; ++j) {
            size_t i = order[order.size() - 1 - j];
            k[i] = 0;
            dropped += std::fabs(w[i]);
        }
    } else {
        for (auto it = order.rbegin(); it != order.rend(); ++it) {
            double nxt = dropped + std::fabs(w[*it]);
            if (nxt > value) break;
            dropped = nxt;
            k[*it] = 0;
        }
    }
    size_t kept = 0;
    for (size_t i = 0; i < n_terms; ++i) {
        keep[i] = k[i];
        kept += k[i];
    }
    if (n_kept) *n_kept = kept;
    if (dropped_abs_sum) *dropped_abs_sum = dropped;
    return VQE_OK;
}
