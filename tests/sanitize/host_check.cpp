// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the fusion planner and its lane-split
// lowering (vqe_circuit_create / vqe_circuit_pass), the Hamiltonian tables
// and the window cover of H psi (vqe_hamiltonian_create / _plan / _info) and
// the cutoff rules (vqe_slim_hamiltonian), on random and structured inputs,
// plus their argument errors.  None of these calls touches a device.  Built
// host-only (no device code) by tests/test_sanitize.py; exits non-zero on
// the first failed expectation, and the sanitizers abort on any memory or
// undefined-behaviour error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "vqe.h"

#define EXPECT(c)                                                             \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n",      \
                         __FILE__, __LINE__, #c, vqe_last_error());           \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

static std::mt19937_64 rng(12345);
static int rint(int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); }

static vqe_gate gate(int kind, int a, int b = 0, int c = 0, int d = 0, int p = -1, double ang = 0.3) {
    vqe_gate g{};
    g.kind = (uint8_t)kind;
    g.q0 = (uint8_t)a;
    g.q1 = (uint8_t)b;
    g.q2 = (uint8_t)c;
    g.q3 = (uint8_t)d;
    g.param_index = p;
    g.angle = ang;
    return g;
}

// distinct qubits
static void pick(int n, int k, int* q) {
    for (int i = 0; i < k; ++i) {
        bool again;
        do {
            q[i] = rint(0, n - 1);
            again = false;
            for (int j = 0; j < i; ++j) again |= q[j] == q[i];
        } while (again);
    }
}

static void check_circuit(int n, const std::vector<vqe_gate>& gs) {
    vqe_circuit* c = nullptr;
    EXPECT(vqe_circuit_create(n, gs.data(), gs.size(), &c) == VQE_OK);
    size_t np = 0, npass = 0;
    EXPECT(vqe_circuit_info(c, &np, &npass) == VQE_OK);
    for (int dt : {VQE_C64, VQE_C128}) {
        size_t covered = 0;
        for (size_t p = 0; p < npass; ++p) {
            int window = 0, qubits[VQE_MAX_WINDOW] = {0};
            size_t ng = 0;
            EXPECT(vqe_circuit_pass(c, dt, p, &window, qubits, &ng, nullptr, 0) == VQE_OK);
            EXPECT(window >= 1 && window <= VQE_MAX_WINDOW && window <= n);
            std::vector<int32_t> idx(ng + 1);
            EXPECT(vqe_circuit_pass(c, dt, p, &window, qubits, &ng, idx.data(), idx.size()) == VQE_OK);
            for (size_t i = 0; i < ng; ++i) EXPECT(idx[i] >= 0 && (size_t)idx[i] < gs.size());
            for (int i = 1; i < window; ++i) EXPECT(qubits[i - 1] < qubits[i]);
            covered += ng;
        }
        EXPECT(covered == gs.size());
        int window = 0, qubits[VQE_MAX_WINDOW];
        size_t ng = 0;
        EXPECT(vqe_circuit_pass(c, dt, npass, &window, qubits, &ng, nullptr, 0) == VQE_ERR_ARG);
    }
    EXPECT(vqe_circuit_free(c) == VQE_OK);
}

static void circuits() {
    for (int it = 0; it < 300; ++it) {
        const int n = rint(1, 34);
        const int ng = rint(0, 120);
        std::vector<vqe_gate> gs;
        int p = 0;
        for (int i = 0; i < ng; ++i) {
            int q[4];
            const int kind = rint(0, 8);
            if ((kind == VQE_GATE_CNOT || kind == VQE_GATE_CZ || kind == VQE_GATE_SEXC) && n < 2) continue;
            if (kind == VQE_GATE_DEXC && n < 4) continue;
            switch (kind) {
                case VQE_GATE_CNOT: case VQE_GATE_CZ: pick(n, 2, q); gs.push_back(gate(kind, q[0], q[1])); break;
                case VQE_GATE_SEXC: pick(n, 2, q); gs.push_back(gate(kind, q[0], q[1], 0, 0, p++)); break;
                case VQE_GATE_DEXC: pick(n, 4, q); gs.push_back(gate(kind, q[0], q[1], q[2], q[3], p++)); break;
                case VQE_GATE_H: case VQE_GATE_X: gs.push_back(gate(kind, rint(0, n - 1))); break;
                default: gs.push_back(gate(kind, rint(0, n - 1), 0, 0, 0, rint(0, 1) ? p++ : -1)); break;
            }
        }
        check_circuit(n, gs);
    }
    for (int n : {12, 20, 28, 32}) {  // the layered ansatz of the workloads
        std::vector<vqe_gate> gs;
        for (int l = 0, p = 0; l < 8; ++l) {
            for (int q = 0; q < n; ++q) gs.push_back(gate(VQE_GATE_RY, q, 0, 0, 0, p++));
            for (int q = 0; q < n; ++q) gs.push_back(gate(VQE_GATE_RZ, q, 0, 0, 0, p++));
            for (int q = 0; q + 1 < n; ++q) gs.push_back(gate(VQE_GATE_CNOT, q, q + 1));
        }
        check_circuit(n, gs);
    }
    vqe_circuit* c = nullptr;
    vqe_gate bad = gate(VQE_GATE_CNOT, 3, 3);
    EXPECT(vqe_circuit_create(5, &bad, 1, &c) == VQE_ERR_ARG);
    bad = gate(VQE_GATE_RY, 9);
    EXPECT(vqe_circuit_create(5, &bad, 1, &c) == VQE_ERR_ARG);
    bad = gate(42, 0);
    EXPECT(vqe_circuit_create(5, &bad, 1, &c) == VQE_ERR_ARG);
}

static void check_hamiltonian(int n, const std::vector<uint64_t>& x, const std::vector<uint64_t>& z,
                              const std::vector<double>& w) {
    vqe_hamiltonian* h = nullptr;
    EXPECT(vqe_hamiltonian_create(n, x.data(), z.data(), w.data(), w.size(), &h) == VQE_OK);
    size_t nt = 0, ngr = 0, nw = 0;
    double id = 0;
    EXPECT(vqe_hamiltonian_info(h, &nt, &ngr, &id) == VQE_OK);
    EXPECT(nt <= w.size() && ngr <= nt + 1);
    EXPECT(vqe_hamiltonian_plan(h, &nw, nullptr, 0) == VQE_OK);
    std::vector<uint64_t> masks(nw + 1);
    EXPECT(vqe_hamiltonian_plan(h, &nw, masks.data(), masks.size()) == VQE_OK);
    for (size_t i = 0; i < nw; ++i) EXPECT(__builtin_popcountll(masks[i]) == VQE_HPSI_WINDOW_QUBITS && (masks[i] & 7) == 7);
    if (nw) EXPECT(vqe_hamiltonian_plan(h, &nw, masks.data(), nw - 1) == VQE_ERR_ARG);
    EXPECT(vqe_hamiltonian_free(h) == VQE_OK);
}

static void hamiltonians() {
    std::normal_distribution<double> nd;
    for (int it = 0; it < 200; ++it) {
        const int n = rint(1, 40);
        const int nt = rint(1, 400);
        const int span = rint(1, std::min(n, 14));  // x masks over a few nearby qubits, as in lattice models
        std::vector<uint64_t> x(nt), z(nt);
        std::vector<double> w(nt);
        const uint64_t all = n == 64 ? ~0ull : ((1ull << n) - 1);
        for (int t = 0; t < nt; ++t) {
            const int lo = rint(0, n - span);
            const uint64_t win = ((span == 64 ? ~0ull : (1ull << span) - 1) << lo) & all;
            x[t] = rng() & win;
            z[t] = rng() & all;
            w[t] = nd(rng);
        }
        check_hamiltonian(n, x, z, w);
    }
    // one X group with more distinct in-window z patterns than a pass holds
    std::vector<uint64_t> x, z;
    std::vector<double> w;
    for (int t = 0; t < 1500; ++t) {
        x.push_back(1);
        z.push_back(rng() & ((1ull << 20) - 1));
        w.push_back(nd(rng));
    }
    for (int q = VQE_HPSI_WINDOW_QUBITS; q < 20; ++q) {
        x.push_back(1ull << q);
        z.push_back(0);
        w.push_back(0.5);
    }
    check_hamiltonian(20, x, z, w);
    vqe_hamiltonian* h = nullptr;
    uint64_t bx = 1ull << 7, bz = 0;
    double bw = 1.0;
    EXPECT(vqe_hamiltonian_create(5, &bx, &bz, &bw, 1, &h) == VQE_ERR_ARG);  // mask beyond n
    bx = 1;
    bw = NAN;
    EXPECT(vqe_hamiltonian_create(5, &bx, &bz, &bw, 1, &h) == VQE_ERR_ARG);  // non-finite weight
}

static void slimming() {
    std::normal_distribution<double> nd;
    for (int it = 0; it < 100; ++it) {
        const size_t nt = (size_t)rint(0, 500);
        std::vector<uint64_t> x(nt), z(nt);
        std::vector<double> w(nt);
        for (size_t t = 0; t < nt; ++t) {
            x[t] = rng() & 0xfff;
            z[t] = rng() & 0xfff;
            w[t] = std::round(nd(rng) * 8) / 8 * std::pow(10.0, -rint(0, 6));
        }
        std::vector<uint8_t> keep(nt + 1);
        size_t nk = 0;
        double dropped = 0;
        for (int mode : {VQE_SLIM_THRESHOLD, VQE_SLIM_REMOVE_PERCENT, VQE_SLIM_BUDGET, VQE_SLIM_KEEP_TOP}) {
            const double v = mode == VQE_SLIM_THRESHOLD ? 1e-3 : mode == VQE_SLIM_REMOVE_PERCENT ? rint(0, 100)
                             : mode == VQE_SLIM_BUDGET ? 0.01 : rint(0, 600);
            EXPECT(vqe_slim_hamiltonian(x.data(), z.data(), w.data(), nt, mode, v, keep.data(), &nk, &dropped) ==
                   VQE_OK);
            EXPECT(nk <= nt && dropped >= 0.0);
        }
    }
    uint64_t x = 1, z = 0;
    double w = 1;
    uint8_t k = 0;
    EXPECT(vqe_slim_hamiltonian(&x, &z, &w, 1, 9, 0.1, &k, nullptr, nullptr) == VQE_ERR_ARG);
    EXPECT(vqe_slim_hamiltonian(&x, &z, &w, 1, VQE_SLIM_KEEP_TOP, 1.5, &k, nullptr, nullptr) == VQE_ERR_ARG);
    EXPECT(vqe_slim_hamiltonian(nullptr, &z, &w, 1, VQE_SLIM_THRESHOLD, 0.1, &k, nullptr, nullptr) == VQE_ERR_ARG);
}

int main() {
    circuits();
    hamiltonians();
    slimming();
    std::printf("host checks passed\n");
    return 0;
}
