// A verified decomposition U = D R(P_t) ... R(P_1) (up to global phase) as a gate list over
// {H, S, S^dag, CNOT, T, T^dag, X, Y, Z} (Sec. 5.3: the Pauli part as conjugated T gates, the
// Clifford part from its action on Paulis).  Host code: a few dozen gates on n <= 4 qubits.
//
// Paulis are codes q in [0, 4^n): x = q & (2^n - 1), z = q >> n, qubit j on bit j, with
// sigma(1,1) = Y = iXZ.  A signed Pauli is (code, sign).  Conjugation rules (U P U^dag):
//   H_j:       swap x_j, z_j; sign flips on Y_j
//   S_j:       z_j ^= x_j;    sign flips on Y_j          (S X S^dag = Y, S Y S^dag = -X)
//   S^dag_j:   z_j ^= x_j;    sign flips on X_j          (S^dag X S = -Y, S^dag Y S = X)
//   CNOT(c,t): x_t ^= x_c, z_c ^= z_t; sign flips iff x_c z_t (x_t xor z_c xor 1)
//   X_j, Z_j, Y_j: sign flips when P anticommutes with them
// R(P) = C^dag R(C P C^dag) C for a Clifford C; with C P C^dag = s Z_q, R(Z_q) = T_q and
// R(-Z_q) = omega T_q^dag.
#include <cstdint>
#include <vector>

#include "tcw.h"

namespace {

struct SP {
    uint32_t code;
    int sign;  // +1 or -1
};

struct Conj {
    int n;
    int xb(uint32_t c, int j) const { return (c >> j) & 1; }
    int zb(uint32_t c, int j) const { return (c >> (n + j)) & 1; }

    void apply(const tcw_gate& g, SP& p) const {
        uint32_t& c = p.code;
        const int j = g.q0;
        switch (g.kind) {
            case TCW_GATE_H: {
                const int x = xb(c, j), z = zb(c, j);
                if (x && z) p.sign = -p.sign;
                c &= ~((1u << j) | (1u << (n + j)));
                c |= ((uint32_t)z << j) | ((uint32_t)x << (n + j));
                break;
            }
            case TCW_GATE_S: {
                const int x = xb(c, j), z = zb(c, j);
                if (x && z) p.sign = -p.sign;
                if (x) c ^= 1u << (n + j);
                break;
            }
            case TCW_GATE_SDG: {
                const int x = xb(c, j), z = zb(c, j);
                if (x && !z) p.sign = -p.sign;
                if (x) c ^= 1u << (n + j);
                break;
            }
            case TCW_GATE_CNOT: {
                const int t = g.q1;
                const int xc = xb(c, j), zc = zb(c, j), xt = xb(c, t), zt = zb(c, t);
                if (xc && zt && ((xt ^ zc ^ 1) & 1)) p.sign = -p.sign;
                if (xc) c ^= 1u << t;
                if (zt) c ^= 1u << (n + j);
                break;
            }
            case TCW_GATE_X:
                if (zb(c, j)) p.sign = -p.sign;
                break;
            case TCW_GATE_Z:
                if (xb(c, j)) p.sign = -p.sign;
                break;
            case TCW_GATE_Y:
                if (xb(c, j) ^ zb(c, j)) p.sign = -p.sign;
                break;
            default:
                break;
        }
    }
};

tcw_gate gate(int kind, int q0, int q1 = -1) { return tcw_gate{kind, q0, q1}; }

tcw_gate inverse(const tcw_gate& g) {
    if (g.kind == TCW_GATE_S) return gate(TCW_GATE_SDG, g.q0);
    if (g.kind == TCW_GATE_SDG) return gate(TCW_GATE_S, g.q0);
    if (g.kind == TCW_GATE_T) return gate(TCW_GATE_TDG, g.q0);
    if (g.kind == TCW_GATE_TDG) return gate(TCW_GATE_T, g.q0);
    return g;  // H, CNOT and the Paulis are self-inverse (up to phase)
}

// Clifford C (gates in application order) with C P C^dag = s Z_q; returns q, sets s.
int to_single_z(const Conj& cj, uint32_t code, std::vector<tcw_gate>& C, int& s) {
    SP p{code, 1};
    auto use = [&](tcw_gate g) {
        cj.apply(g, p);
        C.push_back(g);
    };
    for (int k = 0; k < cj.n; ++k) {
        const int x = cj.xb(p.code, k), z = cj.zb(p.code, k);
        if (x && z) use(gate(TCW_GATE_S, k));  // Y -> -X
        if (x) use(gate(TCW_GATE_H, k));       // X -> Z
    }
    int q = -1;
    for (int k = 0; k < cj.n; ++k)
        if (cj.zb(p.code, k)) {
            if (q < 0) q = k;
            else use(gate(TCW_GATE_CNOT, k, q));  // Z_k Z_q -> Z_q
        }
    s = p.sign;
    return q;
}

// Gates G_1..G_m (applied on the left) reducing the tableau of D to the identity.
bool reduce_clifford(const Conj& cj, std::vector<SP>& img, std::vector<tcw_gate>& G) {
    const int n = cj.n;
    auto use = [&](tcw_gate g) {
        for (auto& p : img) cj.apply(g, p);
        G.push_back(g);
    };
    for (int j = 0; j < n; ++j) {
        SP* a = &img[j];          // image of X_j
        SP* b = &img[n + j];      // image of Z_j
        // the image of X_j acts only on qubits >= j (it commutes with X_i, Z_i for i < j)
        int k0 = -1;
        for (int k = j; k < n; ++k)
            if (cj.xb(a->code, k)) {
                k0 = k;
                break;
            }
        if (k0 < 0) {
            for (int k = j; k < n; ++k)
                if (cj.zb(a->code, k)) {
                    k0 = k;
                    break;
                }
            if (k0 < 0) return false;
            use(gate(TCW_GATE_H, k0));
        }
        if (!cj.xb(a->code, j)) use(gate(TCW_GATE_CNOT, k0, j));
        for (int k = j + 1; k < n; ++k)
            if (cj.xb(a->code, k)) use(gate(TCW_GATE_CNOT, j, k));
        if (cj.zb(a->code, j)) use(gate(TCW_GATE_S, j));
        for (int k = j + 1; k < n; ++k)
            if (cj.zb(a->code, k)) {
                use(gate(TCW_GATE_H, k));
                use(gate(TCW_GATE_CNOT, j, k));
            }
        // the image of Z_j anticommutes with X_j: clear its other qubits keeping X_j fixed
        for (int k = j + 1; k < n; ++k) {
            const int x = cj.xb(b->code, k), z = cj.zb(b->code, k);
            if (!x && !z) continue;
            if (x && z) use(gate(TCW_GATE_S, k));
            if (x) use(gate(TCW_GATE_H, k));
            use(gate(TCW_GATE_CNOT, k, j));
        }
        if (cj.xb(b->code, j)) {
            // Y_j -> Z_j with X_j fixed: H S H maps Y to Z (and X to X)
            use(gate(TCW_GATE_H, j));
            use(gate(TCW_GATE_S, j));
            use(gate(TCW_GATE_H, j));
        }
        if (a->code != (1u << j) || b->code != (1u << (n + j))) return false;
    }
    for (int j = 0; j < n; ++j) {
        if (img[j].sign < 0) use(gate(TCW_GATE_Z, j));
        if (img[n + j].sign < 0) use(gate(TCW_GATE_X, j));
    }
    // generator j (X_0..X_{n-1}, then Z_0..Z_{n-1}) has code 1 << j
    for (int j = 0; j < 2 * n; ++j)
        if (img[j].sign != 1 || img[j].code != (1u << j)) return false;
    return true;
}

// Append g, or drop it together with the previous gate when that one is its inverse.
void push_cancel(std::vector<tcw_gate>& out, const tcw_gate& g) {
    if (!out.empty()) {
        const tcw_gate ib = inverse(out.back());
        if (ib.kind == g.kind && ib.q0 == g.q0 && ib.q1 == g.q1) {
            out.pop_back();
            return;
        }
    }
    out.push_back(g);
}

}  // namespace

extern "C" int tcw_circuit(const tcw_result* res, tcw_gate* gates, int32_t cap, int32_t* count) {
    if (!res || !count || cap < 0 || (cap > 0 && !gates)) return TCW_EINVAL;
    *count = 0;
    const int n = res->n;
    if (res->status != 1 || n < 1 || n > 4 || res->t < 0 || res->t > TCW_MAX_T) return TCW_EINVAL;
    const Conj cj{n};
    const uint32_t R = 1u << (2 * n);
    std::vector<tcw_gate> out;
    // R(P_1) first: res->paulis lists P_t, ..., P_1
    for (int i = res->t - 1; i >= 0; --i) {
        const uint32_t p = res->paulis[i];
        if (p == 0 || p >= R) return TCW_EINVAL;
        std::vector<tcw_gate> C;
        int s = 1;
        const int q = to_single_z(cj, p, C, s);
        if (q < 0) return TCW_EINVAL;
        for (const auto& g : C) push_cancel(out, g);
        push_cancel(out, gate(s > 0 ? TCW_GATE_T : TCW_GATE_TDG, q));
        for (auto it = C.rbegin(); it != C.rend(); ++it) push_cancel(out, inverse(*it));
    }
    // D from its images D P_q D^dag = sign[q] P_perm[q] of the generators X_j, Z_j
    std::vector<SP> img(2 * n);
    for (int j = 0; j < 2 * n; ++j) {
        const uint32_t code = 1u << j;
        const int32_t pc = res->clifford_perm[code];
        const int8_t sg = res->clifford_sign[code];
        if (pc <= 0 || (uint32_t)pc >= R || (sg != 1 && sg != -1)) return TCW_EINVAL;
        img[j] = SP{(uint32_t)pc, sg};
    }
    std::vector<tcw_gate> G;
    if (!reduce_clifford(cj, img, G)) return TCW_EINVAL;
    // G_m ... G_1 D = I, so D = G_1^dag ... G_m^dag: apply G_m^dag first
    for (auto it = G.rbegin(); it != G.rend(); ++it) push_cancel(out, inverse(*it));
    *count = (int32_t)out.size();
    if ((int64_t)out.size() > cap) return gates ? TCW_EOVERFLOW : TCW_OK;
    for (size_t i = 0; i < out.size(); ++i) gates[i] = out[i];
    return TCW_OK;
}
