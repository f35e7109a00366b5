// Gate matrices from (op, angles) and gate validation (host, FP64).
//
// A one-qubit gate is the 2x2 matrix U of the pair update (QVecOpt Sec. III.A
// Eq. 5); a two-qubit gate is a 4x4 on the quadruple of its two qubits
// (Sec. III.C). The paper names no gate set; matrices follow OpenQASM 2,
// global phase included, so amplitudes (not just probabilities) are fixed.
// Diagonal gates are recorded as diagonals so that the planner can let them
// join any pass and the sweeps touch only the part of the state they change.
#include <cmath>

#include "gates.h"

namespace qv {

namespace {

const cd I1(0.0, 1.0);

bool is_diag2(const cd* m) { return m[1] == 0.0 && m[2] == 0.0; }

bool is_diag4(const cd* m)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            if (r != c && m[4 * r + c] != 0.0) return false;
    return true;
}

void set2(HostGate& g, cd a, cd b, cd c, cd d)
{
    g.kind = G_DENSE1;
    g.m[0] = a;
    g.m[1] = b;
    g.m[2] = c;
    g.m[3] = d;
}

void set_diag1(HostGate& g, int q, cd d0, cd d1)
{
    g.kind = G_DIAG;
    g.q[0] = q;
    g.q[1] = -1;
    g.m[0] = d0;
    g.m[1] = d1;
    g.m[2] = d0;
    g.m[3] = d1;
}

void set_diag2(HostGate& g, int qa, int qc, cd d0, cd d1, cd d2, cd d3)
{
    g.kind = G_DIAG;
    g.q[0] = qa;
    g.q[1] = qc;
    g.m[0] = d0;
    g.m[1] = d1;
    g.m[2] = d2;
    g.m[3] = d3;
}

}  // namespace

bool is_two_qubit_op(int op)
{
    return op == SV_OP_MATRIX2 || op == SV_OP_CNOT || op == SV_OP_CZ || op == SV_OP_CP || op == SV_OP_SWAP;
}

std::string check_gate(const sv_gate& g, int n)
{
    if (g.op < SV_OP_MATRIX1 || g.op > SV_OP_SWAP) return "unknown op " + std::to_string(g.op);
    if (g.reserved != 0) return "reserved field must be 0";
    const bool two = is_two_qubit_op(g.op);
    const int nt = two ? 2 : 1;
    uint64_t seen = 0;
    for (int t = 0; t < nt; t++) {
        const int q = g.qubits[t];
        if (q < 0 || q >= n) return "qubit " + std::to_string(q) + " out of range";
        if (seen & (1ull << q)) return "repeated qubit " + std::to_string(q);
        seen |= 1ull << q;
    }
    if (g.n_controls < 0 || g.n_controls > 2) return "n_controls must be 0..2";
    for (int c = 0; c < g.n_controls; c++) {
        const int q = g.controls[c];
        if (q < 0 || q >= n) return "control " + std::to_string(q) + " out of range";
        if (seen & (1ull << q)) return "control " + std::to_string(q) + " repeats a qubit of the gate";
        seen |= 1ull << q;
    }
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(g.angles[a])) return "non-finite angle";
    if (g.op == SV_OP_MATRIX1 || g.op == SV_OP_MATRIX2) {
        const int cnt = g.op == SV_OP_MATRIX1 ? 8 : 32;
        for (int e = 0; e < cnt; e++)
            if (!std::isfinite(g.matrix[e])) return "non-finite matrix entry";
    }
    if (g.param_index < -1) return "param_index must be -1 or a slot";
    if (g.param_index >= 0 && g.op != SV_OP_RX && g.op != SV_OP_RY && g.op != SV_OP_RZ)
        return "only RX/RY/RZ may carry a param_index";
    return "";
}

bool unsupported_gate(const sv_gate& g, std::string* why)
{
    if (is_two_qubit_op(g.op) && g.n_controls > 0) {
        *why = "extra controls on a two-qubit op are not supported";
        return true;
    }
    if (g.param_index >= 0 && g.n_controls > 0) {
        *why = "a trainable gate cannot carry controls";
        return true;
    }
    return false;
}

HostGate build_gate(const sv_gate& g)
{
    HostGate h;
    h.q[0] = g.qubits[0];
    h.param = g.param_index;
    for (int c = 0; c < g.n_controls; c++) h.ctrl |= 1ull << g.controls[c];
    const double th = g.angles[0];
    const double c2 = std::cos(0.5 * th), s2 = std::sin(0.5 * th);
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (g.op) {
    case SV_OP_H: set2(h, r2, r2, r2, -r2); break;
    case SV_OP_X: set2(h, 0.0, 1.0, 1.0, 0.0); break;
    case SV_OP_Y: set2(h, 0.0, -I1, I1, 0.0); break;
    case SV_OP_Z: set_diag1(h, h.q[0], 1.0, -1.0); break;
    case SV_OP_S: set_diag1(h, h.q[0], 1.0, I1); break;
    case SV_OP_SDG: set_diag1(h, h.q[0], 1.0, -I1); break;
    case SV_OP_T: set_diag1(h, h.q[0], 1.0, std::polar(1.0, M_PI / 4)); break;
    case SV_OP_TDG: set_diag1(h, h.q[0], 1.0, std::polar(1.0, -M_PI / 4)); break;
    case SV_OP_RX:
        set2(h, c2, -I1 * s2, -I1 * s2, c2);
        h.gen = GEN_X;
        break;
    case SV_OP_RY:
        set2(h, c2, -s2, s2, c2);
        h.gen = GEN_Y;
        break;
    case SV_OP_RZ:
        set_diag1(h, h.q[0], std::polar(1.0, -0.5 * th), std::polar(1.0, 0.5 * th));
        h.gen = GEN_Z;
        break;
    case SV_OP_P: set_diag1(h, h.q[0], 1.0, std::polar(1.0, th)); break;
    case SV_OP_U3: {
        const double ph = g.angles[1], la = g.angles[2];
        set2(h, c2, -std::polar(s2, la), std::polar(s2, ph), std::polar(c2, ph + la));
        break;
    }
    case SV_OP_MATRIX1: {
        cd m[4];
        for (int e = 0; e < 4; e++) m[e] = cd(g.matrix[2 * e], g.matrix[2 * e + 1]);
        if (is_diag2(m)) set_diag1(h, h.q[0], m[0], m[3]);
        else set2(h, m[0], m[1], m[2], m[3]);
        break;
    }
    case SV_OP_CNOT:
        // X on the target where the control (and any extra control) is 1
        h.q[0] = g.qubits[1];
        h.ctrl |= 1ull << g.qubits[0];
        set2(h, 0.0, 1.0, 1.0, 0.0);
        break;
    case SV_OP_CZ: set_diag2(h, g.qubits[0], g.qubits[1], 1.0, 1.0, 1.0, -1.0); break;
    case SV_OP_CP: set_diag2(h, g.qubits[0], g.qubits[1], 1.0, 1.0, 1.0, std::polar(1.0, th)); break;
    case SV_OP_SWAP:
        h.kind = G_DENSE2;
        h.q[1] = g.qubits[1];
        for (int e = 0; e < 16; e++) h.m[e] = 0.0;
        h.m[0] = 1.0;
        h.m[1 * 4 + 2] = 1.0;
        h.m[2 * 4 + 1] = 1.0;
        h.m[15] = 1.0;
        break;
    case SV_OP_MATRIX2: {
        cd m[16];
        for (int e = 0; e < 16; e++) m[e] = cd(g.matrix[2 * e], g.matrix[2 * e + 1]);
        if (is_diag4(m)) {
            set_diag2(h, g.qubits[0], g.qubits[1], m[0], m[5], m[10], m[15]);
        } else {
            h.kind = G_DENSE2;
            h.q[1] = g.qubits[1];
            for (int e = 0; e < 16; e++) h.m[e] = m[e];
        }
        break;
    }
    default: break;
    }
    return h;
}

HostGate dagger(const HostGate& g)
{
    HostGate d = g;
    if (g.kind == G_DENSE1) {
        d.m[0] = std::conj(g.m[0]);
        d.m[1] = std::conj(g.m[2]);
        d.m[2] = std::conj(g.m[1]);
        d.m[3] = std::conj(g.m[3]);
    } else if (g.kind == G_DENSE2) {
        for (int r = 0; r < 4; r++)
            for (int c = 0; c < 4; c++) d.m[4 * r + c] = std::conj(g.m[4 * c + r]);
    } else {
        for (int e = 0; e < 4; e++) d.m[e] = std::conj(g.m[e]);
    }
    return d;
}

uint64_t dense_bits(const HostGate& g)
{
    if (g.kind == G_DENSE1) return 1ull << g.q[0];
    if (g.kind == G_DENSE2) return (1ull << g.q[0]) | (1ull << g.q[1]);
    return 0;
}

uint64_t diag_bits(const HostGate& g)
{
    uint64_t m = g.ctrl;
    if (g.kind == G_DIAG) {
        if (g.q[0] >= 0) m |= 1ull << g.q[0];
        if (g.q[1] >= 0) m |= 1ull << g.q[1];
    }
    return m;
}

HostGate sweep_form(const HostGate& g)
{
    // A diagonal that is 1 wherever some qubit's bit is 0 only changes the
    // subspace where that bit is 1: move the qubit into the control mask so
    // the diagonal sweep touches only that subspace.
    HostGate h = g;
    if (h.kind != G_DIAG) return h;
    const cd one(1.0, 0.0);
    if (h.q[1] < 0) {
        if (h.m[0] == one) {
            h.ctrl |= 1ull << h.q[0];
            h.m[0] = h.m[1];
            h.q[0] = -1;
        }
        return h;
    }
    if (h.m[0] == one && h.m[1] == one && h.m[2] == one) {  // only |11> changes
        h.ctrl |= (1ull << h.q[0]) | (1ull << h.q[1]);
        h.m[0] = h.m[3];
        h.q[0] = h.q[1] = -1;
    } else if (h.m[0] == one && h.m[1] == one) {  // only bit q1 = 1 changes: diagonal (d2, d3) on q0
        h.ctrl |= 1ull << h.q[1];
        h.m[0] = h.m[2];
        h.m[1] = h.m[3];
        h.q[1] = -1;
    } else if (h.m[0] == one && h.m[2] == one) {  // only bit q0 = 1 changes: diagonal (d1, d3) on q1
        h.ctrl |= 1ull << h.q[0];
        h.m[0] = h.m[1];
        h.m[1] = h.m[3];
        h.q[0] = h.q[1];
        h.q[1] = -1;
    }
    return h;
}

}  // namespace qv
