// Planner: turns an ordered gate list into passes over the state.
//
// A block pass stages blocks of 2^b amplitudes on chip and applies a run of
// gates to them in one HBM round trip. The paper's block storage keeps B
// consecutive amplitudes together (Sec. III.C Eq. 7-8), which holds every
// pair (i, i ^ 2^k) for 2^k < B (the index-aligned partition of Sec. III.E);
// here a block is the set of indices that agree outside a chosen set S of b
// qubits, so S may hold high qubits too, and every pair or quadruple of a
// gate whose qubits lie in S is inside one block. The lowest `coalesce`
// qubits always belong to S, which keeps each block a union of contiguous
// runs in memory. Diagonal gates need no qubit in S (each amplitude's phase
// follows from its global index), nor do controls (a control outside S is
// constant over a block).
//
// Gates are taken greedily in order. A gate may move ahead of an earlier
// gate left for a later pass only when the two commute for certain: on each
// shared qubit both act diagonally (diagonal gates, controls, Z generators).
// So the pass result equals applying the gates one by one (Sec. III.E: one
// traversal for a batch of gates, same result as gate by gate).
#include <algorithm>
#include <functional>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <stdexcept>
#include <utility>

#include "gates.h"
#include "qv_internal.h"

namespace qv {

int default_block_qubits(int n, int elem_bytes, int n_states)
{
    // 2^12 amplitudes per block: a 32 KiB exchange buffer (complex128
    // exchanges real and imaginary parts in turn), three workgroups per CU
    // for complex128 (168 VGPRs), four for complex64 (four waves per SIMD).
    // Measured on MI355X, occupancy beats the fewer passes of larger blocks.
    // The adjoint carries two states and halves the complex128 block.
    const int lb = n_states == 2 ? (elem_bytes == 16 ? 11 : 12) : 12;
    return std::min(n, lb);
}

int reg_bits_for(int elem_bytes, int n_states) { return n_states == 2 ? 3 : 4; }

namespace {

int popc(uint64_t v) { return __builtin_popcountll(v); }

struct ItemBits {
    uint64_t dense;  // qubits acted on non-diagonally (must be local)
    uint64_t diag;   // qubits acted on diagonally (may be outside the block)
    uint64_t want;   // qubits that need not be local but let the gate fuse when they are
    int n_ops;
};

ItemBits bits_of(const PlanItem& it)
{
    ItemBits b{0, 0, 0, 0};
    if (it.gate) {
        b = ItemBits{dense_bits(it.g), diag_bits(it.g), 0, 1};
        if (it.g.kind == G_DENSE1 && it.g.ctrl && !(it.g.ctrl & (it.g.ctrl - 1))) b.want = it.g.ctrl;
        if (it.g.kind == G_DIAG && it.g.q[1] >= 0 && !it.g.ctrl) b.want = (1ull << it.g.q[0]) | (1ull << it.g.q[1]);
    }
    if (it.grad) {
        b.n_ops++;
        if (it.g.gen == GEN_Z) b.diag |= 1ull << it.g.q[0];
        else b.dense |= 1ull << it.g.q[0];
    }
    return b;
}

// Read + write of the amplitudes a sweep touches: all of them, except the
// subspace its controls exclude.
double sweep_bytes(const HostGate& g, int n, int elem)
{
    return 2.0 * std::ldexp(1.0, n - popc(g.ctrl)) * elem;
}

bool is_pauli_x(const HostGate& g)
{
    return g.m[0] == 0.0 && g.m[1] == 1.0 && g.m[2] == 1.0 && g.m[3] == 0.0;
}

bool is_swap(const HostGate& g)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            const bool one = (r == 0 && c == 0) || (r == 3 && c == 3) || (r == 1 && c == 2) || (r == 2 && c == 1);
            if (g.m[4 * r + c] != (one ? 1.0 : 0.0)) return false;
        }
    return true;
}

// Local positions an op acts on non-diagonally / diagonally.
void op_positions(const TileOp& t, uint32_t* dense, uint32_t* diag)
{
    *dense = 0;
    *diag = t.lctrl;
    switch (t.kind) {
    case T_DENSE1:
    case T_XPERM: *dense = 1u << t.a; break;
    case T_DENSE2:
    case T_SWAP: *dense = (1u << t.a) | (1u << t.c); break;
    case T_DIAG:
        if (t.a >= 0) *diag |= 1u << t.a;
        if (t.c >= 0) *diag |= 1u << t.c;
        break;
    case T_GRAD:
        if (t.gen == GEN_Z) {
            if (t.a >= 0) *diag |= 1u << t.a;
        } else {
            *dense = 1u << t.a;
        }
        break;
    default: break;
    }
}

int window_index(const StageHdr& st, int r, int pos)
{
    for (int j = 0; j < r; j++)
        if (st.w[j] == pos) return j;
    return -1;
}

// Split a block pass into register stages. Each stage holds a window of r
// local positions in every thread's registers; the ops of the stage act
// densely only inside the window (diagonal ops and controls may use any
// position). Ops move between stages only past ops they commute with, by the
// same rule as gates between passes.
//
// Thread bits map to the positions outside the window: the low ones (lanes
// of a wave) to the lowest free positions, the top ones (which wave of the
// workgroup) to a set P of wave positions. While P stays out of the windows,
// a window change only moves amplitudes between lanes of one wave, and the
// exchange needs no workgroup barrier. P is chosen among the positions the
// pass's ops use least, windows avoid it while they can, and it moves
// (with a workgroup-wide exchange) only when an op needs one of its bits.
// The first window is the load window (top positions outside P), and
// leftover window slots are filled towards it so that the last stage often
// needs no exchange before the store.
void set_mapping(StageHdr& st, int b, uint32_t W, uint32_t P, int r, int slot_bytes)
{
    int j = 0;
    for (int p = 0; p < b; p++)
        if (W & (1u << p)) st.w[j++] = p;
    st.wmask = W;
    int i = 0;
    for (int p = 0; p < b; p++)
        if (!(W & (1u << p)) && !(P & (1u << p))) st.tpos[i++] = p;
    for (int p = 0; p < b; p++)
        if (P & (1u << p)) st.tpos[i++] = p;
    // exchange-buffer byte offsets of the registers' window bits
    for (int k = 0; k < (1 << r); k++) {
        uint32_t l = 0;
        for (int jj = 0; jj < r; jj++)
            if ((k >> jj) & 1) l |= 1u << st.w[jj];
        st.woff[k] = lds_slot(l, slot_bytes == 16 ? 4 : 5) * (uint32_t)slot_bytes;
    }
}

// `avoid`: positions kept off the wave bits while others are free (those
// whose lanes make contiguous runs at the load or at the store).
uint32_t pick_wave_positions(const std::vector<int>& use, int b, int wb, uint32_t exclude, uint32_t prefer,
                             uint32_t avoid)
{
    uint32_t P = 0;
    for (int k = 0; k < wb; k++) {
        int best = -1;
        for (int p = b - 1; p >= 0; p--) {
            if ((exclude | P) & (1u << p)) continue;
            if (best < 0) { best = p; continue; }
            const bool pp = prefer & (1u << p), pb = prefer & (1u << best);
            const bool low_p = (avoid >> p) & 1u, low_b = (avoid >> best) & 1u;  // keep the run qubits on lanes
            if (low_p != low_b) { if (low_b) best = p; continue; }
            if (use[p] < use[best] || (use[p] == use[best] && pp && !pb)) best = p;
        }
        if (best < 0) break;
        P |= 1u << best;
    }
    return P;
}

// store_first (may be null): the local positions whose bits the store writes
// to the block's lowest qubits, lowest first; null when the store writes each
// position to the qubit it was loaded from (then they are positions 0..).
void plan_stages(PlanPass& pp, int b, int r, int wave_mode, int elem, int xelem, const int* store_first,
                 uint32_t moved_mask)
{
    const int tb = b - r;
    // lanes 0..coal-1 on the lowest positions make each load/store
    // instruction a set of whole 128-byte runs
    const int coal = elem == 16 ? 3 : 4;
    const uint32_t coal_mask = (1u << coal) - 1;
    int sfirst[8];
    uint32_t store_mask = 0;
    bool store_ident = true;
    for (int i = 0; i < coal; i++) {
        sfirst[i] = store_first ? store_first[i] : i;
        store_mask |= 1u << sfirst[i];
        store_ident = store_ident && sfirst[i] == i;
    }
    const uint32_t avoid = coal_mask | store_mask | moved_mask;
    const int wb = (tb > 6 && wave_mode > 0) ? tb - 6 : 0;
    const bool wave_ok = tb <= 6 || wb > 0;  // one wave per block, or wave positions kept apart
    std::vector<TileOp>& ops = pp.ops;
    std::vector<uint32_t> dn(ops.size()), dg(ops.size());
    for (size_t i = 0; i < ops.size(); i++) op_positions(ops[i], &dn[i], &dg[i]);
    std::vector<int> use(b, 0);
    for (size_t i = 0; i < ops.size(); i++)
        for (int p = 0; p < b; p++) use[p] += (dn[i] >> p) & 1;

    // load/store mapping: the default wave bits sit just above the lanes
    const uint32_t default_P = wb ? (((1u << wb) - 1) << (tb - wb)) : 0;
    uint32_t P = wave_mode == 2 ? pick_wave_positions(use, b, wb, 0, default_P, avoid) : default_P;
    uint32_t natural = 0;
    for (int p = b - 1, c = 0; p >= 0 && c < r; p--)
        if (!(P & (1u << p))) {
            natural |= 1u << p;
            c++;
        }
    set_mapping(pp.hdr.nat, b, natural, P, r, xelem);
    pp.hdr.nat.wave_local = XCH_NONE;
    const uint32_t P_nat = P;

    std::vector<char> done(ops.size(), 0);
    std::vector<TileOp> out;
    out.reserve(ops.size());
    pp.stages.clear();
    size_t first = 0;
    uint32_t prev_W = natural;
    std::vector<uint32_t> stage_P;
    while (true) {
        while (first < ops.size() && done[first]) first++;
        if (first >= ops.size()) break;
        uint32_t W = 0;
        uint32_t bd = 0, bg = 0;
        std::vector<size_t> taken;
        for (size_t i = first; i < ops.size(); i++) {
            if (done[i]) continue;
            bool ok = !(dn[i] & (bd | bg)) && !(dg[i] & bd);
            if (ok) {
                const uint32_t need = dn[i] & ~W;
                // a wave position joins the window only for the stage's first op
                if (popc(W | need) > r || ((need & P) && !taken.empty())) ok = false;
                else W |= need;
            }
            if (ok) {
                taken.push_back(i);
            } else {
                bd |= dn[i];
                bg |= dg[i];
            }
        }
        if (taken.empty()) throw std::runtime_error("stage planner made no progress");
        for (size_t i : taken)
            for (int p = 0; p < b; p++) use[p] -= (dn[i] >> p) & 1;
        // leftover window slots: controls of the stage's CNOTs first (a CNOT
        // whose control is in the window is a plain register swap), then the
        // load/store window, never a wave position
        for (size_t i : taken) {
            const TileOp& t = ops[i];
            if (t.kind == T_XPERM && t.lctrl && !(t.lctrl & (t.lctrl - 1)) && popc(W) < r && !(t.lctrl & P))
                W |= t.lctrl;
        }
        for (int p = b - 1; p >= 0 && popc(W) < r; p--)
            if ((natural & (1u << p)) && !(P & (1u << p))) W |= 1u << p;
        for (int p = 0; p < b && popc(W) < r; p++)
            if (!(P & (1u << p))) W |= 1u << p;
        for (int p = 0; p < b && popc(W) < r; p++) W |= 1u << p;
        StageHdr st{};
        const uint32_t P_prev = P, W_prev = prev_W;
        if (W & P) P = pick_wave_positions(use, b, wb, W, P_nat, avoid);  // an op needs a wave position
        set_mapping(st, b, W, P, r, xelem);
        // exchange into this mapping: none if it is unchanged, within waves
        // if the wave positions stay, else across the workgroup
        st.wave_local = (W == W_prev && P == P_prev) ? XCH_NONE : (P == P_prev && wave_ok ? XCH_WAVE : XCH_BLOCK);
        prev_W = W;
        stage_P.push_back(P);
        st.op_begin = (int32_t)out.size();
        st.n_ops = (int32_t)taken.size();
        for (size_t i : taken) {
            done[i] = 1;
            TileOp t = ops[i];
            if (t.kind == T_XPERM && t.lctrl && !(t.lctrl & (t.lctrl - 1))) t.c = __builtin_ctz(t.lctrl);
            t.j0 = t.a >= 0 ? window_index(st, r, t.a) : -1;
            t.j1 = t.c >= 0 ? window_index(st, r, t.c) : -1;
            const bool two = t.kind == T_DENSE2 || t.kind == T_SWAP;
            if (two && t.j0 > t.j1) {
                // order the pair by window bit: swap the roles of a and c, which
                // exchanges matrix rows/columns 1 and 2 (index bit(a) + 2 bit(c))
                std::swap(t.a, t.c);
                std::swap(t.j0, t.j1);
                if (t.kind == T_DENSE2) {
                    cd* m = &pp.mats[t.mat];
                    cd tmp[16];
                    const int perm[4] = {0, 2, 1, 3};
                    for (int rr = 0; rr < 4; rr++)
                        for (int cc = 0; cc < 4; cc++) tmp[4 * rr + cc] = m[4 * perm[rr] + perm[cc]];
                    for (int e = 0; e < 16; e++) m[e] = tmp[e];
                }
            }
            out.push_back(t);
        }
        pp.stages.push_back(st);
    }
    // Load straight into the first stage's mapping, and store straight from
    // the last one, when its lanes keep the 128-byte runs together;
    // otherwise through the natural mapping.
    auto whole_runs = [&](const StageHdr& m, const int* first) {
        for (int i = 0; i < coal; i++)
            if (m.tpos[i] != first[i]) return false;
        return true;
    };
    const int ident[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    uint32_t P_load = P_nat;
    if (!pp.stages.empty() && whole_runs(pp.stages.front(), ident)) {
        pp.hdr.nat = pp.stages.front();
        pp.stages.front().wave_local = XCH_NONE;
        P_load = stage_P.front();
    }
    pp.hdr.nat.wave_local = XCH_NONE;
    if (!pp.stages.empty() && whole_runs(pp.stages.back(), sfirst)) {
        pp.hdr.out = pp.stages.back();
        pp.hdr.final_wave_local = XCH_NONE;
    } else if (store_ident) {
        pp.hdr.out = pp.hdr.nat;
        const bool same = pp.stages.empty() || (prev_W == pp.hdr.nat.wmask && P == P_load);
        pp.hdr.final_wave_local = same ? XCH_NONE : (P == P_load && wave_ok ? XCH_WAVE : XCH_BLOCK);
    } else {
        // A store that moves qubits: lanes 0..coal-1 on the positions written
        // to the lowest qubits, the window on the top positions left over.
        const uint32_t P_cur = pp.stages.empty() ? P_load : P;
        const uint32_t P_st = (P_cur & store_mask) ? pick_wave_positions(use, b, wb, store_mask, P_cur, avoid) : P_cur;
        uint32_t W_st = 0;
        for (int p = b - 1, c = 0; p >= 0 && c < r; p--)
            if (!((P_st | store_mask) & (1u << p))) {
                W_st |= 1u << p;
                c++;
            }
        StageHdr& o = pp.hdr.out;
        o = StageHdr{};
        set_mapping(o, b, W_st, P_st, r, xelem);
        // lanes first: the run positions in store order, then the other free positions
        int i = 0;
        for (int k = 0; k < coal; k++) o.tpos[i++] = sfirst[k];
        for (int p = 0; p < b; p++)
            if (!((W_st | P_st | store_mask) & (1u << p))) o.tpos[i++] = p;
        for (int p = 0; p < b; p++)
            if (P_st & (1u << p)) o.tpos[i++] = p;
        if (i != tb) throw std::runtime_error("store mapping does not cover the thread bits");
        const StageHdr& last = pp.stages.empty() ? pp.hdr.nat : pp.stages.back();
        bool same = last.wmask == o.wmask;
        for (int k = 0; k < tb && same; k++) same = last.tpos[k] == o.tpos[k];
        pp.hdr.final_wave_local = same ? XCH_NONE : (P_st == P_cur && wave_ok ? XCH_WAVE : XCH_BLOCK);
    }
    // A store that moves qubits writes an amplitude to another address of the
    // block than the one it was loaded from. Without a workgroup-wide exchange
    // in the pass each wave keeps its amplitudes from load to store, and its
    // stores stay on the addresses it loaded only if the moved positions
    // avoid the wave positions; otherwise a wave could overwrite what another
    // wave has not loaded yet, and the final exchange becomes workgroup-wide
    // (its barrier separates every wave's loads from every wave's stores).
    if (store_first) {
        bool barrier = pp.hdr.final_wave_local == XCH_BLOCK;
        for (const StageHdr& st : pp.stages) barrier = barrier || st.wave_local == XCH_BLOCK;
        uint32_t wave_pos = 0;
        for (int i = 6; i < tb; i++) wave_pos |= 1u << pp.hdr.out.tpos[i];
        if (!barrier && (moved_mask & wave_pos)) pp.hdr.final_wave_local = XCH_BLOCK;
    }
    pp.hdr.out.wave_local = XCH_NONE;
    (void)coal_mask;
    ops.swap(out);
    pp.hdr.n_stages = (int32_t)pp.stages.size();
}

// Global qubit of each thread bit and element offset of each register in
// the load and store mappings, so that the kernel forms its addresses
// without looking up local positions.
// store_q (may be null): the qubit each local position is written to (a
// permutation of local_q); null: the qubit it was loaded from.
void set_io_offsets(PassHdr& h, int r, const int32_t* store_q)
{
    const int tb = h.b - r;
    auto fill = [&](const StageHdr& m, const int32_t* q_of, int32_t* tq, uint64_t* koff) {
        for (int i = 0; i < kMaxThreadBits; i++) tq[i] = i < tb ? q_of[m.tpos[i]] : 0;
        for (int k = 0; k < (1 << kMaxRegBits); k++) {
            uint64_t o = 0;
            if (k < (1 << r))
                for (int j = 0; j < r; j++)
                    if ((k >> j) & 1) o |= 1ull << q_of[m.w[j]];
            koff[k] = o;
        }
    };
    fill(h.nat, h.local_q, h.nat_tq, h.nat_koff);
    fill(h.out, store_q ? store_q : h.local_q, h.out_tq, h.out_koff);
}

// Flat dispatch code of an op for the register kernel (after stages and
// diagonal merging).
int32_t reg_code(const TileOp& t, bool mfma)
{
    const bool ctrl = t.lctrl != 0;
    switch (t.kind) {
    case T_DENSE1: return (ctrl ? RC_D1C : RC_D1) + t.j0;
    case T_XPERM:
        if (t.j1 >= 0 && t.c >= 0 && t.lctrl == (1u << t.c)) return RC_CX + 5 * t.j0 + t.j1;
        return (ctrl ? RC_XC : RC_X) + t.j0;
    case T_DENSE2: return (ctrl ? RC_D2C : (mfma ? RC_D2M : RC_D2)) + 5 * t.j0 + t.j1;
    case T_SWAP: return (ctrl ? RC_SWC : RC_SW) + 5 * t.j0 + t.j1;
    case T_DIAG: return RC_DIAG;
    case T_PHASE: return RC_PHASE;
    case T_GRAD: return t.gen == GEN_Z ? RC_GZ : RC_GXY + t.j0;
    case T_GRADZ: return RC_GZM;
    case T_SIGN: return RC_SIGN;
    default: return RC_NONE;
    }
}

// A diagonal whose entries are all 1 except a -1 on the all-ones corner (CZ,
// Z, and their controlled forms) multiplies the amplitudes whose bits at its
// qubits (and controls) are all 1 by -1: a sign flip of those amplitudes,
// with the qubits joining the controls. The register kernel selects them as
// it selects the registers of a controlled op and flips their sign bits,
// which is exact, instead of a complex product per amplitude.
void diag_to_sign(PlanPass& pp)
{
    for (TileOp& t : pp.ops) {
        if (t.kind != T_DIAG) continue;
        const cd* d = &pp.mats[t.mat];
        const bool one_q = t.c < 0 && t.oc < 0;
        const bool sign = one_q ? (d[0] == 1.0 && d[1] == -1.0)
                                : (d[0] == 1.0 && d[1] == 1.0 && d[2] == 1.0 && d[3] == -1.0);
        if (!sign) continue;
        if (t.a >= 0) t.lctrl |= 1u << t.a;
        else if (t.oa >= 0) t.gctrl |= 1ull << t.oa;
        if (t.c >= 0) t.lctrl |= 1u << t.c;
        else if (t.oc >= 0) t.gctrl |= 1ull << t.oc;
        t.kind = T_SIGN;
        t.a = t.c = t.oa = t.oc = -1;
        t.j0 = t.j1 = -1;
    }
}

void set_reg_codes(PlanPass& pp, int r, bool mfma)
{
    for (TileOp& t : pp.ops) {
        t.code = reg_code(t, mfma);
        t.tctrl = 0;
        t.kmask = (1u << r) - 1;
    }
    // local controls split into the thread's part and a register mask
    for (const StageHdr& st : pp.stages) {
        for (int o = st.op_begin; o < st.op_begin + st.n_ops; o++) {
            TileOp& t = pp.ops[o];
            const uint32_t wc = t.lctrl & st.wmask;
            t.tctrl = t.lctrl & ~st.wmask;
            uint32_t km = 0;
            for (int k = 0; k < (1 << r); k++) {
                uint32_t l = 0;
                for (int j = 0; j < r; j++)
                    if ((k >> j) & 1) l |= 1u << st.w[j];
                if ((l & wc) == wc) km |= 1u << k;
            }
            t.kmask = km;
        }
    }
}

// Register permutations (X on a window bit, with or without controls, and
// CNOT within the window) only change which register holds which local
// index. When no later op of the stage touches their positions and an
// exchange follows (the next stage's, or the final one before the store),
// the kernel leaves the values where they are and moves the exchange-buffer
// offsets instead: the slot map is linear over XOR, so a register now
// holding index l ^ 2^a takes the offset of its old one XOR the uniform term
// slot(2^a) (times the slot size), for the registers the op moves (kmask:
// those whose window bits meet its controls inside the window) in the
// threads and blocks that meet its other controls (tctrl, gctrl). Such ops
// are kept after a stage's n_ops as its n_exit ops, with that term in aux.
// Their targets are window bits, so the values stay in their thread (and
// wave: after a within-wave exchange, other waves may still be reading the
// slots of their own indices).
void fold_trailing_perms(PlanPass& pp, int r, int slot_bytes)
{
    const int e = slot_bytes == 16 ? 4 : 5;
    auto positions = [](const TileOp& t) {
        uint32_t mine = ~0u;  // phases, reads and the rest: every position
        if (t.kind == T_DENSE1 || t.kind == T_XPERM || t.kind == T_DENSE2 || t.kind == T_SWAP || t.kind == T_DIAG ||
            t.kind == T_SIGN || (t.kind == T_GRAD && t.gen == GEN_Z)) {
            uint32_t dense, diag;
            op_positions(t, &dense, &diag);
            mine = dense | diag;
        }
        return mine;
    };
    auto is_perm = [](const TileOp& t) {
        return t.kind == T_XPERM && ((t.code >= RC_X && t.code < RC_X + kMaxRegBits + 1) ||
                                     (t.code >= RC_XC && t.code < RC_XC + kMaxRegBits + 1) ||
                                     (t.code >= RC_CX && t.code < RC_CX + 25));
    };
    // the op as an exit of a stage whose mapping is m
    auto make_exit = [&](TileOp t, const StageHdr& m) {
        const uint32_t wc = t.lctrl & m.wmask;
        t.tctrl = t.lctrl & ~m.wmask;
        uint32_t fm = 0;
        for (int k = 0; k < (1 << r); k++) {
            uint32_t l = 0;
            for (int j = 0; j < r; j++)
                if ((k >> j) & 1) l |= 1u << m.w[j];
            if ((l & wc) == wc) fm |= 1u << k;
        }
        t.kmask = fm;
        t.aux = (int32_t)(lds_slot(1u << t.a, e) * (uint32_t)slot_bytes);
        return t;
    };
    std::vector<const StageHdr*> eff(pp.stages.size());  // mapping in effect during each stage
    const StageHdr* cur = &pp.hdr.nat;
    for (size_t si = 0; si < pp.stages.size(); si++) {
        if (pp.stages[si].wave_local != XCH_NONE) cur = &pp.stages[si];
        eff[si] = cur;
    }
    for (size_t si = 0; si < pp.stages.size(); si++) {
        StageHdr& st = pp.stages[si];
        st.n_exit = 0;
        const bool xch_next = si + 1 < pp.stages.size() ? pp.stages[si + 1].wave_local != XCH_NONE
                                                        : pp.hdr.final_wave_local != XCH_NONE;
        if (!xch_next || st.n_ops == 0) continue;
        std::vector<TileOp> keep, exits;
        uint32_t later = 0;
        for (int o = st.op_begin + st.n_ops - 1; o >= st.op_begin; o--) {
            const TileOp& t = pp.ops[o];
            const uint32_t mine = positions(t);
            if (is_perm(t) && !(mine & later)) {
                exits.push_back(make_exit(t, *eff[si]));
            } else {
                keep.push_back(t);
            }
            later |= mine;
        }
        if (exits.empty()) continue;
        int o = st.op_begin;
        for (auto it = keep.rbegin(); it != keep.rend(); ++it) pp.ops[o++] = *it;
        for (auto it = exits.rbegin(); it != exits.rend(); ++it) pp.ops[o++] = *it;
        st.n_ops = (int32_t)keep.size();
        st.n_exit = (int32_t)exits.size();
    }
}

// ------------------------------------------------------------ fusion ---
// Inside one block pass, one-qubit gates are folded into neighbouring
// two-qubit gates when that saves work: a 4x4 update of a quadruple costs
// about as much as two 2x2 updates of its pairs, so a two-qubit gate that
// swallows the one-qubit gates before and after it on both of its qubits
// replaces up to four pair sweeps and itself. A two-qubit gate with no
// pending one-qubit work stays as it is (a CNOT is then a register swap, a
// CZ a diagonal). The products are formed on the host in FP64; the result
// equals the gate-by-gate product (Sec. III.A Eq. 5 applied in sequence).

using M2 = std::array<cd, 4>;
using M4 = std::array<cd, 16>;

M2 m2_ident() { return {cd(1), cd(0), cd(0), cd(1)}; }

M2 m2_mul(const M2& A, const M2& B)
{
    M2 r;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) r[2 * i + j] = A[2 * i] * B[j] + A[2 * i + 1] * B[2 + j];
    return r;
}

M4 m4_mul(const M4& A, const M4& B)
{
    M4 r;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cd t = 0;
            for (int k = 0; k < 4; k++) t += A[4 * i + k] * B[4 * k + j];
            r[4 * i + j] = t;
        }
    return r;
}

// u acting on the first (role 0) or second (role 1) qubit of a pair, in the
// pair basis m = bit(first) + 2 bit(second).
M4 m4_embed(const M2& u, int role)
{
    M4 r{};
    for (int mo = 0; mo < 4; mo++)
        for (int mi = 0; mi < 4; mi++) {
            const int xo = role == 0 ? (mo & 1) : (mo >> 1), xi = role == 0 ? (mi & 1) : (mi >> 1);
            const int yo = role == 0 ? (mo >> 1) : (mo & 1), yi = role == 0 ? (mi >> 1) : (mi & 1);
            r[4 * mo + mi] = yo == yi ? u[2 * xo + xi] : cd(0);
        }
    return r;
}

// Exchange the two qubits of the basis (matrix on (q, p) -> on (p, q)).
M4 m4_swap_roles(const M4& g)
{
    static const int perm[4] = {0, 2, 1, 3};
    M4 r;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) r[4 * i + j] = g[4 * perm[i] + perm[j]];
    return r;
}

bool m2_is_diag(const M2& u) { return u[1] == 0.0 && u[2] == 0.0; }

void fuse_ops(PlanPass& pp)
{
    const std::vector<TileOp> in = pp.ops;
    std::vector<TileOp> out;
    std::vector<M4> fused;          // matrices of fused DENSE2 ops, by out index
    std::vector<int> fused_of;      // out index -> fused slot (-1: keep op's own matrix)
    M2 pend[kMaxLocal];
    bool has_pend[kMaxLocal];
    int open[kMaxLocal];            // out index of a fused op that may absorb gates on this position
    int role[kMaxLocal];
    for (int p = 0; p < kMaxLocal; p++) {
        pend[p] = m2_ident();
        has_pend[p] = false;
        open[p] = -1;
        role[p] = 0;
    }
    auto push = [&](const TileOp& t) {
        out.push_back(t);
        fused_of.push_back(-1);
    };
    auto flush = [&](int p) {
        if (!has_pend[p]) return;
        const M2& u = pend[p];
        TileOp t{};
        t.a = p;
        t.c = t.oa = t.oc = -1;
        t.j0 = t.j1 = -1;
        t.gen = GEN_NONE;
        t.slot = -1;
        t.mat = (int32_t)pp.mats.size();
        if (m2_is_diag(u)) {
            t.kind = T_DIAG;
            pp.mats.insert(pp.mats.end(), {u[0], u[3], u[0], u[3]});
        } else {
            t.kind = (u[0] == 0.0 && u[1] == 1.0 && u[2] == 1.0 && u[3] == 0.0) ? T_XPERM : T_DENSE1;
            pp.mats.insert(pp.mats.end(), u.begin(), u.end());
        }
        push(t);
        has_pend[p] = false;
        pend[p] = m2_ident();
    };
    auto barrier = [&](uint32_t mask) {
        for (int p = 0; p < kMaxLocal; p++)
            if (mask & (1u << p)) {
                flush(p);
                open[p] = -1;
            }
    };
    auto one_qubit = [&](int p, const M2& u) {
        if (open[p] >= 0) {
            M4& m = fused[fused_of[open[p]]];
            m = m4_mul(m4_embed(u, role[p]), m);
        } else {
            pend[p] = m2_mul(u, pend[p]);
            has_pend[p] = true;
        }
    };
    // g: matrix on (p, q) in the basis bit(p) + 2 bit(q); bare: the op to emit unfused
    auto two_qubit = [&](int p, int q, const M4& g, const TileOp& bare, bool bare_is_dense2) {
        if (open[p] >= 0 && open[p] == open[q]) {
            const int idx = open[p];
            M4& m = fused[fused_of[idx]];
            m = m4_mul(role[p] == 0 ? g : m4_swap_roles(g), m);
            return;
        }
        open[p] = open[q] = -1;
        const bool dense_pending = (has_pend[p] && !m2_is_diag(pend[p])) || (has_pend[q] && !m2_is_diag(pend[q]));
        if (!dense_pending && !bare_is_dense2) {
            flush(p);
            flush(q);
            push(bare);
            return;
        }
        M4 m = m4_mul(g, m4_mul(m4_embed(pend[p], 0), m4_embed(pend[q], 1)));
        has_pend[p] = has_pend[q] = false;
        pend[p] = pend[q] = m2_ident();
        TileOp t{};
        t.kind = T_DENSE2;
        t.a = p;
        t.c = q;
        t.oa = t.oc = -1;
        t.j0 = t.j1 = -1;
        t.gen = GEN_NONE;
        t.slot = -1;
        out.push_back(t);
        fused_of.push_back((int)fused.size());
        fused.push_back(m);
        open[p] = open[q] = (int)out.size() - 1;
        role[p] = 0;
        role[q] = 1;
    };

    for (const TileOp& t : in) {
        const cd* mt = pp.mats.data() + t.mat;
        const bool plain = t.lctrl == 0 && t.gctrl == 0;
        if (t.kind == T_DENSE1 && plain) {
            one_qubit(t.a, {mt[0], mt[1], mt[2], mt[3]});
        } else if (t.kind == T_XPERM && plain) {
            one_qubit(t.a, {cd(0), cd(1), cd(1), cd(0)});
        } else if (t.kind == T_DIAG && plain && t.a >= 0 && t.c < 0 && t.oc < 0) {
            one_qubit(t.a, {mt[0], cd(0), cd(0), mt[1]});
        } else if (t.kind == T_DIAG && plain && t.a >= 0 && t.c >= 0) {
            M4 g{};
            for (int e = 0; e < 4; e++) g[5 * e] = mt[e];
            two_qubit(t.a, t.c, g, t, false);
        } else if (t.kind == T_XPERM && t.gctrl == 0 && t.lctrl && !(t.lctrl & (t.lctrl - 1))) {
            // CNOT with a local control: X on a where bit c is 1, basis bit(a) + 2 bit(c)
            const int c = __builtin_ctz(t.lctrl);
            M4 g{};
            g[0] = g[5] = 1.0;
            g[4 * 2 + 3] = g[4 * 3 + 2] = 1.0;
            two_qubit(t.a, c, g, t, false);
        } else if ((t.kind == T_DENSE2 || t.kind == T_SWAP) && plain) {
            M4 g{};
            for (int e = 0; e < 16; e++) g[e] = mt[e];
            two_qubit(t.a, t.c, g, t, t.kind == T_DENSE2);
        } else {
            uint32_t mask = t.lctrl;
            if (t.a >= 0) mask |= 1u << t.a;
            if (t.c >= 0) mask |= 1u << t.c;
            barrier(mask);
            push(t);
        }
    }
    for (int p = 0; p < kMaxLocal; p++) flush(p);
    for (size_t i = 0; i < out.size(); i++) {
        if (fused_of[i] < 0) continue;
        out[i].mat = (int32_t)pp.mats.size();
        const M4& m = fused[fused_of[i]];
        pp.mats.insert(pp.mats.end(), m.begin(), m.end());
    }
    pp.ops.swap(out);
    pp.hdr.n_ops = (int32_t)pp.ops.size();
}

// Whole-circuit version of the same fusion, on global qubits, before the
// passes are formed: a two-qubit gate with one-qubit work pending on its
// qubits becomes a 4x4 that also takes the one-qubit gates that follow it
// (until another gate touches the qubit). In layered circuits this makes
// every other layer of two-qubit gates absorb the one-qubit gates on both
// sides, and leaves the layers in between as plain CNOTs / CZs.
std::vector<HostGate> prefuse_gates(const std::vector<HostGate>& in)
{
    std::vector<HostGate> out;
    std::vector<int> open(kMaxQubits + 1, -1), role(kMaxQubits + 1, 0);
    std::vector<M2> pend(kMaxQubits + 1, m2_ident());
    std::vector<char> has_pend(kMaxQubits + 1, 0);
    auto emit_pending = [&](int q) {
        if (!has_pend[q]) return;
        HostGate g;
        const M2& u = pend[q];
        g.q[0] = q;
        if (m2_is_diag(u)) {
            g.kind = G_DIAG;
            g.m[0] = u[0];
            g.m[1] = u[3];
            g.m[2] = u[0];
            g.m[3] = u[3];
        } else {
            g.kind = G_DENSE1;
            for (int e = 0; e < 4; e++) g.m[e] = u[e];
        }
        out.push_back(g);
        has_pend[q] = 0;
        pend[q] = m2_ident();
    };
    auto barrier = [&](uint64_t mask) {
        for (int q = 0; q < kMaxQubits; q++)
            if (mask & (1ull << q)) {
                emit_pending(q);
                open[q] = -1;
            }
    };
    auto m4_of = [&](int idx) {
        M4 m;
        for (int e = 0; e < 16; e++) m[e] = out[idx].m[e];
        return m;
    };
    auto set_m4 = [&](int idx, const M4& m) {
        for (int e = 0; e < 16; e++) out[idx].m[e] = m[e];
    };
    for (const HostGate& g : in) {
        const bool one_q = (g.kind == G_DENSE1 && !g.ctrl) || (g.kind == G_DIAG && !g.ctrl && g.q[1] < 0);
        if (one_q) {
            const int q = g.q[0];
            const M2 u = g.kind == G_DENSE1 ? M2{g.m[0], g.m[1], g.m[2], g.m[3]} : M2{g.m[0], cd(0), cd(0), g.m[1]};
            if (open[q] >= 0) {
                set_m4(open[q], m4_mul(m4_embed(u, role[q]), m4_of(open[q])));
            } else {
                pend[q] = m2_mul(u, pend[q]);
                has_pend[q] = 1;
            }
            continue;
        }
        // two-qubit forms: CNOT (one control), CZ/CP (two-qubit diagonal), 4x4
        int p = -1, q = -1;
        M4 gm{};
        if (g.kind == G_DENSE1 && g.ctrl && !(g.ctrl & (g.ctrl - 1))) {
            p = g.q[0];
            q = __builtin_ctzll(g.ctrl);
            // X (or any 2x2) on p where bit q is 1, basis bit(p) + 2 bit(q)
            gm[0] = gm[5] = 1.0;
            gm[4 * 2 + 2] = g.m[0];
            gm[4 * 2 + 3] = g.m[1];
            gm[4 * 3 + 2] = g.m[2];
            gm[4 * 3 + 3] = g.m[3];
        } else if (g.kind == G_DIAG && !g.ctrl && g.q[1] >= 0) {
            p = g.q[0];
            q = g.q[1];
            for (int e = 0; e < 4; e++) gm[5 * e] = g.m[e];
        } else if (g.kind == G_DENSE2 && !g.ctrl) {
            p = g.q[0];
            q = g.q[1];
            for (int e = 0; e < 16; e++) gm[e] = g.m[e];
        } else {
            barrier(dense_bits(g) | diag_bits(g));
            out.push_back(g);
            continue;
        }
        if (open[p] >= 0 && open[p] == open[q]) {
            const int idx = open[p];
            set_m4(idx, m4_mul(role[p] == 0 ? gm : m4_swap_roles(gm), m4_of(idx)));
            continue;
        }
        open[p] = open[q] = -1;
        const bool dense_pending = (has_pend[p] && !m2_is_diag(pend[p])) || (has_pend[q] && !m2_is_diag(pend[q]));
        if (!dense_pending && g.kind != G_DENSE2) {
            emit_pending(p);
            emit_pending(q);
            out.push_back(g);
            continue;
        }
        const M4 m = m4_mul(gm, m4_mul(m4_embed(pend[p], 0), m4_embed(pend[q], 1)));
        has_pend[p] = has_pend[q] = 0;
        pend[p] = pend[q] = m2_ident();
        HostGate f;
        f.kind = G_DENSE2;
        f.q[0] = p;
        f.q[1] = q;
        for (int e = 0; e < 16; e++) f.m[e] = m[e];
        out.push_back(f);
        open[p] = open[q] = (int)out.size() - 1;
        role[p] = 0;
        role[q] = 1;
    }
    for (int q = 0; q < kMaxQubits; q++) emit_pending(q);
    return out;
}

constexpr int kPhaseMinRun = 4;  // shorter runs of diagonal gates stay separate ops

bool mergeable_diag(const TileOp& t, const PlanPass& pp)
{
    if (t.kind != T_DIAG || t.lctrl != 0 || t.gctrl != 0) return false;
    for (int e = 0; e < 4; e++)
        if (std::abs(std::abs(pp.mats[t.mat + e]) - 1.0) > 1e-12) return false;
    return true;
}

uint32_t dense_positions(const TileOp& t)
{
    uint32_t dn, dg;
    op_positions(t, &dn, &dg);
    return dn;
}

uint32_t local_positions(const TileOp& t)
{
    uint32_t m = 0;
    if (t.a >= 0) m |= 1u << t.a;
    if (t.c >= 0) m |= 1u << t.c;
    return m;
}

// Phase polynomial of a run of diagonal gates for a stage's window. A
// diagonal d on bits (x, y) has phase angle a(x, y) = a00 + (a10 - a00) x +
// (a01 - a00) y + (a11 - a10 - a01 + a00) x y, which is exact on {0, 1}^2;
// the run's phase is the sum over its gates.
TileOp make_phase(const std::vector<TileOp>& run, const StageHdr& st, int r, PlanPass& pp)
{
    std::map<std::array<int32_t, 5>, double> acc;
    auto win = [&](int p) { return p < 64 ? window_index(st, r, p) : -1; };
    auto add_lin = [&](int p, double th) {
        const int j = win(p);
        if (j >= 0) acc[{PH_WLIN, j, -1, -1, -1}] += th;
        else acc[{PH_THREAD, -1, -1, p, -1}] += th;
    };
    auto add_quad = [&](int p, int q, double th) {
        int jp = win(p), jq = win(q);
        if (jp >= 0 && jq >= 0) {
            if (jp > jq) std::swap(jp, jq);
            acc[{PH_WQUAD, jp, jq, -1, -1}] += th;
        } else if (jp >= 0) {
            acc[{PH_MIXED, jp, -1, q, -1}] += th;
        } else if (jq >= 0) {
            acc[{PH_MIXED, jq, -1, p, -1}] += th;
        } else {
            acc[{PH_THREAD, -1, -1, std::min(p, q), std::max(p, q)}] += th;
        }
    };
    for (const TileOp& d : run) {
        double al[4];
        for (int e = 0; e < 4; e++) al[e] = std::arg(pp.mats[d.mat + e]) / (2.0 * M_PI);
        const int pa = d.a >= 0 ? d.a : 64 + d.oa;
        const bool two = d.c >= 0 || d.oc >= 0;
        acc[{PH_CONST, -1, -1, -1, -1}] += al[0];
        add_lin(pa, al[1] - al[0]);
        if (two) {
            const int pc = d.c >= 0 ? d.c : 64 + d.oc;
            add_lin(pc, al[2] - al[0]);
            add_quad(pa, pc, al[3] - al[2] - al[1] + al[0]);
        }
    }
    TileOp t{};
    t.kind = T_PHASE;
    t.a = t.c = t.oa = t.oc = -1;
    t.j0 = t.j1 = -1;
    t.gen = GEN_NONE;
    t.slot = -1;
    // window-only part (constant, window-linear, window-quadratic terms) as a
    // table of 2^r unit complex numbers, one per register
    std::vector<double> wang(1u << r, 0.0);
    // the rest as mask records: for A (target 0) and for each window bit's
    // coefficient (target 1 + j)
    std::vector<std::vector<PhaseTerm>> groups(r + 1);
    auto add_bit = [&](PhaseTerm& pt, int p) {
        if (p >= 64) {
            pt.omask |= 1ull << (p - 64);
            return;
        }
        for (int i = 0; i < pp.hdr.b - r; i++)
            if (st.tpos[i] == p) {
                pt.tmask |= 1u << i;
                return;
            }
        throw std::runtime_error("phase term on a position that is neither thread nor window");
    };
    for (const auto& kv : acc) {
        double th = kv.second - std::nearbyint(kv.second);  // angles are periodic in turns
        if (th == 0.0) continue;
        const int kind = kv.first[0];
        if (kind == PH_CONST || kind == PH_WLIN || kind == PH_WQUAD) {
            for (int k = 0; k < (1 << r); k++) {
                const bool on = kind == PH_CONST ||
                                (kind == PH_WLIN && ((k >> kv.first[1]) & 1)) ||
                                (kind == PH_WQUAD && ((k >> kv.first[1]) & 1) && ((k >> kv.first[2]) & 1));
                if (on) wang[k] += th;
            }
            continue;
        }
        PhaseTerm pt{};
        pt.th = th;
        add_bit(pt, kv.first[3]);
        if (kind == PH_THREAD && kv.first[4] >= 0) add_bit(pt, kv.first[4]);
        groups[kind == PH_THREAD ? 0 : 1 + kv.first[1]].push_back(pt);
    }
    PhaseHead head{};
    t.aux = (int32_t)pp.phase.size();
    pp.phase.push_back(PhaseTerm{});  // the head, filled below
    int total = 0;
    for (int g = 0; g <= r; g++) {
        while (groups[g].size() % 4) groups[g].push_back(PhaseTerm{});  // th = 0: adds nothing
        head.count[g] = (int32_t)groups[g].size();
        total += head.count[g];
        pp.phase.insert(pp.phase.end(), groups[g].begin(), groups[g].end());
    }
    std::memcpy(&pp.phase[t.aux], &head, sizeof(head));
    t.cnt = total;
    t.mat = (int32_t)pp.mats.size();
    for (int k = 0; k < (1 << r); k++) {
        const double a = wang[k] - std::nearbyint(wang[k]);
        pp.mats.push_back(cd(std::cos(2.0 * M_PI * a), std::sin(2.0 * M_PI * a)));
    }
    return t;
}

// Move each diagonal gate of a pass as late as it may go (until a later op
// acts densely on one of its bits, or the end of the pass) so that diagonal
// gates gather into runs, and turn each run into one phase-polynomial op.
void merge_diagonals(PlanPass& pp, int r)
{
    const size_t n_st = pp.stages.size();
    std::vector<std::vector<TileOp>> out(n_st);
    std::vector<TileOp> pending;
    uint32_t pending_pos = 0;
    auto flush = [&](size_t si) {
        if (pending.empty()) return;
        if ((int)pending.size() >= kPhaseMinRun) out[si].push_back(make_phase(pending, pp.stages[si], r, pp));
        else for (const TileOp& d : pending) out[si].push_back(d);
        pending.clear();
        pending_pos = 0;
    };
    for (size_t si = 0; si < n_st; si++) {
        const StageHdr& st = pp.stages[si];
        for (int o = 0; o < st.n_ops; o++) {
            const TileOp& t = pp.ops[st.op_begin + o];
            if (mergeable_diag(t, pp)) {
                pending.push_back(t);
                pending_pos |= local_positions(t);
                continue;
            }
            const uint32_t dp = dense_positions(t);
            if (dp & pending_pos) {
                // Only the pending diagonals that share a position with this op
                // must be applied before it; the others commute with it and
                // stay pending, so that later diagonals join them.
                std::vector<TileOp> keep;
                uint32_t keep_pos = 0;
                for (size_t k = 0; k < pending.size();) {
                    if (local_positions(pending[k]) & dp) {
                        k++;
                    } else {
                        keep.push_back(pending[k]);
                        keep_pos |= local_positions(pending[k]);
                        pending.erase(pending.begin() + (long)k);
                    }
                }
                flush(si);
                pending.swap(keep);
                pending_pos = keep_pos;
            }
            out[si].push_back(t);
        }
    }
    if (n_st) flush(n_st - 1);
    std::vector<TileOp> ops;
    for (size_t si = 0; si < n_st; si++) {
        pp.stages[si].op_begin = (int32_t)ops.size();
        pp.stages[si].n_ops = (int32_t)out[si].size();
        ops.insert(ops.end(), out[si].begin(), out[si].end());
    }
    pp.ops.swap(ops);
    pp.hdr.n_ops = (int32_t)pp.ops.size();
}

// Z reads of the adjoint sweep (Im <lambda|Z_q|phi>) commute with every op
// that does not act densely on q (diagonal gates, other reads, gates on other
// qubits), so each read may wait until such an op or the end of the pass.
// When one waiting read has to be taken, all are taken there, and reads
// taken together become one op that passes over the registers once:
// with p_k = Im(conj(lambda_k) phi_k), a read of window bit j is
// sum_k (-1)^(k_j) p_k, and a read of a thread bit or of a qubit outside the
// block is +-sum_k p_k (the same sums, in the same order, as one read alone).
void group_z_reads(PlanPass& pp, int r)
{
    const size_t n_st = pp.stages.size();
    const int tb = pp.hdr.b - r;
    std::vector<std::vector<TileOp>> out(n_st);
    std::vector<TileOp> pending;
    auto emit = [&](size_t si, const std::vector<TileOp>& reads) {
        if (reads.empty()) return;
        if (reads.size() == 1) {
            out[si].push_back(reads[0]);
            return;
        }
        const StageHdr& st = pp.stages[si];
        TileOp t{};
        t.kind = T_GRADZ;
        t.a = t.c = t.oa = t.oc = -1;
        t.j0 = t.j1 = -1;
        t.gen = GEN_Z;
        t.slot = -1;
        t.aux = (int32_t)pp.phase.size();
        t.cnt = (int32_t)reads.size();
        for (const TileOp& g : reads) {
            ReadZ z{};
            z.j = z.tbit = z.oa = -1;
            z.slot = g.slot;
            if (g.a >= 0) {
                z.j = window_index(st, r, g.a);
                if (z.j < 0)
                    for (int i = 0; i < tb; i++)
                        if (st.tpos[i] == g.a) z.tbit = i;
                if (z.j < 0 && z.tbit < 0) throw std::runtime_error("Z read on an unmapped position");
            } else {
                z.oa = g.oa;
            }
            PhaseTerm rec;
            std::memcpy(&rec, &z, sizeof(rec));
            pp.phase.push_back(rec);
        }
        out[si].push_back(t);
    };
    for (size_t si = 0; si < n_st; si++) {
        const StageHdr& st = pp.stages[si];
        for (int o = 0; o < st.n_ops; o++) {
            const TileOp& t = pp.ops[st.op_begin + o];
            if (t.kind == T_GRAD && t.gen == GEN_Z) {
                pending.push_back(t);
                continue;
            }
            if (t.kind != T_GRAD) {
                // when this op changes the qubit of a waiting read, every
                // waiting read is taken here, before it: each has waited only
                // past ops that are not dense on its qubit, so any point up to
                // its own qubit's next dense op is right for it, and reads
                // taken together share one pass over the registers
                const uint32_t dp = dense_positions(t);
                bool hit = false;
                for (const TileOp& g : pending) hit = hit || (g.a >= 0 && ((dp >> g.a) & 1u));
                if (hit) {
                    emit(si, pending);
                    pending.clear();
                }
            }
            out[si].push_back(t);
        }
    }
    if (n_st) emit(n_st - 1, pending);
    std::vector<TileOp> ops;
    for (size_t si = 0; si < n_st; si++) {
        pp.stages[si].op_begin = (int32_t)ops.size();
        pp.stages[si].n_ops = (int32_t)out[si].size();
        ops.insert(ops.end(), out[si].begin(), out[si].end());
    }
    pp.ops.swap(ops);
    pp.hdr.n_ops = (int32_t)pp.ops.size();
}

}  // namespace

// Every mapping of a staged pass places each local position exactly once,
// and the store writes the block's own qubits (a permutation of local_q), so
// that every load and store address stays inside the block.
void check_mappings(const PlanPass& pp, int r, const int32_t* store_q)
{
    const int b = pp.hdr.b, tb = b - r;
    auto check = [&](const StageHdr& m) {
        uint32_t seen = 0;
        for (int j = 0; j < r; j++) seen |= 1u << m.w[j];
        for (int i = 0; i < tb; i++) {
            if (m.tpos[i] < 0 || m.tpos[i] >= b || (seen & (1u << m.tpos[i])))
                throw std::runtime_error("pass mapping repeats a local position");
            seen |= 1u << m.tpos[i];
        }
        if (seen != ((1u << b) - 1)) throw std::runtime_error("pass mapping misses a local position");
    };
    check(pp.hdr.nat);
    check(pp.hdr.out);
    for (const StageHdr& st : pp.stages) check(st);
    if (store_q) {
        uint64_t a = 0, c = 0;
        for (int j = 0; j < b; j++) {
            a |= 1ull << pp.hdr.local_q[j];
            c |= 1ull << store_q[j];
        }
        if (a != c || popc(c) != b) throw std::runtime_error("store map is not a permutation of the block's qubits");
    }
}

void plan_circuit_stream(int n, const std::vector<PlanItem>& items_in, const PlanOptions& opt, int elem,
                         const std::function<bool(PlanPass&&)>& emit)
{
    if (n < 1 || n > kMaxQubits) throw std::runtime_error("qubit count out of range");
    const int b = std::min(opt.b, n);
    if (b > kMaxLocal) throw std::runtime_error("block too large");
    const uint64_t all = (n == 64) ? ~0ull : ((1ull << n) - 1);
    const int n_states = opt.n_states;

    std::vector<PlanItem> fused_items;
    const std::vector<PlanItem>* src = &items_in;
    if (opt.prefuse) {
        bool any_grad = false;
        for (const PlanItem& it : items_in) any_grad |= it.grad;
        if (!any_grad) {
            std::vector<HostGate> gs;
            gs.reserve(items_in.size());
            for (const PlanItem& it : items_in) gs.push_back(it.g);
            for (const HostGate& g : prefuse_gates(gs)) {
                PlanItem it;
                it.g = g;
                fused_items.push_back(it);
            }
            src = &fused_items;
        }
    }
    const std::vector<PlanItem>& items = *src;
    std::vector<ItemBits> ib(items.size());
    for (size_t i = 0; i < items.size(); i++) ib[i] = bits_of(items[i]);

    std::vector<char> done(items.size(), 0);
    const int coal = (b == n) ? 0 : std::min(opt.coalesce, b);
    const bool staged = opt.reg_bits > 0 && b - opt.reg_bits >= 6 && b - opt.reg_bits <= 9;
    // Qubit moves: items keep their own (logical) qubit numbers; logical qubit
    // q sits at state bit phys[q]. The block always holds state bits
    // 0..coal-1 (contiguous runs); with `park`, a pass's store may permute its
    // local qubits, so that the logical qubits the next pass needs sit on
    // those bits and take no extra room in its block. The last pass sends
    // every qubit back to its own bit (an extra pass with no gates if the last
    // one cannot). A permutation of local qubits at the store only changes
    // where each amplitude is written, so the result equals applying the
    // gates in order.
    const bool park = opt.park && staged && n_states == 1 && coal > 0 && b < n;
    int phys[64], logi[64];
    for (int q = 0; q < 64; q++) phys[q] = logi[q] = q;
    auto to_phys = [&](uint64_t m) {
        uint64_t r = 0;
        for (int q = 0; q < n; q++)
            if (m & (1ull << q)) r |= 1ull << phys[q];
        return r;
    };

    // In-order scan from the first pending item: an item is taken when its
    // dense qubits are (or, with `grow`, can still be made) local and no
    // skipped earlier item it does not commute with blocks it. Returns the
    // number taken; fills `taken` and the final local set when given.
    auto scan = [&](size_t first, uint64_t& S, bool grow, std::vector<size_t>* taken) {
        uint64_t blk_dense = 0, blk_diag = 0;
        int ops = 0, grads = 0, scanned = 0, count = 0;
        for (size_t i = first; i < items.size() && scanned < opt.lookahead; i++) {
            if (done[i]) continue;
            scanned++;
            const ItemBits& it = ib[i];
            bool ok = !(it.dense & (blk_dense | blk_diag)) && !(it.diag & blk_dense);
            if (ok) {
                const uint64_t need = it.dense & ~S;
                if ((need && (!grow || popc(S | need) > b)) || ops + it.n_ops > opt.max_ops ||
                    (items[i].grad && grads >= kMaxGradPerPass))
                    ok = false;
                else S |= need;
                if (ok && grow && opt.want_local) {
                    const uint64_t w = it.want & ~S;
                    if (w && popc(S | w) <= b - opt.want_reserve) S |= w;
                }
            }
            if (ok) {
                if (taken) taken->push_back(i);
                count++;
                ops += it.n_ops;
                grads += items[i].grad ? 1 : 0;
            } else {
                blk_dense |= it.dense;
                blk_diag |= it.diag;
                if ((blk_dense & all) == all) break;  // nothing later can be taken
            }
        }
        return count;
    };
    // Local set of a pass that must hold S0 (logical qubits): first choice,
    // grown in item order (each item's qubits join while there is room);
    // second choice, from the first pending item's qubits, add one candidate
    // item's missing qubits at a time, the ones that let the most further
    // items in per added qubit. Keeps whichever set takes more items.
    // skip_first: in the first growth step, pass over the skip_first best
    // additions (a different start for the lookahead's candidates).
    auto choose = [&](size_t first, uint64_t S0, std::vector<size_t>& taken, int skip_first = 0,
                      bool greedy = true) {
        uint64_t S = S0;
        taken.clear();
        if (greedy) scan(first, S, true, &taken);
        if (opt.best_gain && b < n) {
            uint64_t S1 = S0 | ib[first].dense;
            if (popc(S1) <= b) {
                int step = 0;
                while (true) {
                    uint64_t t = S1;
                    const int base = scan(first, t, false, nullptr);
                    std::vector<std::pair<double, uint64_t>> cand;
                    int seen = 0;
                    for (size_t i = first; i < items.size() && seen < opt.gain_candidates; i++) {
                        if (done[i]) continue;
                        seen++;
                        const uint64_t need = ib[i].dense & ~S1;
                        if (!need || popc(S1 | need) > b) continue;
                        uint64_t u = S1 | need;
                        const double gain = (double)(scan(first, u, false, nullptr) - base) / popc(need);
                        if (gain > 0) cand.push_back({gain, S1 | need});
                    }
                    // best gain first; equal gains keep item order
                    std::stable_sort(cand.begin(), cand.end(),
                                     [](const std::pair<double, uint64_t>& x, const std::pair<double, uint64_t>& y) {
                                         return x.first > y.first;
                                     });
                    // distinct sets only
                    cand.erase(std::unique(cand.begin(), cand.end(),
                                           [](const std::pair<double, uint64_t>& x,
                                              const std::pair<double, uint64_t>& y) { return x.second == y.second; }),
                               cand.end());
                    const size_t pick = step == 0 ? (size_t)skip_first : 0;
                    if (pick >= cand.size()) break;
                    S1 = cand[pick].second;
                    step++;
                }
                if (skip_first > 0 && step == 0) return (uint64_t)0;  // no such start
                std::vector<size_t> taken1;
                uint64_t u = S1;
                scan(first, u, false, &taken1);
                if (!greedy || taken1.size() >= taken.size()) {
                    taken.swap(taken1);
                    S = S1;
                }
            }
        }
        return S;
    };
    // With lookahead_sets > 0: more candidate local sets (best-gain growths
    // whose first step takes the 1st, 2nd, ... best addition instead of the
    // best), each scored by the items it takes plus the items the following
    // pass would take after it (chosen without lookahead); the best score
    // wins, ties going to the set that takes more now. On the 29-qubit random
    // U3 + CNOT circuit of depth 40 this plans 39 passes instead of 43 (8
    // candidates), at about 1 ms of host time per pass.
    auto choose_la = [&](size_t first, uint64_t S0, std::vector<size_t>& taken) {
        uint64_t S = choose(first, S0, taken);
        if (opt.lookahead_sets <= 0 || b >= n) return S;
        auto next_count = [&](const std::vector<size_t>& tk) {
            for (size_t i : tk) done[i] = 1;
            size_t f = first;
            while (f < items.size() && done[f]) f++;
            size_t c = 0;
            if (f < items.size()) {
                std::vector<size_t> t2;
                choose(f, S0, t2);
                c = t2.size();
            }
            for (size_t i : tk) done[i] = 0;
            return c;
        };
        size_t best = taken.size() + next_count(taken);
        for (int v = 0; v <= opt.lookahead_sets; v++) {
            std::vector<size_t> tk;
            const uint64_t Sv = choose(first, S0, tk, v, false);
            if (!Sv || tk.empty()) continue;
            const size_t sc = tk.size() + next_count(tk);
            if (sc > best || (sc == best && tk.size() > taken.size())) {
                best = sc;
                taken.swap(tk);
                S = Sv;
            }
        }
        return S;
    };

    size_t first = 0;
    while (true) {
        while (first < items.size() && done[first]) first++;
        if (first >= items.size()) break;

        uint64_t S0 = 0;
        if (b == n) {
            S0 = all;
        } else {
            for (int q = 0; q < coal; q++) S0 |= 1ull << logi[q];
        }
        std::vector<size_t> taken;
        uint64_t S = choose_la(first, S0, taken);
        if (taken.empty()) throw std::runtime_error("planner made no progress");
        // fill with qubits away from their own bit (so that they can go back),
        // then with the lowest qubits
        for (int q = 0; q < n && popc(S) < b; q++)
            if (phys[q] != q) S |= 1ull << q;
        for (int q = 0; q < n && popc(S) < b; q++) S |= 1ull << q;
        int grads = 0;
        for (size_t i : taken) {
            done[i] = 1;
            grads += items[i].grad ? 1 : 0;
        }

        PlanPass pp;
        const bool single = taken.size() == 1 && !items[taken[0]].grad;
        if (single && opt.single_gate_sweeps && n_states == 1) {
            HostGate g = items[taken[0]].g;
            for (int e = 0; e < 2; e++)
                if (g.q[e] >= 0) g.q[e] = phys[g.q[e]];
            g.ctrl = to_phys(g.ctrl);
            pp.kind = g.kind == G_DENSE1 ? PlanPass::SWEEP1 : g.kind == G_DENSE2 ? PlanPass::SWEEP2
                                                                                : PlanPass::SWEEPDIAG;
            pp.gate = pp.kind == PlanPass::SWEEPDIAG ? sweep_form(g) : g;
            pp.bytes = sweep_bytes(pp.gate, n, elem);
            if (!emit(std::move(pp))) return;
            continue;
        }

        pp.kind = PlanPass::BLOCK;
        PassHdr& h = pp.hdr;
        h.b = b;
        h.n_outer = n - b;
        const uint64_t Sp = to_phys(S);
        int pos_of[64];  // local position of each logical qubit of S
        for (int q = 0; q < 64; q++) pos_of[q] = -1;
        int j = 0, o = 0;
        for (int p = 0; p < n; p++) {
            if (Sp & (1ull << p)) {
                pos_of[logi[p]] = j;
                h.local_q[j++] = p;
            } else {
                h.outer_q[o++] = p;
            }
        }
        auto local_mask = [&](uint64_t m) {
            uint32_t r = 0;
            for (int q = 0; q < n; q++)
                if ((m & (1ull << q)) && pos_of[q] >= 0) r |= 1u << pos_of[q];
            return r;
        };
        auto phys_of = [&](int q) { return q >= 0 ? phys[q] : -1; };
        for (size_t i : taken) {
            const PlanItem& it = items[i];
            const HostGate& g = it.g;
            if (it.grad) {
                TileOp t{};
                t.kind = T_GRAD;
                t.a = pos_of[g.q[0]];
                t.oa = phys_of(g.q[0]);
                t.c = -1;
                t.oc = -1;
                t.slot = it.grad_slot;
                t.mat = 0;
                if (g.gen == GEN_Z) {
                    t.gen = GEN_Z;
                } else {
                    // X, Y and rotated reads share one form: cx X + cy Y
                    t.gen = GEN_XY;
                    t.mat = (int32_t)pp.mats.size();
                    pp.mats.push_back(g.gen == GEN_X ? cd(1.0, 0.0) : g.gen == GEN_Y ? cd(0.0, 1.0) : it.gcoef);
                }
                pp.ops.push_back(t);
            }
            if (!it.gate) continue;
            TileOp t{};
            t.kind = g.kind == G_DENSE1 ? T_DENSE1 : g.kind == G_DENSE2 ? T_DENSE2 : T_DIAG;
            t.lctrl = local_mask(g.ctrl);
            t.gctrl = to_phys(g.ctrl & ~S);
            t.mat = (int32_t)pp.mats.size();
            t.gen = GEN_NONE;
            t.slot = -1;
            if (g.kind == G_DENSE1) {
                t.a = pos_of[g.q[0]];
                t.c = -1;
                t.oa = t.oc = -1;
                if (is_pauli_x(g)) t.kind = T_XPERM;
                for (int e = 0; e < 4; e++) pp.mats.push_back(g.m[e]);
            } else if (g.kind == G_DENSE2) {
                t.a = pos_of[g.q[0]];
                t.c = pos_of[g.q[1]];
                t.oa = t.oc = -1;
                if (is_swap(g)) t.kind = T_SWAP;
                for (int e = 0; e < 16; e++) pp.mats.push_back(g.m[e]);
            } else {
                t.a = g.q[0] >= 0 ? pos_of[g.q[0]] : -1;
                t.oa = phys_of(g.q[0]);
                t.c = g.q[1] >= 0 ? pos_of[g.q[1]] : -1;
                t.oc = phys_of(g.q[1]);
                for (int e = 0; e < 4; e++) pp.mats.push_back(g.m[e]);
            }
            pp.ops.push_back(t);
        }
        h.n_ops = (int32_t)pp.ops.size();
        h.n_grad = grads;

        // Where the store writes each local position (park only).
        int32_t store_q[kMaxLocal];
        int store_first[8];
        bool moved = false;
        if (park) {
            size_t nf = first;
            while (nf < items.size() && done[nf]) nf++;
            // new state bit of each logical qubit of S, starting from where it is
            int np[64], nl[64];
            for (int q = 0; q < n; q++) {
                np[q] = phys[q];
                nl[phys[q]] = q;
            }
            auto put = [&](int x, int slot) {  // logical x onto state bit `slot` (both in the block)
                const int y = nl[slot], px = np[x];
                np[x] = slot;
                nl[slot] = x;
                np[y] = px;
                nl[px] = y;
            };
            int want[8], slot_of[8];
            int nw = 0;
            const bool last = nf >= items.size();
            if (!last) {
                // the logical qubits the next pass would hold with a free choice
                std::vector<size_t> t2;
                const uint64_t Sn = choose(nf, 0, t2) & S;
                auto add_want = [&](int q) {
                    for (int k = 0; k < nw; k++)
                        if (want[k] == q) return;
                    want[nw++] = q;
                };
                // those of the block first (the ones already on the run bits
                // before the others), then the block's qubits in the order the
                // pending items first use them
                for (int k = 0; k < coal; k++)
                    if (Sn & (1ull << nl[k])) add_want(nl[k]);
                for (int q = 0; q < n && nw < coal; q++)
                    if (Sn & (1ull << q)) add_want(q);
                for (size_t i = nf; i < items.size() && nw < coal; i++) {
                    if (done[i]) continue;
                    const uint64_t d = ib[i].dense & S;
                    for (int q = 0; q < n && nw < coal; q++)
                        if (d & (1ull << q)) add_want(q);
                }
                // a wanted qubit already on a run bit stays there; the others
                // take the run bits left
                bool used_slot[8] = {false};
                for (int k = 0; k < nw; k++) {
                    slot_of[k] = np[want[k]] < coal ? np[want[k]] : -1;
                    if (slot_of[k] >= 0) used_slot[slot_of[k]] = true;
                }
                for (int k = 0; k < nw; k++)
                    if (slot_of[k] < 0)
                        for (int sl = 0; sl < coal; sl++)
                            if (!used_slot[sl]) {
                                slot_of[k] = sl;
                                used_slot[sl] = true;
                                break;
                            }
            } else {
                // last pass: the qubits of the run bits back to them
                for (int k = 0; k < coal; k++)
                    if (S & (1ull << k)) {
                        want[nw] = k;
                        slot_of[nw++] = k;
                    }
            }
            for (int k = 0; k < nw; k++) put(want[k], slot_of[k]);
            // the others back to their own bit where that bit is in the block and
            // holds a qubit not on a run bit
            for (int q = coal; q < n; q++) {
                if (!(S & (1ull << q)) || np[q] == q || np[q] < coal) continue;
                if (!(Sp & (1ull << q))) continue;
                const int y = nl[q];
                if (np[y] < coal) continue;
                put(q, q);
            }
            for (int jj = 0; jj < b; jj++) {
                const int x = logi[h.local_q[jj]];
                store_q[jj] = np[x];
                if (np[x] != h.local_q[jj]) moved = true;
            }
            if (moved) {
                for (int k = 0; k < coal; k++) {
                    store_first[k] = -1;
                    for (int jj = 0; jj < b; jj++)
                        if (store_q[jj] == k) store_first[k] = jj;
                    if (store_first[k] < 0) throw std::runtime_error("store map lost a run bit");
                }
                for (int q = 0; q < n; q++) {
                    phys[q] = np[q];
                    logi[np[q]] = q;
                }
            }
        }
        if (staged) {
            if (opt.fuse_gates) fuse_ops(pp);
            uint32_t moved_mask = 0;
            if (moved)
                for (int jj = 0; jj < b; jj++)
                    if (store_q[jj] != h.local_q[jj]) moved_mask |= 1u << jj;
            plan_stages(pp, b, opt.reg_bits, opt.wave_mode, elem, opt.lds_elem > 0 ? opt.lds_elem : elem,
                        moved ? store_first : nullptr, moved_mask);
            pp.reg_bits = opt.reg_bits;
            if (opt.merge_diagonals) merge_diagonals(pp, opt.reg_bits);
            if (opt.group_reads && grads > 1) group_z_reads(pp, opt.reg_bits);
            diag_to_sign(pp);
            set_reg_codes(pp, opt.reg_bits, opt.mfma && elem == 8 && opt.n_states == 1);
            if (opt.fold_perms) fold_trailing_perms(pp, opt.reg_bits, opt.lds_elem > 0 ? opt.lds_elem : elem);
            set_io_offsets(pp.hdr, opt.reg_bits, moved ? store_q : nullptr);
            check_mappings(pp, opt.reg_bits, moved ? store_q : nullptr);
        }
        pp.bytes = 2.0 * n_states * std::ldexp(1.0, n) * elem;
        if (!emit(std::move(pp))) return;
    }
    // Qubits still away from their own bit: passes with no gates that move
    // them back, a few pairs (qubit, holder of its bit) at a time.
    while (park) {
        uint64_t away = 0;
        for (int q = 0; q < n; q++)
            if (phys[q] != q) away |= 1ull << q;
        if (!away) break;
        uint64_t S = 0;
        for (int k = 0; k < coal; k++) S |= 1ull << logi[k];
        // whole cycles of the permutation while they fit, else pairs
        for (int q = 0; q < n; q++) {
            if (!(away & (1ull << q)) || (S & (1ull << q))) continue;
            uint64_t cyc = 0;
            for (int x = q; !(cyc & (1ull << x)); x = logi[x]) cyc |= 1ull << x;
            if (popc(S | cyc) <= b) S |= cyc;
        }
        for (int q = 0; q < n && popc(S) < b - 1; q++) {
            if (!(away & (1ull << q)) || (S & (1ull << q))) continue;
            S |= (1ull << q) | (1ull << logi[q]);
        }
        for (int q = 0; q < n && popc(S) < b; q++) S |= 1ull << q;
        PlanPass pp;
        pp.kind = PlanPass::BLOCK;
        PassHdr& h = pp.hdr;
        h.b = b;
        h.n_outer = n - b;
        const uint64_t Sp = to_phys(S);
        int j = 0, o = 0;
        for (int p = 0; p < n; p++) {
            if (Sp & (1ull << p)) h.local_q[j++] = p;
            else h.outer_q[o++] = p;
        }
        int np[64], nl[64];
        for (int q = 0; q < n; q++) {
            np[q] = phys[q];
            nl[phys[q]] = q;
        }
        for (int q = 0; q < n; q++) {
            if (!(S & (1ull << q)) || np[q] == q || !(Sp & (1ull << q))) continue;
            const int y = nl[q], pq = np[q];
            np[q] = q;
            nl[q] = q;
            np[y] = pq;
            nl[pq] = y;
        }
        // the run bits must stay in the block's run positions
        int32_t store_q[kMaxLocal];
        int store_first[8];
        for (int jj = 0; jj < b; jj++) store_q[jj] = np[logi[h.local_q[jj]]];
        for (int k = 0; k < coal; k++) {
            store_first[k] = -1;
            for (int jj = 0; jj < b; jj++)
                if (store_q[jj] == k) store_first[k] = jj;
            if (store_first[k] < 0) throw std::runtime_error("restore map lost a run bit");
        }
        bool progress = false;
        for (int q = 0; q < n; q++) {
            progress |= np[q] == q && phys[q] != q;
            phys[q] = np[q];
            logi[np[q]] = q;
        }
        if (!progress) throw std::runtime_error("qubit restore made no progress");
        h.n_ops = 0;
        h.n_grad = 0;
        uint32_t moved_mask = 0;
        for (int jj = 0; jj < b; jj++)
            if (store_q[jj] != h.local_q[jj]) moved_mask |= 1u << jj;
        plan_stages(pp, b, opt.reg_bits, opt.wave_mode, elem, opt.lds_elem > 0 ? opt.lds_elem : elem, store_first,
                    moved_mask);
        pp.reg_bits = opt.reg_bits;
        diag_to_sign(pp);
        set_reg_codes(pp, opt.reg_bits, opt.mfma && elem == 8 && opt.n_states == 1);
        set_io_offsets(pp.hdr, opt.reg_bits, store_q);
        check_mappings(pp, opt.reg_bits, store_q);
        pp.bytes = 2.0 * n_states * std::ldexp(1.0, n) * elem;
        if (!emit(std::move(pp))) return;
    }
}

std::vector<PlanPass> plan_circuit(int n, const std::vector<PlanItem>& items, const PlanOptions& opt, int elem)
{
    std::vector<PlanPass> passes;
    plan_circuit_stream(n, items, opt, elem, [&](PlanPass&& pp) {
        passes.push_back(std::move(pp));
        return true;
    });
    return passes;
}

}  // namespace qv
