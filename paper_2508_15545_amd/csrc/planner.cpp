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
#include <cmath>
#include <stdexcept>

#include "gates.h"
#include "qv_internal.h"

namespace qv {

int default_block_qubits(int n, int elem_bytes, int n_states)
{
    // 64 KiB of LDS per workgroup: 4096 complex128 / 8192 complex64
    // amplitudes, halved when two states share the block.
    const int lb = (elem_bytes == 16 ? 12 : 13) - (n_states == 2 ? 1 : 0);
    return std::min(n, lb);
}

namespace {

int popc(uint64_t v) { return __builtin_popcountll(v); }

struct ItemBits {
    uint64_t dense;  // qubits acted on non-diagonally (must be local)
    uint64_t diag;   // qubits acted on diagonally (may be outside the block)
    int n_ops;
};

ItemBits bits_of(const PlanItem& it)
{
    ItemBits b{dense_bits(it.g), diag_bits(it.g), 1};
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

}  // namespace

std::vector<PlanPass> plan_circuit(int n, const std::vector<PlanItem>& items, const PlanOptions& opt, int elem)
{
    if (n < 1 || n > kMaxQubits) throw std::runtime_error("qubit count out of range");
    const int b = std::min(opt.b, n);
    if (b > kMaxLocal) throw std::runtime_error("block too large");
    const uint64_t all = (n == 64) ? ~0ull : ((1ull << n) - 1);
    const int n_states = opt.n_states;

    std::vector<ItemBits> ib(items.size());
    for (size_t i = 0; i < items.size(); i++) ib[i] = bits_of(items[i]);

    std::vector<char> done(items.size(), 0);
    std::vector<PlanPass> passes;
    size_t first = 0;
    while (true) {
        while (first < items.size() && done[first]) first++;
        if (first >= items.size()) break;

        uint64_t S = 0;
        if (b == n) {
            S = all;
        } else {
            for (int q = 0; q < std::min(opt.coalesce, b); q++) S |= 1ull << q;
        }
        uint64_t blk_dense = 0, blk_diag = 0;
        std::vector<size_t> taken;
        int ops = 0;
        int scanned = 0;
        for (size_t i = first; i < items.size() && scanned < opt.lookahead; i++) {
            if (done[i]) continue;
            scanned++;
            const ItemBits& it = ib[i];
            bool ok = !(it.dense & (blk_dense | blk_diag)) && !(it.diag & blk_dense);
            if (ok) {
                const uint64_t need = it.dense & ~S;
                if (popc(S | need) > b || ops + it.n_ops > opt.max_ops) ok = false;
                else S |= need;
            }
            if (ok) {
                taken.push_back(i);
                ops += it.n_ops;
            } else {
                blk_dense |= it.dense;
                blk_diag |= it.diag;
                if ((blk_dense & all) == all) break;  // nothing later can be taken
            }
        }
        if (taken.empty()) throw std::runtime_error("planner made no progress");
        for (int q = 0; q < n && popc(S) < b; q++) S |= 1ull << q;  // fill with the lowest qubits
        for (size_t i : taken) done[i] = 1;

        PlanPass pp;
        const bool single = taken.size() == 1 && !items[taken[0]].grad;
        if (single && opt.single_gate_sweeps && n_states == 1) {
            const HostGate& g = items[taken[0]].g;
            pp.kind = g.kind == G_DENSE1 ? PlanPass::SWEEP1 : g.kind == G_DENSE2 ? PlanPass::SWEEP2
                                                                                : PlanPass::SWEEPDIAG;
            pp.gate = pp.kind == PlanPass::SWEEPDIAG ? sweep_form(g) : g;
            pp.bytes = sweep_bytes(pp.gate, n, elem);
            passes.push_back(pp);
            continue;
        }

        pp.kind = PlanPass::BLOCK;
        PassHdr& h = pp.hdr;
        h.b = b;
        h.n_outer = n - b;
        int pos_of[64];
        for (int q = 0; q < 64; q++) pos_of[q] = -1;
        int j = 0, o = 0;
        for (int q = 0; q < n; q++) {
            if (S & (1ull << q)) {
                pos_of[q] = j;
                h.local_q[j++] = q;
            } else {
                h.outer_q[o++] = q;
            }
        }
        auto local_mask = [&](uint64_t m) {
            uint32_t r = 0;
            for (int q = 0; q < n; q++)
                if ((m & (1ull << q)) && pos_of[q] >= 0) r |= 1u << pos_of[q];
            return r;
        };
        for (size_t i : taken) {
            const PlanItem& it = items[i];
            const HostGate& g = it.g;
            if (it.grad) {
                TileOp t{};
                t.kind = T_GRAD;
                t.gen = g.gen;
                t.a = pos_of[g.q[0]];
                t.oa = g.q[0];
                t.c = -1;
                t.oc = -1;
                t.slot = it.grad_slot;
                t.mat = 0;
                pp.ops.push_back(t);
            }
            TileOp t{};
            t.kind = g.kind == G_DENSE1 ? T_DENSE1 : g.kind == G_DENSE2 ? T_DENSE2 : T_DIAG;
            t.lctrl = local_mask(g.ctrl);
            t.gctrl = g.ctrl & ~S;
            t.mat = (int32_t)pp.mats.size();
            t.gen = GEN_NONE;
            t.slot = -1;
            if (g.kind == G_DENSE1) {
                t.a = pos_of[g.q[0]];
                t.c = -1;
                t.oa = t.oc = -1;
                for (int e = 0; e < 4; e++) pp.mats.push_back(g.m[e]);
            } else if (g.kind == G_DENSE2) {
                t.a = pos_of[g.q[0]];
                t.c = pos_of[g.q[1]];
                t.oa = t.oc = -1;
                for (int e = 0; e < 16; e++) pp.mats.push_back(g.m[e]);
            } else {
                t.a = g.q[0] >= 0 ? pos_of[g.q[0]] : -1;
                t.oa = g.q[0];
                t.c = g.q[1] >= 0 ? pos_of[g.q[1]] : -1;
                t.oc = g.q[1];
                for (int e = 0; e < 4; e++) pp.mats.push_back(g.m[e]);
            }
            pp.ops.push_back(t);
        }
        h.n_ops = (int32_t)pp.ops.size();
        pp.bytes = 2.0 * n_states * std::ldexp(1.0, n) * elem;
        passes.push_back(std::move(pp));
    }
    return passes;
}

}  // namespace qv
