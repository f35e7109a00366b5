// Host emulation of the planner's single-state block passes, for CPU tests.
//
// Each block pass is executed at the level of local indices, reading the pass
// exactly as the register kernel does where it matters for the result: the
// load and store mappings (global qubit of each thread bit and element offset
// of each register), the ops' local positions and controls, the phase ops'
// window tables and thread/block term records. The state after all passes is
// compared with the same gates applied one by one. Structural checks: every
// within-wave exchange keeps each wave's set of local indices; without a
// workgroup-wide exchange in a pass, each wave stores only to addresses it
// loaded; a pass with no final exchange stores from the mapping it is in.
//
// Input (stdin): one gate per line, "op q0 q1 a0 a1 a2" (sv_op code, qubits,
// angles). Arguments: n, bytes per amplitude (16 or 8), 1 to let passes move
// qubits between state bits. Prints the maximum difference; exit status 0
// when every check holds and the difference is below 1e-10.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gates.h"
#include "qv_internal.h"

using namespace qv;
typedef std::complex<double> C;

static void apply_host(std::vector<C>& psi, int n, const HostGate& g)
{
    const uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; i++) {
        if ((i & g.ctrl) != g.ctrl) continue;
        if (g.kind == G_DENSE1) {
            const uint64_t kb = 1ull << g.q[0];
            if (i & kb) continue;
            C a = psi[i], b = psi[i | kb];
            psi[i] = g.m[0] * a + g.m[1] * b;
            psi[i | kb] = g.m[2] * a + g.m[3] * b;
        } else if (g.kind == G_DENSE2) {
            const uint64_t ka = 1ull << g.q[0], kc = 1ull << g.q[1];
            if (i & (ka | kc)) continue;
            uint64_t id[4] = {i, i | ka, i | kc, i | ka | kc};
            C x[4], y[4];
            for (int e = 0; e < 4; e++) x[e] = psi[id[e]];
            for (int r = 0; r < 4; r++) {
                y[r] = 0;
                for (int c = 0; c < 4; c++) y[r] += g.m[4 * r + c] * x[c];
            }
            for (int e = 0; e < 4; e++) psi[id[e]] = y[e];
        } else {
            int s = (g.q[0] >= 0 ? (int)((i >> g.q[0]) & 1) : 0) + 2 * (g.q[1] >= 0 ? (int)((i >> g.q[1]) & 1) : 0);
            psi[i] *= g.m[s];
        }
    }
}

static int bit(uint64_t x, int p) { return (int)((x >> p) & 1); }

static void run_block_pass(std::vector<C>& psi, int n, const PlanPass& pp)
{
    const PassHdr& h = pp.hdr;
    const int b = h.b, r = pp.reg_bits, tb = b - r;
    const uint64_t nblocks = 1ull << (n - b);
    auto lidx = [&](const StageHdr& m, uint32_t tid, uint32_t k) {
        uint32_t l = 0;
        for (int i = 0; i < tb; i++) l |= ((tid >> i) & 1u) << m.tpos[i];
        for (int j = 0; j < r; j++) l |= ((k >> j) & 1u) << m.w[j];
        return l;
    };
    for (uint64_t bi = 0; bi < nblocks; bi++) {
        std::vector<C> blk(1u << b);
        uint64_t base = bi;
        for (int j = 0; j < b; j++) {
            const int q = h.local_q[j];
            base = ((base >> q) << 1 << q) | (base & ((1ull << q) - 1));
        }
        // load
        for (uint32_t tid = 0; tid < (1u << tb); tid++) {
            uint64_t tg = 0;
            for (int i = 0; i < tb; i++) tg |= (uint64_t)((tid >> i) & 1) << h.nat_tq[i];
            for (uint32_t k = 0; k < (1u << r); k++) blk[lidx(h.nat, tid, k)] = psi[(base | tg) + h.nat_koff[k]];
        }
        // ops by stage
        for (size_t si = 0; si < pp.stages.size(); si++) {
            const StageHdr& st = pp.stages[si];
            // the stage's ops, then its exit permutations (which the kernel
            // applies to the registers' exchange offsets) as ops at its end
            for (int o = st.op_begin; o < st.op_begin + st.n_ops + st.n_exit; o++) {
                const TileOp& t = pp.ops[o];
                if ((base & t.gctrl) != t.gctrl) continue;
                const cd* M = pp.mats.data() + t.mat;
                const uint32_t L = 1u << b;
                if (t.kind == T_DENSE1 || t.kind == T_XPERM) {
                    for (uint32_t l = 0; l < L; l++) {
                        if (bit(l, t.a) || (l & t.lctrl) != t.lctrl) continue;
                        const uint32_t l1 = l | (1u << t.a);
                        C x = blk[l], y = blk[l1];
                        if (t.kind == T_XPERM) { blk[l] = y; blk[l1] = x; }
                        else { blk[l] = M[0] * x + M[1] * y; blk[l1] = M[2] * x + M[3] * y; }
                    }
                } else if (t.kind == T_DENSE2 || t.kind == T_SWAP) {
                    for (uint32_t l = 0; l < L; l++) {
                        if (bit(l, t.a) || bit(l, t.c) || (l & t.lctrl) != t.lctrl) continue;
                        uint32_t id[4] = {l, l | (1u << t.a), l | (1u << t.c), l | (1u << t.a) | (1u << t.c)};
                        C x[4], y[4];
                        for (int e = 0; e < 4; e++) x[e] = blk[id[e]];
                        if (t.kind == T_SWAP) { y[0] = x[0]; y[1] = x[2]; y[2] = x[1]; y[3] = x[3]; }
                        else for (int rr = 0; rr < 4; rr++) { y[rr] = 0; for (int c = 0; c < 4; c++) y[rr] += M[4 * rr + c] * x[c]; }
                        for (int e = 0; e < 4; e++) blk[id[e]] = y[e];
                    }
                } else if (t.kind == T_DIAG) {
                    for (uint32_t l = 0; l < L; l++) {
                        if ((l & t.lctrl) != t.lctrl) continue;
                        const int ba = t.a >= 0 ? bit(l, t.a) : (t.oa >= 0 ? bit(base, t.oa) : 0);
                        const int bc = t.c >= 0 ? bit(l, t.c) : (t.oc >= 0 ? bit(base, t.oc) : 0);
                        blk[l] *= M[ba + 2 * bc];
                    }
                } else if (t.kind == T_SIGN) {
                    for (uint32_t l = 0; l < L; l++)
                        if ((l & t.lctrl) == t.lctrl) blk[l] = -blk[l];
                } else if (t.kind == T_PHASE) {
                    const PhaseHead& ph = *reinterpret_cast<const PhaseHead*>(&pp.phase[t.aux]);
                    for (uint32_t tid = 0; tid < (1u << tb); tid++) {
                        const PhaseTerm* pt = pp.phase.data() + t.aux + 1;
                        double grp[8] = {0};
                        if (t.cnt) {
                            for (int g = 0; g <= r; g++) {
                                for (int u = 0; u < ph.count[g]; u++) {
                                    const PhaseTerm& x = pt[u];
                                    if ((base & x.omask) == x.omask && (tid & x.tmask) == x.tmask) grp[g] += x.th;
                                }
                                pt += ph.count[g];
                            }
                        }
                        for (uint32_t k = 0; k < (1u << r); k++) {
                            double ang = grp[0];
                            for (int j = 0; j < r; j++) if ((k >> j) & 1) ang += grp[1 + j];
                            C f = std::polar(1.0, 2 * M_PI * ang) * C(M[k].real(), M[k].imag());
                            blk[lidx(st, tid, k)] *= f;
                        }
                    }
                } else {
                    fprintf(stderr, "op kind %d\n", t.kind);
                    exit(2);
                }
            }
        }
        // store
        for (uint32_t tid = 0; tid < (1u << tb); tid++) {
            uint64_t go = base;
            for (int i = 0; i < tb; i++) go |= (uint64_t)((tid >> i) & 1) << h.out_tq[i];
            for (uint32_t k = 0; k < (1u << r); k++) psi[go + h.out_koff[k]] = blk[lidx(h.out, tid, k)];
        }
    }
}

static int g_slot_bytes = 8;     // exchange slot size of the kernel the plan is for
static int g_bank_conflicts = 0;  // (mapping, register) pairs whose lowest lanes share a bank row slot

static int check_structure(const std::vector<PlanPass>& passes)
{
    int bad = 0;
    for (size_t pi = 0; pi < passes.size(); pi++) {
        const PlanPass& pp = passes[pi];
        if (pp.kind != PlanPass::BLOCK || pp.reg_bits == 0) continue;
        const PassHdr& h = pp.hdr;
        const int b = h.b, r = pp.reg_bits, tb = b - r;
        const int nwaves = tb > 6 ? 1 << (tb - 6) : 1;
        auto index_of = [&](const StageHdr& m, uint32_t tid, uint32_t k) {
            uint32_t l = 0;
            for (int i = 0; i < tb; i++) l |= ((tid >> i) & 1u) << m.tpos[i];
            for (int j = 0; j < r; j++) l |= ((k >> j) & 1u) << m.w[j];
            return l;
        };
        auto wave_set = [&](const StageHdr& m, int w) {
            std::vector<uint32_t> v;
            for (uint32_t tid = (uint32_t)w * 64; tid < (uint32_t)(w + 1) * 64 && tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) v.push_back(index_of(m, tid, k));
            std::sort(v.begin(), v.end());
            return v;
        };
        // the index each (thread, register) holds in the current mapping: its
        // own, until exit permutations at a stage's end move the values
        // (the kernel then writes it at the offset of the index it holds)
        std::vector<uint32_t> held;
        auto reset_held = [&](const StageHdr& m) {
            held.assign((size_t)1 << b, 0);
            for (uint32_t tid = 0; tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) held[(tid << r) | k] = index_of(m, tid, k);
        };
        auto held_wave_set = [&](int w) {
            std::vector<uint32_t> v;
            for (uint32_t tid = (uint32_t)w * 64; tid < (uint32_t)(w + 1) * 64 && tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) v.push_back(held[(tid << r) | k]);
            std::sort(v.begin(), v.end());
            return v;
        };
        bool block_xch = h.final_wave_local == XCH_BLOCK;
        const StageHdr* cur = &h.nat;
        // Exchange-buffer byte offset of (thread, register) under a mapping,
        // as the kernel forms it: the slot of the thread part (lds_slot) and
        // the register's window part from the stage table.
        auto offset_of = [&](const StageHdr& m, uint32_t tid, uint32_t k) {
            const uint32_t e = g_slot_bytes == 16 ? 4 : 5;
            uint32_t tl = 0;
            for (int i = 0; i < tb; i++) tl |= ((tid >> i) & 1u) << m.tpos[i];
            return lds_slot(tl, (int)e) * (uint32_t)g_slot_bytes ^ m.woff[k];
        };
        // Every exchange: the write of the current mapping fills each slot
        // once, and the read of the new one finds in each register the
        // amplitude of its own local index. Lanes 0..2^e-1 of a wave (2^e
        // slots of 256 / 2^e bytes: one row of LDS banks) that share a row
        // position are counted as bank conflicts (reported, not required).
        auto lds_round_trip = [&](const StageHdr& to) {
            const uint32_t sb = (uint32_t)g_slot_bytes, e = sb == 16 ? 4 : 5;
            const uint32_t nslots = 1u << b;
            std::vector<int64_t> buf(nslots, -1);
            for (uint32_t tid = 0; tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) {
                    const uint32_t o = offset_of(*cur, tid, k);
                    if (o % sb || o / sb >= nslots || buf[o / sb] >= 0) {
                        std::printf("pass %zu: exchange write collides or leaves the buffer\n", pi);
                        bad++;
                        return;
                    }
                    buf[o / sb] = index_of(*cur, tid, k);
                }
            for (uint32_t tid = 0; tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) {
                    const uint32_t o = offset_of(to, tid, k);
                    if (o / sb >= nslots || buf[o / sb] != (int64_t)index_of(to, tid, k)) {
                        std::printf("pass %zu: exchange read finds another amplitude\n", pi);
                        bad++;
                        return;
                    }
                }
            for (const StageHdr* m : {cur, &to})
                for (uint32_t k = 0; k < (1u << r); k++) {
                    uint32_t seen = 0;
                    for (uint32_t lane = 0; lane < (1u << e); lane++) seen |= 1u << ((offset_of(*m, lane, k) / sb) & ((1u << e) - 1));
                    if (seen != (uint32_t)((1ull << (1u << e)) - 1)) g_bank_conflicts++;
                }
        };
        auto check_xch = [&](const StageHdr& to, int kind) {
            if (kind == XCH_BLOCK) block_xch = true;
            if (kind != XCH_NONE) lds_round_trip(to);
            if (kind != XCH_WAVE) return;
            for (int w = 0; w < nwaves; w++)
                if (held_wave_set(w) != wave_set(to, w)) {
                    std::printf("pass %zu: a within-wave exchange changes wave %d's indices\n", pi, w);
                    bad++;
                    return;
                }
        };
        reset_held(*cur);
        for (size_t si = 0; si < pp.stages.size(); si++) {
            const StageHdr& st = pp.stages[si];
            if (st.wave_local != XCH_NONE) {
                check_xch(st, st.wave_local);
                cur = &st;
                reset_held(*cur);
            }
            if (st.n_exit == 0) continue;
            // the values move as the exits say (blocks that meet their outer
            // controls: the within-wave check must hold for them too)
            for (int o = st.op_begin + st.n_ops; o < st.op_begin + st.n_ops + st.n_exit; o++) {
                const TileOp& t = pp.ops[o];
                for (uint32_t& l : held)
                    if ((l & t.lctrl) == t.lctrl) l ^= 1u << t.a;
            }
            // exit permutations: an exchange follows, and XOR-ing the term
            // into the offsets of the registers in kmask gives each of them
            // the offset of its partner index in the mapping in effect
            const bool xch_next = si + 1 < pp.stages.size() ? pp.stages[si + 1].wave_local != XCH_NONE
                                                            : h.final_wave_local != XCH_NONE;
            if (!xch_next) {
                std::printf("pass %zu: stage %zu has exit permutations but no exchange after it\n", pi, si);
                bad++;
            }
            // element (thread, register) of each local index in the mapping in effect
            std::vector<std::pair<uint32_t, uint32_t>> elem_of(1u << b);
            for (uint32_t tid = 0; tid < (1u << tb); tid++)
                for (uint32_t k = 0; k < (1u << r); k++) elem_of[index_of(*cur, tid, k)] = {tid, k};
            for (int o = st.op_begin + st.n_ops; o < st.op_begin + st.n_ops + st.n_exit; o++) {
                const TileOp& t = pp.ops[o];
                bool ok = t.kind == T_XPERM && t.a >= 0 && t.a < b && !((t.lctrl >> t.a) & 1u);
                // values stay in their wave: other waves may still be reading
                // the slots of their own indices (within-wave exchanges)
                for (int i = 6; i < tb; i++)
                    if (cur->tpos[i] == t.a) {
                        std::printf("pass %zu: exit permutation %d moves values between waves\n", pi, o);
                        bad++;
                    }
                // kmask: the registers whose window bits meet the op's controls
                // inside the window; tctrl: its controls on thread bits
                const uint32_t wc = t.lctrl & cur->wmask;
                ok = ok && t.tctrl == (t.lctrl & ~cur->wmask);
                for (uint32_t k = 0; ok && k < (1u << r); k++) {
                    uint32_t wl = 0;
                    for (int j = 0; j < r; j++)
                        if ((k >> j) & 1u) wl |= 1u << cur->w[j];
                    ok = (((t.kmask >> k) & 1u) != 0) == ((wl & wc) == wc);
                }
                // every element the op moves: its offset XOR the term is the
                // offset of the element holding its partner index
                for (uint32_t tid = 0; ok && tid < (1u << tb); tid++) {
                    uint32_t tl = 0;
                    for (int i = 0; i < tb; i++) tl |= ((tid >> i) & 1u) << cur->tpos[i];
                    if ((tl & t.tctrl) != t.tctrl) continue;
                    for (uint32_t k = 0; ok && k < (1u << r); k++) {
                        if (!((t.kmask >> k) & 1u)) continue;
                        const auto pe = elem_of[index_of(*cur, tid, k) ^ (1u << t.a)];
                        ok = (offset_of(*cur, tid, k) ^ (uint32_t)t.aux) == offset_of(*cur, pe.first, pe.second);
                    }
                }
                if (!ok) {
                    std::printf("pass %zu: exit permutation %d does not map the offsets of its registers\n", pi, o);
                    bad++;
                }
            }
        }
        if (h.final_wave_local != XCH_NONE) {
            check_xch(h.out, h.final_wave_local);
        } else {
            bool same = cur->wmask == h.out.wmask;
            for (int i = 0; i < tb; i++) same = same && cur->tpos[i] == h.out.tpos[i];
            for (int j = 0; j < r; j++) same = same && cur->w[j] == h.out.w[j];
            if (!same) {
                std::printf("pass %zu: stores from another mapping than the one it is in\n", pi);
                bad++;
            }
        }
        if (block_xch) continue;
        for (int w = 0; w < nwaves; w++) {
            std::vector<uint64_t> L, S;
            for (uint32_t tid = (uint32_t)w * 64; tid < (uint32_t)(w + 1) * 64 && tid < (1u << tb); tid++) {
                uint64_t tg = 0, go = 0;
                for (int i = 0; i < tb; i++) {
                    tg |= (uint64_t)((tid >> i) & 1) << h.nat_tq[i];
                    go |= (uint64_t)((tid >> i) & 1) << h.out_tq[i];
                }
                for (uint32_t k = 0; k < (1u << r); k++) {
                    L.push_back(tg + h.nat_koff[k]);
                    S.push_back(go + h.out_koff[k]);
                }
            }
            std::sort(L.begin(), L.end());
            std::sort(S.begin(), S.end());
            if (L != S) {
                std::printf("pass %zu: wave %d stores outside what it loaded, with no workgroup barrier\n", pi, w);
                bad++;
                break;
            }
        }
    }
    return bad;
}

int main(int argc, char** argv)
{
    if (argc < 4) return 2;
    const int n = std::atoi(argv[1]), elem = std::atoi(argv[2]);
    std::vector<HostGate> gates;
    std::vector<PlanItem> items;
    int op, q0, q1;
    double a0, a1, a2;
    while (std::scanf("%d %d %d %lf %lf %lf", &op, &q0, &q1, &a0, &a1, &a2) == 6) {
        sv_gate g{};
        g.op = op;
        g.qubits[0] = q0;
        g.qubits[1] = q1;
        g.param_index = -1;
        g.angles[0] = a0;
        g.angles[1] = a1;
        g.angles[2] = a2;
        PlanItem it;
        it.g = build_gate(g);
        items.push_back(it);
        gates.push_back(it.g);
    }
    // the options the library uses for a single state on the register kernel
    PlanOptions o;
    o.b = std::min(default_block_qubits(n, elem, 1), std::min(n, 12));
    o.coalesce = elem == 16 ? 3 : 4;
    if (argc > 4 && std::atoi(argv[4]) > 0) o.coalesce = std::atoi(argv[4]);  // the QVEC_COALESCE knob
    o.reg_bits = 4;
    o.lds_elem = elem == 16 ? 8 : elem;
    g_slot_bytes = o.lds_elem;
    o.prefuse = true;
    o.park = std::atoi(argv[3]) > 0;
    if (argc > 5) o.lookahead_sets = std::atoi(argv[5]);  // candidate local sets scored with the next pass
    if (argc > 6) o.fold_perms = std::atoi(argv[6]) > 0;  // exit permutations (default on)
    const std::vector<PlanPass> passes = plan_circuit(n, items, o, elem);
    const int bad = check_structure(passes);
    if (argc > 7 && std::atoi(argv[7]) > 0) {  // plan structure only (sizes too large to emulate)
        int exits = 0;
        for (const PlanPass& pp : passes)
            for (const StageHdr& st : pp.stages) exits += st.n_exit;
        std::printf("n=%d elem=%d passes=%zu structure_errors=%d exit_perms=%d (structure only)\n", n, elem,
                    passes.size(), bad, exits);
        return bad == 0 ? 0 : 1;
    }
    std::vector<C> psi(1ull << n), ref;
    uint64_t seed = 0x9E3779B97F4A7C15ull;
    double nn = 0;
    for (C& x : psi) {
        seed = seed * 6364136223846793005ull + 1442695040888963407ull;
        const double re = (double)(seed >> 11) / 9007199254740992.0 - 0.5;
        seed = seed * 6364136223846793005ull + 1442695040888963407ull;
        const double im = (double)(seed >> 11) / 9007199254740992.0 - 0.5;
        x = C(re, im);
        nn += std::norm(x);
    }
    for (C& x : psi) x /= std::sqrt(nn);
    ref = psi;
    for (const HostGate& g : gates) apply_host(ref, n, g);
    for (const PlanPass& pp : passes) {
        if (pp.kind == PlanPass::BLOCK) run_block_pass(psi, n, pp);
        else apply_host(psi, n, pp.gate);
    }
    double err = 0;
    for (size_t i = 0; i < psi.size(); i++) err = std::max(err, std::abs(psi[i] - ref[i]));
    int exits = 0;
    for (const PlanPass& pp : passes)
        for (const StageHdr& st : pp.stages) exits += st.n_exit;
    std::printf("n=%d elem=%d passes=%zu structure_errors=%d bank_conflicts=%d exit_perms=%d maxerr=%.3e\n", n,
                elem, passes.size(), bad, g_bank_conflicts, exits, err);
    return (bad == 0 && err < 1e-10) ? 0 : 1;
}
