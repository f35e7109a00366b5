// C ABI of the state-vector engine: handles, argument checks, gate-table
// upload, pass execution, FP64 reductions and the adjoint sweep.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/sv.h"
#include "gates.h"
#include "qv_internal.h"

using namespace qv;

namespace {

thread_local std::string g_err;

sv_status fail(sv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(SV_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

struct TimingRec {
    int kind;
    hipEvent_t e0, e1;
};

}  // namespace

struct sv_state_t {
    int n = 0;
    sv_dtype dtype = SV_C128;
    size_t elem = 16;
    void* buf = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    int device = 0;

    // gate tables: pinned host staging + device copy
    unsigned char* h_table = nullptr;
    size_t h_table_cap = 0;
    void* d_table = nullptr;
    size_t d_table_cap = 0;
    hipEvent_t table_done = nullptr;
    bool table_pending = false;

    // reduction scratch
    double* d_part = nullptr;
    size_t d_part_cap = 0;  // doubles
    double* d_res = nullptr;
    size_t d_res_cap = 0;   // doubles
    double* h_res = nullptr;
    size_t h_res_cap = 0;   // doubles (pinned)

    // timing
    bool timing = false;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    double acc_ms[KF_COUNT] = {};
    int64_t acc_n[KF_COUNT] = {};
};

namespace {

// Keeps the caller's current device and restores it on exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

sv_status ensure_device(void** p, size_t* cap, size_t bytes, hipStream_t st)
{
    if (*cap >= bytes) return SV_OK;
    if (*p) {
        HIP_TRY(hipStreamSynchronize(st));  // older launches may still read it
        HIP_TRY(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    size_t want = bytes < 4096 ? 4096 : bytes + bytes / 2;
    if (hipMalloc(p, want) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SV_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    *cap = want;
    return SV_OK;
}

sv_status ensure_part(sv_state s, size_t doubles)
{
    size_t cap = s->d_part_cap * sizeof(double);
    void* p = s->d_part;
    sv_status st = ensure_device(&p, &cap, doubles * sizeof(double), s->stream);
    s->d_part = (double*)p;
    s->d_part_cap = cap / sizeof(double);
    return st;
}

sv_status ensure_res(sv_state s, size_t doubles)
{
    size_t cap = s->d_res_cap * sizeof(double);
    void* p = s->d_res;
    sv_status st = ensure_device(&p, &cap, doubles * sizeof(double), s->stream);
    s->d_res = (double*)p;
    s->d_res_cap = cap / sizeof(double);
    if (st != SV_OK) return st;
    if (s->h_res_cap < doubles) {
        if (s->h_res) {
            HIP_TRY(hipStreamSynchronize(s->stream));
            HIP_TRY(hipHostFree(s->h_res));
            s->h_res = nullptr;
            s->h_res_cap = 0;
        }
        const size_t want = doubles < 512 ? 512 : doubles + doubles / 2;
        if (hipHostMalloc((void**)&s->h_res, want * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->h_res = nullptr;
            return fail(SV_ENOMEM, "pinned host allocation failed");
        }
        s->h_res_cap = want;
    }
    return SV_OK;
}

// ----------------------------------------------------------- timing ---

hipEvent_t take_event(sv_state s)
{
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct LaunchTimer {
    sv_state s;
    int kind;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LaunchTimer(sv_state s_, int kind_) : s(s_), kind(kind_)
    {
        if (s->timing) {
            e0 = take_event(s);
            e1 = take_event(s);
            if (e0) (void)hipEventRecord(e0, s->stream);
        }
    }
    ~LaunchTimer()
    {
        if (s->timing && e0 && e1) {
            (void)hipEventRecord(e1, s->stream);
            s->recs.push_back({kind, e0, e1});
        }
    }
};

sv_status drain_timing(sv_state s)
{
    if (s->recs.empty()) return SV_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (auto& r : s->recs) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, r.e0, r.e1));
        s->acc_ms[r.kind] += ms;
        s->acc_n[r.kind] += 1;
        s->pool.push_back(r.e0);
        s->pool.push_back(r.e1);
    }
    s->recs.clear();
    return SV_OK;
}

// --------------------------------------------------------- validation ---

sv_status check_state(sv_state s)
{
    if (!s) return fail(SV_EINVAL, "null state handle");
    return SV_OK;
}

sv_status build_gates(sv_state s, const sv_gate* gates, int n_gates, std::vector<HostGate>* out)
{
    if (n_gates < 0) return fail(SV_EINVAL, "n_gates < 0");
    if (n_gates > 0 && !gates) return fail(SV_EINVAL, "null gate array");
    out->clear();
    out->reserve(n_gates);
    for (int i = 0; i < n_gates; i++) {
        const std::string why = check_gate(gates[i], s->n);
        if (!why.empty()) return fail(SV_EINVAL, "gate " + std::to_string(i) + ": " + why);
        std::string uns;
        if (unsupported_gate(gates[i], &uns)) return fail(SV_EUNSUPPORTED, "gate " + std::to_string(i) + ": " + uns);
        out->push_back(build_gate(gates[i]));
    }
    return SV_OK;
}

sv_status check_terms(sv_state s, const sv_pauli* terms, int n_terms)
{
    if (n_terms < 0) return fail(SV_EINVAL, "n_terms < 0");
    if (n_terms > 0 && !terms) return fail(SV_EINVAL, "null term array");
    const uint64_t all = (1ull << s->n) - 1;
    for (int t = 0; t < n_terms; t++) {
        if ((terms[t].x_mask | terms[t].z_mask) & ~all)
            return fail(SV_EINVAL, "term " + std::to_string(t) + " acts on a qubit >= n");
        if (!std::isfinite(terms[t].coeff)) return fail(SV_EINVAL, "non-finite coefficient");
    }
    return SV_OK;
}

// Terms grouped by x mask (first-appearance order), at most kTermsPerLaunch
// per batch, terms of one mask in their input order; coefficients carry
// i^{#Y}. Each batch is handed to f as it is formed, with no heap
// allocation (the non-allocating expectation uses this too); a mask is
// grouped where it first appears, so the scan is quadratic in n_terms.
template <typename F>
void visit_batches(const sv_pauli* terms, int n_terms, F&& f)
{
    static const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
    for (int t = 0; t < n_terms; t++) {
        const uint64_t x = terms[t].x_mask;
        bool seen = false;
        for (int u = 0; u < t && !seen; u++) seen = terms[u].x_mask == x;
        if (seen) continue;
        TermBatch tb{};
        tb.x_mask = x;
        for (int u = t; u < n_terms; u++) {
            const sv_pauli& p = terms[u];
            if (p.x_mask != x) continue;
            const int ny = __builtin_popcountll(p.x_mask & p.z_mask) & 3;
            tb.z_mask[tb.n_terms] = p.z_mask;
            tb.coeff_re[tb.n_terms] = p.coeff * re[ny];
            tb.coeff_im[tb.n_terms] = p.coeff * im[ny];
            if (++tb.n_terms == kTermsPerLaunch) {
                f(tb);
                tb = TermBatch{};
                tb.x_mask = x;
            }
        }
        if (tb.n_terms > 0) f(tb);
    }
}

std::vector<TermBatch> batch_terms(const sv_pauli* terms, int n_terms)
{
    std::vector<TermBatch> out;
    visit_batches(terms, n_terms, [&](const TermBatch& tb) { out.push_back(tb); });
    return out;
}

// ------------------------------------------------------ plan execution ---

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct TableOffsets {
    std::vector<size_t> hdr;  // byte offset of each block pass's header
    size_t stages = 0, ops = 0, mats = 0, phase = 0;
};

template <typename T>
sv_status upload_tables(sv_state s, const std::vector<PlanPass>& passes, TableOffsets* off)
{
    size_t n_hdr = 0, n_st = 0, n_ops = 0, n_mats = 0, n_ph = 0;
    for (const auto& p : passes)
        if (p.kind == PlanPass::BLOCK) {
            n_hdr++;
            n_st += p.stages.size();
            n_ops += p.ops.size();
            n_mats += p.mats.size();
            n_ph += p.phase.size();
        }
    off->hdr.clear();
    if (n_hdr == 0) return SV_OK;
    off->stages = align_up(n_hdr * sizeof(PassHdr), 256);
    off->ops = align_up(off->stages + n_st * sizeof(StageHdr), 256);
    off->mats = align_up(off->ops + n_ops * sizeof(TileOp), 256);
    off->phase = align_up(off->mats + n_mats * sizeof(T), 256);
    const size_t total = off->phase + n_ph * sizeof(PhaseTerm);

    if (s->table_pending) {  // the staging buffer may still feed the last copy
        HIP_TRY(hipEventSynchronize(s->table_done));
        s->table_pending = false;
    }
    if (s->h_table_cap < total) {
        if (s->h_table) HIP_TRY(hipHostFree(s->h_table));
        s->h_table = nullptr;
        const size_t want = total + total / 2 + 4096;
        if (hipHostMalloc((void**)&s->h_table, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->h_table_cap = 0;
            return fail(SV_ENOMEM, "pinned host allocation failed");
        }
        s->h_table_cap = want;
    }
    sv_status st = ensure_device(&s->d_table, &s->d_table_cap, total, s->stream);
    if (st != SV_OK) return st;

    PassHdr* H = reinterpret_cast<PassHdr*>(s->h_table);
    StageHdr* S = reinterpret_cast<StageHdr*>(s->h_table + off->stages);
    TileOp* O = reinterpret_cast<TileOp*>(s->h_table + off->ops);
    T* M = reinterpret_cast<T*>(s->h_table + off->mats);
    PhaseTerm* P = reinterpret_cast<PhaseTerm*>(s->h_table + off->phase);
    size_t ih = 0, is = 0, io = 0, im = 0, ip = 0;
    for (const auto& p : passes) {
        if (p.kind != PlanPass::BLOCK) continue;
        PassHdr h = p.hdr;
        h.op_begin = (int32_t)io;
        h.stage_begin = (int32_t)is;
        h.n_stages = (int32_t)p.stages.size();
        H[ih] = h;
        off->hdr.push_back(ih * sizeof(PassHdr));
        ih++;
        for (const StageHdr& sh : p.stages) S[is++] = sh;
        for (const TileOp& op : p.ops) {
            TileOp t = op;
            t.mat += (int32_t)im;
            if (t.kind == T_PHASE || t.kind == T_GRADZ) t.aux += (int32_t)ip;
            O[io++] = t;
        }
        for (const PhaseTerm& pt : p.phase) P[ip++] = pt;
        for (const cd& v : p.mats) {
            using R = std::remove_reference_t<decltype(M[0].x)>;
            T e;
            e.x = (R)v.real();
            e.y = (R)v.imag();
            M[im++] = e;
        }
    }
    HIP_TRY(hipMemcpyAsync(s->d_table, s->h_table, total, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipEventRecord(s->table_done, s->stream));
    s->table_pending = true;
    return SV_OK;
}

// Run a plan on one state (s1 == nullptr) or on phi and lambda (adjoint);
// grad rows of each block pass are summed into d_gvals + running offset.
template <typename T>
sv_status run_plan(sv_state s, const std::vector<PlanPass>& passes, T* s0, T* s1, int n_states,
                   std::vector<int>* grad_rows_per_pass, double* d_gvals)
{
    TableOffsets off;
    sv_status st = upload_tables<T>(s, passes, &off);
    if (st != SV_OK) return st;
    const unsigned char* base = reinterpret_cast<const unsigned char*>(s->d_table);
    const PassHdr* d_hdr = reinterpret_cast<const PassHdr*>(base);
    const StageHdr* d_stages = reinterpret_cast<const StageHdr*>(base + off.stages);
    const TileOp* d_ops = reinterpret_cast<const TileOp*>(base + off.ops);
    const T* d_mats = reinterpret_cast<const T*>(base + off.mats);
    const PhaseTerm* d_phase = reinterpret_cast<const PhaseTerm*>(base + off.phase);

    size_t ih = 0;
    int64_t gval_off = 0;
    for (size_t p = 0; p < passes.size(); p++) {
        const PlanPass& pp = passes[p];
        if (pp.kind == PlanPass::BLOCK) {
            const int b = pp.hdr.b;
            const int64_t nblocks = (int64_t)1 << (s->n - b);
            const int rows = grad_rows_per_pass ? (*grad_rows_per_pass)[p] : 0;
            if (rows > 0) {
                st = ensure_part(s, (size_t)rows * nblocks);
                if (st != SV_OK) return st;
            }
            {
                LaunchTimer tm(s, n_states == 2 ? KF_ADJ_BLOCK : KF_BLOCK);
                const PassHdr* h = d_hdr + off.hdr[ih] / sizeof(PassHdr);
                if (pp.reg_bits > 0) {  // register kernel (a pass of it may have no stages: a pure permutation)
                    HIP_TRY((launch_block_reg<T>(s0, s1, s->n, n_states, pp.reg_bits, h, d_stages, d_ops, d_mats,
                                                 d_phase, b, s->d_part, nblocks, s->stream)));
                } else {
                    HIP_TRY((launch_block_pass<T>(s0, s1, s->n, n_states, h, d_ops, d_mats, b, s->d_part, nblocks,
                                                  s->stream)));
                }
            }
            ih++;
            if (rows > 0) {
                LaunchTimer tm(s, KF_REDUCE);
                HIP_TRY(launch_sum_rows(s->d_part, rows, nblocks, nblocks, d_gvals + gval_off, s->stream));
                gval_off += rows;
            }
        } else {
            for (int k = 0; k < n_states; k++) {
                T* tgt = k == 0 ? s0 : s1;
                if (pp.kind == PlanPass::SWEEP1) {
                    LaunchTimer tm(s, KF_SWEEP1);
                    HIP_TRY(launch_sweep1<T>(tgt, s->n, pp.gate, s->stream));
                } else if (pp.kind == PlanPass::SWEEP2) {
                    LaunchTimer tm(s, KF_SWEEP2);
                    HIP_TRY(launch_sweep2<T>(tgt, s->n, pp.gate, s->stream));
                } else {
                    LaunchTimer tm(s, KF_DIAG);
                    HIP_TRY(launch_sweep_diag<T>(tgt, s->n, pp.gate, s->stream));
                }
            }
        }
    }
    return SV_OK;
}

// One pass of a streamed plan (sv_apply_fused on large states): the
// pass's tables go to the next free region of the pinned staging buffer and
// of the device table (from *cursor), are copied on the state's stream and
// the pass is launched at once, so that the host plans the next pass while
// this one runs. A region is never rewritten while a copy from it may be
// pending: the caller starts at 0 only after the previous call's last copy
// (table_done), and a pass that does not fit waits for the stream before the
// buffers grow and the cursor goes back to 0.
template <typename T>
sv_status run_pass_streamed(sv_state s, const PlanPass& pp, T* psi, size_t* cursor)
{
    if (pp.kind != PlanPass::BLOCK) {
        if (pp.kind == PlanPass::SWEEP1) {
            LaunchTimer tm(s, KF_SWEEP1);
            HIP_TRY(launch_sweep1<T>(psi, s->n, pp.gate, s->stream));
        } else if (pp.kind == PlanPass::SWEEP2) {
            LaunchTimer tm(s, KF_SWEEP2);
            HIP_TRY(launch_sweep2<T>(psi, s->n, pp.gate, s->stream));
        } else {
            LaunchTimer tm(s, KF_DIAG);
            HIP_TRY(launch_sweep_diag<T>(psi, s->n, pp.gate, s->stream));
        }
        return SV_OK;
    }
    const size_t o_st = align_up(sizeof(PassHdr), 256);
    const size_t o_ops = align_up(o_st + pp.stages.size() * sizeof(StageHdr), 256);
    const size_t o_mats = align_up(o_ops + pp.ops.size() * sizeof(TileOp), 256);
    const size_t o_ph = align_up(o_mats + pp.mats.size() * sizeof(T), 256);
    const size_t size = align_up(o_ph + pp.phase.size() * sizeof(PhaseTerm), 256);
    if (*cursor + size > s->h_table_cap || *cursor + size > s->d_table_cap) {
        HIP_TRY(hipStreamSynchronize(s->stream));  // nothing reads either buffer after this
        s->table_pending = false;
        *cursor = 0;
        const size_t want = std::max<size_t>(size * 64, (size_t)1 << 20);
        if (s->h_table_cap < want) {
            if (s->h_table) HIP_TRY(hipHostFree(s->h_table));
            s->h_table = nullptr;
            s->h_table_cap = 0;
            if (hipHostMalloc((void**)&s->h_table, want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(SV_ENOMEM, "pinned host allocation failed");
            }
            s->h_table_cap = want;
        }
        sv_status st = ensure_device(&s->d_table, &s->d_table_cap, want, s->stream);
        if (st != SV_OK) return st;
    }
    unsigned char* h = s->h_table + *cursor;
    PassHdr hdr = pp.hdr;
    hdr.op_begin = 0;
    hdr.stage_begin = 0;
    hdr.n_stages = (int32_t)pp.stages.size();
    std::memcpy(h, &hdr, sizeof(hdr));
    StageHdr* S = reinterpret_cast<StageHdr*>(h + o_st);
    for (size_t i = 0; i < pp.stages.size(); i++) S[i] = pp.stages[i];
    TileOp* O = reinterpret_cast<TileOp*>(h + o_ops);
    for (size_t i = 0; i < pp.ops.size(); i++) O[i] = pp.ops[i];
    T* M = reinterpret_cast<T*>(h + o_mats);
    for (size_t i = 0; i < pp.mats.size(); i++) {
        using R = std::remove_reference_t<decltype(M[0].x)>;
        M[i].x = (R)pp.mats[i].real();
        M[i].y = (R)pp.mats[i].imag();
    }
    PhaseTerm* P = reinterpret_cast<PhaseTerm*>(h + o_ph);
    for (size_t i = 0; i < pp.phase.size(); i++) P[i] = pp.phase[i];
    unsigned char* d = static_cast<unsigned char*>(s->d_table) + *cursor;
    HIP_TRY(hipMemcpyAsync(d, h, size, hipMemcpyHostToDevice, s->stream));
    *cursor += size;
    const int b = pp.hdr.b;
    const int64_t nblocks = (int64_t)1 << (s->n - b);
    LaunchTimer tm(s, KF_BLOCK);
    const PassHdr* d_hdr = reinterpret_cast<const PassHdr*>(d);
    if (pp.reg_bits > 0) {
        HIP_TRY((launch_block_reg<T>(psi, nullptr, s->n, 1, pp.reg_bits, d_hdr,
                                     reinterpret_cast<const StageHdr*>(d + o_st),
                                     reinterpret_cast<const TileOp*>(d + o_ops), reinterpret_cast<const T*>(d + o_mats),
                                     reinterpret_cast<const PhaseTerm*>(d + o_ph), b, s->d_part, nblocks, s->stream)));
    } else {
        HIP_TRY((launch_block_pass<T>(psi, nullptr, s->n, 1, d_hdr, reinterpret_cast<const TileOp*>(d + o_ops),
                                      reinterpret_cast<const T*>(d + o_mats), b, s->d_part, nblocks, s->stream)));
    }
    return SV_OK;
}

template <typename F>
sv_status dispatch(sv_state s, F&& f)
{
    if (s->dtype == SV_C128) return f(static_cast<d2*>(s->buf));
    return f(static_cast<f2*>(s->buf));
}

bool g_reg_kernel = true;  // register-resident block passes (QVEC_BLOCK_KERNEL=lds turns them off)

PlanOptions plan_options(int n, size_t elem, int n_states)
{
    PlanOptions o;
    o.n_states = n_states;
    o.b = default_block_qubits(n, (int)elem, n_states);
    // keep 128-byte runs contiguous in memory: 8 complex128 / 16 complex64
    o.coalesce = elem == 16 ? 3 : 4;
    const char* co = std::getenv("QVEC_COALESCE");  // lowest qubits kept in every block (2..6)
    if (co && co[0] >= '2' && co[0] <= '6' && co[1] == 0) o.coalesce = co[0] - '0';
    const char* env = std::getenv("QVEC_BLOCK_KERNEL");
    const bool reg = g_reg_kernel && !(env && std::strcmp(env, "lds") == 0);
    o.reg_bits = reg ? reg_bits_for((int)elem, n_states) : 0;
    const char* rb = std::getenv("QVEC_REG_BITS");  // register-window width override (3 or 4)
    if (reg && rb && (std::strcmp(rb, "3") == 0 || std::strcmp(rb, "4") == 0)) o.reg_bits = rb[0] - '0';
    // the single-state complex128 register kernel exchanges 8-byte halves
    o.lds_elem = (o.reg_bits > 0 && elem == 16 && n_states == 1) ? 8 : (int)elem;
    const char* sel = std::getenv("QVEC_PASS_SELECT");  // "greedy": local sets grown in gate order only
    if (sel && std::strcmp(sel, "greedy") == 0) o.best_gain = false;
    const char* fuse = std::getenv("QVEC_FUSE");  // "0": keep gates as given (no 4x4 fusion)
    o.fuse_gates = !(fuse && std::strcmp(fuse, "0") == 0);
    o.prefuse = o.fuse_gates && o.reg_bits > 0;
    // "1": passes may move qubits between state bits (fewer passes, but on
    // MI355X the extra store exchanges cost more than the passes saved)
    const char* gr = std::getenv("QVEC_GROUP_READS");  // "0": every Z read of the adjoint sweep on its own
    o.group_reads = !(gr && std::strcmp(gr, "0") == 0);
    const char* mf = std::getenv("QVEC_MFMA");  // "1": complex64 4x4 updates on the matrix cores
    o.mfma = o.reg_bits > 0 && elem == 8 && n_states == 1 && mf && std::strcmp(mf, "1") == 0;
    const char* fp = std::getenv("QVEC_FOLD_PERMS");  // "0": register permutations stay in the op loop
    o.fold_perms = !(fp && std::strcmp(fp, "0") == 0);
    const char* pk = std::getenv("QVEC_PARK");
    o.park = o.reg_bits > 0 && pk && std::strcmp(pk, "1") == 0;
    const char* wm = std::getenv("QVEC_WAVE_MODE");  // "0" | "1" | "2": see PlanOptions::wave_mode
    if (wm && wm[0] >= '0' && wm[0] <= '2' && wm[1] == 0) o.wave_mode = wm[0] - '0';
    const char* bq = std::getenv("QVEC_BLOCK_QUBITS");  // block size override (local qubits)
    if (bq) {
        const int v = std::atoi(bq);
        if (v >= 1 && v <= kMaxLocal) o.b = std::min(n, v);
    }
    // Keep the block within what the chosen kernel can hold: the register
    // kernel's exchange buffer (kRegLdsBytesPerState per state) and at most
    // 512 threads; the LDS kernel has a fixed 64 KiB block.
    if (o.reg_bits > 0) {
        while (o.b > 1 && ((size_t)1 << o.b) * (size_t)o.lds_elem > (size_t)kRegLdsBytesPerState) o.b--;
        while (o.b - o.reg_bits > 9) o.b--;
    } else {
        o.b = std::min(o.b, (elem == 16 ? 12 : 13) - (n_states == 2 ? 1 : 0));
    }
    // Lookahead in each pass's choice of local qubits (fewer passes for more
    // host time: about 1 ms per pass with 8 candidates) on states of 4 GiB
    // and more, where a pass takes milliseconds on the GPU and
    // sv_apply_fused plans each pass while the previous one runs. 16
    // candidates for complex64 (29-qubit benchmark step: 42 instead of 44
    // passes, 125.3 against 127.1 ms), 8 for complex128 (16 found no fewer
    // passes there and were slower).
    // QVEC_LOOKAHEAD=<k> sets the candidates (0: off).
    const uint64_t state_bytes = ((uint64_t)1 << n) * (uint64_t)elem * (uint64_t)n_states;
    o.lookahead_sets = (n_states == 1 && state_bytes >= (4ull << 30)) ? (elem == 8 ? 16 : 8) : 0;
    const char* la = std::getenv("QVEC_LOOKAHEAD");
    if (la) {
        const int v = std::atoi(la);
        if (v >= 0 && v <= 64) o.lookahead_sets = v;
    }
    return o;
}

std::vector<PlanItem> forward_items(const std::vector<HostGate>& hg)
{
    std::vector<PlanItem> items(hg.size());
    for (size_t i = 0; i < hg.size(); i++) items[i].g = hg[i];
    return items;
}

// Sum rows of per-block partials into d_res[0..rows), copy to h_res, wait.
sv_status finish_rows(sv_state s, int rows, int64_t count)
{
    sv_status st = ensure_res(s, rows);
    if (st != SV_OK) return st;
    {
        LaunchTimer tm(s, KF_REDUCE);
        HIP_TRY(launch_sum_rows(s->d_part, rows, count, count, s->d_res, s->stream));
    }
    HIP_TRY(hipMemcpyAsync(s->h_res, s->d_res, rows * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

template <typename T>
sv_status expect_impl(sv_state s, T* psi, const std::vector<TermBatch>& batches, double* out)
{
    const int np = kReduceBlocks;
    if (batches.empty()) {
        *out = 0;
        return SV_OK;
    }
    sv_status st = ensure_part(s, batches.size() * (size_t)np);
    if (st != SV_OK) return st;
    for (size_t k = 0; k < batches.size(); k++) {
        LaunchTimer tm(s, KF_REDUCE);
        HIP_TRY(launch_pauli_expect<T>(psi, s->n, batches[k], s->d_part + k * np, np, s->stream));
    }
    st = finish_rows(s, (int)batches.size(), np);
    if (st != SV_OK) return st;
    double f = 0;
    for (size_t k = 0; k < batches.size(); k++) f += s->h_res[k];
    *out = f;
    return SV_OK;
}

template <typename T>
sv_status pauli_apply_impl(sv_state s, const T* psi, T* dst, const std::vector<TermBatch>& batches)
{
    if (batches.empty()) {
        TermBatch zero{};
        LaunchTimer tm(s, KF_REDUCE);
        HIP_TRY(launch_pauli_apply<T>(psi, dst, s->n, zero, false, s->stream));
        return SV_OK;
    }
    for (size_t k = 0; k < batches.size(); k += kBatchesPerLaunch) {
        const int cnt = (int)std::min(batches.size() - k, (size_t)kBatchesPerLaunch);
        LaunchTimer tm(s, KF_REDUCE);
        HIP_TRY(launch_pauli_apply_multi<T>(psi, dst, s->n, batches.data() + k, cnt, k > 0, s->stream));
    }
    return SV_OK;
}

}  // namespace

// ================================================================= C ABI ===

// ------------------------------------------------------------ host tier ---
// The state stays in pinned host memory and moves through the GPU in chunks
// (QVecOpt Sec. III.B-C: a slower tier holds the state in blocks, a window of
// blocks is staged, every queued gate whose pairs lie inside is applied, the
// blocks are written back). A chunk is the set of 2^c indices that agree
// outside c local qubits: the lowest m = c - h qubits (contiguous runs of 2^m
// amplitudes) and h high qubits chosen per pass, so one chunk is 2^h runs.
// A pass takes the gates whose qubits (targets and controls) fit in its
// chunk and that commute with the gates it leaves for later; each chunk is
// then a c-qubit state for the device planner. Three device buffers and three streams overlap the copy-in of one
// chunk, the passes over another and the copy-out of a third.
namespace {

struct HostPass {
    std::vector<int> high;          // high local qubits (ascending), h of them
    std::vector<sv_gate> gates;     // gates with qubits renumbered to chunk positions
};

// High local qubits of a chunk: up to 8 (runs of 2^(c-8) amplitudes stay
// large DMA copies), none when the chunk is the whole state.
int host_high_qubits(int n, int c)
{
    if (n == c) return 0;
    int h = 8;
    const char* e = std::getenv("QVEC_HOST_HIGH");  // override (measurement knob)
    if (e && std::atoi(e) >= 1 && std::atoi(e) <= 12) h = std::atoi(e);
    return std::min(h, c / 2);
}

sv_status plan_host_passes(int n, int c, const sv_gate* gates, const std::vector<HostGate>& hg,
                           std::vector<HostPass>* out)
{
    // Each pass scans the pending gates in order and takes every gate whose
    // qubits fit in the chunk (the low qubits plus up to h high ones, chosen
    // as the scan meets them) and that commutes with the gates it skips (on
    // each shared qubit both act diagonally), as the device planner does for
    // blocks; the taken gates keep their order.
    const int h = host_high_qubits(n, c), m = c - h;
    const uint64_t low = m >= 64 ? ~0ull : ((1ull << m) - 1);
    const size_t ng = hg.size();
    std::vector<char> done(ng, 0);
    size_t first = 0;
    out->clear();
    while (true) {
        while (first < ng && done[first]) first++;
        if (first >= ng) break;
        HostPass cur;
        uint64_t high = 0, blk_dense = 0, blk_diag = 0;
        for (size_t i = first; i < ng; i++) {
            if (done[i]) continue;
            const uint64_t dn = dense_bits(hg[i]), dg = diag_bits(hg[i]);
            const uint64_t add = (dn | dg) & ~low & ~high;
            const bool free = !(dn & (blk_dense | blk_diag)) && !(dg & blk_dense);
            if (free && __builtin_popcountll(high | add) <= h) {
                high |= add;
                cur.gates.push_back(gates[i]);
                done[i] = 1;
            } else {
                blk_dense |= dn;
                blk_diag |= dg;
            }
        }
        if (cur.gates.empty())
            return fail(SV_EUNSUPPORTED, "gate " + std::to_string(first) + " needs more high qubits than a chunk holds");
        // fill the high set to h qubits (lowest first) so that every chunk has 2^c amplitudes
        for (int q = m; q < n && __builtin_popcountll(high) < h; q++) high |= 1ull << q;
        for (int q = m; q < n; q++)
            if (high >> q & 1) cur.high.push_back(q);
        int pos[64];
        for (int q = 0; q < 64; q++) pos[q] = q < m ? q : -1;
        for (int k = 0; k < h; k++) pos[cur.high[k]] = m + k;
        for (sv_gate& g : cur.gates) {
            const bool two = g.op == SV_OP_MATRIX2 || g.op == SV_OP_CNOT || g.op == SV_OP_CZ || g.op == SV_OP_CP ||
                             g.op == SV_OP_SWAP;
            g.qubits[0] = pos[g.qubits[0]];
            if (two) g.qubits[1] = pos[g.qubits[1]];
            for (int k = 0; k < g.n_controls; k++) g.controls[k] = pos[g.controls[k]];
        }
        out->push_back(std::move(cur));
    }
    return SV_OK;
}

}  // namespace

extern "C" {

const char* sv_last_error(void) { return g_err.c_str(); }

sv_status sv_alloc(sv_state* out, int n_qubits, sv_dtype dtype, void* device_buf, size_t buf_bytes,
                   void* hip_stream)
{
    g_err.clear();
    if (!out) return fail(SV_EINVAL, "null output handle");
    *out = nullptr;
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (n_qubits < 1 || n_qubits > kMaxQubits) return fail(SV_EINVAL, "n_qubits must be in [1, 34]");
    const size_t elem = dtype == SV_C128 ? 16 : 8;
    const size_t need = ((size_t)1 << n_qubits) * elem;
    if (device_buf) {
        if (buf_bytes < need)
            return fail(SV_EINVAL, "buffer of " + std::to_string(buf_bytes) + " bytes < 2^n * " +
                                       std::to_string(elem) + " = " + std::to_string(need));
        if (reinterpret_cast<uintptr_t>(device_buf) % 16) return fail(SV_EINVAL, "buffer not 16-byte aligned");
    }
    sv_state s = new (std::nothrow) sv_state_t;
    if (!s) return fail(SV_ENOMEM, "host allocation failed");
    s->n = n_qubits;
    s->dtype = dtype;
    s->elem = elem;
    s->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(SV_EDEVICE, "no HIP device");
    }
    if (device_buf) {
        s->buf = device_buf;
    } else {
        if (hipMalloc(&s->buf, need) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(SV_ENOMEM, "device allocation of the state failed");
        }
        s->owns = true;
    }
    if (hipEventCreateWithFlags(&s->table_done, hipEventDisableTiming) != hipSuccess) {
        if (s->owns) (void)hipFree(s->buf);
        delete s;
        return fail(SV_EDEVICE, "event creation failed");
    }
    *out = s;
    return SV_OK;
}

sv_status sv_free(sv_state s)
{
    g_err.clear();
    if (!s) return SV_OK;
    DeviceGuard dg(s->device);
    sv_status st = SV_OK;
    if (hipStreamSynchronize(s->stream) != hipSuccess) st = fail(SV_EDEVICE, "stream failed before free");
    for (auto& r : s->recs) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    for (auto e : s->pool) (void)hipEventDestroy(e);
    if (s->table_done) (void)hipEventDestroy(s->table_done);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->h_table) (void)hipHostFree(s->h_table);
    if (s->d_part) (void)hipFree(s->d_part);
    if (s->d_res) (void)hipFree(s->d_res);
    if (s->h_res) (void)hipHostFree(s->h_res);
    if (s->owns && s->buf) (void)hipFree(s->buf);
    delete s;
    return st;
}

void* sv_data(sv_state s) { return s ? s->buf : nullptr; }
int sv_num_qubits(sv_state s) { return s ? s->n : 0; }
sv_dtype sv_get_dtype(sv_state s) { return s ? s->dtype : SV_C128; }

sv_status sv_set_basis(sv_state s, uint64_t x)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (x >> s->n) return fail(SV_EINVAL, "basis index >= 2^n");
    DeviceGuard dg(s->device);
    LaunchTimer tm(s, KF_INIT);
    return dispatch(s, [&](auto* psi) -> sv_status {
        HIP_TRY(launch_init_basis(psi, s->n, x, s->stream));
        return SV_OK;
    });
}

sv_status sv_apply_gate(sv_state s, int n_targets, const int* targets, int n_controls, const int* controls,
                        const double* matrix)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (n_targets != 1 && n_targets != 2) return fail(SV_EINVAL, "n_targets must be 1 or 2");
    if (!targets || !matrix) return fail(SV_EINVAL, "null targets or matrix");
    if (n_controls < 0 || n_controls > 2) return fail(SV_EINVAL, "n_controls must be 0..2");
    if (n_controls > 0 && !controls) return fail(SV_EINVAL, "null controls");
    sv_gate g{};
    g.op = n_targets == 1 ? SV_OP_MATRIX1 : SV_OP_MATRIX2;
    g.qubits[0] = targets[0];
    g.qubits[1] = n_targets == 2 ? targets[1] : 0;
    g.n_controls = n_controls;
    for (int c = 0; c < n_controls; c++) g.controls[c] = controls[c];
    g.param_index = -1;
    std::memcpy(g.matrix, matrix, sizeof(double) * (n_targets == 1 ? 8 : 32));
    return sv_apply_unfused(s, &g, 1);
}

sv_status sv_apply_unfused(sv_state s, const sv_gate* gates, int n_gates)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    std::vector<HostGate> hg;
    sv_status st = build_gates(s, gates, n_gates, &hg);
    if (st != SV_OK) return st;
    DeviceGuard dg(s->device);
    return dispatch(s, [&](auto* psi) -> sv_status {
        using T = std::remove_pointer_t<decltype(psi)>;
        for (const HostGate& g : hg) {
            if (g.kind == G_DENSE1) {
                LaunchTimer tm(s, KF_SWEEP1);
                HIP_TRY(launch_sweep1<T>(psi, s->n, g, s->stream));
            } else if (g.kind == G_DENSE2) {
                LaunchTimer tm(s, KF_SWEEP2);
                HIP_TRY(launch_sweep2<T>(psi, s->n, g, s->stream));
            } else {
                LaunchTimer tm(s, KF_DIAG);
                HIP_TRY(launch_sweep_diag<T>(psi, s->n, sweep_form(g), s->stream));
            }
        }
        return SV_OK;
    });
}

sv_status sv_apply_fused(sv_state s, const sv_gate* gates, int n_gates)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    std::vector<HostGate> hg;
    sv_status st = build_gates(s, gates, n_gates, &hg);
    if (st != SV_OK) return st;
    if (hg.empty()) return SV_OK;
    DeviceGuard dg(s->device);
    const PlanOptions opt = plan_options(s->n, s->elem, 1);
    // States of 1 GiB and more (a pass takes half a millisecond or more on
    // the GPU): each pass is launched as soon as it is planned.
    // QVEC_STREAM_PLAN=0 / 1 turns this off / on at any size.
    const char* sp = std::getenv("QVEC_STREAM_PLAN");
    const bool stream = sp ? std::strcmp(sp, "1") == 0 : (((uint64_t)1 << s->n) * s->elem >= (1ull << 30));
    if (stream) {
        return dispatch(s, [&](auto* psi) -> sv_status {
            using T = std::remove_pointer_t<decltype(psi)>;
            if (s->table_pending) {  // the staging buffer may still feed the last call's copy
                HIP_TRY(hipEventSynchronize(s->table_done));
                s->table_pending = false;
            }
            size_t cursor = 0;
            sv_status st = SV_OK;
            bool any = false;
            try {
                plan_circuit_stream(s->n, forward_items(hg), opt, (int)s->elem, [&](PlanPass&& pp) {
                    st = run_pass_streamed<T>(s, pp, psi, &cursor);
                    any = true;
                    return st == SV_OK;
                });
            } catch (const std::exception& e) {
                (void)hipStreamSynchronize(s->stream);
                return fail(SV_EINVAL, std::string("planner: ") + e.what() +
                                           (any ? " (the passes planned before it were applied)" : ""));
            }
            if (any) {
                HIP_TRY(hipEventRecord(s->table_done, s->stream));
                s->table_pending = true;
            }
            return st;
        });
    }
    std::vector<PlanPass> passes;
    try {
        passes = plan_circuit(s->n, forward_items(hg), opt, (int)s->elem);
    } catch (const std::exception& e) {
        return fail(SV_EINVAL, std::string("planner: ") + e.what());
    }
    return dispatch(s, [&](auto* psi) -> sv_status {
        using T = std::remove_pointer_t<decltype(psi)>;
        return run_plan<T>(s, passes, psi, nullptr, 1, nullptr, nullptr);
    });
}

sv_status sv_plan(int n_qubits, sv_dtype dtype, const sv_gate* gates, int n_gates, sv_plan_stats* out)
{
    g_err.clear();
    if (!out) return fail(SV_EINVAL, "null output");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
    if (n_qubits < 1 || n_qubits > kMaxQubits) return fail(SV_EINVAL, "n_qubits must be in [1, 34]");
    sv_state_t tmp;
    tmp.n = n_qubits;
    tmp.dtype = dtype;
    tmp.elem = dtype == SV_C128 ? 16 : 8;
    std::vector<HostGate> hg;
    sv_status st = build_gates(&tmp, gates, n_gates, &hg);
    if (st != SV_OK) return st;
    std::memset(out, 0, sizeof(*out));
    out->n_gates = n_gates;
    const PlanOptions o = plan_options(n_qubits, tmp.elem, 1);
    out->block_qubits = std::min(o.b, n_qubits);
    if (hg.empty()) return SV_OK;
    try {
        const auto passes = plan_circuit(n_qubits, forward_items(hg), o, (int)tmp.elem);
        for (const auto& p : passes) {
            out->n_passes++;
            if (p.kind == PlanPass::BLOCK) out->n_block_passes++;
            out->bytes_moved += p.bytes;
            out->n_stages += (int64_t)p.stages.size();
            out->n_ops += (int64_t)p.ops.size();
            for (const auto& op : p.ops) out->n_phase_ops += op.kind == T_PHASE ? 1 : 0;
        }
    } catch (const std::exception& e) {
        return fail(SV_EINVAL, std::string("planner: ") + e.what());
    }
    return SV_OK;
}

sv_status sv_host_apply(void* host_state, int n_qubits, sv_dtype dtype, const sv_gate* gates, int n_gates,
                        int chunk_qubits, sv_host_stats* stats)
{
    g_err.clear();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!host_state) return fail(SV_EINVAL, "null host state");
    if (reinterpret_cast<uintptr_t>(host_state) % 16) return fail(SV_EINVAL, "host state not 16-byte aligned");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (n_qubits < 1 || n_qubits > kMaxQubits) return fail(SV_EINVAL, "n_qubits must be in [1, 34]");
    if (chunk_qubits < 1 || chunk_qubits > kMaxQubits) return fail(SV_EINVAL, "chunk_qubits must be in [1, 34]");
    const size_t elem = dtype == SV_C128 ? 16 : 8;
    sv_state_t tmp;
    tmp.n = n_qubits;
    tmp.dtype = dtype;
    tmp.elem = elem;
    std::vector<HostGate> hg;
    sv_status st = build_gates(&tmp, gates, n_gates, &hg);
    if (st != SV_OK) return st;
    const int n = n_qubits, c = std::min(chunk_qubits, n_qubits);
    std::vector<HostPass> hp;
    st = plan_host_passes(n, c, gates, hg, &hp);
    if (st != SV_OK) return st;
    const int h = host_high_qubits(n, c), m = c - h;
    const uint64_t n_chunks = 1ull << (n - c), n_runs = 1ull << h;
    const size_t run_bytes = ((size_t)1 << m) * elem, chunk_bytes = ((size_t)1 << c) * elem;
    if (stats) {
        stats->n_passes = (int64_t)hp.size();
        stats->n_chunks = (int64_t)n_chunks;
        stats->chunk_qubits = c;
        stats->high_qubits = h;
    }
    if (hp.empty()) return SV_OK;
    const auto t0 = std::chrono::steady_clock::now();

    // Three device buffers in rotation: the copy-in of chunk k + 1 waits only
    // for the copy-out of chunk k - 2, so copies in and out overlap while
    // chunk k is on the device.
    constexpr int NB = 3;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    void* dbuf[NB] = {};
    sv_state hs[NB] = {};
    hipEvent_t ev[3 * NB + 1] = {};  // in_done[NB], comp_done[NB], out_done[NB], pass_done
    hipEvent_t *in_done = ev, *comp_done = ev + NB, *out_done = ev + 2 * NB, &pass_done = ev[3 * NB];
    auto body = [&]() -> sv_status {
        HIP_TRY(hipStreamCreate(&s_in));
        HIP_TRY(hipStreamCreate(&s_comp));
        HIP_TRY(hipStreamCreate(&s_out));
        for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (int b = 0; b < NB; b++) {
            if (hipMalloc(&dbuf[b], chunk_bytes) != hipSuccess) {
                (void)hipGetLastError();
                dbuf[b] = nullptr;
                return fail(SV_ENOMEM, "device allocation of a chunk buffer failed");
            }
            sv_status a = sv_alloc(&hs[b], c, dtype, dbuf[b], chunk_bytes, s_comp);
            if (a != SV_OK) return a;
        }
        bool used[NB] = {}, have_pass = false;
        for (const HostPass& p : hp) {
            std::vector<HostGate> cg;
            sv_status bs = build_gates(hs[0], p.gates.data(), (int)p.gates.size(), &cg);
            if (bs != SV_OK) return bs;
            std::vector<PlanPass> plan;
            try {
                plan = plan_circuit(c, forward_items(cg), plan_options(c, elem, 1), (int)elem);
            } catch (const std::exception& e) {
                return fail(SV_EINVAL, std::string("planner: ") + e.what());
            }
            uint64_t local = (m >= 64) ? ~0ull : ((1ull << m) - 1);
            for (int q : p.high) local |= 1ull << q;
            int outer[64], n_outer = 0;
            for (int q = 0; q < n; q++)
                if (!(local >> q & 1)) outer[n_outer++] = q;
            for (uint64_t k = 0; k < n_chunks; k++) {
                const int b = (int)(k % NB);
                uint64_t base = 0;
                for (int i = 0; i < n_outer; i++) base |= ((k >> i) & 1ull) << outer[i];
                if (used[b]) HIP_TRY(hipStreamWaitEvent(s_in, out_done[b], 0));
                if (have_pass) HIP_TRY(hipStreamWaitEvent(s_in, pass_done, 0));
                for (uint64_t r = 0; r < n_runs; r++) {
                    uint64_t off = base;
                    for (int i = 0; i < h; i++) off |= ((r >> i) & 1ull) << p.high[i];
                    HIP_TRY(hipMemcpyAsync(static_cast<char*>(dbuf[b]) + r * run_bytes,
                                           static_cast<const char*>(host_state) + off * elem, run_bytes,
                                           hipMemcpyHostToDevice, s_in));
                }
                HIP_TRY(hipEventRecord(in_done[b], s_in));
                HIP_TRY(hipStreamWaitEvent(s_comp, in_done[b], 0));
                sv_status rs = dispatch(hs[b], [&](auto* psi) -> sv_status {
                    using T = std::remove_pointer_t<decltype(psi)>;
                    return run_plan<T>(hs[b], plan, psi, nullptr, 1, nullptr, nullptr);
                });
                if (rs != SV_OK) return rs;
                HIP_TRY(hipEventRecord(comp_done[b], s_comp));
                HIP_TRY(hipStreamWaitEvent(s_out, comp_done[b], 0));
                for (uint64_t r = 0; r < n_runs; r++) {
                    uint64_t off = base;
                    for (int i = 0; i < h; i++) off |= ((r >> i) & 1ull) << p.high[i];
                    HIP_TRY(hipMemcpyAsync(static_cast<char*>(host_state) + off * elem,
                                           static_cast<const char*>(dbuf[b]) + r * run_bytes, run_bytes,
                                           hipMemcpyDeviceToHost, s_out));
                }
                HIP_TRY(hipEventRecord(out_done[b], s_out));
                used[b] = true;
            }
            // the next pass reads what this one writes back
            HIP_TRY(hipEventRecord(pass_done, s_out));
            have_pass = true;
        }
        HIP_TRY(hipStreamSynchronize(s_out));
        return SV_OK;
    };
    sv_status res = body();
    const std::string err = g_err;  // sv_free below clears the message
    // release in dependency order; a failure above still drains the streams
    for (hipStream_t q : {s_in, s_comp, s_out})
        if (q && hipStreamSynchronize(q) != hipSuccess && res == SV_OK) res = fail(SV_EDEVICE, "host tier stream failed");
    for (int b = 0; b < NB; b++) {
        if (hs[b]) (void)sv_free(hs[b]);
        if (dbuf[b]) (void)hipFree(dbuf[b]);
    }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : {s_in, s_comp, s_out})
        if (q) (void)hipStreamDestroy(q);
    if (res != SV_OK) g_err = err;
    if (res == SV_OK && stats) {
        stats->bytes_h2d = (double)hp.size() * (double)n_chunks * (double)chunk_bytes;
        stats->bytes_d2h = stats->bytes_h2d;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return res;
}

sv_status sv_norm2(sv_state s, double* out)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (!out) return fail(SV_EINVAL, "null output");
    DeviceGuard dg(s->device);
    sv_pauli one{1.0, 0, 0};
    const auto batches = batch_terms(&one, 1);
    return dispatch(s, [&](auto* psi) { return expect_impl(s, psi, batches, out); });
}

sv_status sv_expect(sv_state s, const sv_pauli* terms, int n_terms, double* out)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (!out) return fail(SV_EINVAL, "null output");
    sv_status st = check_terms(s, terms, n_terms);
    if (st != SV_OK) return st;
    DeviceGuard dg(s->device);
    const auto batches = batch_terms(terms, n_terms);
    return dispatch(s, [&](auto* psi) { return expect_impl(s, psi, batches, out); });
}

sv_status sv_apply_pauli_sum(sv_state s, const sv_pauli* terms, int n_terms, void* dst_buf, size_t dst_bytes)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    sv_status st = check_terms(s, terms, n_terms);
    if (st != SV_OK) return st;
    const size_t need = ((size_t)1 << s->n) * s->elem;
    if (!dst_buf || dst_bytes < need) return fail(SV_EINVAL, "destination buffer missing or too small");
    if (reinterpret_cast<uintptr_t>(dst_buf) % 16) return fail(SV_EINVAL, "destination not 16-byte aligned");
    const char* a = static_cast<const char*>(s->buf);
    const char* d = static_cast<const char*>(dst_buf);
    if (d < a + need && a < d + need) return fail(SV_EINVAL, "destination overlaps the state");
    DeviceGuard dg(s->device);
    const auto batches = batch_terms(terms, n_terms);
    return dispatch(s, [&](auto* psi) -> sv_status {
        using T = std::remove_pointer_t<decltype(psi)>;
        return pauli_apply_impl<T>(s, psi, static_cast<T*>(dst_buf), batches);
    });
}

// Reverse-sweep rewrite: a one-qubit diagonal gate D followed by an X/Y
// gradient read and a one-qubit gate U on the same qubit. The read sees both
// states after D, and Im <D lam| G |D phi> = Im <lam| D^dag G D |phi>, where
// D^dag G D is again a combination of X and Y. So the read moves before D
// with the rotated generator, and D joins U as the single matrix U D. The
// item that held D keeps only its own read (a Z read, which D does not
// change), or disappears if it had none. This saves one pass over the
// registers per such pair (RZ then RY in hardware-efficient ansatze).
static void fold_diagonals_into_reads(std::vector<PlanItem>& items)
{
    std::vector<PlanItem> out;
    out.reserve(items.size());
    for (size_t i = 0; i < items.size(); i++) {
        PlanItem a = items[i];
        if (i + 1 < items.size() && a.gate && a.g.kind == G_DIAG && a.g.q[1] < 0 && a.g.ctrl == 0) {
            PlanItem& b = items[i + 1];
            const bool xy = b.grad && (b.g.gen == GEN_X || b.g.gen == GEN_Y || b.g.gen == GEN_XY);
            if (xy && b.gate && b.g.kind == G_DENSE1 && b.g.ctrl == 0 && b.g.q[0] == a.g.q[0]) {
                const cd d0 = a.g.m[0], d1 = a.g.m[1];
                // G = cx X + cy Y has off-diagonal entry g01 = cx - i cy
                const cd c = b.g.gen == GEN_X ? cd(1.0, 0.0) : b.g.gen == GEN_Y ? cd(0.0, 1.0) : b.gcoef;
                const cd g01 = std::conj(d0) * cd(c.real(), -c.imag()) * d1;
                b.gcoef = cd(g01.real(), -g01.imag());
                b.g.gen = GEN_XY;
                // U D: column c of U times d_c
                b.g.m[0] *= d0;
                b.g.m[1] *= d1;
                b.g.m[2] *= d0;
                b.g.m[3] *= d1;
                if (!a.grad) continue;  // nothing left of this item
                a.gate = false;
            }
        }
        out.push_back(a);
    }
    items.swap(out);
}

sv_status sv_adjoint_grad(sv_state s, const sv_gate* gates, int n_gates, const sv_pauli* terms, int n_terms,
                          void* work_buf, size_t work_bytes, double* grad_out, int n_params, double* expval_out)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (n_params < 0) return fail(SV_EINVAL, "n_params < 0");
    if (n_params > 0 && !grad_out) return fail(SV_EINVAL, "null grad_out");
    sv_status st = check_terms(s, terms, n_terms);
    if (st != SV_OK) return st;
    const size_t need = ((size_t)1 << s->n) * s->elem;
    if (!work_buf || work_bytes < need) return fail(SV_EINVAL, "work buffer missing or too small");
    if (reinterpret_cast<uintptr_t>(work_buf) % 16) return fail(SV_EINVAL, "work buffer not 16-byte aligned");
    {
        const char* a = static_cast<const char*>(s->buf);
        const char* d = static_cast<const char*>(work_buf);
        if (d < a + need && a < d + need) return fail(SV_EINVAL, "work buffer overlaps the state");
    }
    std::vector<HostGate> hg;
    st = build_gates(s, gates, n_gates, &hg);
    if (st != SV_OK) return st;
    for (int i = 0; i < n_gates; i++)
        if (hg[i].param >= n_params)
            return fail(SV_EINVAL, "gate " + std::to_string(i) + ": param_index >= n_params");
    DeviceGuard dg(s->device);

    return dispatch(s, [&](auto* psi) -> sv_status {
        using T = std::remove_pointer_t<decltype(psi)>;
        T* lam = static_cast<T*>(work_buf);
        // lambda = H psi and f = <psi|lambda> go to the device first; the
        // reverse sweep is planned on the host while they run.
        const auto batches = batch_terms(terms, n_terms);
        sv_status st2 = pauli_apply_impl<T>(s, psi, lam, batches);
        if (st2 != SV_OK) return st2;
        const int np = kReduceBlocks;
        st2 = ensure_part(s, 2 * (size_t)np);
        if (st2 != SV_OK) return st2;
        {
            LaunchTimer tm(s, KF_REDUCE);
            HIP_TRY(launch_inner<T>(psi, lam, s->n, s->d_part, np, s->stream));
        }

        // Reverse sweep items: gradient read, then the inverse gate. A grad
        // item's slot is its position among the grad items (reverse gate order).
        std::vector<PlanItem> items;
        std::vector<int> slot_gate;  // grad slot -> gate index
        items.reserve(hg.size());
        for (int l = n_gates - 1; l >= 0; l--) {
            PlanItem it;
            it.g = dagger(hg[l]);
            it.g.gen = hg[l].gen;
            if (hg[l].param >= 0) {
                it.grad = true;
                it.grad_slot = (int32_t)slot_gate.size();
                slot_gate.push_back(l);
            }
            items.push_back(it);
        }
        fold_diagonals_into_reads(items);
        std::vector<PlanPass> passes;
        try {
            PlanOptions o = plan_options(s->n, s->elem, 2);
            o.single_gate_sweeps = false;
            passes = plan_circuit(s->n, items, o, (int)s->elem);
        } catch (const std::exception& e) {
            (void)hipStreamSynchronize(s->stream);  // the launches above read psi and write lambda
            return fail(SV_EINVAL, std::string("planner: ") + e.what());
        }
        // Renumber the grad reads pass by pass: the rows of one pass are
        // contiguous in the device result array, in op order.
        std::vector<int> rows_per_pass(passes.size(), 0);
        std::vector<int> row_gate;  // result row -> gate index
        for (size_t p = 0; p < passes.size(); p++) {
            int local = 0;
            for (TileOp& op : passes[p].ops) {
                if (op.kind == T_GRAD) {
                    row_gate.push_back(slot_gate[op.slot]);
                    op.slot = local++;
                } else if (op.kind == T_GRADZ) {
                    for (int e = 0; e < op.cnt; e++) {
                        ReadZ z;
                        std::memcpy(&z, &passes[p].phase[op.aux + e], sizeof(z));
                        row_gate.push_back(slot_gate[z.slot]);
                        z.slot = local++;
                        std::memcpy(&passes[p].phase[op.aux + e], &z, sizeof(z));
                    }
                }
            }
            rows_per_pass[p] = local;
        }
        const int n_grad = (int)row_gate.size();

        // f = Re <psi|H psi>
        st2 = finish_rows(s, 2, np);
        if (st2 != SV_OK) return st2;
        const double f = s->h_res[0];
        st2 = ensure_res(s, (size_t)(n_grad > 0 ? n_grad : 1));
        if (st2 != SV_OK) return st2;
        st2 = run_plan<T>(s, passes, psi, lam, 2, &rows_per_pass, s->d_res);
        if (st2 != SV_OK) return st2;
        if (n_grad > 0)
            HIP_TRY(hipMemcpyAsync(s->h_res, s->d_res, n_grad * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        std::vector<double> per_gate(hg.size(), 0.0);
        for (int r = 0; r < n_grad; r++) per_gate[row_gate[r]] = s->h_res[r];
        for (int p = 0; p < n_params; p++) grad_out[p] = 0;
        for (size_t l = 0; l < hg.size(); l++)
            if (hg[l].param >= 0) grad_out[hg[l].param] += per_gate[l];
        if (expval_out) *expval_out = f;
        return SV_OK;
    });
}

sv_status sv_compare(sv_state a, sv_state b, sv_diff* out)
{
    g_err.clear();
    if (!a || !b) return fail(SV_EINVAL, "null state handle");
    if (!out) return fail(SV_EINVAL, "null output");
    if (a->n != b->n) return fail(SV_EINVAL, "qubit counts differ");
    if (a->device != b->device) return fail(SV_EINVAL, "states on different devices");
    DeviceGuard dg(a->device);
    const int np = kReduceBlocks;
    HIP_TRY(hipStreamSynchronize(b->stream));  // b's pending work lands before a's stream reads it
    sv_status st = ensure_part(a, 6 * (size_t)np);
    if (st != SV_OK) return st;
    st = ensure_res(a, 6);
    if (st != SV_OK) return st;
    {
        LaunchTimer tm(a, KF_REDUCE);
        hipError_t e;
        if (a->dtype == SV_C128 && b->dtype == SV_C128)
            e = launch_compare<d2, d2>((const d2*)a->buf, (const d2*)b->buf, a->n, a->d_part, np, a->stream);
        else if (a->dtype == SV_C128)
            e = launch_compare<d2, f2>((const d2*)a->buf, (const f2*)b->buf, a->n, a->d_part, np, a->stream);
        else if (b->dtype == SV_C128)
            e = launch_compare<f2, d2>((const f2*)a->buf, (const d2*)b->buf, a->n, a->d_part, np, a->stream);
        else
            e = launch_compare<f2, f2>((const f2*)a->buf, (const f2*)b->buf, a->n, a->d_part, np, a->stream);
        HIP_TRY(e);
        HIP_TRY(launch_compare_finish(a->d_part, np, a->d_res, a->stream));
    }
    HIP_TRY(hipMemcpyAsync(a->h_res, a->d_res, 6 * sizeof(double), hipMemcpyDeviceToHost, a->stream));
    HIP_TRY(hipStreamSynchronize(a->stream));
    out->max_abs = a->h_res[0];
    out->l2 = std::sqrt(a->h_res[1]);
    out->inner_re = a->h_res[2];
    out->inner_im = a->h_res[3];
    out->norm2_a = a->h_res[4];
    out->norm2_b = a->h_res[5];
    return SV_OK;
}

sv_status sv_copy(sv_state s, void* dst, const void* src, size_t bytes)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (!dst || !src) return fail(SV_EINVAL, "null pointer");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | bytes) % 16)
        return fail(SV_EINVAL, "pointers and size must be multiples of 16 bytes");
    const char* a = static_cast<const char*>(src);
    const char* d = static_cast<const char*>(dst);
    if (bytes && d < a + bytes && a < d + bytes) return fail(SV_EINVAL, "ranges overlap");
    if (!bytes) return SV_OK;
    DeviceGuard dg(s->device);
    LaunchTimer tm(s, KF_COPY);
    HIP_TRY(launch_copy(dst, src, bytes, s->stream));
    return SV_OK;
}

sv_status sv_sync(sv_state s)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    DeviceGuard dg(s->device);
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

sv_status sv_timing_enable(sv_state s, int on)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    s->timing = on != 0;
    return SV_OK;
}

sv_status sv_timing_reset(sv_state s)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    DeviceGuard dg(s->device);
    sv_status st = drain_timing(s);
    for (int k = 0; k < KF_COUNT; k++) {
        s->acc_ms[k] = 0;
        s->acc_n[k] = 0;
    }
    return st;
}

sv_status sv_timing_read(sv_state s, int kernel, int64_t* launches, double* total_ms)
{
    g_err.clear();
    if (check_state(s)) return SV_EINVAL;
    if (kernel < 0 || kernel >= KF_COUNT) return fail(SV_EINVAL, "kernel family out of range");
    if (!launches || !total_ms) return fail(SV_EINVAL, "null output");
    DeviceGuard dg(s->device);
    sv_status st = drain_timing(s);
    if (st != SV_OK) return st;
    *launches = s->acc_n[kernel];
    *total_ms = s->acc_ms[kernel];
    return SV_OK;
}

}  // extern "C"

// ------------------------------------------------- non-allocating calls ---
// sv_expect_noalloc keeps its reduction scratch (per-block partials of each
// term batch, then one sum per batch) in a fixed device array instead of
// buffers the library allocates: one copy per GPU, held until the process
// ends, shared by every call on that GPU.
namespace {

constexpr int kNoAllocMaxBatches = 64;
constexpr size_t kNoAllocScratchDoubles = (size_t)kNoAllocMaxBatches * kReduceBlocks + kNoAllocMaxBatches;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current GPU's copy of `scratch`, looked up once
// per device with that device current. Host code passes this address to
// kernels; the array's name is only a host-side stand-in.
sv_status scratch_for_device(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(SV_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SV_OK;
}

}  // namespace

extern "C" {

sv_status sv_expect_noalloc(const void* state, int n_qubits, sv_dtype dtype, const sv_pauli* terms, int n_terms,
                            double* d_out, void* hip_stream)
{
    g_err.clear();
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (n_qubits < 1 || n_qubits > kMaxQubits) return fail(SV_EINVAL, "n_qubits must be in [1, 34]");
    if (!state || !d_out) return fail(SV_EINVAL, "null state or output");
    if (reinterpret_cast<uintptr_t>(state) % 16) return fail(SV_EINVAL, "state not 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_out) % 8) return fail(SV_EINVAL, "output not 8-byte aligned");
    if (n_terms < 0) return fail(SV_EINVAL, "n_terms < 0");
    if (n_terms > 0 && !terms) return fail(SV_EINVAL, "null term array");
    const uint64_t all = (1ull << n_qubits) - 1;
    for (int t = 0; t < n_terms; t++) {
        if ((terms[t].x_mask | terms[t].z_mask) & ~all) return fail(SV_EINVAL, "a term acts on a qubit >= n");
        if (!std::isfinite(terms[t].coeff)) return fail(SV_EINVAL, "non-finite coefficient");
    }
    int nb = 0;
    visit_batches(terms, n_terms, [&](const TermBatch&) { nb++; });
    if (nb > kNoAllocMaxBatches)
        return fail(SV_EINVAL, "more than 64 term batches (a batch is up to 16 terms sharing one x mask)");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    double* part = nullptr;
    sv_status st = scratch_for_device(dev, &part);
    if (st != SV_OK) return st;
    double* rows = part + (size_t)kNoAllocMaxBatches * kReduceBlocks;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int np = kReduceBlocks;
    // The launches and the order of the sums are those of sv_expect, so the
    // two give the same double.
    int k = 0;
    hipError_t err = hipSuccess;
    visit_batches(terms, n_terms, [&](const TermBatch& tb) {
        if (err != hipSuccess) return;
        err = dtype == SV_C128
                  ? launch_pauli_expect<d2>(static_cast<const d2*>(state), n_qubits, tb, part + (size_t)k * np, np,
                                            stream)
                  : launch_pauli_expect<f2>(static_cast<const f2*>(state), n_qubits, tb, part + (size_t)k * np, np,
                                            stream);
        k++;
    });
    HIP_TRY(err);
    HIP_TRY(launch_sum_rows(part, nb, np, np, rows, stream));
    HIP_TRY(launch_sum_ordered(rows, nb, d_out, stream));
    return SV_OK;
}

}  // extern "C"
