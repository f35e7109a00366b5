// HIP kernels for gfx950 (MI355X): amplitude-pairing sweeps, block passes
// and FP64 reductions over a 2^n complex state held in HBM.
//
// Amplitudes are native 2-vectors (re, im): d2 (complex128, 16 B) or f2
// (complex64, 8 B), so every amplitude moves with one 16-/8-byte access.
// All indices are 64-bit (2^34 amplitudes at most).
#include <type_traits>

#include "device_common.h"

namespace qv {

static unsigned grid_for(uint64_t items, uint64_t per_block)
{
    const uint64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g ? g : 1);
}

// A dispatch holds fewer than 2^32 work-items, so large states give each
// thread more items: the smallest of pref, 2, 4, 8, 16 that keeps the grid
// at 2^31 work-items or fewer (2^34 amplitudes need 8).
static int items_per_thread(uint64_t items, int pref)
{
    int p = pref;
    while (p < 16 && (items + p - 1) / p > (1ull << 31)) p *= 2;
    return p;
}

// Calls f(std::integral_constant<int, P>) for P = items_per_thread(items, pref).
template <typename F>
static void with_per_thread(uint64_t items, int pref, F&& f)
{
    switch (items_per_thread(items, pref)) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 16>{}); break;
    }
}

// ----------------------------------------------------------- basis init ---

template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_init_basis(T* __restrict__ psi, uint64_t N, uint64_t x)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        if (i < N) {
            T v;
            v.x = (i == x) ? 1 : 0;
            v.y = 0;
            st_nt(psi + i, v);
        }
    }
}

template <typename T>
hipError_t launch_init_basis(T* psi, int n, uint64_t x, hipStream_t st)
{
    // one amplitude per thread (as for the copy) while the grid allows
    const uint64_t N = 1ull << n;
    with_per_thread(N, 1, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_init_basis<T, P>), dim3(grid_for(N, kThreads * P)), dim3(kThreads), 0, st, psi, N,
                           x);
    });
    return hipGetLastError();
}

// ------------------------------------------------------ one-qubit sweep ---
// Eq. 5 on every pair (i, i | 2^k) with bit k of i clear and all control
// bits set. Each thread owns P pairs spaced kThreads apart so that each
// wave's loads are contiguous runs; all 2P loads are issued before any math.

// Workgroup index with the XCD index moved: workgroups are dispatched
// round-robin over the eight XCDs, so the low three bits of blockIdx.x name
// the XCD; with sb >= 0 they become bits sb..sb+2 of the index (the grid is
// a multiple of 2^(sb+3) then), and each XCD sweeps runs of 2^sb
// consecutive workgroups. sb < 0 keeps the dispatch order.
__device__ __forceinline__ uint64_t xcd_block(int sb)
{
    uint64_t blk = blockIdx.x;
    if (sb >= 0) {
        const uint64_t j = blk & 7, r = blk >> 3;
        blk = ((r >> sb) << (sb + 3)) | (j << sb) | (r & ((1ull << sb) - 1));
    }
    return blk;
}

template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep1(T* __restrict__ psi, uint64_t npairs, int k, Ins ins,
                                                     uint64_t ctrl, T u00, T u01, T u10, T u11, int sb)
{
    const uint64_t base = xcd_block(sb) * (kThreads * P) + threadIdx.x;
    const uint64_t kb = 1ull << k;
    T x[P], y[P];
    uint64_t i0[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        i0[r] = insert_zeros(p < npairs ? p : 0, ins) | ctrl;
        if (p < npairs) {
            x[r] = ld_nt(psi + i0[r]);
            y[r] = ld_nt(psi + (i0[r] | kb));
        }
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        if (p < npairs) {
            const T a = cmul2(u00, x[r], u01, y[r]);
            const T c = cmul2(u10, x[r], u11, y[r]);
            st_nt(psi + i0[r], a);
            st_nt(psi + (i0[r] | kb), c);
        }
    }
}

// The same without controls: the pair index gains one zero bit at k, a
// shift and a mask instead of the general insertion.
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep1_plain(T* __restrict__ psi, uint64_t npairs, int k, T u00,
                                                           T u01, T u10, T u11, int sb)
{
    const uint64_t base = xcd_block(sb) * (kThreads * P) + threadIdx.x;
    const uint64_t kb = 1ull << k, lo = kb - 1;
    T x[P], y[P];
    uint64_t i0[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        i0[r] = ((p & ~lo) << 1) | (p & lo);
        if (p < npairs) {
            x[r] = ld_nt(psi + i0[r]);
            y[r] = ld_nt(psi + (i0[r] | kb));
        }
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        if (p < npairs) {
            st_nt(psi + i0[r], cmul2(u00, x[r], u01, y[r]));
            st_nt(psi + (i0[r] | kb), cmul2(u10, x[r], u11, y[r]));
        }
    }
}

// Low targets without controls (2^k <= 32): every lane loads one amplitude,
// so each wave reads and writes whole contiguous runs, and takes the
// partner amplitude i ^ 2^k from lane (lane ^ 2^k) of the same wave. Each
// lane computes its own output row of Eq. 5.
template <typename T>
__device__ __forceinline__ T shfl_xor_amp(T v, int m)
{
    T r;
    if constexpr (sizeof(T) == 16) {
        r.x = __shfl_xor(v.x, m, 64);
        r.y = __shfl_xor(v.y, m, 64);
    } else {
        r.x = __shfl_xor(v.x, m, 64);
        r.y = __shfl_xor(v.y, m, 64);
    }
    return r;
}

template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep1_lane(T* __restrict__ psi, uint64_t N, int k, T u00, T u01,
                                                          T u10, T u11)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
    const int m = 1 << k;
    const bool hi = (threadIdx.x & m) != 0;  // bit k of the index (kThreads is a multiple of 2^k)
    // row of Eq. 5 this lane produces: own amplitude x, partner y
    const T a_own = hi ? u11 : u00, a_par = hi ? u10 : u01;
    T v[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        if (i < N) v[r] = ld_nt(psi + i);
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        const T y = shfl_xor_amp(v[r], m);  // every lane takes part in the shuffle
        if (i < N) st_nt(psi + i, cmul2(a_own, v[r], a_par, y));
    }
}

// Gates whose qubits (targets and controls) all lie among the lowest five:
// their pairs and quadruples sit inside groups of 32 lanes, and a sweep over
// only the touched amplitudes would use a fraction of each 128-byte line.
// One coalesced pass instead: every lane loads its amplitude, takes the
// partners of its quadruple by lane shuffles, writes its own output row, and
// writes its amplitude back unchanged where the controls are not all 1.
// KIND 0: 2x2 on qa; KIND 1: 4x4 on (qa, qc), index bit(qa) + 2 bit(qc);
// KIND 2: diagonal d[bit(qa) + 2 bit(qc)] (qa / qc < 0: bit 0).
constexpr int kLaneQubits = 5;

// A 4x4 (or 2x2, or diagonal) complex matrix by value, (re, im) pairs.
struct Mat4 {
    double v[32];
};

template <typename T, int P, int KIND>
__global__ __launch_bounds__(kThreads) void k_gate_lane(T* __restrict__ psi, uint64_t N, int qa, int qc,
                                                        uint32_t ctrl, Mat4 m)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
    using R = typename RealOf<T>::type;
    auto U = [&](int e) {
        T u;
        u.x = (R)m.v[2 * e];
        u.y = (R)m.v[2 * e + 1];
        return u;
    };
    const uint32_t li = threadIdx.x;  // the index's low bits (kThreads is a multiple of 32)
    const bool on = (li & ctrl) == ctrl;
    const int ba = qa >= 0 ? (int)((li >> qa) & 1) : 0;
    const int bc = qc >= 0 ? (int)((li >> qc) & 1) : 0;
    const int row = ba + 2 * bc;
    T v[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        if (i < N) v[r] = ld_nt(psi + i);
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        T out = v[r];
        if constexpr (KIND == 0) {
            const T y = shfl_xor_amp(v[r], 1 << qa);  // every lane takes part in the shuffle
            const T own = ba ? U(3) : U(0), par = ba ? U(2) : U(1);
            if (on) out = cmul2(own, v[r], par, y);
        } else if constexpr (KIND == 1) {
            // x[e] for e = row ^ f: the partner across the bits set in f
            const T p1 = shfl_xor_amp(v[r], 1 << qa), p2 = shfl_xor_amp(v[r], 1 << qc),
                    p3 = shfl_xor_amp(v[r], (1 << qa) | (1 << qc));
            if (on) {
                const T a0 = cmul2(U(4 * row + row), v[r], U(4 * row + (row ^ 1)), p1);
                const T a1 = cmul2(U(4 * row + (row ^ 2)), p2, U(4 * row + (row ^ 3)), p3);
                out.x = a0.x + a1.x;
                out.y = a0.y + a1.y;
            }
        } else {
            if (on) out = cmul(U(row), v[r]);
        }
        if (i < N) st_nt(psi + i, out);
    }
}

// True when every qubit of g (targets and controls) is below kLaneQubits and
// the state has whole waves of amplitudes.
static bool lane_gate(const HostGate& g, int n)
{
    uint64_t bits = g.ctrl;
    if (g.q[0] >= 0) bits |= 1ull << g.q[0];
    if (g.q[1] >= 0) bits |= 1ull << g.q[1];
    return n >= 8 && (bits >> kLaneQubits) == 0;
}

template <typename T, int KIND>
static hipError_t launch_gate_lane(T* psi, int n, const HostGate& g, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    Mat4 m{};
    const int cnt = KIND == 0 ? 4 : KIND == 1 ? 16 : 4;
    for (int e = 0; e < cnt; e++) {
        m.v[2 * e] = g.m[e].real();
        m.v[2 * e + 1] = g.m[e].imag();
    }
    with_per_thread(N, 1, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_gate_lane<T, P, KIND>), dim3(grid_for(N, kThreads * P)), dim3(kThreads), 0, st, psi,
                           N, g.q[0], g.q[1], (uint32_t)g.ctrl, m);
    });
    return hipGetLastError();
}

// Index bit that takes the XCD index (xcd_block) in a one-qubit sweep on
// target k, controlled or not (mask: the target and control bits), from
// sweeps of every split bit against every target and several control /
// target pairs at 29 qubits on MI355X, complex128 and complex64. A partner
// 8 MiB or more away (partner byte bit X >= 23) runs best with the split on
// amplitude byte bit 17 + (X mod 4): 6.0-6.5 TB/s, where the dispatch order
// gives 5.5-5.9 and a split chosen without regard to X drops to 5.2-5.7 for
// one X in two. Other partners, and a control on that bit, take index bit
// 15 (6.1-6.7 TB/s), or 16 at X = 20 (6.19 against 5.94 TB/s).
static int sweep_xcd_bit(int k, uint64_t mask, size_t elem)
{
    const int eb = elem == 16 ? 4 : 3;  // log2 of the amplitude's bytes
    const int X = k + eb;
    if (X >= 23) {
        const int A = 17 + (X & 3) - eb;  // amplitude bit
        if (!((mask >> A) & 1)) return A - __builtin_popcountll(mask & ((1ull << A) - 1));
    }
    return X == 20 ? 16 : 15;
}

// xcd_block's sb for index bit `bit` with P items per thread, or -1 where the
// grid is too small to be cut that way.
static int xcd_shift(int bit, int P, unsigned grid)
{
    const int sb = bit - 8 - __builtin_ctz(P);
    return (sb < 0 || grid % (8u << sb) != 0) ? -1 : sb;
}

template <typename T>
hipError_t launch_sweep1(T* psi, int n, const HostGate& g, hipStream_t st)
{
    if (g.ctrl != 0 && lane_gate(g, n)) return launch_gate_lane<T, 0>(psi, n, g, st);
    // Measured on MI355X at 29 qubits: one amplitude per lane with the
    // partner taken by a lane shuffle for targets 0-5 (6.75 TB/s); one pair
    // per thread above, with the eight XCDs' share of the workgroups placed
    // by sweep_xcd_bit (6.0-6.7 TB/s against 5.6-5.85 with the dispatch
    // order and one or four pairs per thread). Without such a split (small
    // grids), four pairs per thread once the partner stride reaches 2^20.
    const int k = g.q[0];
    const uint64_t mask = g.ctrl | (1ull << k);
    const Ins ins = make_ins(mask);
    const uint64_t npairs = 1ull << (n - ins.cnt);
    const T u00 = to_dev<T>(g.m[0]), u01 = to_dev<T>(g.m[1]), u10 = to_dev<T>(g.m[2]), u11 = to_dev<T>(g.m[3]);
    const int bit = sweep_xcd_bit(k, mask, sizeof(T));
    const bool split = xcd_shift(bit, 1, grid_for(npairs, kThreads)) >= 0;
    if (g.ctrl == 0 && k < 6 && n >= 8) {
        const uint64_t N = 1ull << n;
        with_per_thread(N, 1, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            hipLaunchKernelGGL((k_sweep1_lane<T, P>), dim3(grid_for(N, kThreads * P)), dim3(kThreads), 0, st, psi,
                               N, k, u00, u01, u10, u11);
        });
    } else if (g.ctrl == 0) {
        with_per_thread(npairs, split || k < 20 ? 1 : 4, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            const unsigned grid = grid_for(npairs, kThreads * P);
            hipLaunchKernelGGL((k_sweep1_plain<T, P>), dim3(grid), dim3(kThreads), 0, st, psi, npairs, k, u00, u01,
                               u10, u11, xcd_shift(bit, P, grid));
        });
    } else {
        with_per_thread(npairs, split || k < 20 ? 1 : 4, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            const unsigned grid = grid_for(npairs, kThreads * P);
            hipLaunchKernelGGL((k_sweep1<T, P>), dim3(grid), dim3(kThreads), 0, st, psi, npairs, k, ins, g.ctrl,
                               u00, u01, u10, u11, xcd_shift(bit, P, grid));
        });
    }
    return hipGetLastError();
}

// ------------------------------------------------------ two-qubit sweep ---
// 4x4 update of every quadruple {i, i|2^a, i|2^c, i|2^a|2^c} with bits a, c
// of i clear (index bit(a) + 2 bit(c)) and all control bits set.


template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep2(T* __restrict__ psi, uint64_t nquads, int qa, int qc,
                                                     Ins ins, uint64_t ctrl, Mat4 m)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
    const uint64_t ba = 1ull << qa, bc = 1ull << qc;
    T u[16];
#pragma unroll
    for (int e = 0; e < 16; e++) {
        u[e].x = (typename RealOf<T>::type)m.v[2 * e];
        u[e].y = (typename RealOf<T>::type)m.v[2 * e + 1];
    }
    T v[P][4];
    uint64_t i0[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        i0[r] = insert_zeros(p < nquads ? p : 0, ins) | ctrl;
        if (p < nquads) {
            v[r][0] = ld_nt(psi + i0[r]);
            v[r][1] = ld_nt(psi + (i0[r] | ba));
            v[r][2] = ld_nt(psi + (i0[r] | bc));
            v[r][3] = ld_nt(psi + (i0[r] | ba | bc));
        }
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        if (p < nquads) {
            T w[4];
#pragma unroll
            for (int row = 0; row < 4; row++) {
                w[row] = cmul2(u[4 * row + 0], v[r][0], u[4 * row + 1], v[r][1]);
                const T t = cmul2(u[4 * row + 2], v[r][2], u[4 * row + 3], v[r][3]);
                w[row].x += t.x;
                w[row].y += t.y;
            }
            st_nt(psi + i0[r], w[0]);
            st_nt(psi + (i0[r] | ba), w[1]);
            st_nt(psi + (i0[r] | bc), w[2]);
            st_nt(psi + (i0[r] | ba | bc), w[3]);
        }
    }
}

// SWAP of qubits a and c (controls allowed): only the amplitudes whose bits
// a and c differ move, so each of the 2^(n-2) pairs (i | 2^a, i | 2^c) with
// bits a, c of i clear is read and written once (2^n amplitudes of traffic,
// half that of a 4x4 sweep).
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep_swap(T* __restrict__ psi, uint64_t npairs, int qa, int qc,
                                                         Ins ins, uint64_t ctrl, int sb)
{
    const uint64_t base = xcd_block(sb) * (kThreads * P) + threadIdx.x;
    const uint64_t ba = 1ull << qa, bc = 1ull << qc;
    T x[P], y[P];
    uint64_t i0[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        i0[r] = insert_zeros(p < npairs ? p : 0, ins) | ctrl;
        if (p < npairs) {
            x[r] = ld_nt(psi + (i0[r] | ba));
            y[r] = ld_nt(psi + (i0[r] | bc));
        }
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        if (p < npairs) {
            st_nt(psi + (i0[r] | ba), y[r]);
            st_nt(psi + (i0[r] | bc), x[r]);
        }
    }
}

static bool is_swap_matrix(const HostGate& g)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            const bool one = (r == c && (r == 0 || r == 3)) || (r == 1 && c == 2) || (r == 2 && c == 1);
            if (g.m[4 * r + c] != cd(one ? 1.0 : 0.0, 0.0)) return false;
        }
    return true;
}

// A general 4x4 (no controls) on one qubit below 6 (ql) and one at 6 or
// above (qh): each lane loads amplitude i (bit qh clear; the 64 lanes of a
// wave hold 64 consecutive indices) and i | 2^qh, takes the ql-partners of
// both by lane shuffles and writes its own two rows, so that every load and
// store instruction of a wave covers a whole contiguous kilobyte (complex128)
// where the quadruple sweep would touch half of each 128-byte line per
// instruction. qa / qc keep the gate's own order: index bit(qa) + 2 bit(qc).
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep2_lane(T* __restrict__ psi, uint64_t nhalf, int ql, int qh,
                                                          bool low_is_a, Mat4 m)
{
    using R = typename RealOf<T>::type;
    auto U = [&](int e) {
        T u;
        u.x = (R)m.v[2 * e];
        u.y = (R)m.v[2 * e + 1];
        return u;
    };
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
    const uint64_t hb = 1ull << qh, lo = hb - 1;
    const int bl = (int)((threadIdx.x >> ql) & 1);  // bit ql of the index (kThreads is a multiple of 64)
    // quadruple index of (bit ql, bit qh) in the gate's order
    auto idx = [&](int l, int h) { return low_is_a ? l + 2 * h : h + 2 * l; };
    T v0[P] = {}, v1[P] = {};
    uint64_t i0[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        i0[r] = ((p & ~lo) << 1) | (p & lo);
        if (p < nhalf) {
            v0[r] = ld_nt(psi + i0[r]);
            v1[r] = ld_nt(psi + (i0[r] | hb));
        }
    }
    const int r0 = idx(bl, 0), r1 = idx(bl, 1);  // this lane's two output rows
    const int c_own0 = idx(bl, 0), c_own1 = idx(bl, 1), c_par0 = idx(bl ^ 1, 0), c_par1 = idx(bl ^ 1, 1);
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        const T p0 = shfl_xor_amp(v0[r], 1 << ql), p1 = shfl_xor_amp(v1[r], 1 << ql);  // every lane shuffles
        const T a0 = cmul2(U(4 * r0 + c_own0), v0[r], U(4 * r0 + c_par0), p0);
        const T b0 = cmul2(U(4 * r0 + c_own1), v1[r], U(4 * r0 + c_par1), p1);
        const T a1 = cmul2(U(4 * r1 + c_own0), v0[r], U(4 * r1 + c_par0), p0);
        const T b1 = cmul2(U(4 * r1 + c_own1), v1[r], U(4 * r1 + c_par1), p1);
        T o0, o1;
        o0.x = a0.x + b0.x;
        o0.y = a0.y + b0.y;
        o1.x = a1.x + b1.x;
        o1.y = a1.y + b1.y;
        if (p < nhalf) {
            st_nt(psi + i0[r], o0);
            st_nt(psi + (i0[r] | hb), o1);
        }
    }
}

template <typename T>
hipError_t launch_sweep2(T* psi, int n, const HostGate& g, hipStream_t st)
{
    if (lane_gate(g, n)) return launch_gate_lane<T, 1>(psi, n, g, st);
    if (is_swap_matrix(g)) {
        const Ins ins = make_ins(g.ctrl | (1ull << g.q[0]) | (1ull << g.q[1]));
        const uint64_t npairs = 1ull << (n - ins.cnt);
        // XCD placement as for the one-qubit sweeps, keyed on the higher
        // qubit; where both qubits' byte bits agree mod 4 (no placement
        // separates them), index bit 15. Measured at 29 qubits complex128:
        // (11,20) 5.46 -> 6.09, (20,28) 5.26 -> 5.49, (27,5) 5.59 -> 6.05,
        // (2,11) 3.63 -> 3.85 TB/s against two pairs per thread in dispatch
        // order.
        const int qh = g.q[0] > g.q[1] ? g.q[0] : g.q[1], ql = g.q[0] > g.q[1] ? g.q[1] : g.q[0];
        const int eb = sizeof(T) == 16 ? 4 : 3;
        const int bit = ((qh + eb) & 3) == ((ql + eb) & 3)
                            ? 15
                            : sweep_xcd_bit(qh, g.ctrl | (1ull << g.q[0]) | (1ull << g.q[1]), sizeof(T));
        const bool split = xcd_shift(bit, 1, grid_for(npairs, kThreads)) >= 0;
        with_per_thread(npairs, split ? 1 : 2, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            const unsigned grid = grid_for(npairs, kThreads * P);
            hipLaunchKernelGGL((k_sweep_swap<T, P>), dim3(grid), dim3(kThreads), 0, st, psi, npairs, g.q[0], g.q[1],
                               ins, g.ctrl, split ? xcd_shift(bit, P, grid) : -1);
        });
        return hipGetLastError();
    }
    const uint64_t mask = g.ctrl | (1ull << g.q[0]) | (1ull << g.q[1]);
    const Ins ins = make_ins(mask);
    const uint64_t nquads = 1ull << (n - ins.cnt);
    Mat4 m;
    for (int e = 0; e < 16; e++) {
        m.v[2 * e] = g.m[e].real();
        m.v[2 * e + 1] = g.m[e].imag();
    }
    const int qlo = g.q[0] < g.q[1] ? g.q[0] : g.q[1], qhi = g.q[0] < g.q[1] ? g.q[1] : g.q[0];
    if (g.ctrl == 0 && qlo < 6 && qhi >= 6 && n >= 8) {
        const uint64_t nhalf = 1ull << (n - 1);
        with_per_thread(nhalf, 1, [&](auto pc) {
            constexpr int P = decltype(pc)::value;
            hipLaunchKernelGGL((k_sweep2_lane<T, P>), dim3(grid_for(nhalf, kThreads * P)), dim3(kThreads), 0, st,
                               psi, nhalf, qlo, qhi, g.q[0] == qlo, m);
        });
        return hipGetLastError();
    }
    // 4 quadruples per thread when both qubits are 11 or above (measured 2-3%
    // faster there at 29 qubits), 2 otherwise
    with_per_thread(nquads, qlo >= 11 ? 4 : 2, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_sweep2<T, P>), dim3(grid_for(nquads, kThreads * P)), dim3(kThreads), 0, st, psi,
                           nquads, g.q[0], g.q[1], ins, g.ctrl, m);
    });
    return hipGetLastError();
}

// ------------------------------------------------------- diagonal sweep ---
// alpha_i *= d[bit(qa) + 2 bit(qc)] over the subspace where every control
// bit is 1 (qa / qc < 0: bit taken as 0). Only that subspace is touched.

template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_sweep_diag(T* __restrict__ psi, uint64_t count, Ins ins,
                                                         uint64_t ctrl, int qa, int qc, T d0, T d1, T d2v, T d3,
                                                         int sb)
{
    const uint64_t base = xcd_block(sb) * (kThreads * P) + threadIdx.x;
    T v[P];
    uint64_t idx[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        idx[r] = insert_zeros(p < count ? p : 0, ins) | ctrl;
        if (p < count) v[r] = ld_nt(psi + idx[r]);
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t p = base + (uint64_t)r * kThreads;
        if (p < count) {
            const int ba = qa >= 0 ? (int)((idx[r] >> qa) & 1) : 0;
            const int bc = qc >= 0 ? (int)((idx[r] >> qc) & 1) : 0;
            const int s = ba + 2 * bc;
            const T d = s == 0 ? d0 : s == 1 ? d1 : s == 2 ? d2v : d3;
            st_nt(psi + idx[r], cmul(d, v[r]));
        }
    }
}

template <typename T>
hipError_t launch_sweep_diag(T* psi, int n, const HostGate& g, hipStream_t st)
{
    if (lane_gate(g, n)) return launch_gate_lane<T, 2>(psi, n, g, st);
    const Ins ins = make_ins(g.ctrl);
    const uint64_t count = 1ull << (n - ins.cnt);
    // One amplitude per thread with each XCD's workgroups on index bit 15
    // (as for the one-qubit sweeps' near partners): CZ and CP on (11,20),
    // (20,28), (27,5) 5.4-5.9 -> 6.4-6.6 TB/s, on (2,11) 2.75 -> 3.43 TB/s of
    // their algorithmic bytes, against four per thread in dispatch order.
    const int bit = 15;
    const bool split = xcd_shift(bit, 1, grid_for(count, kThreads)) >= 0;
    with_per_thread(count, split ? 1 : 4, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const unsigned grid = grid_for(count, kThreads * P);
        hipLaunchKernelGGL((k_sweep_diag<T, P>), dim3(grid), dim3(kThreads), 0, st, psi, count, ins, g.ctrl, g.q[0],
                           g.q[1], to_dev<T>(g.m[0]), to_dev<T>(g.m[1]), to_dev<T>(g.m[2]), to_dev<T>(g.m[3]),
                           split ? xcd_shift(bit, P, grid) : -1);
    });
    return hipGetLastError();
}

// ------------------------------------------------------------ block pass ---
// One workgroup per block of 2^b amplitudes whose indices share the bits of
// the qubits outside the block (the block's base) and range over all values
// of the b local qubits hdr->local_q[0..b). The block is staged in LDS, the
// pass's ops are applied in order with a barrier between them, and the block
// is written back: one HBM round trip for the whole run of gates. With
// NS == 2 every op acts on two states (phi and lambda of the adjoint sweep)
// and T_GRAD ops write per-block partials of Im <lambda|G|phi>.

template <typename T, int LB, int NS>
__global__ __launch_bounds__(kThreads) void k_block(T* __restrict__ s0, T* __restrict__ s1,
                                                    const PassHdr* __restrict__ hdr,
                                                    const TileOp* __restrict__ ops, const T* __restrict__ mats,
                                                    double* __restrict__ gpart, int64_t gstride)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* lds0 = reinterpret_cast<T*>(smem_raw);
    T* lds1 = lds0 + (1 << LB);
    __shared__ double red[kThreads / 64];

    const int b = hdr->b;
    const int nloc = 1 << b;
    const int tid = threadIdx.x;
    const uint64_t blk = blockIdx.x;

    uint64_t base = 0;
    for (int j = 0; j < hdr->n_outer; j++) base |= ((blk >> j) & 1ull) << hdr->outer_q[j];

    // Global offset of local index l = tid + 256 r: low 8 bits are tid's.
    uint64_t dlo = 0;
    const int blo = b < 8 ? b : 8;
    for (int j = 0; j < blo; j++) dlo |= (uint64_t)((tid >> j) & 1) << hdr->local_q[j];

    constexpr int U = 8;
    for (int l0 = 0; l0 < nloc; l0 += kThreads * U) {
        T v0[U], v1[U];
        uint64_t g[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int l = l0 + u * kThreads + tid;
            uint64_t dhi = 0;
            const int r = l >> 8;
            for (int j = 8; j < b; j++) dhi |= (uint64_t)((r >> (j - 8)) & 1) << hdr->local_q[j];
            g[u] = base | dlo | dhi;
            if (l < nloc) {
                v0[u] = ld_nt(s0 + g[u]);
                if (NS == 2) v1[u] = ld_nt(s1 + g[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int l = l0 + u * kThreads + tid;
            if (l < nloc) {
                lds0[l] = v0[u];
                if (NS == 2) lds1[l] = v1[u];
            }
        }
    }
    __syncthreads();

    const int n_ops = hdr->n_ops;
    const TileOp* po = ops + hdr->op_begin;
    for (int o = 0; o < n_ops; o++) {
        const TileOp op = po[o];
        if ((base & op.gctrl) != op.gctrl) continue;  // uniform over the block
        const uint32_t lc = op.lctrl;
        if (op.kind == T_DENSE1) {
            const T u00 = mats[op.mat], u01 = mats[op.mat + 1], u10 = mats[op.mat + 2], u11 = mats[op.mat + 3];
            const int a = op.a;
            const int lowm = (1 << a) - 1;
            for (int p = tid; p < (nloc >> 1); p += kThreads) {
                const int i0 = ((p & ~lowm) << 1) | (p & lowm);
                if ((i0 & lc) != lc) continue;
                const int i1 = i0 | (1 << a);
                {
                    const T x = lds0[i0], y = lds0[i1];
                    lds0[i0] = cmul2(u00, x, u01, y);
                    lds0[i1] = cmul2(u10, x, u11, y);
                }
                if (NS == 2) {
                    const T x = lds1[i0], y = lds1[i1];
                    lds1[i0] = cmul2(u00, x, u01, y);
                    lds1[i1] = cmul2(u10, x, u11, y);
                }
            }
        } else if (op.kind == T_XPERM) {
            const int a = op.a;
            const int lowm = (1 << a) - 1;
            for (int p = tid; p < (nloc >> 1); p += kThreads) {
                const int i0 = ((p & ~lowm) << 1) | (p & lowm);
                if ((i0 & lc) != lc) continue;
                const int i1 = i0 | (1 << a);
                const T x = lds0[i0];
                lds0[i0] = lds0[i1];
                lds0[i1] = x;
                if (NS == 2) {
                    const T y = lds1[i0];
                    lds1[i0] = lds1[i1];
                    lds1[i1] = y;
                }
            }
        } else if (op.kind == T_SWAP) {
            const int a = op.a, c = op.c;
            const int lo = a < c ? a : c, hi = a < c ? c : a;
            const int mlo = (1 << lo) - 1, mhi = (1 << hi) - 1;
            for (int p = tid; p < (nloc >> 2); p += kThreads) {
                int i0 = ((p & ~mlo) << 1) | (p & mlo);
                i0 = ((i0 & ~mhi) << 1) | (i0 & mhi);
                if ((i0 & lc) != lc) continue;
                const int ia = i0 | (1 << a), ic = i0 | (1 << c);
                const T x = lds0[ia];
                lds0[ia] = lds0[ic];
                lds0[ic] = x;
                if (NS == 2) {
                    const T y = lds1[ia];
                    lds1[ia] = lds1[ic];
                    lds1[ic] = y;
                }
            }
        } else if (op.kind == T_DENSE2) {
            const int a = op.a, c = op.c;
            const int lo = a < c ? a : c, hi = a < c ? c : a;
            const int mlo = (1 << lo) - 1, mhi = (1 << hi) - 1;
            for (int p = tid; p < (nloc >> 2); p += kThreads) {
                int i0 = ((p & ~mlo) << 1) | (p & mlo);
                i0 = ((i0 & ~mhi) << 1) | (i0 & mhi);
                if ((i0 & lc) != lc) continue;
                const int idx[4] = {i0, i0 | (1 << a), i0 | (1 << c), i0 | (1 << a) | (1 << c)};
#pragma unroll
                for (int s = 0; s < NS; s++) {
                    T* L = s == 0 ? lds0 : lds1;
                    T v[4], w[4];
#pragma unroll
                    for (int e = 0; e < 4; e++) v[e] = L[idx[e]];
#pragma unroll
                    for (int row = 0; row < 4; row++) {
                        w[row] = cmul2(mats[op.mat + 4 * row], v[0], mats[op.mat + 4 * row + 1], v[1]);
                        const T t = cmul2(mats[op.mat + 4 * row + 2], v[2], mats[op.mat + 4 * row + 3], v[3]);
                        w[row].x += t.x;
                        w[row].y += t.y;
                    }
#pragma unroll
                    for (int e = 0; e < 4; e++) L[idx[e]] = w[e];
                }
            }
        } else if (op.kind == T_DIAG) {
            const T d0 = mats[op.mat], d1 = mats[op.mat + 1], dd2 = mats[op.mat + 2], d3 = mats[op.mat + 3];
            const int a = op.a, c = op.c;
            const int ua = a < 0 ? (op.oa >= 0 ? (int)((base >> op.oa) & 1) : 0) : 0;
            const int uc = c < 0 ? (op.oc >= 0 ? (int)((base >> op.oc) & 1) : 0) : 0;
            for (int l = tid; l < nloc; l += kThreads) {
                if ((l & lc) != lc) continue;
                const int ba = a >= 0 ? ((l >> a) & 1) : ua;
                const int bc = c >= 0 ? ((l >> c) & 1) : uc;
                const int s = ba + 2 * bc;
                const T d = s == 0 ? d0 : s == 1 ? d1 : s == 2 ? dd2 : d3;
                lds0[l] = cmul(d, lds0[l]);
                if (NS == 2) lds1[l] = cmul(d, lds1[l]);
            }
        } else if (NS == 2 && op.kind == T_GRAD) {
            // Im <lambda|G|phi> over the block; s0 = phi, s1 = lambda.
            double acc = 0;
            if (op.gen == GEN_Z) {
                const int a = op.a;
                const int ua = a < 0 ? (int)((base >> op.oa) & 1) : 0;
                for (int l = tid; l < nloc; l += kThreads) {
                    const int bit = a >= 0 ? ((l >> a) & 1) : ua;
                    const T f = lds0[l], m = lds1[l];
                    const double im = (double)m.x * (double)f.y - (double)m.y * (double)f.x;  // Im(conj(m) f)
                    acc += bit ? -im : im;
                }
            } else {
                // G = cx X + cy Y on bit a
                const int a = op.a;
                const double cx = (double)mats[op.mat].x, cy = (double)mats[op.mat].y;
                for (int l = tid; l < nloc; l += kThreads) {
                    const int bit = (l >> a) & 1;
                    const T f = lds0[l ^ (1 << a)], m = lds1[l];
                    // conj(m) * f
                    const double re = (double)m.x * (double)f.x + (double)m.y * (double)f.y;
                    const double im = (double)m.x * (double)f.y - (double)m.y * (double)f.x;
                    // X: (X phi)_l = phi_{l^a}; Y: (Y phi)_l = (bit ? i : -i) phi_{l^a},
                    // and Im(conj(m) * (+-i) f) = +-Re(conj(m) f)
                    acc += cx * im + cy * (bit ? re : -re);
                }
            }
            const double t = block_sum(acc, red);
            if (tid == 0) gpart[(int64_t)op.slot * gstride + (int64_t)blk] = t;
        }
        __syncthreads();
    }

    for (int l0 = 0; l0 < nloc; l0 += kThreads * U) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int l = l0 + u * kThreads + tid;
            if (l < nloc) {
                uint64_t dhi = 0;
                const int r = l >> 8;
                for (int j = 8; j < b; j++) dhi |= (uint64_t)((r >> (j - 8)) & 1) << hdr->local_q[j];
                const uint64_t g = base | dlo | dhi;
                st_nt(s0 + g, lds0[l]);
                if (NS == 2) st_nt(s1 + g, lds1[l]);
            }
        }
    }
}

template <typename T>
constexpr int block_lb(int ns)
{
    // 64 KiB of LDS per workgroup: two workgroups fit one CU's 160 KiB.
    return (sizeof(T) == 16 ? 12 : 13) - (ns == 2 ? 1 : 0);
}

template <typename T, int LB, int NS>
static hipError_t launch_block_t(T* s0, T* s1, int n, const PassHdr* d_hdr, const TileOp* d_ops, const T* d_mats,
                                 int b, double* gp, int64_t gs, hipStream_t st)
{
    static bool attr_set = false;
    const size_t lds = (size_t)NS * ((size_t)1 << LB) * sizeof(T);
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_block<T, LB, NS>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const uint64_t nblocks = 1ull << (n - b);
    hipLaunchKernelGGL((k_block<T, LB, NS>), dim3((unsigned)nblocks), dim3(kThreads), lds, st, s0, s1, d_hdr,
                       d_ops, d_mats, gp, gs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_block_pass(T* s0, T* s1, int n, int n_states, const PassHdr* d_hdr, const TileOp* d_ops,
                             const T* d_mats, int b, double* gp, int64_t gs, hipStream_t st)
{
    if (b > block_lb<T>(n_states)) return hipErrorInvalidValue;  // the block must fit the kernel's LDS
    if (n_states == 2)
        return launch_block_t<T, block_lb<T>(2), 2>(s0, s1, n, d_hdr, d_ops, d_mats, b, gp, gs, st);
    return launch_block_t<T, block_lb<T>(1), 1>(s0, s1, n, d_hdr, d_ops, d_mats, b, gp, gs, st);
}

// ------------------------------------------------------------ reductions ---
// Fixed grid of kReduceBlocks workgroups with a grid-stride loop: every
// thread sums a fixed set of indices in a fixed order, so the partials (and
// the final sums) are bit-reproducible run to run.

template <typename T>
__device__ __forceinline__ void to_double(T v, double& re, double& im)
{
    re = (double)v.x;
    im = (double)v.y;
}

// Per term t (all sharing x_mask): coeff_t * Re(i^{#Y} sum_j (-1)^{|j & z_t|} conj(a_{j^x}) a_j)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pauli_expect(const T* __restrict__ psi, int n, TermBatch tb,
                                                           double* __restrict__ partials)
{
    __shared__ double red[kThreads / 64];
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    double acc = 0;
    if (tb.x_mask == 0) {
        for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < N; j += stride) {
            double re, im;
            to_double(psi[j], re, im);
            const double w = re * re + im * im;
            double s = 0;
            for (int t = 0; t < tb.n_terms; t++) s += (__popcll(j & tb.z_mask[t]) & 1) ? -tb.coeff_re[t] : tb.coeff_re[t];
            acc += w * s;
        }
    } else {
        const int h = 63 - __clzll(tb.x_mask);
        const uint64_t hm = (1ull << h) - 1;
        for (uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x; p < (N >> 1); p += stride) {
            const uint64_t j = ((p & ~hm) << 1) | (p & hm);
            const uint64_t j2 = j ^ tb.x_mask;
            double ar, ai, br, bi;
            to_double(psi[j], ar, ai);
            to_double(psi[j2], br, bi);
            // q = conj(b) * a
            const double qr = br * ar + bi * ai, qi = br * ai - bi * ar;
            for (int t = 0; t < tb.n_terms; t++) {
                const double s1 = (__popcll(j & tb.z_mask[t]) & 1) ? -1.0 : 1.0;
                const double s2 = (__popcll(j2 & tb.z_mask[t]) & 1) ? -1.0 : 1.0;
                // Re(c s1 q + c s2 conj(q)), c = coeff_re + i coeff_im
                acc += s1 * (tb.coeff_re[t] * qr - tb.coeff_im[t] * qi) + s2 * (tb.coeff_re[t] * qr + tb.coeff_im[t] * qi);
            }
        }
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_pauli_expect(const T* psi, int n, const TermBatch& tb, double* partials, int n_part, hipStream_t st)
{
    hipLaunchKernelGGL((k_pauli_expect<T>), dim3(n_part), dim3(kThreads), 0, st, psi, n, tb, partials);
    return hipGetLastError();
}

// dst_j (+)= sum_t c_t (P_t psi)_j with (P psi)_j = i^{#Y} (-1)^{|j2 & z|} psi_{j2}, j2 = j ^ x.
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_pauli_apply(const T* __restrict__ psi, T* __restrict__ dst, int n,
                                                          TermBatch tb, int accumulate)
{
    const uint64_t N = 1ull << n;
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t j = base + (uint64_t)r * kThreads;
        if (j >= N) continue;
        const uint64_t j2 = j ^ tb.x_mask;
        double vr, vi;
        to_double(psi[j2], vr, vi);
        double cr = 0, ci = 0;
        for (int t = 0; t < tb.n_terms; t++) {
            const double s = (__popcll(j2 & tb.z_mask[t]) & 1) ? -1.0 : 1.0;
            cr += s * tb.coeff_re[t];
            ci += s * tb.coeff_im[t];
        }
        double outr = cr * vr - ci * vi, outi = cr * vi + ci * vr;
        if (accumulate) {
            double dr, di;
            to_double(dst[j], dr, di);
            outr += dr;
            outi += di;
        }
        T o;
        o.x = (typename RealOf<T>::type)outr;
        o.y = (typename RealOf<T>::type)outi;
        dst[j] = o;
    }
}

template <typename T>
hipError_t launch_pauli_apply(const T* psi, T* dst, int n, const TermBatch& tb, bool accumulate, hipStream_t st)
{
    with_per_thread(1ull << n, 4, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_pauli_apply<T, P>), dim3(grid_for(1ull << n, kThreads * P)), dim3(kThreads), 0, st,
                           psi, dst, n, tb, accumulate ? 1 : 0);
    });
    return hipGetLastError();
}

// The same for up to kBatchesPerLaunch x-mask groups in one pass: every
// output sums its terms from all the groups in FP64 registers and is written
// once (added to dst when accumulating).
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_pauli_apply_multi(const T* __restrict__ psi, T* __restrict__ dst,
                                                                int n, TermBatchSet set, int accumulate)
{
    const uint64_t N = 1ull << n;
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t j = base + (uint64_t)r * kThreads;
        if (j >= N) continue;
        double outr = 0, outi = 0;
        if (accumulate) to_double(dst[j], outr, outi);
        for (int b = 0; b < set.count; b++) {
            const TermBatch& tb = set.b[b];
            const uint64_t j2 = j ^ tb.x_mask;
            double vr, vi;
            to_double(psi[j2], vr, vi);
            double cr = 0, ci = 0;
            for (int t = 0; t < tb.n_terms; t++) {
                const double sg = (__popcll(j2 & tb.z_mask[t]) & 1) ? -1.0 : 1.0;
                cr += sg * tb.coeff_re[t];
                ci += sg * tb.coeff_im[t];
            }
            outr += cr * vr - ci * vi;
            outi += cr * vi + ci * vr;
        }
        T o;
        o.x = (typename RealOf<T>::type)outr;
        o.y = (typename RealOf<T>::type)outi;
        dst[j] = o;
    }
}

template <typename T>
hipError_t launch_pauli_apply_multi(const T* psi, T* dst, int n, const TermBatch* batches, int count,
                                    bool accumulate, hipStream_t st)
{
    if (count < 1 || count > kBatchesPerLaunch) return hipErrorInvalidValue;
    TermBatchSet set{};
    set.count = count;
    for (int b = 0; b < count; b++) set.b[b] = batches[b];
    with_per_thread(1ull << n, 4, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_pauli_apply_multi<T, P>), dim3(grid_for(1ull << n, kThreads * P)), dim3(kThreads), 0,
                           st, psi, dst, n, set, accumulate ? 1 : 0);
    });
    return hipGetLastError();
}

// <a|b> = sum conj(a_j) b_j -> partials rows 0 (re) and 1 (im), n_part each.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_inner(const T* __restrict__ a, const T* __restrict__ b, int n,
                                                    double* __restrict__ partials, int n_part)
{
    __shared__ double red[kThreads / 64];
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    double sr = 0, si = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < N; j += stride) {
        double ar, ai, br, bi;
        to_double(a[j], ar, ai);
        to_double(b[j], br, bi);
        sr += ar * br + ai * bi;
        si += ar * bi - ai * br;
    }
    const double tr = block_sum(sr, red);
    const double ti = block_sum(si, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = tr;
        partials[n_part + blockIdx.x] = ti;
    }
}

template <typename T>
hipError_t launch_inner(const T* a, const T* b, int n, double* partials, int n_part, hipStream_t st)
{
    hipLaunchKernelGGL((k_inner<T>), dim3(n_part), dim3(kThreads), 0, st, a, b, n, partials, n_part);
    return hipGetLastError();
}

// Im <lam|G|phi> for G = X/Y/Z on qubit q.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_grad_sweep(const T* __restrict__ phi, const T* __restrict__ lam, int n,
                                                         int q, int gen, double* __restrict__ partials)
{
    __shared__ double red[kThreads / 64];
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    const uint64_t qb = 1ull << q;
    double acc = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < N; j += stride) {
        const int bit = (j & qb) ? 1 : 0;
        double fr, fi, mr, mi;
        to_double(phi[gen == GEN_Z ? j : (j ^ qb)], fr, fi);
        to_double(lam[j], mr, mi);
        const double re = mr * fr + mi * fi, im = mr * fi - mi * fr;
        if (gen == GEN_Z) acc += bit ? -im : im;
        else if (gen == GEN_X) acc += im;
        else acc += bit ? re : -re;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_grad_sweep(const T* phi, const T* lam, int n, int q, int gen, double* partials, int n_part,
                             hipStream_t st)
{
    hipLaunchKernelGGL((k_grad_sweep<T>), dim3(n_part), dim3(kThreads), 0, st, phi, lam, n, q, gen, partials);
    return hipGetLastError();
}

// Six rows of partials: max |a-b|, sum |a-b|^2, Re<a|b>, Im<a|b>, <a|a>, <b|b>.
template <typename Ta, typename Tb>
__global__ __launch_bounds__(kThreads) void k_compare(const Ta* __restrict__ a, const Tb* __restrict__ b, int n,
                                                      double* __restrict__ partials, int n_part)
{
    __shared__ double red[kThreads / 64];
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    double mx = 0, d2s = 0, ir = 0, ii = 0, na = 0, nb = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < N; j += stride) {
        double ar, ai, br, bi;
        to_double(a[j], ar, ai);
        to_double(b[j], br, bi);
        const double dr = ar - br, di = ai - bi;
        const double dd = dr * dr + di * di;
        mx = fmax(mx, sqrt(dd));
        d2s += dd;
        ir += ar * br + ai * bi;
        ii += ar * bi - ai * br;
        na += ar * ar + ai * ai;
        nb += br * br + bi * bi;
    }
    const double vals[6] = {block_max(mx, red), block_sum(d2s, red), block_sum(ir, red),
                            block_sum(ii, red), block_sum(na, red), block_sum(nb, red)};
    if (threadIdx.x == 0)
        for (int r = 0; r < 6; r++) partials[(int64_t)r * n_part + blockIdx.x] = vals[r];
}

template <typename Ta, typename Tb>
hipError_t launch_compare(const Ta* a, const Tb* b, int n, double* partials, int n_part, hipStream_t st)
{
    hipLaunchKernelGGL((k_compare<Ta, Tb>), dim3(n_part), dim3(kThreads), 0, st, a, b, n, partials, n_part);
    return hipGetLastError();
}

// One workgroup per row; fixed-order sum (or max for rows flagged in max_rows).
__global__ __launch_bounds__(kThreads) void k_sum_rows(const double* __restrict__ partials, int64_t count,
                                                       int64_t stride, double* __restrict__ out, int max_row0)
{
    __shared__ double red[kThreads / 64];
    const int row = blockIdx.x;
    const double* p = partials + (int64_t)row * stride;
    const bool is_max = max_row0 && row == 0;
    double acc = 0;
    for (int64_t c = threadIdx.x; c < count; c += kThreads) acc = is_max ? fmax(acc, p[c]) : acc + p[c];
    const double t = is_max ? block_max(acc, red) : block_sum(acc, red);
    if (threadIdx.x == 0) out[row] = t;
}

hipError_t launch_sum_rows(const double* partials, int rows, int64_t count, int64_t stride, double* out,
                           hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_rows, dim3(rows), dim3(kThreads), 0, st, partials, count, stride, out, 0);
    return hipGetLastError();
}

// out[0] = ((0 + rows[0]) + rows[1]) + ... + rows[count - 1]: one thread,
// in index order (the same additions a host loop over the rows makes).
__global__ __launch_bounds__(64) void k_sum_ordered(const double* __restrict__ rows, int count,
                                                    double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double f = 0;
    for (int k = 0; k < count; k++) f += rows[k];
    out[0] = f;
}

hipError_t launch_sum_ordered(const double* rows, int count, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(64), 0, st, rows, count, out);
    return hipGetLastError();
}

hipError_t launch_compare_finish(const double* partials, int n_part, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_rows, dim3(6), dim3(kThreads), 0, st, partials, (int64_t)n_part, (int64_t)n_part, out,
                       1);
    return hipGetLastError();
}

// ------------------------------------------------------------------ copy ---

template <int P>
__global__ __launch_bounds__(kThreads) void k_copy(d2* __restrict__ dst, const d2* __restrict__ src, uint64_t n16)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * P) + threadIdx.x;
    d2 v[P];
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        if (i < n16) v[r] = ld_nt(src + i);
    }
#pragma unroll
    for (int r = 0; r < P; r++) {
        const uint64_t i = base + (uint64_t)r * kThreads;
        if (i < n16) st_nt(dst + i, v[r]);
    }
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    // one element per thread while the grid allows: 6.6 TB/s on MI355X, against 5.8 with 4
    const uint64_t n16 = bytes / 16;
    with_per_thread(n16, 1, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        hipLaunchKernelGGL((k_copy<P>), dim3(grid_for(n16, kThreads * P)), dim3(kThreads), 0, st,
                           reinterpret_cast<d2*>(dst), reinterpret_cast<const d2*>(src), n16);
    });
    return hipGetLastError();
}

// --------------------------------------------------------- instantiation ---

#define QV_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_init_basis<T>(T*, int, uint64_t, hipStream_t);                               \
    template hipError_t launch_sweep1<T>(T*, int, const HostGate&, hipStream_t);                            \
    template hipError_t launch_sweep2<T>(T*, int, const HostGate&, hipStream_t);                            \
    template hipError_t launch_sweep_diag<T>(T*, int, const HostGate&, hipStream_t);                        \
    template hipError_t launch_block_pass<T>(T*, T*, int, int, const PassHdr*, const TileOp*, const T*, int, \
                                             double*, int64_t, hipStream_t);                                \
    template hipError_t launch_pauli_expect<T>(const T*, int, const TermBatch&, double*, int, hipStream_t);  \
    template hipError_t launch_pauli_apply_multi<T>(const T*, T*, int, const TermBatch*, int, bool, hipStream_t); \
    template hipError_t launch_pauli_apply<T>(const T*, T*, int, const TermBatch&, bool, hipStream_t);        \
    template hipError_t launch_inner<T>(const T*, const T*, int, double*, int, hipStream_t);                \
    template hipError_t launch_grad_sweep<T>(const T*, const T*, int, int, int, double*, int, hipStream_t);

QV_INSTANTIATE(d2)
QV_INSTANTIATE(f2)

template hipError_t launch_compare<d2, d2>(const d2*, const d2*, int, double*, int, hipStream_t);
template hipError_t launch_compare<d2, f2>(const d2*, const f2*, int, double*, int, hipStream_t);
template hipError_t launch_compare<f2, d2>(const f2*, const d2*, int, double*, int, hipStream_t);
template hipError_t launch_compare<f2, f2>(const f2*, const f2*, int, double*, int, hipStream_t);

}  // namespace qv
