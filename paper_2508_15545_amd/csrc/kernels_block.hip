// Register-resident block pass for gfx950.
//
// One workgroup owns a block of 2^b amplitudes (the indices that agree
// outside the pass's local qubits; block storage of QVecOpt Sec. III.C,
// generalised to any qubit set). Each thread holds R = 2^r of them in
// registers: the ones whose local positions in the current window W (r
// positions) vary while the other b - r positions are fixed by the thread
// index. Gates acting densely inside the window are applied in registers
// (pairs and quadruples of Sec. III.A Eq. 5 / Sec. III.C are register pairs
// and quadruples of one thread); diagonal gates and controls may use any
// bit because each amplitude knows its index. Moving to the next window is a
// transpose through LDS (write all, barrier, read all), so LDS traffic is
// one round trip per window change instead of one per gate, and HBM sees
// the block once per pass.
//
// The block is loaded and stored with the natural mapping (lanes run over
// the lowest local positions, which hold the lowest qubits and so
// contiguous runs of memory); the planner starts and, when it can, ends on
// that window.
#include <cstdio>
#include <cstdlib>

#include "device_common.h"

namespace qv {

// The single-state complex128 kernel exchanges real and imaginary parts in
// two rounds through a buffer of 8-byte slots (half the block's bytes), so
// that three workgroups share a CU's LDS instead of two. Its slot map is
// the 8-byte one, as for complex64.
template <typename T, int NS>
constexpr bool split_exchange() { return sizeof(T) == 16 && NS == 1; }

template <typename T, int NS>
constexpr uint32_t xch_slot_bytes() { return split_exchange<T, NS>() ? 8u : (uint32_t)sizeof(T); }

template <typename T, int NS>
__device__ __forceinline__ uint32_t lds_swizzle(uint32_t l)
{
    return lds_slot(l, xch_slot_bytes<T, NS>() == 16 ? 4 : 5);
}

// Local index bits contributed by the thread index: thread bit i sits at
// local position tpos[i].
__device__ __forceinline__ uint32_t thread_part(const int32_t* tpos, int tb, int tid)
{
    uint32_t tl = 0;
    // Unrolled with a guard, so that the positions arrive in one scalar
    // load; the opaque copy of tid keeps the bit extractions here instead of
    // in registers held across the whole kernel.
    int t = tid;
    asm volatile("" : "+v"(t));
    int tp[kMaxThreadBits];
#pragma unroll
    for (int i = 0; i < kMaxThreadBits; i++) tp[i] = tpos[i];
#pragma unroll
    for (int i = 0; i < kMaxThreadBits; i++)
        if (i < tb) tl |= (uint32_t)((t >> i) & 1) << tp[i];
    return tl;
}

// Orders this wave's LDS writes before its later LDS reads (a wave's LDS
// operations execute in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int RB>
__device__ __forceinline__ uint32_t window_part(int k, const int (&w)[kMaxRegBits])
{
    uint32_t l = 0;
#pragma unroll
    for (int j = 0; j < RB; j++) l |= (uint32_t)((k >> j) & 1) << w[j];
    return l;
}

// e^{2 pi i x} for x in turns (reduced to [-1/2, 1/2] first)
template <typename T>
__device__ __forceinline__ T cis_turns(double x)
{
    x -= rint(x);
    T f;
    if constexpr (sizeof(T) == 16) {
        double sn, cs;
        sincospi(2.0 * x, &sn, &cs);
        f.x = cs;
        f.y = sn;
    } else {
        float sn, cs;
        sincospif((float)(2.0 * x), &sn, &cs);
        f.x = cs;
        f.y = sn;
    }
    return f;
}

// The op fields every op needs, in the order they lead TileOp.
struct OpHot {
    int32_t code;
    int32_t mat;
    uint32_t tctrl;
    uint32_t kmask;
    uint64_t gctrl;
};

// Ops that read the state without changing it (the adjoint's gradient reads).
__device__ __forceinline__ bool is_read_code(int code)
{
    return code == RC_GZ || code == RC_GZM || (code >= RC_GXY && code < RC_GXY + kMaxRegBits);
}

__device__ __forceinline__ OpHot op_hot(const TileOp* p)
{
    OpHot h;
    h.code = p->code;
    h.mat = p->mat;
    h.tctrl = p->tctrl;
    h.kmask = p->kmask;
    h.gctrl = p->gctrl;
    return h;
}

// Transpose the thread's registers from one mapping to another through LDS.
// The slot map is linear over XOR and the thread and window parts of an
// index have disjoint bits, so slot(tl | wl) = slot(tl) ^ slot(wl): one
// per-thread term and one uniform term per register, the latter read from the
// stage table (wo_new: byte offsets, uniform scalar loads). The offsets of
// the current mapping are kept in registers from one exchange to the next.
template <typename T, int RB, int NS>
__device__ __forceinline__ void exchange(T (&v)[NS][1 << RB], T* lds, int nloc, uint32_t (&aoff)[1 << RB],
                                         uint32_t tl_new, const uint32_t* __restrict__ wo_new, bool wave_only)
{
    // aoff: the registers' byte offsets in the current mapping (kept from the
    // previous exchange); on return, those of the new mapping.
    constexpr int R = 1 << RB;
    constexpr uint32_t sb = xch_slot_bytes<T, NS>();
    unsigned char* base = reinterpret_cast<unsigned char*>(lds);
    const uint32_t sn = lds_swizzle<T, NS>(tl_new) * sb;
    uint32_t noff[R];
#pragma unroll
    for (int k = 0; k < R; k++) noff[k] = sn ^ wo_new[k];
    // Within-wave exchanges (the wave positions did not move) read only what
    // the same wave wrote: no workgroup barrier.
    auto sync = [&]() {
        if (wave_only) wave_lds_sync();
        else __syncthreads();
    };
    if constexpr (split_exchange<T, NS>()) {
        using R8 = typename RealOf<T>::type;
#pragma unroll
        for (int part = 0; part < 2; part++) {
#pragma unroll
            for (int k = 0; k < R; k++) {
                R8* d = reinterpret_cast<R8*>(base + aoff[k]);
                *d = part ? v[0][k].y : v[0][k].x;
            }
            sync();
#pragma unroll
            for (int k = 0; k < R; k++) {
                const R8 x = *reinterpret_cast<const R8*>(base + noff[k]);
                if (part) v[0][k].y = x;
                else v[0][k].x = x;
            }
            sync();
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; k++) {
#pragma unroll
            for (int s = 0; s < NS; s++)
                *reinterpret_cast<T*>(base + (size_t)s * nloc * sizeof(T) + aoff[k]) = v[s][k];
        }
        sync();
#pragma unroll
        for (int k = 0; k < R; k++) {
#pragma unroll
            for (int s = 0; s < NS; s++)
                v[s][k] = *reinterpret_cast<const T*>(base + (size_t)s * nloc * sizeof(T) + noff[k]);
        }
        sync();
    }
#pragma unroll
    for (int k = 0; k < R; k++) aoff[k] = noff[k];
}

template <typename T, int RB, int NS, int J, bool CTRL>
__device__ __forceinline__ void reg_dense1(T (&v)[NS][1 << RB], T u00, T u01, T u10, T u11, uint32_t cm)
{
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & (1 << J)) continue;
        const int k1 = k | (1 << J);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const T x = v[s][k], y = v[s][k1];
            const T a = cmul2(u00, x, u01, y), c = cmul2(u10, x, u11, y);
            if (CTRL) {
                const bool on = (cm >> k) & 1u;
                v[s][k] = on ? a : x;
                v[s][k1] = on ? c : y;
            } else {
                v[s][k] = a;
                v[s][k1] = c;
            }
        }
    }
}

// x with the sign bits of both components XORed with m (0 or 0x80000000):
// x or -x exactly.
__device__ __forceinline__ d2 flip_sign(d2 x, uint32_t m)
{
    const uint64_t mm = (uint64_t)m << 32;
    x.x = __longlong_as_double(__double_as_longlong(x.x) ^ (long long)mm);
    x.y = __longlong_as_double(__double_as_longlong(x.y) ^ (long long)mm);
    return x;
}
__device__ __forceinline__ f2 flip_sign(f2 x, uint32_t m)
{
    x.x = __int_as_float(__float_as_int(x.x) ^ (int)m);
    x.y = __int_as_float(__float_as_int(x.y) ^ (int)m);
    return x;
}

// A register copy the compiler cannot see through: a multiplication by
// `one`, 1.0 read at run time (exact; four cycles per FP64 value, the cost
// of a 64-bit move). The op loop alternates between two register sets, and
// each op must define every register of the set it writes: a plain
// assignment would let the register allocator merge the two sets along that
// path, and every other op would then end in a copy of the whole state.
// Permutations (X, CNOT, SWAP), registers an op leaves alone, and ops that
// only read the state write through this.
template <typename T>
__device__ __forceinline__ T fresh(T x, typename RealOf<T>::type one)
{
    T r;
    r.x = x.x * one;
    r.y = x.y * one;
    return r;
}

// Every register through fresh (with two register sets; with one set the
// registers stay where they are).
template <bool PP, typename T, int NS, int R>
__device__ __forceinline__ void fresh_all(T (&v)[NS][R], typename RealOf<T>::type z)
{
    if constexpr (!PP) return;
#pragma unroll
    for (int s = 0; s < NS; s++)
#pragma unroll
        for (int k = 0; k < R; k++) v[s][k] = fresh(v[s][k], z);
}

template <typename T, int RB, int NS, int J, bool CTRL>
__device__ __forceinline__ void reg_xperm(T (&v)[NS][1 << RB], uint32_t cm, typename RealOf<T>::type z)
{
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & (1 << J)) continue;
        const int k1 = k | (1 << J);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const T x = v[s][k], y = v[s][k1];
            if (CTRL) {
                const bool on = (cm >> k) & 1u;
                v[s][k] = on ? y : x;
                v[s][k1] = on ? x : y;
            } else {
                v[s][k] = fresh(y, z);
                v[s][k1] = fresh(x, z);
            }
        }
    }
}

// CNOT with target window bit JT and control window bit JC: swap the
// register pairs whose control bit is set.
template <bool PP, typename T, int RB, int NS, int JT, int JC>
__device__ __forceinline__ void reg_cx(T (&v)[NS][1 << RB], typename RealOf<T>::type z)
{
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & (1 << JT)) continue;
        const int k1 = k | (1 << JT);
        const bool swap = (k & (1 << JC)) != 0;
        if (!swap && !PP) continue;
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const T x = v[s][k], y = v[s][k1];
            v[s][k] = fresh(swap ? y : x, z);
            v[s][k1] = fresh(swap ? x : y, z);
        }
    }
}

template <typename T, int RB, int NS, int J0, int J1, bool CTRL>
__device__ __forceinline__ void reg_dense2(T (&v)[NS][1 << RB], const T* __restrict__ m, uint32_t cm)
{
    T u[16];
#pragma unroll
    for (int e = 0; e < 16; e++) u[e] = m[e];
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & ((1 << J0) | (1 << J1))) continue;
        const int idx[4] = {k, k | (1 << J0), k | (1 << J1), k | (1 << J0) | (1 << J1)};
        const bool on = !CTRL || ((cm >> k) & 1u);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            T x[4], w[4];
#pragma unroll
            for (int e = 0; e < 4; e++) x[e] = v[s][idx[e]];
#pragma unroll
            for (int r = 0; r < 4; r++)
                w[r] = cdot4(u[4 * r], x[0], u[4 * r + 1], x[1], u[4 * r + 2], x[2], u[4 * r + 3], x[3]);
#pragma unroll
            for (int e = 0; e < 4; e++) v[s][idx[e]] = CTRL ? (on ? w[e] : x[e]) : w[e];
        }
    }
}

// The 4x4 update of reg_dense2 on the matrix cores (complex64, one state).
// v_mfma_f32_4x4x1f32 treats the wave as 16 blocks of 4 lanes; in block b it
// adds A[i] * B[j] to output register i of lane 4b + j, with A[i] taken from
// lane 4b + i and B[j] from lane 4b + j. With B = element e of a lane's own
// quadruple and A = column e of the matrix (lane 4b + i holding row i), one
// instruction adds M[i][e] x_e to output i of every lane's quadruple, so the
// quadruple stays in its lane's registers. Real and imaginary parts take
// four such steps per e: yr += Mr x_r - Mi x_i, yi += Mi x_r + Mr x_i.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int RB, int J0, int J1>
__device__ __forceinline__ void reg_dense2_mfma(f2 (&v)[1][1 << RB], const f2* __restrict__ m, int lane)
{
    const f2* row = m + 4 * (lane & 3);  // this lane's A operands: row (lane mod 4) of the matrix
    float ar[4], ai[4], an[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const f2 u = row[e];
        ar[e] = u.x;
        ai[e] = u.y;
        an[e] = -u.y;
    }
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & ((1 << J0) | (1 << J1))) continue;
        const int idx[4] = {k, k | (1 << J0), k | (1 << J1), k | (1 << J0) | (1 << J1)};
        f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const f2 x = v[0][idx[e]];
            yr = __builtin_amdgcn_mfma_f32_4x4x1f32(ar[e], x.x, yr, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_4x4x1f32(ai[e], x.x, yi, 0, 0, 0);
            yr = __builtin_amdgcn_mfma_f32_4x4x1f32(an[e], x.y, yr, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_4x4x1f32(ar[e], x.y, yi, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            v[0][idx[i]].x = yr[i];
            v[0][idx[i]].y = yi[i];
        }
    }
}

template <bool PP, typename T, int RB, int NS, int J0, int J1, bool CTRL>
__device__ __forceinline__ void reg_swap(T (&v)[NS][1 << RB], uint32_t cm, typename RealOf<T>::type z)
{
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        if (k & ((1 << J0) | (1 << J1))) continue;
        const int a = k | (1 << J0), c = k | (1 << J1), d = a | c;
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const T x = v[s][a], y = v[s][c];
            if (CTRL) {
                const bool on = (cm >> k) & 1u;
                v[s][a] = on ? y : x;
                v[s][c] = on ? x : y;
            } else {
                v[s][a] = fresh(y, z);
                v[s][c] = fresh(x, z);
            }
            // the pairs whose two bits agree stay
            if constexpr (PP) {
                v[s][k] = fresh(v[s][k], z);
                v[s][d] = fresh(v[s][d], z);
            }
        }
    }
}

// Im <lambda|G|phi> contributions of the thread's registers for
// G = cx X + cy Y on window bit J (v[0] = phi, v[1] = lambda). The per-thread
// partial is formed in the state's precision (FP32 for complex64: the
// thread's 2^RB products per component, summed in registers) and handed to
// the FP64 reductions across lanes, waves and blocks.
template <typename T, int RB, int J>
__device__ __forceinline__ double reg_grad_xy(const T (&v)[2][1 << RB], double cx, double cy)
{
    using R = typename RealOf<T>::type;
    R sx = 0, sy = 0;
#pragma unroll
    for (int k = 0; k < (1 << RB); k++) {
        const int p = k ^ (1 << J);
        const T f = v[0][p], m = v[1][k];
        const R re = m.x * f.x + m.y * f.y;
        const R im = m.x * f.y - m.y * f.x;
        const bool bit = (k >> J) & 1;
        // X: Im(conj(m) f); Y: (Y phi)_l = (bit ? i : -i) phi_{l ^ J}
        sx += im;
        sy += bit ? re : -re;
    }
    return cx * (double)sx + cy * (double)sy;
}

#define QV_J1_CASES(F)                                   \
    case 0: F(0); break;                                 \
    case 1: F(1); break;                                 \
    case 2: F(2); break;                                 \
    case 3: if constexpr (RB > 3) { F(3); } break;       \
    case 4: if constexpr (RB > 4) { F(4); } break;

// Occupancy target per SIMD: the narrow single-state variant is held to
// 128 VGPRs so that two 512-thread workgroups (LDS-limited) fill a CU.
// With prefetch (PF) the next block's registers are live as well, and the
// target drops to three waves per SIMD.
// The single-state complex128 kernel with r = 4 is held to 168 VGPRs, three
// waves per SIMD, which its half-size exchange buffer lets the LDS hold; the
// single-state complex64 one to 128 VGPRs, four waves per SIMD (its two
// register sets need more than the 96 of five; two sets at four waves
// measured 2% faster than one set at five).
template <typename T, int RB, int NS, bool PF, bool MF = false>
constexpr int block_waves_per_eu()
{
    return MF ? 4
         : (RB == 3 && NS == 1) ? (PF ? 3 : 4)
         : (split_exchange<T, NS>() && !PF) ? 3
         : (sizeof(T) == 8 && NS == 1 && !PF) ? 4 : 1;
}

// MF: the variant whose plans may hold matrix-core 4x4 ops (RC_D2M); a kernel
// of its own, so that their registers do not weigh on the default kernel.
template <typename T, int RB, int NS, bool PF, bool MF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(block_waves_per_eu<T, RB, NS, PF, MF>())))
void k_block_reg(T* __restrict__ s0, T* __restrict__ s1,
                                                   const PassHdr* __restrict__ hdr,
                                                   const StageHdr* __restrict__ stages,
                                                   const TileOp* __restrict__ ops, const T* __restrict__ mats,
                                                   const PhaseTerm* __restrict__ phase, double* __restrict__ gpart,
                                                   int64_t gstride)
{
    constexpr int R = 1 << RB;
    __shared__ __attribute__((aligned(16))) unsigned char smem_raw[NS * kRegLdsBytesPerState];
    T* lds = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[NS == 2 ? kMaxGradPerPass * 8 : 1];

    const int b = hdr->b;
    const int nloc = 1 << b;
    const int tb = b - RB;
    // two register sets in the op loop (see there); the one-set loop stays
    // for comparison (measured 2% slower for complex64 at five waves per SIMD
    // than two sets at four)
    constexpr bool PP = true;
    // 1.0, read at run time (see fresh)
    const typename RealOf<T>::type one = (typename RealOf<T>::type)(hdr->pad + 1);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint64_t nblocks = 1ull << hdr->n_outer;

    // Load/store mapping (lanes on the lowest positions, see the planner).
    int wn[kMaxRegBits];
#pragma unroll
    for (int j = 0; j < kMaxRegBits; j++) wn[j] = hdr->nat.w[j];
    const uint32_t tl_nat = thread_part(hdr->nat.tpos, tb, tid);
    // The thread's bits of the global index in the load mapping, and its
    // registers' element offsets (hdr->nat_koff): the two have disjoint bits.
    uint64_t tg = 0;
#pragma unroll
    for (int i = 0; i < kMaxThreadBits; i++) {
        if (i < tb) tg |= (uint64_t)((tid >> i) & 1) << hdr->nat_tq[i];
    }
    // Block index -> global index of its first amplitude: the index's bits go
    // to the qubits outside the block, i.e. a zero is inserted at each local
    // qubit (ascending).
    auto block_base = [&](uint64_t blk) {
        uint64_t bb = blk;
#pragma unroll
        for (int j = 0; j < kMaxLocal; j++) {
            const int q = hdr->local_q[j] & 63;
            const uint64_t ins = ((bb >> q) << 1 << q) | (bb & ((1ull << q) - 1));
            bb = j < b ? ins : bb;
        }
        return bb;
    };
    auto load_block = [&](T (&dst)[NS][R], uint64_t g0) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint64_t g = g0 + hdr->nat_koff[k];
            dst[0][k] = ld_nt(s0 + g);
            if (NS == 2) dst[NS - 1][k] = ld_nt(s1 + g);
        }
    };

    // With PF the grid is sized to the resident workgroups and each one
    // issues the loads of its next block before working on the current one,
    // so that HBM reads overlap the register work.
    T nx[PF ? NS : 1][PF ? R : 1];
    if constexpr (PF) {
        if (blockIdx.x < nblocks) load_block(nx, block_base(blockIdx.x) | tg);
        // Nothing outstanding at the loop entry: the loop's own waits then
        // count only the loop's loads and stores.
        __builtin_amdgcn_s_waitcnt(0);
    }
    // One block per workgroup; with PF, a grid smaller than the block count
    // walks the blocks in strides.
    auto run_block = [&](const uint64_t blk) {
    const uint64_t base = block_base(blk);
    const uint64_t gt = base | tg;

    T v[NS][R];
    if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < NS; s++)
#pragma unroll
            for (int k = 0; k < R; k++) v[s][k] = nx[s][k];
        // unconditional, so that the wait for these loads has a fixed
        // count (the last block reloads itself; those values go unused)
        const uint64_t nb = blk + gridDim.x < nblocks ? blk + gridDim.x : blk;
        load_block(nx, block_base(nb) | tg);
    } else {
        load_block(v, gt);
    }

    int cur_w[kMaxRegBits];
#pragma unroll
    for (int j = 0; j < kMaxRegBits; j++) cur_w[j] = wn[j];
    uint32_t cur_tl = tl_nat;
    uint32_t aoff[R];  // exchange-buffer offsets of the registers in the current mapping
    {
        const uint32_t s_nat = lds_swizzle<T, NS>(tl_nat) * xch_slot_bytes<T, NS>();
#pragma unroll
        for (int k = 0; k < R; k++) aoff[k] = s_nat ^ hdr->nat.woff[k];
    }

    const TileOp* po = ops + hdr->op_begin;
    const int n_stages = hdr->n_stages;
    for (int si = 0; si < n_stages; si++) {
        const StageHdr& sh = stages[hdr->stage_begin + si];  // read in place (uniform scalar loads)
        if (sh.wave_local != XCH_NONE) {
            int w_new[kMaxRegBits];
#pragma unroll
            for (int j = 0; j < kMaxRegBits; j++) w_new[j] = sh.w[j];
            const uint32_t tl_new = thread_part(sh.tpos, tb, tid);
            exchange<T, RB, NS>(v, lds, nloc, aoff, tl_new, sh.woff, sh.wave_local == XCH_WAVE);
            cur_tl = tl_new;
#pragma unroll
            for (int j = 0; j < kMaxRegBits; j++) cur_w[j] = w_new[j];
        }
        const TileOp* sop = po + sh.op_begin;
        const int nops = sh.n_ops;
        // Ops alternate between two register sets (vb = op(v), then
        // v = op(vb)): each op writes its results into the other set, so a
        // dense update is not copied back into the registers it read before
        // the next op (with one set, every op ends in a copy of the state).
        // Gradient reads (Im <lambda|G|phi> into the wave's LDS slots) leave
        // the state as it is; with two register sets they run on whichever
        // set holds the state, between the ops that change it.
        auto read_body = [&](const T (&v)[NS][R], const OpHot& cur, const TileOp& op) __attribute__((always_inline)) {
            if ((base & cur.gctrl) != cur.gctrl) return;  // uniform over the block
            switch (cur.code) {
#define QV_C1(BASE, J, STMT) \
    case BASE + J:           \
        if constexpr (J < RB) { STMT; } \
        break;
#define QV_ALL1(BASE, F) QV_C1(BASE, 0, F(0)) QV_C1(BASE, 1, F(1)) QV_C1(BASE, 2, F(2)) QV_C1(BASE, 3, F(3)) QV_C1(BASE, 4, F(4))
            case RC_GZ: {
                if constexpr (NS == 2) {
                    // per-thread partial in the state's precision, FP64 beyond
                    typename RealOf<T>::type pacc = 0;
                    const int a = op.a;
                    const int ua = a < 0 ? (int)((base >> op.oa) & 1) : 0;
                    uint32_t tlx = cur_tl;
                    asm volatile("" : "+v"(tlx));
#pragma unroll
                    for (int k = 0; k < R; k++) {
                        const uint32_t l = tlx | window_part<RB>(k, cur_w);
                        const int bit = a >= 0 ? (int)((l >> a) & 1) : ua;
                        const T f = v[0][k], m = v[1][k];
                        const auto im = m.x * f.y - m.y * f.x;
                        pacc += bit ? -im : im;
                    }
                    const double acc = wave_total((double)pacc);
                    if (lane == 0) red[op.slot * 8 + wave] = acc;
                }
                break;
            }
            case RC_GZM: {
                // several Z reads: p_k = Im(conj(lambda_k) phi_k) once, then a
                // read of window bit j is sum_k (-1)^(k_j) p_k and a read of a
                // thread bit or an outer qubit is +-sum_k p_k
                if constexpr (NS == 2) {
                    // per-thread sums in the state's precision, FP64 beyond
                    using RT = typename RealOf<T>::type;
                    RT S = 0, D[RB];
#pragma unroll
                    for (int j = 0; j < RB; j++) D[j] = 0;
#pragma unroll
                    for (int k = 0; k < R; k++) {
                        const T f = v[0][k], m = v[1][k];
                        const RT p = m.x * f.y - m.y * f.x;
                        S += p;
#pragma unroll
                        for (int j = 0; j < RB; j++) D[j] += ((k >> j) & 1) ? -p : p;
                    }
                    const ReadZ* rz = reinterpret_cast<const ReadZ*>(phase + op.aux);
                    const uint32_t utid = (uint32_t)tid;
                    for (int e = 0; e < op.cnt; e++) {
                        const int zj = rz[e].j, ztb = rz[e].tbit, zoa = rz[e].oa, zslot = rz[e].slot;
                        RT pv;
                        if (zj >= 0) {
                            pv = D[0];
#pragma unroll
                            for (int j = 1; j < RB; j++) pv = zj == j ? D[j] : pv;
                        } else {
                            const bool bit = ztb >= 0 ? ((utid >> ztb) & 1u) != 0 : ((base >> zoa) & 1ull) != 0;
                            pv = bit ? -S : S;
                        }
                        const double val = wave_total((double)pv);
                        if (lane == 0) red[zslot * 8 + wave] = val;
                    }
                }
                break;
            }
#define F_G(J)                                                                                        \
    if constexpr (NS == 2) {                                                                          \
        double acc = reg_grad_xy<T, RB, J>(v, (double)mats[cur.mat].x, (double)mats[cur.mat].y);      \
        acc = wave_total(acc);                                                                        \
        if (lane == 0) red[op.slot * 8 + wave] = acc;                                                 \
    }
                QV_ALL1(RC_GXY, F_G)
#undef F_G
#undef QV_ALL1
#undef QV_C1
            default: break;
            }
        };
        auto op_body = [&](T (&v)[NS][R], const OpHot& cur, const TileOp& op) __attribute__((always_inline)) {
            if ((base & cur.gctrl) == cur.gctrl) {  // uniform over the block
            const int code = cur.code;
            // registers the op acts on (all, for ops without local controls)
            const uint32_t cm = (cur_tl & cur.tctrl) == cur.tctrl ? cur.kmask : 0u;
            switch (code) {
#define QV_C1(BASE, J, STMT) \
    case BASE + J:           \
        if constexpr (J < RB) { STMT; } else { fresh_all<PP>(v, one); } \
        break;
#define QV_ALL1(BASE, F) QV_C1(BASE, 0, F(0)) QV_C1(BASE, 1, F(1)) QV_C1(BASE, 2, F(2)) QV_C1(BASE, 3, F(3)) QV_C1(BASE, 4, F(4))
#define QV_C2(BASE, A, B, F) \
    case BASE + 5 * A + B:   \
        if constexpr (A < RB && B < RB && A != B) { F(A, B); } else { fresh_all<PP>(v, one); } \
        break;
#define QV_PAIRS(BASE, F) \
    QV_C2(BASE, 0, 1, F) QV_C2(BASE, 0, 2, F) QV_C2(BASE, 0, 3, F) QV_C2(BASE, 0, 4, F) QV_C2(BASE, 1, 2, F) \
    QV_C2(BASE, 1, 3, F) QV_C2(BASE, 1, 4, F) QV_C2(BASE, 2, 3, F) QV_C2(BASE, 2, 4, F) QV_C2(BASE, 3, 4, F)
#define QV_ORDERED(BASE, F) \
    QV_PAIRS(BASE, F) \
    QV_C2(BASE, 1, 0, F) QV_C2(BASE, 2, 0, F) QV_C2(BASE, 3, 0, F) QV_C2(BASE, 4, 0, F) QV_C2(BASE, 2, 1, F) \
    QV_C2(BASE, 3, 1, F) QV_C2(BASE, 4, 1, F) QV_C2(BASE, 3, 2, F) QV_C2(BASE, 4, 2, F) QV_C2(BASE, 4, 3, F)
#define QV_M2 mats[cur.mat], mats[cur.mat + 1], mats[cur.mat + 2], mats[cur.mat + 3]
#define F_D1(J) reg_dense1<T, RB, NS, J, false>(v, QV_M2, cm)
#define F_D1C(J) reg_dense1<T, RB, NS, J, true>(v, QV_M2, cm)
#define F_X(J) reg_xperm<T, RB, NS, J, false>(v, cm, one)
#define F_XC(J) reg_xperm<T, RB, NS, J, true>(v, cm, one)
#define F_CX(A, B) reg_cx<PP, T, RB, NS, A, B>(v, one)
#define F_D2(A, B) reg_dense2<T, RB, NS, A, B, false>(v, mats + cur.mat, cm)
#define F_D2C(A, B) reg_dense2<T, RB, NS, A, B, true>(v, mats + cur.mat, cm)
#define F_SW(A, B) reg_swap<PP, T, RB, NS, A, B, false>(v, cm, one)
#define F_D2M(A, B) if constexpr (MF && sizeof(T) == 8 && NS == 1) { reg_dense2_mfma<RB, A, B>(v, mats + cur.mat, lane); } else { fresh_all<PP>(v, one); }
#define F_SWC(A, B) reg_swap<PP, T, RB, NS, A, B, true>(v, cm, one)
                QV_ALL1(RC_D1, F_D1)
                QV_ALL1(RC_D1C, F_D1C)
                QV_ALL1(RC_X, F_X)
                QV_ALL1(RC_XC, F_XC)
                QV_ORDERED(RC_CX, F_CX)
                QV_PAIRS(RC_D2, F_D2)
                QV_PAIRS(RC_D2C, F_D2C)
                QV_PAIRS(RC_D2M, F_D2M)
                QV_PAIRS(RC_SW, F_SW)
                QV_PAIRS(RC_SWC, F_SWC)
            case RC_DIAG: {
                const T d0 = mats[cur.mat], d1 = mats[cur.mat + 1], dd2 = mats[cur.mat + 2], d3 = mats[cur.mat + 3];
                const int a = op.a, c = op.c;
                const bool ctrl = op.lctrl != 0;
                const int ua = a < 0 ? (op.oa >= 0 ? (int)((base >> op.oa) & 1) : 0) : 0;
                const int uc = c < 0 ? (op.oc >= 0 ? (int)((base >> op.oc) & 1) : 0) : 0;
                uint32_t tlx = cur_tl;  // opaque: the indices are formed here, not held across the op loop
                asm volatile("" : "+v"(tlx));
#pragma unroll
                for (int k = 0; k < R; k++) {
                    const uint32_t l = tlx | window_part<RB>(k, cur_w);
                    const int ba = a >= 0 ? (int)((l >> a) & 1) : ua;
                    const int bc = c >= 0 ? (int)((l >> c) & 1) : uc;
                    const int sel = ba + 2 * bc;
                    const T d = sel == 0 ? d0 : sel == 1 ? d1 : sel == 2 ? dd2 : d3;
                    const bool on = !ctrl || ((cm >> k) & 1u);
#pragma unroll
                    for (int s = 0; s < NS; s++) {
                        const T x = v[s][k];
                        const T y = cmul(d, x);
                        v[s][k] = on ? y : x;
                    }
                }
                break;
            }
            case RC_SIGN: {
                // flip the sign of the registers the op acts on: the thread's
                // part of the condition is one sign mask, the register part
                // (kmask) is uniform, so each register is a uniform test and
                // two exclusive ors per component pair
                const uint32_t tsign = (cur_tl & cur.tctrl) == cur.tctrl ? 0x80000000u : 0u;
#pragma unroll
                for (int k = 0; k < R; k++) {
                    const bool flip = (cur.kmask >> k) & 1u;
#pragma unroll
                    for (int s = 0; s < NS; s++) v[s][k] = flip ? flip_sign(v[s][k], tsign) : PP ? fresh(v[s][k], one) : v[s][k];
                }
                break;
            }
            case RC_PHASE: {
                // angle(k) = A + sum_j k_j eff[j] + (window-only part, tabulated
                // as unit complex numbers at mats[cur.mat + k]); A and eff[j]
                // depend on the thread's bits (terms padded to groups of 4)
                if (op.cnt == 0) {  // window-only: the table is the whole phase
#pragma unroll
                    for (int k = 0; k < R; k++) {
                        const T g = mats[cur.mat + k];
#pragma unroll
                        for (int s = 0; s < NS; s++) v[s][k] = cmul(g, v[s][k]);
                    }
                    break;
                }
                const PhaseHead& ph = *reinterpret_cast<const PhaseHead*>(phase + op.aux);
                const PhaseTerm* pt = phase + op.aux + 1;
                const uint32_t utid = (uint32_t)tid;
                auto sum_terms = [&](int cnt) -> double {
                    double acc = 0;
                    for (int t = 0; t < cnt; t += 4) {
                        // four records in one batch of scalar loads
                        const uint64_t* rec = reinterpret_cast<const uint64_t*>(pt + t);
                        uint64_t w[16];
#pragma unroll
                        for (int i = 0; i < 16; i++) w[i] = rec[i];
                        // every word in hand before use: one batch of loads, no per-record waits
#pragma unroll
                        for (int i = 0; i < 16; i++) asm volatile("" : : "s"(w[i]));
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            const uint64_t omask = w[4 * u];
                            const uint32_t tmask = (uint32_t)w[4 * u + 1];
                            // the block part of the condition is uniform (an
                            // integer select, so the angle's load is not branched on)
                            const uint64_t keep_th = (base & omask) == omask ? ~0ull : 0ull;
                            const double th = __longlong_as_double((long long)(w[4 * u + 2] & keep_th));
                            // acc + th or acc, exactly as an add or no add
                            acc = fma(th, (utid & tmask) == tmask ? 1.0 : 0.0, acc);
                        }
                    }
                    pt += cnt;
                    return acc;
                };
                const double A = sum_terms(ph.count[0]);
                double eff[RB];
#pragma unroll
                for (int j = 0; j < RB; j++) eff[j] = sum_terms(ph.count[1 + j]);
                // e^{2 pi i angle(k)} as products of RB + 1 unit factors
                T f[R];
                f[0] = cis_turns<T>(A);
#pragma unroll
                for (int j = 0; j < RB; j++) {
                    const T e = cis_turns<T>(eff[j]);
#pragma unroll
                    for (int k = 0; k < (1 << j); k++) f[k | (1 << j)] = cmul(f[k], e);
                }
#pragma unroll
                for (int k = 0; k < R; k++) {
                    const T g = cmul(mats[cur.mat + k], f[k]);
#pragma unroll
                    for (int s = 0; s < NS; s++) v[s][k] = cmul(g, v[s][k]);
                }
                break;
            }
            case RC_GZ:
            case RC_GZM:
                read_body(v, cur, op);
                fresh_all<PP>(v, one);
                break;
#define F_G(J)                     \
    read_body(v, cur, op);         \
    fresh_all<PP>(v, one)
                QV_ALL1(RC_GXY, F_G)
#undef F_G
#undef F_D1
#undef F_D1C
#undef F_X
#undef F_XC
#undef F_CX
#undef F_D2
#undef F_D2C
#undef F_SW
#undef F_SWC
#undef F_D2M
#undef QV_M2
#undef QV_ORDERED
#undef QV_PAIRS
#undef QV_C2
#undef QV_ALL1
#undef QV_C1
            default: fresh_all<PP>(v, one); break;
            }
            } else {
                fresh_all<PP>(v, one);
            }
        };
        auto apply_op = [&](const T (&src)[NS][R], T (&dst)[NS][R], const OpHot& cur,
                            const TileOp& op) __attribute__((always_inline)) {
            T w[NS][R];
#pragma unroll
            for (int s = 0; s < NS; s++)
#pragma unroll
                for (int k = 0; k < R; k++) w[s][k] = src[s][k];
            op_body(w, cur, op);
#pragma unroll
            for (int s = 0; s < NS; s++)
#pragma unroll
                for (int k = 0; k < R; k++) dst[s][k] = w[s][k];
        };
        // The hot fields of the next op are loaded while the current op runs,
        // so that each op waits for one round of scalar loads (its matrix)
        // instead of three.
        OpHot cur = op_hot(sop);
        if constexpr (PP && NS == 1) {
            // no reads: ops in pairs, the second of an odd tail a copy
            T vb[NS][R];
            for (int o = 0; o < nops; o += 2) {
                const OpHot h1 = op_hot(sop + (o + 1 < nops ? o + 1 : o));
                apply_op(v, vb, cur, sop[o]);
                const OpHot h2 = op_hot(sop + (o + 2 < nops ? o + 2 : o));
                if (o + 1 < nops) {
                    apply_op(vb, v, h1, sop[o + 1]);
                } else {
#pragma unroll
                    for (int s = 0; s < NS; s++)
#pragma unroll
                        for (int k = 0; k < R; k++) v[s][k] = fresh(vb[s][k], one);
                }
                cur = h2;
            }
        } else if constexpr (PP) {
            T vb[NS][R];
            int o = 0;
            // a gradient read right after an op runs on the set that op wrote,
            // instead of taking a turn of its own (which copies the state);
            // a read that follows another read still takes a turn (letting up
            // to three ride along measured no faster: more code per op)
            auto read_after = [&](const T (&cs)[NS][R]) __attribute__((always_inline)) {
                if constexpr (NS == 2) {
                    if (o < nops && is_read_code(cur.code)) {
                        const OpHot nxt = op_hot(sop + (o + 1 < nops ? o + 1 : o));
                        read_body(cs, cur, sop[o]);
                        o++;
                        cur = nxt;
                    }
                }
            };
            while (o < nops) {
                const OpHot h1 = op_hot(sop + (o + 1 < nops ? o + 1 : o));
                apply_op(v, vb, cur, sop[o]);
                o++;
                cur = h1;
                read_after(vb);
                if (o < nops) {
                    const OpHot h2 = op_hot(sop + (o + 1 < nops ? o + 1 : o));
                    apply_op(vb, v, cur, sop[o]);
                    o++;
                    cur = h2;
                    read_after(v);
                } else {
#pragma unroll
                    for (int s = 0; s < NS; s++)
#pragma unroll
                        for (int k = 0; k < R; k++) v[s][k] = fresh(vb[s][k], one);
                }
            }
        } else {
            for (int o = 0; o < nops; o++) {
                const OpHot nxt = op_hot(sop + (o + 1 < nops ? o + 1 : o));
                op_body(v, cur, sop[o]);
                cur = nxt;
            }
        }
        // Register permutations that end the stage (the n_exit ops after its
        // n_ops; an exchange follows) move the registers' exchange offsets
        // instead of their values: register k's offset becomes that of the
        // index it now holds, the current one XOR a uniform term (aux) for
        // the registers in kmask, where the block and the thread meet the
        // op's controls.
        const int nexit = sh.n_exit;
        for (int e = 0; e < nexit; e++) {
            const TileOp& x = sop[nops + e];
            if ((base & x.gctrl) != x.gctrl) continue;  // uniform over the block
            const uint32_t d = (cur_tl & x.tctrl) == x.tctrl ? (uint32_t)x.aux : 0u;
            const uint32_t fm = x.kmask;
#pragma unroll
            for (int k = 0; k < R; k++) aoff[k] ^= ((fm >> k) & 1u) ? d : 0u;
        }
    }

    // Store mapping (the last stage's, when its lanes keep the 128-byte runs
    // together, else the load mapping).
    const StageHdr& so = hdr->out;
    if (hdr->final_wave_local != XCH_NONE) {
        exchange<T, RB, NS>(v, lds, nloc, aoff, thread_part(so.tpos, tb, tid), so.woff,
                            hdr->final_wave_local == XCH_WAVE);
    }
    {
        uint64_t go = base;
#pragma unroll
        for (int i = 0; i < kMaxThreadBits; i++) {
            if (i < tb) go |= (uint64_t)((tid >> i) & 1) << hdr->out_tq[i];
        }
#pragma unroll
        for (int k = 0; k < R; k++) {
            const uint64_t g = go + hdr->out_koff[k];
            st_nt(s0 + g, v[0][k]);
            if (NS == 2) st_nt(s1 + g, v[NS - 1][k]);
        }
    }

    if constexpr (NS == 2) {
        const int ng = hdr->n_grad;
        if (ng > 0) {
            __syncthreads();
            const int nw = (int)(blockDim.x >> 6);
            for (int sl = tid; sl < ng; sl += blockDim.x) {
                double t = 0;
                for (int w = 0; w < nw; w++) t += red[sl * 8 + w];
                gpart[(int64_t)sl * gstride + (int64_t)blk] = t;
            }
            __syncthreads();  // red[] is rewritten by the next block
        }
    }
    };  // run_block
    if constexpr (PF) {
        for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) run_block(blk);
    } else {
        if (blockIdx.x < nblocks) run_block(blockIdx.x);
    }
}

#undef QV_J1_CASES

// Register prefetch of the next block (QVEC_PREFETCH=1). Off by default:
// its extra registers cost a wave per SIMD, and on the 29-qubit benchmark
// occupancy hides the load latency better than the prefetch does.
template <typename T>
static bool prefetch_on()
{
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("QVEC_PREFETCH");
        v = e ? (e[0] == '1' ? 1 : 0) : 0;
    }
    return v == 1;
}

// Matrix-core 4x4 updates for complex64 (QVEC_MFMA=1; the planner emits
// RC_D2M ops only then, and those passes run the MF kernel).
static bool mfma_on()
{
    const char* e = std::getenv("QVEC_MFMA");
    return e && e[0] == '1' && e[1] == 0;
}

static int cu_count()
{
    static int cus = 0;
    if (!cus && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess) cus = 256;
    return cus;
}

template <typename T, int RB, int NS, bool PF, bool MF = false>
static hipError_t launch_reg_k(T* s0, T* s1, int n, const PassHdr* d_hdr, const StageHdr* d_stages,
                               const TileOp* d_ops, const T* d_mats, const PhaseTerm* d_phase, int b, double* gp,
                               int64_t gs, hipStream_t st)
{
    const void* fn = reinterpret_cast<const void*>(&k_block_reg<T, RB, NS, PF, MF>);
    // the exchange buffer is a static array of the kernel
    if ((size_t)NS * ((size_t)1 << b) * xch_slot_bytes<T, NS>() > (size_t)NS * kRegLdsBytesPerState)
        return hipErrorInvalidValue;
    const size_t lds = 0;
    const uint64_t nblocks = 1ull << (n - b);
    const unsigned threads = 1u << (b - RB);
    uint64_t grid = nblocks;
    if (PF) {
        // one workgroup per resident slot
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)threads, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        const char* pe = std::getenv("QVEC_PF_PER_CU");  // experiment: workgroups per CU
        if (pe && std::atoi(pe) > 0) per_cu = std::atoi(pe);
        static bool said = false;
        if (!said && std::getenv("QVEC_VERBOSE")) {
            std::fprintf(stderr, "k_block_reg prefetch: %d workgroups per CU, %u threads, %zu B LDS\n", per_cu,
                         threads, (size_t)NS * kRegLdsBytesPerState);
            said = true;
        }
        const uint64_t g = (uint64_t)per_cu * (uint64_t)cu_count();
        if (g < grid) grid = g;
    }
    hipLaunchKernelGGL((k_block_reg<T, RB, NS, PF, MF>), dim3((unsigned)grid), dim3(threads), lds, st, s0, s1,
                       d_hdr, d_stages, d_ops, d_mats, d_phase, gp, gs);
    return hipGetLastError();
}

template <typename T, int RB, int NS>
static hipError_t launch_reg_t(T* s0, T* s1, int n, const PassHdr* d_hdr, const StageHdr* d_stages,
                               const TileOp* d_ops, const T* d_mats, const PhaseTerm* d_phase, int b, double* gp,
                               int64_t gs, hipStream_t st)
{
    if constexpr (NS == 1) {
        if (prefetch_on<T>())
            return launch_reg_k<T, RB, NS, true>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
        if constexpr (sizeof(T) == 8 && RB == 4) {
            if (mfma_on())
                return launch_reg_k<T, RB, NS, false, true>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp,
                                                            gs, st);
        }
    }
    return launch_reg_k<T, RB, NS, false>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
}

template <typename T>
hipError_t launch_block_reg(T* s0, T* s1, int n, int n_states, int rb, const PassHdr* d_hdr,
                            const StageHdr* d_stages, const TileOp* d_ops, const T* d_mats,
                            const PhaseTerm* d_phase, int b, double* gp, int64_t gs, hipStream_t st)
{
    if (b - rb < 6 || b - rb > 9) return hipErrorInvalidValue;  // whole waves, at most 512 threads
    if (n_states == 2) {
        if (rb == 3) return launch_reg_t<T, 3, 2>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
        if (rb == 4) return launch_reg_t<T, 4, 2>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
        return hipErrorInvalidValue;
    }
    if (rb == 3) return launch_reg_t<T, 3, 1>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
    if (rb == 4) return launch_reg_t<T, 4, 1>(s0, s1, n, d_hdr, d_stages, d_ops, d_mats, d_phase, b, gp, gs, st);
    return hipErrorInvalidValue;
}

// QV_BLOCK_ELEM (16 or 8) limits a translation unit to one element type, so
// that the two sets of kernels compile in parallel (kernels_block_c128.hip,
// kernels_block_c64.hip); without it this file instantiates both.
#if !defined(QV_BLOCK_ELEM) || QV_BLOCK_ELEM == 16
template hipError_t launch_block_reg<d2>(d2*, d2*, int, int, int, const PassHdr*, const StageHdr*, const TileOp*,
                                         const d2*, const PhaseTerm*, int, double*, int64_t, hipStream_t);
#endif
#if !defined(QV_BLOCK_ELEM) || QV_BLOCK_ELEM == 8
template hipError_t launch_block_reg<f2>(f2*, f2*, int, int, int, const PassHdr*, const StageHdr*, const TileOp*,
                                         const f2*, const PhaseTerm*, int, double*, int64_t, hipStream_t);
#endif

}  // namespace qv
