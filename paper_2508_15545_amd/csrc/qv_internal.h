// Internal types of the state-vector engine: host gate records, the block-pass
// program format read by the kernels, and the kernel launchers.
#pragma once

#include <complex>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

namespace qv {

using cd = std::complex<double>;

// Device amplitude types: (re, im) as one native 2-vector.
typedef double d2 __attribute__((ext_vector_type(2)));  // complex128, 16 bytes
typedef float f2 __attribute__((ext_vector_type(2)));   // complex64, 8 bytes

// ------------------------------------------------------------ host gates ---

// A gate after its matrix has been built (global qubit numbers).
enum GateKind : int32_t {
    G_DENSE1 = 0,  // 2x2 on q[0]
    G_DENSE2 = 1,  // 4x4 on (q[0], q[1]), index bit(q0) + 2 bit(q1)
    G_DIAG = 2,    // diagonal on q[0] (and q[1] if >= 0): d[bit(q0) + 2 bit(q1)]
};

// Generator of a trainable gate exp(-i theta G / 2).
// Generators of parametric gates; GEN_XY is a read of cx X + cy Y with the
// coefficients (cx, cy) given next to it (a rotated X/Y generator).
enum GenKind : int32_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_XY = 4 };

struct HostGate {
    int32_t kind = G_DENSE1;
    int32_t q[2] = {-1, -1};
    uint64_t ctrl = 0;   // control mask: acts only where all these bits are 1
    cd m[16];            // DENSE1: m[0..3]; DENSE2: m[0..15]; DIAG: d[0..3]
    int32_t param = -1;  // gradient slot
    int32_t gen = GEN_NONE;
};

// Conjugate transpose (the inverse of a unitary gate).
HostGate dagger(const HostGate& g);

// Bits the gate acts on non-diagonally / diagonally (controls are diagonal).
uint64_t dense_bits(const HostGate& g);
uint64_t diag_bits(const HostGate& g);

// ------------------------------------------------------- block programs ---

enum TileKind : int32_t {
    T_DENSE1 = 0,  // a = local target
    T_DENSE2 = 1,  // a, c = local targets (index bit(a) + 2 bit(c))
    T_DIAG = 2,    // qubits (qa, qc): local position a / c, or -1 with the
                   // global qubit in oa / oc (bit taken from the block base),
                   // or both -1 for an absent second qubit
    T_GRAD = 3,    // Im <s1|G|s0> over the block -> partial[slot]; gen in `gen`
    T_XPERM = 4,   // Pauli X on local target a (a swap; controls allowed)
    T_SWAP = 5,    // exchange of local qubits a and c
    T_PHASE = 6,   // product of diagonal gates as one phase per amplitude:
                   // terms phase[mat .. mat + cnt) (register kernel only)
    T_GRADZ = 7,   // several Z reads in one pass over the registers: ReadZ
                   // records phase[aux .. aux + cnt) (register kernel only)
    T_SIGN = 8,    // negate the amplitudes whose local bits cover lctrl (the
                   // block base covering gctrl): CZ, Z and controlled Z
                   // (register kernel only)
};

struct TileOp {
    // The register kernel's per-op fields come first (one scalar load).
    int32_t code;      // register kernel: flat dispatch code (RegCode)
    int32_t mat;       // offset of the matrix in the pass matrix array (complex
                       // entries); T_PHASE: its table of 2^r window phases
    // register kernel: the op acts on register k of a thread iff the thread's
    // bits cover tctrl (local controls outside the window) and bit k of
    // kmask is set (registers whose window bits cover the other controls)
    uint32_t tctrl;
    uint32_t kmask;
    uint64_t gctrl;    // control bits outside the block (global): block base must have them
    int32_t kind;
    int32_t a, c;      // local positions (-1: not local)
    int32_t oa, oc;    // global qubits for non-local diagonal bits (-1: none)
    uint32_t lctrl;    // control bits inside the block (local positions)
    int32_t gen;       // T_GRAD: GEN_Z, or GEN_XY with (cx, cy) at mats[mat]
    int32_t slot;      // T_GRAD: partial row
    int32_t j0, j1;    // register-window bits of a / c (register kernel; j0 < j1)
    int32_t cnt;       // T_PHASE: number of thread terms (a multiple of 4)
    int32_t aux;       // T_PHASE: offset of its first thread term in the phase array
};

// Flat dispatch codes of the register kernel: one switch case per op kind,
// window bits and control flavour, so that every op has one merge point.
enum RegCode : int32_t {
    RC_NONE = 0,
    RC_D1 = 1,      // + j0: dense 2x2 on window bit j0
    RC_D1C = 8,     // + j0: the same with local controls
    RC_X = 16,      // + j0: Pauli X (register swap)
    RC_XC = 24,     // + j0: X with local controls outside the window
    RC_CX = 32,     // + 5 jt + jc: X on jt controlled by window bit jc
    RC_D2 = 64,     // + 5 j0 + j1: dense 4x4 on window bits j0 < j1
    RC_D2C = 96,    // + 5 j0 + j1: the same with local controls
    RC_SW = 128,    // + 5 j0 + j1: SWAP
    RC_SWC = 160,   // + 5 j0 + j1: controlled SWAP
    RC_DIAG = 192,  // diagonal on any bits
    RC_PHASE = 193, // phase polynomial
    RC_GZ = 194,    // gradient read, G = Z
    RC_GZM = 195,   // several gradient reads with G = Z (T_GRADZ)
    RC_GXY = 200,   // + j0: gradient read, G = X or Y on window bit j0
    RC_D2M = 224,   // + 5 j0 + j1: dense 4x4 on window bits j0 < j1 on the matrix
                    // cores (complex64 single-state kernel only)
    RC_SIGN = 248,  // sign flip of the registers the op acts on (T_SIGN)
};

// Terms of a phase polynomial, angles in turns (1 = 2 pi). The phase of an
// amplitude is the sum of its terms; bit(p) is the amplitude's bit at local
// position p (p < 64) or at global qubit p - 64 (outside the block). The
// planner sorts them by the bits they involve (PhaseKind, host side only):
// the window-only part goes into a per-register table, the rest into
// PhaseTerm records for the register kernel.
enum PhaseKind : int32_t {
    PH_THREAD = 0,  // A += th * bit(p1) * bit(p2) (p2 < 0: linear); p1, p2 outside the window
    PH_MIXED = 1,   // eff[j] += th * bit(p1): window bit j times a bit outside the window
    PH_WLIN = 2,    // eff[j] += th: window bit j
    PH_WQUAD = 3,   // qq[j][j2] += th: window bits j < j2
    PH_CONST = 4,   // A += th
};

// A thread-dependent phase term of a T_PHASE op: it adds th (turns) when the
// thread index covers tmask (thread bit i = bit i of the thread index) and
// the block's global base index covers omask.
struct PhaseTerm {
    uint64_t omask;
    uint32_t tmask;
    uint32_t pad;
    double th;
    double pad2;
};
// First record of a T_PHASE op's range: the number of terms for A (the
// per-thread constant part) and for each window bit j's coefficient, in
// that order; each group is padded to a multiple of 4 with zero terms.
struct PhaseHead {
    int32_t count[8];  // [0]: A, [1 + j]: window bit j
};
static_assert(sizeof(PhaseHead) == sizeof(PhaseTerm), "phase records share one array");
// One read of a T_GRADZ op: Im <lambda|Z_q|phi> into partial row `slot`, with
// q's bit at window bit j, else at thread bit tbit, else global qubit oa.
struct ReadZ {
    int32_t j;
    int32_t tbit;
    int32_t oa;
    int32_t slot;
    uint64_t pad[2];
};
static_assert(sizeof(ReadZ) == sizeof(PhaseTerm), "read records share the phase array");

// A stage of a register-resident block pass: the amplitudes whose local
// positions are w[0..r) are held by one thread (register bit j <-> position
// w[j]); ops of the stage only act densely on those positions.
constexpr int kMaxRegBits = 5;
constexpr int kMaxThreadBits = 10;
struct StageHdr {
    int32_t w[kMaxRegBits];
    uint32_t wmask;
    int32_t n_ops;
    int32_t op_begin;  // relative to the pass's first op
    // thread bit i holds local position tpos[i]: lane bits first (ascending
    // positions), then the wave-index bits
    int32_t tpos[kMaxThreadBits];
    int32_t wave_local;  // exchange into this mapping: XCH_NONE / XCH_WAVE / XCH_BLOCK
    // register kernel: ops after the n_ops of the stage that are register
    // permutations applied to the registers' exchange offsets, not to their
    // values (see fold_trailing_perms)
    int32_t n_exit;
    // byte offset in the exchange buffer of register k's window bits
    // (lds_slot of the window part, times the slot size: 8 bytes for
    // complex64 and for the single-state complex128 kernel, which exchanges
    // real and imaginary parts separately; 16 bytes otherwise)
    uint32_t woff[1 << kMaxRegBits];
};

// LDS slot of local index l in the register kernel's exchange buffer: the
// index bits above the e lowest (e = 4 for 16-byte, 5 for 8-byte amplitudes,
// so that 2^e slots make a 256-byte row) are XOR-folded into the e lowest,
// which spreads power-of-two strides over the banks. The map is linear over
// XOR, so the slot of (thread bits | window bits) is the XOR of their slots.
constexpr uint32_t lds_slot(uint32_t l, int e)
{
    return l ^ (((l >> e) ^ (l >> (2 * e)) ^ (l >> (3 * e))) & ((1u << e) - 1));
}
// Kinds of register-window exchange: none (same mapping), within each wave
// (the wave positions stay, so no workgroup barrier), across the workgroup.
enum XchKind : int32_t { XCH_NONE = 0, XCH_WAVE = 1, XCH_BLOCK = 2 };
constexpr int kMaxGradPerPass = 128;
// Exchange buffer of the register kernel per state carried (a static LDS
// array, so that its addresses fold into the LDS instructions): 2^12 8-byte
// slots, or 2^11 16-byte ones for the two-state complex128 kernel.
constexpr int kRegLdsBytesPerState = 32768;

constexpr int kMaxLocal = 16;
constexpr int kMaxQubits = 34;

struct PassHdr {
    int32_t b;          // local qubits of the block (2^b amplitudes)
    int32_t n_outer;    // n - b
    int32_t n_ops;
    int32_t op_begin;   // first op in the op array
    int32_t local_q[kMaxLocal];   // global qubit of local position j (ascending)
    int32_t outer_q[kMaxQubits];  // global qubits not in the block (ascending)
    int32_t n_stages;   // register kernel: stages of this pass
    int32_t stage_begin;
    int32_t n_grad;     // gradient reads in this pass
    int32_t pad;
    StageHdr nat;       // register kernel: the load mapping
    StageHdr out;       // register kernel: the store mapping
    int32_t final_wave_local;  // exchange into `out` before the store (XchKind)
    int32_t pad3;
    // register kernel, derived from nat / out and local_q by the planner:
    // global qubit of thread bit i, and element offset of register k's
    // window bits, in the load and in the store mapping
    int32_t nat_tq[kMaxThreadBits];
    int32_t out_tq[kMaxThreadBits];
    uint64_t nat_koff[1 << kMaxRegBits];
    uint64_t out_koff[1 << kMaxRegBits];
};
static_assert(offsetof(PassHdr, nat_koff) % 8 == 0, "64-bit offsets are aligned");

// One launch of a plan.
struct PlanPass {
    enum Kind { BLOCK, SWEEP1, SWEEP2, SWEEPDIAG } kind = BLOCK;
    PassHdr hdr{};             // BLOCK
    std::vector<TileOp> ops;   // BLOCK (in stage order when stages are planned)
    std::vector<cd> mats;      // BLOCK: matrices referenced by ops
    std::vector<StageHdr> stages;  // BLOCK, register kernel
    std::vector<PhaseTerm> phase;  // BLOCK, register kernel: T_PHASE terms
    int reg_bits = 0;              // BLOCK, register kernel: window bits r
    HostGate gate;             // SWEEP*
    double bytes = 0;          // algorithmic HBM bytes
};

struct PlanOptions {
    int b = 12;            // local qubits per block
    int coalesce = 3;      // lowest qubits always kept in a block (contiguous runs)
    int n_states = 1;      // 2 for the adjoint sweep (phi and lambda together)
    int max_ops = 2048;    // ops per block pass
    int lookahead = 4096;  // gates scanned when filling a pass
    bool best_gain = true;     // also try growing each pass's local set by best gain per qubit
    int gain_candidates = 64;  // pending items tried as additions per growth step
    int lookahead_sets = 0;    // extra candidate local sets scored with the next pass (0: off)
    bool single_gate_sweeps = true;  // a pass holding one gate uses its sweep kernel
    int reg_bits = 0;      // register-window bits r (0: no stage planning)
    bool merge_diagonals = true;  // runs of diagonal gates become phase polynomials
    bool fuse_gates = true;       // one-qubit gates fold into two-qubit 4x4 updates
    bool prefuse = false;         // fuse one-qubit gates into two-qubit gates over the whole circuit first
    bool want_local = false;      // also bring controls / diagonal partners into a pass when there is room
    int want_reserve = 0;         // ... keeping this many local slots free for later targets
    int lds_elem = 0;             // bytes per exchange-buffer slot (0: the amplitude size)
    int wave_mode = 2;            // 0: workgroup-wide exchanges only; 1: fixed wave positions,
                                  // within-wave exchanges while they hold; 2: wave positions picked
                                  // from the pass's least-used positions
    bool park = false;            // move qubits between passes: each pass's store may permute its
                                  // local qubits (single-state register passes only)
    bool group_reads = true;      // Z reads waiting together share one op (register kernel)
    bool mfma = false;            // uncontrolled 4x4 updates as matrix-core ops (RC_D2M; complex64,
                                  // single state)
    bool fold_perms = true;       // register permutations at the end of a stage into the next
                                  // exchange's offsets (register kernel)
};

// A unit of planning: a gate, optionally preceded by a gradient read of its
// generator (adjoint sweep: the read happens before the gate is applied).
struct PlanItem {
    HostGate g;
    bool gate = true;      // false: only the gradient read
    bool grad = false;
    int32_t grad_slot = -1;
    cd gcoef = cd(0.0);    // g.gen == GEN_XY: the read is of real(gcoef) X + imag(gcoef) Y
};

std::vector<PlanPass> plan_circuit(int n, const std::vector<PlanItem>& items, const PlanOptions& opt,
                                   int elem_bytes);

// The same plan, each pass handed to `emit` as soon as it is complete, in
// order (a pass is not changed after that, so it can run while the next one
// is planned); emit returns false to stop planning.
void plan_circuit_stream(int n, const std::vector<PlanItem>& items, const PlanOptions& opt, int elem_bytes,
                         const std::function<bool(PlanPass&&)>& emit);

// Block size in local qubits for a state of n qubits.
int default_block_qubits(int n, int elem_bytes, int n_states);

// Register-window bits r of the register kernel (each thread holds 2^r
// amplitudes of each state); a block of b qubits runs on it when b - r is
// 6..9 (whole waves, at most 512 threads).
int reg_bits_for(int elem_bytes, int n_states);

// ---------------------------------------------------------- launchers ---

enum KernelFamily : int {
    KF_BLOCK = 0, KF_SWEEP1 = 1, KF_SWEEP2 = 2, KF_DIAG = 3, KF_REDUCE = 4, KF_INIT = 5,
    KF_COPY = 6, KF_ADJ_BLOCK = 7, KF_COUNT = 8
};

// Device Pauli-term batch for one x-mask group.
constexpr int kTermsPerLaunch = 16;
struct TermBatch {
    uint64_t x_mask;
    int32_t n_terms;
    int32_t pad;
    uint64_t z_mask[kTermsPerLaunch];
    double coeff_re[kTermsPerLaunch];  // coeff * Re(i^{#Y})
    double coeff_im[kTermsPerLaunch];  // coeff * Im(i^{#Y})
};

// All launchers enqueue on `st` and return the launch status.
template <typename T>
hipError_t launch_init_basis(T* psi, int n, uint64_t x, hipStream_t st);
template <typename T>
hipError_t launch_sweep1(T* psi, int n, const HostGate& g, hipStream_t st);
template <typename T>
hipError_t launch_sweep2(T* psi, int n, const HostGate& g, hipStream_t st);
template <typename T>
hipError_t launch_sweep_diag(T* psi, int n, const HostGate& g, hipStream_t st);
template <typename T>
hipError_t launch_block_pass(T* s0, T* s1, int n, int n_states, const PassHdr* d_hdr, const TileOp* d_ops,
                             const T* d_mats, int b, double* grad_partials, int64_t grad_stride,
                             hipStream_t st);
// Register-resident block pass (stages planned); same arguments plus the
// stage table.
template <typename T>
hipError_t launch_block_reg(T* s0, T* s1, int n, int n_states, int reg_bits, const PassHdr* d_hdr,
                            const StageHdr* d_stages, const TileOp* d_ops, const T* d_mats,
                            const PhaseTerm* d_phase, int b, double* grad_partials, int64_t grad_stride,
                            hipStream_t st);
template <typename T>
hipError_t launch_pauli_expect(const T* psi, int n, const TermBatch& tb, double* partials, int n_part,
                               hipStream_t st);
template <typename T>
hipError_t launch_pauli_apply(const T* psi, T* dst, int n, const TermBatch& tb, bool accumulate,
                              hipStream_t st);
// Up to kBatchesPerLaunch x-mask groups in one pass over the state.
constexpr int kBatchesPerLaunch = 8;
struct TermBatchSet {
    int32_t count;
    int32_t pad;
    TermBatch b[kBatchesPerLaunch];
};
template <typename T>
hipError_t launch_pauli_apply_multi(const T* psi, T* dst, int n, const TermBatch* batches, int count,
                                    bool accumulate, hipStream_t st);
template <typename T>
hipError_t launch_inner(const T* a, const T* b, int n, double* partials, int n_part, hipStream_t st);
template <typename T>
hipError_t launch_grad_sweep(const T* phi, const T* lam, int n, int q, int gen, double* partials, int n_part,
                             hipStream_t st);
template <typename Ta, typename Tb>
hipError_t launch_compare(const Ta* a, const Tb* b, int n, double* partials, int n_part, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// out[r] = sum over c of partials[r * stride + c], c < count, fixed order.
hipError_t launch_sum_rows(const double* partials, int rows, int64_t count, int64_t stride, double* out,
                           hipStream_t st);
// out[0] = sum of rows[0..count) added one after another in index order.
hipError_t launch_sum_ordered(const double* rows, int count, double* out, hipStream_t st);
// Compare partial rows combine: max for row 0, sums for the rest (6 rows).
hipError_t launch_compare_finish(const double* partials, int n_part, double* out, hipStream_t st);

constexpr int kReduceBlocks = 2048;  // fixed partial count of the reductions

}  // namespace qv
