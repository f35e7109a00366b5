// Internal types of the state-vector engine: host gate records, the block-pass
// program format read by the kernels, and the kernel launchers.
#pragma once

#include <complex>
#include <cstdint>
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
enum GenKind : int32_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3 };

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
};

struct TileOp {
    int32_t kind;
    int32_t a, c;      // local positions (-1: not local)
    int32_t oa, oc;    // global qubits for non-local diagonal bits (-1: none)
    uint32_t lctrl;    // control bits inside the block (local positions)
    int32_t gen;       // T_GRAD: GEN_X / GEN_Y / GEN_Z
    int32_t slot;      // T_GRAD: partial row
    uint64_t gctrl;    // control bits outside the block (global): block base must have them
    int32_t mat;       // offset of the matrix in the pass matrix array (complex entries)
    int32_t pad;
};

constexpr int kMaxLocal = 16;
constexpr int kMaxQubits = 34;

struct PassHdr {
    int32_t b;          // local qubits of the block (2^b amplitudes)
    int32_t n_outer;    // n - b
    int32_t n_ops;
    int32_t op_begin;   // first op in the op array
    int32_t local_q[kMaxLocal];   // global qubit of local position j (ascending)
    int32_t outer_q[kMaxQubits];  // global qubits not in the block (ascending)
    int32_t pad[2];
};

// One launch of a plan.
struct PlanPass {
    enum Kind { BLOCK, SWEEP1, SWEEP2, SWEEPDIAG } kind = BLOCK;
    PassHdr hdr{};             // BLOCK
    std::vector<TileOp> ops;   // BLOCK
    std::vector<cd> mats;      // BLOCK: matrices referenced by ops
    HostGate gate;             // SWEEP*
    double bytes = 0;          // algorithmic HBM bytes
};

struct PlanOptions {
    int b = 12;            // local qubits per block
    int coalesce = 3;      // lowest qubits always kept in a block (contiguous runs)
    int n_states = 1;      // 2 for the adjoint sweep (phi and lambda together)
    int max_ops = 2048;    // ops per block pass
    int lookahead = 4096;  // gates scanned when filling a pass
    bool single_gate_sweeps = true;  // a pass holding one gate uses its sweep kernel
};

// A unit of planning: a gate, optionally preceded by a gradient read of its
// generator (adjoint sweep: the read happens before the gate is applied).
struct PlanItem {
    HostGate g;
    bool grad = false;
    int32_t grad_slot = -1;
};

std::vector<PlanPass> plan_circuit(int n, const std::vector<PlanItem>& items, const PlanOptions& opt,
                                   int elem_bytes);

// Block size in local qubits for a state of n qubits.
int default_block_qubits(int n, int elem_bytes, int n_states);

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
template <typename T>
hipError_t launch_pauli_expect(const T* psi, int n, const TermBatch& tb, double* partials, int n_part,
                               hipStream_t st);
template <typename T>
hipError_t launch_pauli_apply(const T* psi, T* dst, int n, const TermBatch& tb, bool accumulate,
                              hipStream_t st);
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
// Compare partial rows combine: max for row 0, sums for the rest (6 rows).
hipError_t launch_compare_finish(const double* partials, int n_part, double* out, hipStream_t st);

constexpr int kReduceBlocks = 2048;  // fixed partial count of the reductions

}  // namespace qv
