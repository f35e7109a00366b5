/*
 * sv.h - C ABI of the MI355X state-vector gate engine (libqvec.so).
 *
 * The engine applies quantum gates to a dense vector of 2^n complex
 * amplitudes held in device memory (QVecOpt, arXiv 2508.15545, Sec. II
 * Eq. 1-2), by amplitude pairing: a one-qubit gate on qubit k updates every
 * pair (i, i XOR 2^k) with its 2x2 matrix (Sec. III.A Eq. 5), a two-qubit
 * gate updates the quadruples spanned by its two qubits (Sec. III.C). Runs
 * of gates are executed together on blocks of amplitudes staged on chip
 * (the block storage of Sec. III.C Eq. 7-8, and the one-traversal batching
 * of Sec. III.E), with the same result as applying them one by one.
 *
 * Conventions for every call:
 *   - Qubit k is bit k of the amplitude index (the partner of i is i ^ 2^k).
 *   - Amplitudes are interleaved (re, im): SV_C128 stores two doubles
 *     (16 bytes, the paper's S_state), SV_C64 two floats (8 bytes).
 *   - Host matrices are row-major complex, stored as (re, im) pairs of
 *     doubles; for two-target matrices the row/column index is
 *     m = bit(targets[0]) + 2 * bit(targets[1]). SV_C64 rounds them to
 *     float once; all reductions accumulate in double for both dtypes.
 *   - Every call returns an sv_status and never throws. On an argument
 *     error it returns SV_EINVAL (or SV_EUNSUPPORTED) before touching the
 *     device and the state is left unchanged; sv_last_error() then gives a
 *     message (thread-local, valid until the next call on that thread).
 *   - Apply calls only enqueue work on the handle's HIP stream and return.
 *     A device fault surfaces as SV_EDEVICE at the next call that waits for
 *     the stream (sv_norm2, sv_expect, sv_adjoint_grad, sv_compare, sv_sync).
 *   - Host arrays passed in are read during the call only.
 *   - Calls on one handle must not overlap (one host thread at a time).
 */
#ifndef QVEC_SV_H
#define QVEC_SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sv_status {
    SV_OK = 0,
    SV_EINVAL = 1,       /* bad argument; nothing was enqueued */
    SV_ENOMEM = 2,       /* a device or pinned-host allocation failed */
    SV_EDEVICE = 3,      /* a HIP runtime call or kernel failed */
    SV_EUNSUPPORTED = 4  /* valid but not implemented (e.g. controls on a two-target gate) */
} sv_status;

typedef enum sv_dtype {
    SV_C64 = 1,  /* complex64: 8 bytes per amplitude */
    SV_C128 = 2  /* complex128: 16 bytes per amplitude */
} sv_dtype;

/* Gate kinds. Matrices follow OpenQASM 2 (global phase included):
 *   RX/RY/RZ(t) = exp(-i t P / 2) for P = X/Y/Z; P(l) = diag(1, e^{il});
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]];
 *   CNOT/CZ/CP use qubits = (control, target); CP(l) puts e^{il} on |11>;
 *   SWAP exchanges its two qubits; MATRIX1/MATRIX2 take `matrix`. */
typedef enum sv_op {
    SV_OP_MATRIX1 = 0,
    SV_OP_MATRIX2 = 1,
    SV_OP_H = 2,
    SV_OP_X = 3,
    SV_OP_Y = 4,
    SV_OP_Z = 5,
    SV_OP_S = 6,
    SV_OP_SDG = 7,
    SV_OP_T = 8,
    SV_OP_TDG = 9,
    SV_OP_RX = 10,
    SV_OP_RY = 11,
    SV_OP_RZ = 12,
    SV_OP_P = 13,
    SV_OP_U3 = 14,
    SV_OP_CNOT = 15,
    SV_OP_CZ = 16,
    SV_OP_CP = 17,
    SV_OP_SWAP = 18
} sv_op;

/* One gate of a circuit (host memory). */
typedef struct sv_gate {
    int32_t op;           /* sv_op */
    int32_t qubits[2];    /* qubits[0] for one-qubit ops; (control, target) for
                             CNOT/CZ/CP; (t0, t1) for SWAP and MATRIX2 */
    int32_t n_controls;   /* 0..2 extra control qubits (one-qubit ops only):
                             the gate acts where every control bit is 1 */
    int32_t controls[2];
    int32_t param_index;  /* gradient slot for RX/RY/RZ (angles[0] is the
                             angle in use), -1 for a fixed gate */
    int32_t reserved;     /* must be 0 */
    double angles[3];     /* RX/RY/RZ/P/CP: angles[0]; U3: (theta, phi, lambda) */
    double matrix[32];    /* MATRIX1: 2x2 (8 doubles), MATRIX2: 4x4 (32 doubles) */
} sv_gate;

/* Pauli string coeff * P: bit k of x_mask / z_mask puts X / Z on qubit k,
 * both bits put Y there (P|j> = i^{#Y} (-1)^{popcount(j & z_mask)} |j ^ x_mask>). */
typedef struct sv_pauli {
    double coeff;
    uint64_t x_mask;
    uint64_t z_mask;
} sv_pauli;

/* Result of sv_compare. */
typedef struct sv_diff {
    double max_abs;   /* max_i |a_i - b_i| */
    double l2;        /* sqrt(sum_i |a_i - b_i|^2) */
    double inner_re;  /* Re <a|b> */
    double inner_im;  /* Im <a|b> */
    double norm2_a;   /* <a|a> */
    double norm2_b;   /* <b|b> */
} sv_diff;

/* Host-side summary of how sv_apply_fused would execute a circuit. */
typedef struct sv_plan_stats {
    int64_t n_gates;        /* gates in the circuit */
    int64_t n_passes;       /* kernel launches that sweep the whole state */
    int64_t n_block_passes; /* of which: block passes (several gates each) */
    int64_t block_qubits;   /* qubits per on-chip block (b) */
    double bytes_moved;     /* algorithmic HBM bytes of all passes */
    int64_t n_stages;       /* register windows over all block passes */
    int64_t n_ops;          /* block-pass ops (after merging diagonal runs) */
    int64_t n_phase_ops;    /* merged diagonal runs */
} sv_plan_stats;

/* Summary of one sv_host_apply call. */
typedef struct sv_host_stats {
    int64_t n_passes;      /* passes over the host state */
    int64_t n_chunks;      /* chunks per pass: 2^(n - c) */
    int64_t chunk_qubits;  /* c: qubits of a chunk (min(chunk_qubits, n)) */
    int64_t high_qubits;   /* h: qubits of a chunk chosen per pass above its contiguous runs */
    double bytes_h2d;      /* bytes copied host -> device */
    double bytes_d2h;      /* bytes copied device -> host */
    double seconds;        /* wall time of the call */
} sv_host_stats;

typedef struct sv_state_t* sv_state;

/* Create a handle for an n-qubit state (Sec. II Eq. 1-2: 2^n amplitudes of
 * S_state bytes).
 *   n_qubits   1..34 (34 only for SV_C64 in practice: 2^34 * 8 = 128 GiB)
 *   device_buf device memory of >= 2^n * S_state bytes, 16-byte aligned,
 *              owned by the caller (e.g. a torch tensor) and not freed by the
 *              library; NULL makes the library allocate (freed by sv_free)
 *   hip_stream hipStream_t the handle enqueues on (NULL = default stream)
 * The contents of the buffer are left as they are (use sv_set_basis).
 * The handle also owns small device/pinned buffers for gate tables and
 * reduction partials. Errors: SV_EINVAL (n out of range, buffer too small
 * or misaligned, null out), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_alloc(sv_state* out, int n_qubits, sv_dtype dtype, void* device_buf,
                   size_t buf_bytes, void* hip_stream);

/* Release the handle (waits for its stream first). NULL is a no-op. */
sv_status sv_free(sv_state s);

/* Raw device pointer, qubit count and dtype of a handle. */
void* sv_data(sv_state s);
int sv_num_qubits(sv_state s);
sv_dtype sv_get_dtype(sv_state s);

/* Set the amplitude vector of Sec. II Eq. 1 to the basis state e_x:
 * alpha_x = 1, every other alpha_i = 0. One write pass over the state.
 * Errors: SV_EINVAL if x >= 2^n. */
sv_status sv_set_basis(sv_state s, uint64_t x);

/* Apply one gate given by its matrix: a one-target 2x2 (Sec. III.A Eq. 5)
 * or a two-target 4x4 (Sec. III.C) on the quadruples of its targets, with
 * 0..2 control qubits for one-target matrices. One sweep over the affected
 * part of the state. Targets and controls must be distinct and < n.
 * matrix: 8 or 32 doubles. Unitarity is the caller's contract. */
sv_status sv_apply_gate(sv_state s, int n_targets, const int* targets, int n_controls,
                        const int* controls, const double* matrix);

/* Apply a circuit gate by gate: one sweep kernel per gate (no fusion). */
sv_status sv_apply_unfused(sv_state s, const sv_gate* gates, int n_gates);

/* Apply a circuit with fusion: consecutive gates are grouped into passes,
 * each one HBM round trip of the state (Sec. III.C block storage, Sec. III.E
 * one traversal for a batch of gates); diagonal gates join any pass. The
 * result equals applying the gates one by one in order (up to rounding).
 * On states of 1 GiB and more each pass is launched as soon as it is planned
 * (QVEC_STREAM_PLAN=0 / 1 turns that off / on at any size).
 * Errors: SV_EINVAL for a bad op, qubit, control or reserved field (the
 * state is unchanged); SV_EINVAL from the planner itself, which valid input
 * does not produce, may come after passes planned before it were applied
 * (its message says so). */
sv_status sv_apply_fused(sv_state s, const sv_gate* gates, int n_gates);

/* Plan statistics for sv_apply_fused of this circuit on an n-qubit state
 * of this dtype (host only; nothing is launched). */
sv_status sv_plan(int n_qubits, sv_dtype dtype, const sv_gate* gates, int n_gates,
                  sv_plan_stats* out);

/* Out-of-core tier (Sec. III.B-C: the state lives in a slower tier and is
 * staged block by block; every queued gate whose pairs lie in a staged block
 * is applied before it is written back). The state is host_state, 2^n
 * amplitudes of S_state bytes in pinned host memory (hipHostMalloc, or a
 * torch tensor with pin_memory), 16-byte aligned, read and written in place.
 * A chunk is the 2^c indices (c = min(chunk_qubits, n)) that agree outside
 * the lowest c - h qubits (contiguous runs) and h high qubits chosen per
 * pass; a pass takes every gate whose qubits (targets and controls) lie in
 * the chunk and that commutes with the gates it leaves for later passes (on
 * each shared qubit both act diagonally), so the result equals applying the
 * gates in order; each chunk of a pass goes host -> device,
 * through the fused device path (as sv_apply_fused on a c-qubit state) and
 * back. Three device buffers of 2^c * S_state bytes are allocated for the call
 * and freed before it returns; copies in, passes and copies out of three
 * chunks overlap on three streams of the current device. Synchronous: the
 * host state holds the result on return. stats may be NULL.
 * Errors: SV_EINVAL (null or misaligned state, n or chunk_qubits out of
 * range, a bad gate), SV_EUNSUPPORTED (a gate needs more high qubits than a
 * chunk holds), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_host_apply(void* host_state, int n_qubits, sv_dtype dtype, const sv_gate* gates,
                        int n_gates, int chunk_qubits, sv_host_stats* stats);

/* The calls from here to sv_adjoint_grad are additions of this engine, not
 * part of the paper's method (which only applies gates): FP64 reductions
 * over the state and the adjoint gradient of an expectation value.
 *
 * out = <psi|psi> = sum_i |alpha_i|^2 over the amplitudes of Sec. II Eq. 1
 * (1 for a normalized state), accumulated in double. Waits for the stream. */
sv_status sv_norm2(sv_state s, double* out);

/* out = <psi|H|psi> for H = sum_t terms[t].coeff * P_t (an addition: the
 * paper defines no observable), accumulated in double with a fixed-shape
 * (deterministic) reduction. Waits for the stream.
 * Errors: SV_EINVAL if a mask has bits >= n. */
sv_status sv_expect(sv_state s, const sv_pauli* terms, int n_terms, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * expectation of sv_expect on a raw device state, with no handle and no
 * allocation. Enqueues on hip_stream (NULL = default stream) of the current
 * device, which must hold state and d_out, and returns without waiting.
 *   state   2^n_qubits amplitudes of dtype, device memory, 16-byte aligned
 *   terms   n_terms Pauli strings (host, read during the call); the terms
 *           form batches of up to 16 terms sharing one x_mask, at most 64
 *   d_out   one double in device memory (8-byte aligned): on completion it
 *           holds <psi|H|psi>, bit-identical to what sv_expect returns for
 *           the same state and terms (same launches, same order of sums)
 * Its scratch is a fixed 1 MiB device array per GPU (64 batches x 2048
 * partial sums, then 64 batch sums), held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU (on
 * different streams, or from different threads) race on it and must be
 * ordered by the caller. Errors: SV_EINVAL (bad dtype, n_qubits, pointer,
 * alignment, mask >= 2^n, non-finite coefficient, more than 64 batches),
 * SV_EDEVICE; on an error nothing is enqueued. */
sv_status sv_expect_noalloc(const void* state, int n_qubits, sv_dtype dtype, const sv_pauli* terms,
                            int n_terms, double* d_out, void* hip_stream);

/* dst = H psi (an addition: the seed of the adjoint sweep; same dtype and
 * size as s; dst_buf is caller device memory of >= 2^n * S_state bytes, 16-byte
 * aligned, not overlapping the state). Enqueue only. */
sv_status sv_apply_pauli_sum(sv_state s, const sv_pauli* terms, int n_terms, void* dst_buf,
                             size_t dst_bytes);

/* Adjoint gradient of f(theta) = <psi|H|psi> with psi = U_L .. U_1 psi_0 (an
 * addition: the paper has no parameterized circuits; the reverse sweep
 * applies each inverse gate by the same pair updates, Sec. III.A Eq. 5).
 * On entry s holds psi = U_L .. U_1 psi_0 (the caller ran the circuit);
 * on return it holds the state recomputed back to psi_0 by applying the
 * inverse gates (no checkpoints). work_buf (>= 2^n * S_state bytes, device,
 * caller-owned) holds lambda = H psi during the sweep. For each trainable
 * gate U_l = exp(-i theta G / 2) (RX/RY/RZ with param_index >= 0),
 * grad_out[param_index] += Im <lambda_l | G | phi_l>; gates sharing a slot
 * add up. grad_out (n_params doubles, host) is overwritten; expval_out
 * (host, may be NULL) receives f. Waits for the stream. */
sv_status sv_adjoint_grad(sv_state s, const sv_gate* gates, int n_gates, const sv_pauli* terms,
                          int n_terms, void* work_buf, size_t work_bytes, double* grad_out,
                          int n_params, double* expval_out);

/* Compare two states of the same qubit count (any dtypes) on the device,
 * in double: max-abs and l2 of the difference, <a|b>, norms. Waits. */
sv_status sv_compare(sv_state a, sv_state b, sv_diff* out);

/* Copy bytes device-to-device with the library's streaming copy kernel on
 * s's stream (the bandwidth reference for the sweeps). dst and src must be
 * 16-byte aligned, bytes a multiple of 16, and must not overlap. */
sv_status sv_copy(sv_state s, void* dst, const void* src, size_t bytes);

/* Wait for all work enqueued on the handle's stream. */
sv_status sv_sync(sv_state s);

/* Per-kernel timing with HIP events on the handle's stream. While enabled,
 * every launch is bracketed by events; sv_timing_read waits for the stream
 * and returns, for kernel family `kernel` (0 = block pass, 1 = one-qubit
 * sweep, 2 = two-qubit sweep, 3 = diagonal sweep, 4 = reductions, 5 = basis
 * init, 6 = copy, 7 = adjoint block pass), the launch count and total
 * milliseconds since the last reset. */
sv_status sv_timing_enable(sv_state s, int on);
sv_status sv_timing_reset(sv_state s);
sv_status sv_timing_read(sv_state s, int kernel, int64_t* launches, double* total_ms);

/* Message of the last error on this thread ("" if none). */
const char* sv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
