"""Benchmark: gate-applications/s of the state-vector engine on one MI355X.

Workload (one step): on a 29-qubit complex128 state (8 GiB in HBM)
  (a) reset to |0..0>, run the random circuit of depth 40 (per layer U3 with
      seeded angles on every qubit, then CNOTs on a seeded random matching:
      1720 gates), then the FP64 norm;
  (b) reset to a seeded random basis state, run the textbook QFT (449 gates),
      then the FP64 norm.
value = gates applied per second over the timed steps (2169 gates per step),
which run without per-launch instrumentation. The same steps are then run
again with HIP events around every launch on the launch stream (library
timing) for the dominant kernel's achieved bandwidth; the CPU baseline is
the FP64 oracle on bounded samples of the same workload.

Besides the headline value the line carries, measured in the same run:
  sweeps            one-qubit sweep kernel bandwidth for every target qubit;
  two_qubit_sweeps  unfused CNOT / SWAP / CZ / CP / 4x4 sweeps on several
                    qubit pairs, against each one's algorithmic bytes;
  copy              the library's streaming copy kernel (bandwidth reference);
  c64_vs_c128       33-qubit random U3 + CZ circuit, depth 30, in complex128
                    and complex64 (speedup and the device-side difference);
  adjoint           24-qubit hardware-efficient ansatz, 20 layers (960
                    parameters), complex64: forward, adjoint backward, their
                    ratio, 2 x 960 parameter-shift evaluations, gradient
                    error against the complex128 adjoint;
  host_tier         30-qubit complex128 state in pinned host memory through
                    the GPU in chunks, beside a pinned-copy probe.

Prints one JSON line. Flags: --gpus (only 1), --steps, --warmup, --n,
--dtype c128|c64, --no-cpu (skip the oracle leg), --no-extras, and the probe
modes listed by --help.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import circuits as C  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


# The block kernel's HBM traffic per launch is read from the committed
# rocprofv3 summary, and only while the kernel sources still hash to what
# was profiled (otherwise the figure no longer describes this kernel).
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_block_reg_29q_c128_bench.md")
KERNEL_SOURCES = ["kernels_block.hip", "device_common.h", "qv_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2508_15545_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(n: int, dtype: str):
    """Counter bytes per block-pass launch for the profiled workload, or None."""
    if n != 29 or dtype != "c128" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    rec = {}
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            if line.startswith("traffic-record:"):
                rec = dict(kv.split("=", 1) for kv in line.split(":", 1)[1].split())
    if rec.get("source-sha256") != kernel_source_hash():
        return None
    return float(rec["bytes-per-launch"])


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(n: int):
    rand = C.random_u3_layers(n, 40, seed=0, entangler="cx")
    x = C.random_basis_index(n, seed=0)
    qft = C.qft(n)
    return rand, x, qft


def run_step(st, rand, x, qft):
    st.set_basis(0).apply(rand)
    n1 = st.norm2()
    st.set_basis(x).apply(qft)
    n2 = st.norm2()
    return n1, n2


def host_cpus() -> int:
    """CPUs this process may run on (what nproc reports)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def gate_bytes(g, n, elem):
    """Algorithmic HBM bytes of one unfused gate on an n-qubit state: a dense
    one-qubit gate (and RZ, which phases both halves) or a general 4x4 reads
    and writes every amplitude; CNOT and SWAP move half the state each way,
    CZ and CP the |11> quarter."""
    S = (1 << n) * elem
    if g.op in ("cx", "swap"):
        return S
    if g.op in ("cz", "cp"):
        return S / 2
    return 2 * S


def _oracle_rate(oracle, n, s, gates, budget):
    """Apply gates one by one to s until the time budget is crossed; return
    (gates done, seconds) around the gate loop only."""
    t0 = time.perf_counter()
    done = 0
    for g in gates:
        oracle.apply_gate(s, n, g)
        done += 1
        if time.perf_counter() - t0 > budget:
            break
    return done, time.perf_counter() - t0


def cpu_baseline(n: int, rand, x, qft, budget: float = 8.0):
    """The FP64 oracle on bounded samples of the same workload (the same
    gates on the same 2^n-amplitude state), timed around the gate loop only:
    the random circuit from |0..0> and the QFT from the seeded basis state on
    all the oracle's threads, then the random circuit again on one thread.
    Each leg stops after the gate that crosses its time budget."""
    import oracle

    threads = oracle.num_threads()
    s = oracle.basis_state(n, 0)
    d_r, t_r = _oracle_rate(oracle, n, s, rand, budget)
    s = oracle.basis_state(n, x)
    d_q, t_q = _oracle_rate(oracle, n, s, qft, budget / 2)
    oracle.set_threads(1)
    s = oracle.basis_state(n, 0)
    d_1, t_1 = _oracle_rate(oracle, n, s, rand, budget)
    oracle.set_threads(threads)
    del s
    moved = sum(gate_bytes(g, n, 16) for g in rand[:d_r]) + sum(gate_bytes(g, n, 16) for g in qft[:d_q])
    return {
        "value": (d_r + d_q) / (t_r + t_q),
        "unit": "gate-applications/s",
        "cores": threads,
        "effective_gbs": moved / (t_r + t_q) / 1e9,
        "effective_gbs_1_thread": sum(gate_bytes(g, n, 16) for g in rand[:d_1]) / t_1 / 1e9,
        "kind": "oracle",
        "sample": f"{n}-qubit complex128 state: first {d_r} gates of the random U3 + CNOT circuit ({t_r:.1f} s) "
                  f"and first {d_q} gates of the QFT ({t_q:.1f} s) on {threads} threads; "
                  f"first {d_1} gates of the random circuit on 1 thread ({t_1:.1f} s)",
        "value_1_thread": d_1 / t_1,
        "host_cpus": host_cpus(),
        "host_mem_gib": round(os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 2 ** 30, 1),
    }


def copy_probe(qv, B, n, dtype, elem, reps):
    print(json.dumps({"copy_probe": copy_rate(qv, B, n, dtype, elem, reps)}), flush=True)
    return 0


def copy_rate(qv, B, n, dtype, elem, reps):
    """Read + write bandwidth of the library's copy kernel at the state size."""
    torch.cuda.set_device(0)
    st = qv.State(n, dtype, device="cuda:0")
    src = st.tensor
    src.zero_()
    dst = torch.empty_like(src)
    qv.copy(st, dst, src)
    st.timing(True)
    st.timing_reset()
    for _ in range(reps):
        qv.copy(st, dst, src)
    launches, ms = st.timing_read(B.KF_COPY)
    nbytes = (1 << n) * elem
    gbs = 2.0 * nbytes * launches / (ms / 1e3) / 1e9
    del st, src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_launch_read": nbytes, "bytes_per_launch_write": nbytes, "launches": launches,
            "avg_ms": ms / launches, "gbs": gbs}


def sweep_rates(qv, B, n, dtype, elem, reps):
    """HBM GB/s of the one-qubit sweep kernel (unfused U3) for every target:
    each sweep reads and writes the whole state once."""
    torch.cuda.set_device(0)
    st = qv.State(n, dtype, device="cuda:0").set_basis(0)
    rng = C.rng_for(1)
    out = {}
    for k in range(n):
        g = [C.gate("u3", k, params=rng.uniform(0, 2 * math.pi, 3))]
        st.apply(g, fused=False)  # warm
        st.timing(True)
        st.timing_reset()
        for _ in range(reps):
            st.apply(g, fused=False)
        launches, ms = st.timing_read(B.KF_SWEEP1)
        st.timing(False)
        out[k] = 2.0 * (1 << n) * elem / (ms / launches / 1e3) / 1e9
    vals = list(out.values())
    return {"gbs_by_target": out, "min_gbs": min(vals), "mean_gbs": sum(vals) / len(vals),
            "frac_of_peak_min": min(vals) / HBM_PEAK_GBS, "frac_of_peak_mean": sum(vals) / len(vals) / HBM_PEAK_GBS}


TWO_QUBIT_PAIRS = [(0, 1), (2, 11), (11, 20), (20, 28), (27, 5)]


def two_qubit_sweep_rates(qv, B, n, dtype, elem, reps):
    """Unfused two-qubit gates, one sweep kernel each: CNOT (the controlled
    one-qubit sweep over the control-1 half), SWAP (the pairs whose two bits
    differ), CZ and CP (the |11> quarter) and a general 4x4 (every
    quadruple), for several qubit pairs. GB/s against the algorithmic bytes
    of each: CNOT and SWAP 2^n S, CZ and CP 2^(n-1) S, 4x4 2 * 2^n S."""
    torch.cuda.set_device(0)
    st = qv.State(n, dtype, device="cuda:0").set_basis(0)
    rng = C.rng_for(2)
    S = (1 << n) * elem
    kinds = {"cx": (B.KF_SWEEP1, S), "swap": (B.KF_SWEEP2, S), "cz": (B.KF_DIAG, S / 2),
             "cp": (B.KF_DIAG, S / 2), "mat2": (B.KF_SWEEP2, 2 * S)}
    out = {}
    for kind, (fam, nbytes) in kinds.items():
        rates = {}
        for a, b in TWO_QUBIT_PAIRS:
            if kind == "mat2":
                g = C.gate("mat2", a, b, params=C.matrix_params(C.random_unitary(4, rng)))
            elif kind == "cp":
                g = C.gate("cp", a, b, params=(0.7,))
            else:
                g = C.gate(kind, a, b)
            st.apply([g], fused=False)
            st.timing(True)
            st.timing_reset()
            for _ in range(reps):
                st.apply([g], fused=False)
            launches, ms = st.timing_read(fam)
            st.timing(False)
            rates[f"{a},{b}"] = round(nbytes / (ms / launches / 1e3) / 1e9)
        out[kind] = {"gbs_by_pair": rates, "min_gbs": min(rates.values()),
                     "frac_of_peak_min": min(rates.values()) / HBM_PEAK_GBS}
    del st
    torch.cuda.empty_cache()
    return out


def timed(fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, r


def pcie_probe(gib: int = 2, reps: int = 3):
    """Pinned host <-> device copy bandwidth (the host tier's roofline): one
    direction at a time, then both at once on two streams, each copy a
    single large transfer of `gib` GiB."""
    n = gib << 27  # complex128 elements
    h_in = torch.empty(n, dtype=torch.complex128, pin_memory=True)
    h_out = torch.empty(n, dtype=torch.complex128, pin_memory=True)
    d_in = torch.empty(n, dtype=torch.complex128, device="cuda")
    d_out = torch.empty(n, dtype=torch.complex128, device="cuda")
    h_in.zero_()
    d_out.zero_()
    nbytes = n * 16
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def run(h2d, d2h):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if h2d:
                with torch.cuda.stream(s1):
                    d_in.copy_(h_in, non_blocking=True)
            if d2h:
                with torch.cuda.stream(s2):
                    h_out.copy_(d_out, non_blocking=True)
        torch.cuda.synchronize()
        return (h2d + d2h) * nbytes * reps / (time.perf_counter() - t0) / 1e9

    run(True, True)
    out = {"h2d_gbs": run(True, False), "d2h_gbs": run(False, True), "both_gbs": run(True, True),
           "bytes_per_copy": nbytes}
    del h_in, h_out, d_in, d_out
    torch.cuda.empty_cache()
    torch._C._host_emptyCache()
    return out


def host_tier(qv, n=30, chunk=28, depth=4):
    """Out-of-core tier: the random U3 + CNOT circuit on a complex128 state in
    pinned host memory, chunks of 2^chunk amplitudes through the GPU. The
    state is allocated and set outside the timed call; the call's own clock
    covers the copies in and out and the device passes. The circuit runs
    twice and the second call is the figure (the first pays for first-touch
    costs of the pinned pages and the chunk buffers); the norm is taken after
    both. The pinned-copy probe beside it is the PCIe roofline of the tier."""
    import gc
    probe = pcie_probe()
    st = torch.zeros(1 << n, dtype=torch.complex128, pin_memory=True)
    st[0] = 1
    circ = C.random_u3_layers(n, depth, 0)
    first = qv.host_apply(st, circ, chunk)
    s = qv.host_apply(st, circ, chunk)
    step = 1 << 24  # norm in slices, so no state-sized temporaries
    norm = sum(float(torch.sum(st[i:i + step].abs() ** 2)) for i in range(0, 1 << n, step))
    del st
    gc.collect()
    # hand the pinned block back while the HIP runtime is up, rather than
    # from the host allocator's cache at interpreter exit
    torch._C._host_emptyCache()
    moved = s["bytes_h2d"] + s["bytes_d2h"]
    gbs = moved / s["seconds"] / 1e9
    return {"n_qubits": n, "dtype": "complex128", "state_gib": (1 << n) * 16 / 2 ** 30, "gates": len(circ),
            "depth": depth, "chunk_qubits": s["chunk_qubits"], "high_qubits": s["high_qubits"],
            "chunks_per_pass": s["n_chunks"], "passes": s["n_passes"], "seconds": s["seconds"],
            "first_call_seconds": first["seconds"],
            "gate_app_per_s": len(circ) / s["seconds"], "pcie_gbs_both_directions": gbs,
            "pcie_probe": probe, "frac_of_probe_both": gbs / probe["both_gbs"],
            "norm_error": abs(norm - 1)}


def c64_vs_c128(qv, n=33, depth=30):
    """Random U3 + CZ matching on n qubits in both dtypes on one GPU."""
    free = torch.cuda.mem_get_info()[0]
    if free < (1 << n) * 24 + (8 << 30):
        return {"skipped": f"needs {((1 << n) * 24) / 2**30:.0f} GiB free"}
    circ = C.random_u3_layers(n, depth, seed=0, entangler="cz")
    a = qv.State(n, torch.complex128)
    b = qv.State(n, torch.complex64)
    a.set_basis(0).apply(circ)
    b.set_basis(0).apply(circ)
    # median of three timed runs each, after the warm run above
    t128 = sorted(timed(lambda: a.set_basis(0).apply(circ))[0] for _ in range(3))[1]
    t64 = sorted(timed(lambda: b.set_basis(0).apply(circ))[0] for _ in range(3))[1]
    d = a.compare(b)
    fid = (d["inner_re"] ** 2 + d["inner_im"] ** 2) / (d["norm2_a"] * d["norm2_b"])
    out = {"n_qubits": n, "gates": len(circ), "depth": depth,
           "c128_s": t128, "c64_s": t64, "speedup": t128 / t64,
           "c128_gate_app_per_s": len(circ) / t128, "c64_gate_app_per_s": len(circ) / t64,
           "max_abs_c64_vs_c128": d["max_abs"], "l2_c64_vs_c128": d["l2"], "fidelity": fid,
           "passes_c128": qv.plan_stats(n, torch.complex128, circ)["n_passes"],
           "passes_c64": qv.plan_stats(n, torch.complex64, circ)["n_passes"]}
    del a, b
    torch.cuda.empty_cache()
    return out


def adjoint_figures(qv, n=24, layers=20, dtype=torch.complex64, shift_evals=True):
    """Hardware-efficient ansatz: forward (circuit + FP64 expectation),
    adjoint backward, and the parameter-shift alternative."""
    P = 2 * n * layers
    th = C.hea_params(n, layers, seed=0)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    st = qv.State(n, dtype)
    work = torch.empty_like(st.tensor)

    def fwd():
        return st.set_basis(0).apply(circ).expect(H)

    fwd()
    t_fwd, f = timed(fwd, reps=5)

    def fwd_bwd():
        st.set_basis(0).apply(circ)
        return st.adjoint_grad(circ, H, P, work=work)

    fwd_bwd()
    t_fb, (f2, g) = timed(fwd_bwd, reps=3)
    ref = qv.State(n, torch.complex128)
    ref.set_basis(0).apply(circ)
    f_ref, g_ref = ref.adjoint_grad(circ, H, P)
    del ref
    out = {"n_qubits": n, "layers": layers, "params": P, "gates": len(circ), "dtype": str(dtype).split(".")[-1],
           "forward_s": t_fwd, "forward_plus_adjoint_s": t_fb,
           "grad_over_fwd": (t_fb - t_fwd) / t_fwd, "total_over_fwd": t_fb / t_fwd,
           "grad_max_abs_err_vs_c128": float(np.max(np.abs(g - g_ref))), "f": f, "f_err_vs_c128": abs(f - f_ref)}
    if shift_evals:
        def shift_all():
            for p in range(P):
                for sgn in (1.0, -1.0):
                    e = th.copy()
                    e[p] += sgn * math.pi / 2
                    st.set_basis(0).apply(C.with_params(circ, e)).expect(H)
        t_ps, _ = timed(shift_all)
        out["param_shift_2P_s"] = t_ps
        out["param_shift_over_adjoint"] = t_ps / t_fb
    return out


def mfma_probe(qv, B, n, steps):
    """complex64 benchmark step with the 4x4 updates on the VALU (default)
    and on the matrix cores (QVEC_MFMA=1): block-pass launch time and the
    device-side difference of the two final states."""
    rand, x, qft = workload(n)
    out = {}
    states = {}
    for knob in ("0", "1", "0"):
        os.environ["QVEC_MFMA"] = knob
        st = qv.State(n, torch.complex64)
        run_step(st, rand, x, qft)
        st.timing(True)
        st.timing_reset()
        for _ in range(steps):
            run_step(st, rand, x, qft)
        launches, ms = st.timing_read(B.KF_BLOCK)
        st.timing(False)
        st.set_basis(0).apply(rand)
        states[knob] = st
        out[f"mfma{knob}_block_ms_per_launch"] = ms / launches
        out[f"mfma{knob}_block_ms_per_step"] = ms / steps
    os.environ.pop("QVEC_MFMA", None)
    d = states["0"].compare(states["1"])
    out["max_abs_diff_random_circuit"] = d["max_abs"]
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=29)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time the library's streaming copy kernel on two state-sized buffers")
    ap.add_argument("--sweeps", action="store_true",
                    help="only time one unfused U3 sweep per target qubit (the one-qubit sweep kernel)")
    ap.add_argument("--two-qubit-sweeps", action="store_true",
                    help="only time unfused CNOT / SWAP / CZ / CP / 4x4 sweeps on several qubit pairs")
    ap.add_argument("--adjoint", action="store_true",
                    help="only the 24-qubit ansatz forward and adjoint figures (no parameter shift)")
    ap.add_argument("--c64-vs-c128", action="store_true",
                    help="only the 33-qubit random U3 + CZ circuit in complex128 and complex64")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only the block-pass time of the step in complex64 with and without matrix-core 4x4 updates")
    ap.add_argument("--host-tier", action="store_true",
                    help="only the host tier on a 30-qubit complex128 state in pinned host memory")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the engine keeps the whole state in one GPU's HBM; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import paper_2508_15545_amd as qv
    from paper_2508_15545_amd import _binding as B

    n = args.n
    dtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    elem = 16 if args.dtype == "c128" else 8
    if args.copy_probe:
        return copy_probe(qv, B, n, dtype, elem, args.steps)
    if args.sweeps:
        print(json.dumps({"sweeps": sweep_rates(qv, B, n, dtype, elem, args.steps)}), flush=True)
        return 0
    if args.adjoint:
        print(json.dumps({"adjoint": adjoint_figures(qv, shift_evals=False)}), flush=True)
        return 0
    if args.two_qubit_sweeps:
        print(json.dumps({"two_qubit_sweeps": two_qubit_sweep_rates(qv, B, n, dtype, elem, args.steps)}),
              flush=True)
        return 0
    if args.host_tier:
        print(json.dumps({"host_tier": host_tier(qv)}), flush=True)
        return 0
    if args.c64_vs_c128:
        print(json.dumps({"c64_vs_c128": c64_vs_c128(qv)}), flush=True)
        return 0
    if args.mfma_probe:
        print(json.dumps({"mfma_probe": mfma_probe(qv, B, n, args.steps)}), flush=True)
        return 0
    rand, x, qft = workload(n)
    gates_per_step = len(rand) + len(qft)
    plan_r = qv.plan_stats(n, dtype, rand)
    plan_q = qv.plan_stats(n, dtype, qft)
    log(f"n={n} dtype={args.dtype} gates/step={gates_per_step} passes: random {plan_r['n_passes']} "
        f"qft {plan_q['n_passes']}")

    torch.cuda.set_device(0)
    st = qv.State(n, dtype, device="cuda:0")
    for w in range(args.warmup):
        run_step(st, rand, x, qft)
        log(f"warmup {w + 1}/{args.warmup} done")

    # The headline: the steps alone, no per-launch instrumentation.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = []
    for k in range(args.steps):
        norms.append(run_step(st, rand, x, qft))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # The same steps again with HIP events around every launch on the launch
    # stream: per-kernel launch counts and durations for the roofline.
    st.timing(True)
    st.timing_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        run_step(st, rand, x, qft)
    torch.cuda.synchronize()
    elapsed_instr = time.perf_counter() - t1
    st.timing(False)
    log(f"instrumented repeat of {args.steps} steps done")

    fams = {"block": B.KF_BLOCK, "sweep1": B.KF_SWEEP1, "sweep2": B.KF_SWEEP2, "diag": B.KF_DIAG,
            "reduce": B.KF_REDUCE, "init": B.KF_INIT}
    kt = {name: st.timing_read(f) for name, f in fams.items()}
    dominant = max(kt, key=lambda k: kt[k][1])
    launches, ms = kt[dominant]
    state_bytes = (1 << n) * elem
    # a block pass and a dense one-qubit sweep read and write the whole state once
    per_launch = 2.0 * state_bytes
    avg_s = ms / 1e3 / max(1, launches)
    achieved = per_launch / avg_s / 1e9 if launches else 0.0

    ms_per_step = elapsed / args.steps * 1e3
    value = gates_per_step * args.steps / elapsed
    alg_bytes = (plan_r["bytes_moved"] + plan_q["bytes_moved"] + 2 * state_bytes  # two basis inits (write)
                 + 2 * state_bytes)  # two norms (read)
    out = {
        "metric": "gate-applications/s",
        "value": value,
        "unit": "gate-applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_instrumented": elapsed_instr / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic (seeded circuits)",
        "config": {
            "workload": f"{n}-qubit {args.dtype} state: random U3+CNOT-matching circuit depth 40 "
                        f"({len(rand)} gates) + textbook QFT of a seeded random basis state ({len(qft)} gates), "
                        f"norm after each",
            "n_qubits": n,
            "state_gib": state_bytes / 2 ** 30,
            "gates_per_step": gates_per_step,
            "passes_per_step": plan_r["n_passes"] + plan_q["n_passes"],
            "parallelism": "1 GPU",
        },
        "hbm_gbs_algorithmic": alg_bytes / (ms_per_step / 1e3) / 1e9,
        "roofline": {
            "kernel": {"block": "k_block (fused block pass)", "sweep1": "k_sweep1"}.get(dominant, dominant),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(n, args.dtype) if dominant == "block" else None,
            "launches": launches,
            "avg_launch_ms": avg_s * 1e3,
            "bytes_per_launch": per_launch,
        },
        "kernel_ms": {k: v[1] for k, v in kt.items()},
        "norm_error": max(abs(a - 1) for pair in norms for a in pair),
    }
    del st
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("sweeps ...")
        sw = sweep_rates(qv, B, n, dtype, elem, 5)
        out["sweeps"] = {"min_gbs": sw["min_gbs"], "mean_gbs": sw["mean_gbs"],
                         "frac_of_peak_min": sw["frac_of_peak_min"], "frac_of_peak_mean": sw["frac_of_peak_mean"],
                         "gbs_by_target": {k: round(v) for k, v in sw["gbs_by_target"].items()}}
        log("two-qubit sweeps ...")
        out["two_qubit_sweeps"] = two_qubit_sweep_rates(qv, B, n, dtype, elem, 5)
        log("copy ...")
        out["copy"] = copy_rate(qv, B, n, dtype, elem, 5)
        out["sweeps"]["frac_of_copy_mean"] = sw["mean_gbs"] / out["copy"]["gbs"]
        # the dominant kernel against the measured copy rate as well as the nominal peak
        out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / out["copy"]["gbs"]
        log("c64 vs c128 (33 qubits) ...")
        out["c64_vs_c128"] = c64_vs_c128(qv)
        log("adjoint (24-qubit ansatz) ...")
        out["adjoint"] = adjoint_figures(qv)
        log("host tier (30 qubits in pinned host memory) ...")
        out["host_tier"] = host_tier(qv)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, rand, x, qft)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
