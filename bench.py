"""Benchmark: gate-applications/s of the state-vector engine on one MI355X.

Workload (one step): on a 29-qubit complex128 state (8 GiB in HBM)
  (a) reset to |0..0>, run the random circuit of depth 40 (per layer U3 with
      seeded angles on every qubit, then CNOTs on a seeded random matching:
      1720 gates), then the FP64 norm;
  (b) reset to a seeded random basis state, run the textbook QFT (449 gates),
      then the FP64 norm.
value = gates applied per second over the timed steps (2169 gates per step).
The dominant kernel's achieved bandwidth comes from HIP events around each
of its launches (library timing on the launch stream); the CPU baseline is
the FP64 oracle on a bounded sample of the same workload.

Prints one JSON line. Flags: --gpus (only 1), --steps, --warmup, --n,
--dtype c128|c64, --no-cpu (skip the oracle leg), --extras (adjoint and
complex64 figures, slower).
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


def cpu_baseline(n: int, rand, seconds_budget: float = 20.0):
    """The FP64 oracle on the first layer of the random circuit (the same
    gates, the same 2^n-amplitude state), timed around the gate loop only."""
    import oracle

    per_layer = n + n // 2
    sample = rand[:per_layer]
    s = oracle.basis_state(n, 0)
    t0 = time.perf_counter()
    done = 0
    for g in sample:
        oracle.apply_gate(s, n, g)
        done += 1
        if time.perf_counter() - t0 > seconds_budget:
            break
    dt = time.perf_counter() - t0
    del s
    return {
        "value": done / dt,
        "unit": "gate-applications/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"first {done} gates (layer 1: U3 on every qubit + CNOT matching) of the {n}-qubit "
                  f"random circuit on a complex128 state, {dt:.1f} s",
    }


def copy_probe(qv, B, n, dtype, elem, reps):
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
    print(json.dumps({"copy_probe": {"bytes_per_launch_read": nbytes, "bytes_per_launch_write": nbytes,
                                     "launches": launches, "avg_ms": ms / launches, "gbs": gbs}}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=29)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time the library's streaming copy kernel on two state-sized buffers")
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

    st.timing(True)
    st.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = []
    for k in range(args.steps):
        norms.append(run_step(st, rand, x, qft))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st.timing(False)

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
            "traffic": None,
            "launches": launches,
            "avg_launch_ms": avg_s * 1e3,
            "bytes_per_launch": per_launch,
        },
        "kernel_ms": {k: v[1] for k, v in kt.items()},
        "norm_error": max(abs(a - 1) for pair in norms for a in pair),
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, rand)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
