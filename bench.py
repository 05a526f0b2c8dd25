#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Workload (one step): a 30-qubit random brick circuit of depth 20 (a Haar-random 2x2
unitary on every qubit each layer, then CZ on alternating neighbour pairs: 600 + 290
gates) applied to |0...0>, then <sum_i Z_i>.  A step runs state init, every fused tile
pass and the expectation pass; inputs (the state) are resident in HBM throughout.

Reported `value`: achieved HBM throughput of the whole step, i.e. the algorithmic bytes
of every launch (each pass reads and writes the 2^30-amplitude state once; the
expectation reads it once; init writes it once) divided by the step time.  Extra fields
give gates/s, the roofline of the dominant kernel (fused tile pass) from per-launch HIP
event timings taken inside the timed steps, the adjoint-vs-parameter-shift gradient
throughput on the 24-qubit QAOA batch, and the CPU oracle timed on a bounded sample.
"""

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "state-vector HBM GB/s vs peak; adjoint grad evals/s vs parameter-shift"


def cpu_baseline_sample(n, depth, seconds):
    """Time the CPU oracle on the first gates of the same brick circuit (complex128)."""
    import numpy as np

    import workloads as W
    from oracle import statevector as O
    circ, _ = W.brick_workload(n, depth)
    psi = O.zero_state(n)
    done, bytes_ = 0, 0.0
    t0 = time.perf_counter()
    for g in circ["gates"]:
        O.apply_gate(psi, n, g)
        done += 1
        frac = 1.0 if g["kind"] == "MAT1" else 0.25  # CZ touches the |11> quarter
        bytes_ += 2.0 * frac * (2 ** n) * 16
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    assert np.isfinite(psi[0])
    return {"value": bytes_ / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} gate(s) of the {n}-qubit depth-{depth} brick circuit, complex128, "
                      f"numpy single thread, {dt:.1f} s",
            "gates_per_s": done / dt}


def run_cpu_baseline(n, depth, seconds):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--n-qubits", str(n),
           "--depth", str(depth), "--cpu-seconds", str(seconds)]
    out = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    return json.loads(out.stdout.strip().splitlines()[-1])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def qaoa_leg(Q, dtype, ps_sets):
    """Adjoint batch gradient (64 sets) vs GPU parameter shift (ps_sets sets)."""
    import numpy as np

    import workloads as W
    circ, H, params, _ = W.qaoa_workload()
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    s = Q.qsv_state_create(24, dtype)
    Q.qsv_expectation_and_grad_batch(s, c, h, params[:2])  # warm plans and workspaces
    t0 = time.perf_counter()
    E, G = Q.qsv_expectation_and_grad_batch(s, c, h, params)
    t_adj = time.perf_counter() - t0
    log(f"qaoa adjoint batch of {params.shape[0]}: {t_adj:.3f} s")
    t0 = time.perf_counter()
    Eps, Gps = Q.qsv_param_shift_grad_batch(s, c, h, params[:ps_sets])
    t_ps = time.perf_counter() - t0
    log(f"qaoa parameter shift, {ps_sets} set(s): {t_ps:.3f} s")
    adj_rate = params.shape[0] / t_adj
    ps_rate = ps_sets / t_ps
    scale = sum(abs(cf) for cf, _ in H)
    agree = float(np.max(np.abs(G[:ps_sets] - Gps)) / scale)
    del s
    return {"workload": "qaoa24_p8_batch64", "dtype": dtype, "adjoint_grad_evals_per_s": adj_rate,
            "param_shift_grad_evals_per_s": ps_rate, "speedup": adj_rate / ps_rate,
            "max_grad_diff_over_S": agree, "param_shift_sets": ps_sets}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--n-qubits", type=int, default=30)
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--tile", type=int, default=None, help="tile qubits (0: unfused per-gate kernels)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-qaoa", action="store_true")
    ap.add_argument("--ps-sets", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_sample(args.n_qubits, args.depth, args.cpu_seconds)))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the engine keeps a whole state on a single MI355X; "
              "it has no multi-GPU mode (use --gpus 1)", file=sys.stderr)
        return 2

    import torch

    import paper_2406_17248_amd as Q
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, depth = args.n_qubits, args.depth
    circ, H = W.brick_workload(n, depth)
    n_gates = len(circ["gates"])
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    s = Q.qsv_state_create(n, args.dtype)
    if args.tile is not None:
        Q.qsv_state_set_option(s, Q.OPT_TILE_QUBITS, args.tile)

    def step():
        Q.qsv_state_reset(s)
        Q.qsv_apply_circuit(s, c)
        return Q.qsv_expectation(s, h).real

    log(f"brick n={n} depth={depth} dtype={args.dtype}: warmup")
    for _ in range(args.warmup):
        step()
    log("warmup done; timing")
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 1)
    for k in range(5):
        Q.qsv_profile_read(s, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = {k: Q.qsv_profile_read(s, k) for k in range(5)}
    log(f"timed {args.steps} steps: {dt * 1e3:.2f} ms/step")
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 0)

    total_bytes = sum(b for (_, _, b) in prof.values()) / args.steps
    value = total_bytes / dt / 1e9
    dom = Q.K_TILE_FORWARD if prof[Q.K_TILE_FORWARD][1] else Q.K_GATE_STREAM
    ms, launches, b = prof[dom]
    avg_ms = ms / max(launches, 1)
    achieved = (b / max(launches, 1)) / (avg_ms / 1e3) / 1e9 if launches else 0.0
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "tile_pass (fused forward)" if dom == Q.K_TILE_FORWARD else "gate1/gate2/diag_stream",
                "launches_per_step": launches / args.steps, "avg_launch_ms": avg_ms,
                "algorithmic_bytes_per_launch": b / max(launches, 1)}
    kernel_ms = {name: prof[k][0] / args.steps for name, k in
                 (("tile_forward", Q.K_TILE_FORWARD), ("pauli", Q.K_PAULI), ("gate_stream", Q.K_GATE_STREAM),
                  ("other", Q.K_OTHER))}
    del s
    torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.dtype == "c64" else "f64", "data": "synthetic",
           "config": {"workload": f"brick{n}_depth{depth}_sumZ", "n_qubits": n, "depth": depth,
                      "gates": n_gates, "amplitude_type": "complex64" if args.dtype == "c64" else "complex128",
                      "state_bytes": (2 ** n) * (8 if args.dtype == "c64" else 16), "parallelism": "single-gpu"},
           "gates_per_s": n_gates / dt, "expectation": e, "hbm_frac_of_peak": value / HBM_PEAK_GBS,
           "kernel_ms_per_step": kernel_ms, "roofline": roofline}
    if not args.no_qaoa:
        try:
            out["qaoa"] = qaoa_leg(Q, args.dtype, args.ps_sets)
        except Exception as ex:  # report, do not hide, a failure of the secondary leg
            out["qaoa"] = {"error": repr(ex)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, single thread)")
        out["cpu_baseline"] = run_cpu_baseline(n, depth, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
