#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Workload (one step): a 30-qubit random brick circuit of depth 20 (a Haar-random 2x2
unitary on every qubit each layer, then CZ on alternating neighbour pairs: 600 + 290
gates) applied to |0...0>, then <sum_i Z_i>.  A step runs state init, every fused tile
pass and the expectation pass; the state is resident in HBM throughout.

Reported `value`: HBM throughput of the whole step, i.e. the bytes every launch moves by
schedule (each fused pass reads and writes the 2^30-amplitude state once, the
expectation reads it once, init writes it once) divided by the step time.  The fused
passes carry ~40 gates each, so their arithmetic intensity (~14 flop per amplitude per
gate) is above the vector ridge point and the dominant kernel's roofline is the vector
ALU: `roofline` gives its algorithmic flop rate from per-launch HIP event timings taken
inside the timed steps on the library's stream.  Extra fields: gates/s, the same step in
the other precision, adjoint-vs-parameter-shift gradient throughput on the 24-qubit QAOA
batch (with the adjoint pass's own roofline), the 10-qubit ansatz latency, and the CPU
oracle timed on a bounded sample.
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
# Published MI355X vector peaks (256 CUs x 64 lanes x FMA x 2.4 GHz = 78.6 TFLOP/s; FP32
# doubles that only with packed two-wide FP32 instructions, which this library's build
# turns off, so 78.6 is also what complex64 code can reach).
VALU_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}
VALU_NONPACKED_TFLOPS = 78.6
# A 2x2 complex gate: each output amplitude is two complex multiplies and one complex
# add (6 + 6 + 2 flop).  Sign-only gates (CZ) count as zero flop.
FLOP_PER_AMP_DENSE1 = 14
METRIC = "state-vector HBM GB/s vs peak; adjoint grad evals/s vs parameter-shift"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_pass_brick30_traffic.txt")
QAOA_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_pass_adjoint_qaoa24_traffic.txt")
TRAFFIC_SOURCES = ["qsv_kernels.hip", "engine.cpp", "api.cpp"]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_17248_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic(dtype, path=TRAFFIC_FILE):
    """HBM bytes per launch of the profiled pass from a committed rocprofv3 counter summary,
    or None when it is missing or the kernel, planner or launch sources changed since."""
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != sources_digest():
        return None
    try:
        return float(kv[f"{dtype}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    # the 10-qubit hardware-efficient ansatz: one energy-and-gradient evaluation by the oracle
    circ10, H10, p10 = W.hea10_workload()
    t1 = time.perf_counter()
    reps = 0
    while reps < 3 or time.perf_counter() - t1 < 1.0:
        O.grad_adjoint(circ10, H10, p10)
        reps += 1
    hea10_s = (time.perf_counter() - t1) / reps
    return {"value": bytes_ / dt / 1e9, "unit": "GB/s", "cores": 1, "host_cores": os.cpu_count(), "kind": "oracle",
            "sample": f"first {done} gate(s) of the {n}-qubit depth-{depth} brick circuit, complex128, "
                      f"numpy single thread, {dt:.1f} s",
            "gates_per_s": done / dt, "hea10_grad_eval_s": hea10_s}


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


def qaoa_flops(circ, n, adjoint):
    """Algorithmic flop of one evaluation of the QAOA circuit per amplitude-pass, summed over
    gates: a dense 2x2 gate is 14 flop per amplitude (two complex multiplies and a complex
    add per output); a ZZ cost layer is one fused diagonal phase, 6 flop per amplitude (one
    complex multiply; the edge parities are integer work).  The adjoint sweep applies U^dag to
    both psi and lambda (twice the forward cost) and adds, per parameterized gate, 4 flop per
    amplitude for its term Im<lambda|G|psi>.  Returns (forward, adjoint) flop per parameter set."""
    N = float(2 ** n)
    fwd = adj = 0.0
    layer_open = False
    for g in circ["gates"]:
        if g["kind"] == "RZZ":
            if not layer_open:  # one fused diagonal op per cost layer
                fwd += 6 * N
                adj += 2 * 6 * N
                layer_open = True
            adj += 4 * N
        else:
            layer_open = False
            fwd += 14 * N
            if g["kind"] != "H":  # the leading Hadamards act on the start state: never undone
                adj += 2 * 14 * N + (4 * N if g["params"] else 0)
    return fwd, adj


def qaoa_leg(Q, dtype, ps_sets, with_copy=False):
    """Adjoint batch gradient (64 sets) vs GPU parameter shift (ps_sets sets), with per-launch
    HIP event timings of the adjoint evaluation (on the library's stream) for its roofline."""
    import numpy as np

    import workloads as W
    circ, H, params, _ = W.qaoa_workload()
    n = circ["n_qubits"]
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    s = Q.qsv_state_create(n, dtype)
    Q.qsv_expectation_and_grad_batch(s, c, h, params[:2])  # warm plans and workspaces
    Q.qsv_expectation_and_grad_batch(s, c, h, params)
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 1)
    for k in range(5):
        Q.qsv_profile_read(s, k)
    t0 = time.perf_counter()
    E, G = Q.qsv_expectation_and_grad_batch(s, c, h, params)
    t_adj = time.perf_counter() - t0
    prof = {k: Q.qsv_profile_read(s, k) for k in range(5)}
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 0)
    log(f"qaoa adjoint batch of {params.shape[0]}: {t_adj:.3f} s")
    adj_rate = params.shape[0] / t_adj
    ps_rate = agree = None
    if ps_sets > 0:
        t0 = time.perf_counter()
        Eps, Gps = Q.qsv_param_shift_grad_batch(s, c, h, params[:ps_sets])
        t_ps = time.perf_counter() - t0
        log(f"qaoa parameter shift, {ps_sets} set(s): {t_ps:.3f} s")
        ps_rate = ps_sets / t_ps
        scale = sum(abs(cf) for cf, _ in H)
        agree = float(np.max(np.abs(G[:ps_sets] - Gps)) / scale)
    if with_copy:
        # plain copy kernel of known size (reads and writes 2^28 amplitudes once), for the
        # calibration of hardware byte counters
        a, d = Q.qsv_state_create(28, dtype), Q.qsv_state_create(28, dtype)
        Q.qsv_state_copy(d, a)
        Q.qsv_state_synchronize(d)
        del a, d
    del s
    B = params.shape[0]
    f_fwd, f_adj = qaoa_flops(circ, n, True)
    ms, launches, by = prof[Q.K_TILE_ADJOINT]
    launches = max(launches, 1)
    avg_s = ms / launches / 1e3
    flop_launch = f_adj * B / launches
    bytes_launch = by / launches
    peak = VALU_PEAK_TFLOPS[dtype]
    achieved = flop_launch / avg_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": committed_traffic(dtype, QAOA_TRAFFIC_FILE),
            "kernel": "tile_pass_rb adjoint (psi and lambda, reverse sweep)",
            "launches_per_eval": launches, "avg_launch_ms": avg_s * 1e3,
            "algorithmic_flop_per_launch": flop_launch, "algorithmic_bytes_per_launch": bytes_launch,
            "hbm_GBs": bytes_launch / avg_s / 1e9, "hbm_frac": bytes_launch / avg_s / 1e9 / HBM_PEAK_GBS,
            "frac_of_nonpacked_peak": achieved / VALU_NONPACKED_TFLOPS}
    kernel_ms = {name: prof[k][0] for name, k in
                 (("tile_forward", Q.K_TILE_FORWARD), ("tile_adjoint", Q.K_TILE_ADJOINT), ("pauli", Q.K_PAULI),
                  ("other", Q.K_OTHER))}
    return {"workload": "qaoa24_p8_batch64", "dtype": dtype, "adjoint_grad_evals_per_s": adj_rate,
            "param_shift_grad_evals_per_s": ps_rate, "speedup": adj_rate / ps_rate if ps_rate else None,
            "max_grad_diff_over_S": agree, "param_shift_sets": ps_sets,
            "kernel_ms_per_batch": kernel_ms, "roofline": roof}


def hea10_leg(Q, reps):
    """10-qubit hardware-efficient ansatz (80 parameters), complex128: latency of one
    expectation-and-gradient call through the C ABI (its 16 KiB state is latency-bound, no
    roofline applies)."""
    import workloads as W
    circ, H, params = W.hea10_workload()
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    s = Q.qsv_state_create(10, "c128")
    for _ in range(3):
        Q.qsv_expectation_and_grad(s, c, h, params)
    t0 = time.perf_counter()
    for _ in range(reps):
        E, g = Q.qsv_expectation_and_grad(s, c, h, params)
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "hea10_4layers_80params_zzchain", "dtype": "c128", "evals_per_s": 1.0 / dt,
            "ms_per_eval": dt * 1e3, "reps": reps, "energy": E}


def batch_leg(Q, reps=5):
    """512 uneven circuits (8-20 qubits, depth 2-10, 50 Pauli strings each), complex64:
    energy and adjoint gradient of every circuit from one HIP-graph replay, after the
    autotuner picks the tile width and schedule; compared with the same circuits one call at a time."""
    import numpy as np

    import workloads as W
    circs, hams, params = W.uneven_batch_workload()
    b = Q.qsv_batch_create(circs, hams, "c64")
    tile, low = Q.qsv_batch_autotune(b, params, with_schedule=True)
    Q.qsv_batch_expectation_and_grad(b, params)
    t0 = time.perf_counter()
    for _ in range(reps):
        E, g = Q.qsv_batch_expectation_and_grad(b, params)
    t_batch = (time.perf_counter() - t0) / reps
    dev_ms = b.info()["last_ms"]
    states = {}
    for i, c in enumerate(circs):
        n = c["n_qubits"]
        if n not in states:
            states[n] = Q.qsv_state_create(n, "c64")
    t0 = time.perf_counter()
    worst = 0.0
    for i, c in enumerate(circs):
        p_i = params[b.offsets[i]:b.offsets[i + 1]]
        Ei, gi = Q.qsv_expectation_and_grad(states[c["n_qubits"]], c, hams[i], p_i)
        worst = max(worst, abs(Ei - E[i]))
    t_single = time.perf_counter() - t0
    del states, b
    return {"workload": "uneven512_hea_n8-20_depth2-10_50terms", "dtype": "c64", "autotuned_tile": tile,
            "autotuned_low_qubits": low,
            "circuits_per_s": len(circs) / t_batch, "ms_per_batch": t_batch * 1e3, "graph_replay_device_ms": dev_ms,
            "one_call_per_circuit_ms": t_single * 1e3, "speedup_vs_one_call_per_circuit": t_single / t_batch,
            "max_energy_diff_vs_one_call": worst}


def max_cut(edges, n_nodes):
    """Brute-force maximum cut of a small graph (all 2^n bipartitions)."""
    import numpy as np
    x = np.arange(1 << n_nodes, dtype=np.int64)
    cut = np.zeros(1 << n_nodes, dtype=np.int64)
    for (u, v) in edges:
        cut += ((x >> u) ^ (x >> v)) & 1
    return int(cut.max())


def warmstart_leg(n_train, n_test, epochs, restarts, chunk=2048, opt_steps=150):
    """Learned warm start at full size: labels are angles the simulator optimized (Adam on
    adjoint gradients from the linear ramp and from `restarts` random starts, best kept),
    the network is trained on them by the library's kernels, and 1k held-out graphs are
    started from the ramp and from the network's angles; the simulator reports the cut
    reached and the optimizer steps needed to reach the ramp run's final cut."""
    import numpy as np

    import paper_2406_17248_amd as Q
    import workloads as W
    from paper_2406_17248_amd import warmstart as WS
    ramp = W.linear_ramp()
    p2 = ramp.size
    t0 = time.perf_counter()
    train_g = W.warmstart_graphs(n_train, 11)
    test_g = W.warmstart_graphs(n_test, 12)
    rng = np.random.default_rng(5)
    labels = np.zeros((n_train, p2))
    sim_calls = 0
    for s in range(0, n_train, chunk):
        graphs = train_g[s:s + chunk]
        qb = WS.QaoaBatch(graphs, W.qaoa_circuit, W.maxcut_hamiltonian)
        best_x, best_c, _ = WS.optimize(qb, np.tile(ramp, (len(graphs), 1)), steps=opt_steps)
        for _ in range(restarts):
            init = np.concatenate([rng.uniform(-np.pi / 2, 0, (len(graphs), p2 // 2)),
                                   rng.uniform(0, np.pi, (len(graphs), p2 // 2))], axis=1)
            x, c, _ = WS.optimize(qb, init, steps=opt_steps)
            better = c > best_c
            best_x[better], best_c[better] = x[better], c[better]
        sim_calls += (1 + restarts) * (opt_steps + 1)
        labels[s:s + len(graphs)] = best_x
        log(f"warm start labels {s + len(graphs)}/{n_train}")
    t_labels = time.perf_counter() - t0
    masks = np.stack([WS.adjacency_masks(e) for e in train_g])
    net = Q.Mpnn(WS.init_params(1))
    t1 = time.perf_counter()
    losses = WS.train(net, masks, labels, ramp, epochs=epochs, batch_size=256, lr=3e-3)
    t_train = time.perf_counter() - t1
    log(f"trained {epochs} epochs: loss {losses[:10].mean():.4f} -> {losses[-10:].mean():.4f}")
    qb = WS.QaoaBatch(test_g, W.qaoa_circuit, W.maxcut_hamiltonian)
    tmasks = np.stack([WS.adjacency_masks(e) for e in test_g])
    init_r = np.tile(ramp, (n_test, 1))
    init_n = net.predict(tmasks, ramp)
    mc = np.array([max_cut(e, 16) for e in test_g], dtype=np.float64)
    c0_r, _ = qb.cut_and_grad(init_r)
    c0_n, _ = qb.cut_and_grad(init_n)
    _, cf_r, _ = WS.optimize(qb, init_r, steps=opt_steps)
    target = cf_r - 1e-3 * qb.n_edges
    _, _, hit_r = WS.optimize(qb, init_r, steps=opt_steps, target=target)
    _, cf_n, hit_n = WS.optimize(qb, init_n, steps=opt_steps, target=target)
    return {"workload": f"qaoa16_p6_warmstart_{n_train}train_{n_test}test", "dtype": "c64 simulator, fp32 network",
            "label_restarts": 1 + restarts, "optimizer_steps": opt_steps, "epochs": epochs,
            "train_loss_first": float(losses[:10].mean()), "train_loss_last": float(losses[-10:].mean()),
            "approx_ratio_init_ramp": float((c0_r / mc).mean()), "approx_ratio_init_net": float((c0_n / mc).mean()),
            "approx_ratio_opt_ramp": float((cf_r / mc).mean()), "approx_ratio_opt_net": float((cf_n / mc).mean()),
            "steps_to_ramp_final_cut_ramp": float(hit_r.mean()), "steps_to_ramp_final_cut_net": float(hit_n.mean()),
            "steps_saved_frac": float(1.0 - hit_n.mean() / max(hit_r.mean(), 1e-9)),
            "label_simulator_batch_calls": sim_calls, "seconds_labels": t_labels, "seconds_train": t_train}


def brick_leg(Q, torch, circ, H, n, dtype, steps, warmup, tile, with_copy):
    """Time `steps` brick steps in one precision; per-launch times come from HIP events the
    library records on its stream around every launch while profiling is on."""
    n_gates = len(circ["gates"])
    n_dense = sum(1 for g in circ["gates"] if g["kind"] == "MAT1")
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    s = Q.qsv_state_create(n, dtype)
    if tile is not None:
        Q.qsv_state_set_option(s, Q.OPT_TILE_QUBITS, tile)

    def step():
        Q.qsv_state_reset(s)
        Q.qsv_apply_circuit(s, c)
        return Q.qsv_expectation(s, h).real

    log(f"brick n={n} dtype={dtype}: {warmup} warmup step(s)")
    for _ in range(warmup):
        step()
    # the same steps without per-launch events (their cost is two event records per ~20 ms launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t0) / steps
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 1)
    for k in range(5):
        Q.qsv_profile_read(s, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = {k: Q.qsv_profile_read(s, k) for k in range(5)}
    log(f"timed {steps} step(s): {dt * 1e3:.2f} ms/step")
    if with_copy:
        # plain copy kernel of known size (reads and writes the state once), for the
        # calibration of hardware byte counters
        d = Q.qsv_state_create(n, dtype)
        Q.qsv_state_copy(d, s)
        Q.qsv_state_synchronize(d)
        log(f"copy calibration: {(2 ** n) * (8 if dtype == 'c64' else 16) * 2 / 1e9:.3f} GB moved")
        del d
    Q.qsv_state_set_option(s, Q.OPT_PROFILE, 0)
    del s
    torch.cuda.empty_cache()

    total_bytes = sum(b for (_, _, b) in prof.values()) / steps
    fused = bool(prof[Q.K_TILE_FORWARD][1])
    dom = Q.K_TILE_FORWARD if fused else Q.K_GATE_STREAM
    ms, launches, b = prof[dom]
    launches = max(launches, 1)
    avg_s = ms / launches / 1e3
    bytes_per_launch = b / launches
    hbm_gbs = bytes_per_launch / avg_s / 1e9
    flops_per_launch = n_dense * FLOP_PER_AMP_DENSE1 * float(2 ** n) / (launches / steps)
    achieved = flops_per_launch / avg_s / 1e12
    peak = VALU_PEAK_TFLOPS[dtype]
    traffic = committed_traffic(dtype) if fused else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "kernel": "tile_pass_rb (fused forward pass)" if fused else "gate1/gate2/diag_stream",
                "launches_per_step": launches / steps, "avg_launch_ms": avg_s * 1e3,
                "algorithmic_flop_per_launch": flops_per_launch,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "hbm_GBs": hbm_gbs, "hbm_frac": hbm_gbs / HBM_PEAK_GBS,
                "frac_of_nonpacked_peak": achieved / VALU_NONPACKED_TFLOPS}
    kernel_ms = {name: prof[k][0] / steps for name, k in
                 (("tile_forward", Q.K_TILE_FORWARD), ("pauli", Q.K_PAULI), ("gate_stream", Q.K_GATE_STREAM),
                  ("other", Q.K_OTHER))}
    value = total_bytes / dt / 1e9
    state = float(2 ** n) * (8 if dtype == "c64" else 16)
    return {"value": value, "ms_per_step": dt * 1e3, "ms_per_step_without_events": dt_plain * 1e3,
            "gates": n_gates, "gates_per_s": n_gates / dt,
            "expectation": e, "kernel_ms_per_step": kernel_ms, "roofline": roofline,
            "hbm_frac_of_peak": value / HBM_PEAK_GBS, "state_bytes": int(state)}


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
    ap.add_argument("--no-other-dtype", action="store_true", help="skip the second precision")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-circuit batch leg")
    ap.add_argument("--no-hea10", action="store_true", help="skip the 10-qubit ansatz latency leg")
    ap.add_argument("--hea10-reps", type=int, default=200)
    ap.add_argument("--with-copy", action="store_true",
                    help="after the timed steps, run one plain state copy (counter calibration)")
    ap.add_argument("--ps-sets", type=int, default=1)
    ap.add_argument("--qaoa-only", action="store_true", help="run only the QAOA adjoint leg in --dtype")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--warmstart", action="store_true",
                    help="run only the learned warm-start experiment (20k train / 1k test graphs)")
    ap.add_argument("--ws-train", type=int, default=20000)
    ap.add_argument("--ws-test", type=int, default=1000)
    ap.add_argument("--ws-epochs", type=int, default=40)
    ap.add_argument("--ws-restarts", type=int, default=2)
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
    if args.warmstart:
        print(json.dumps(warmstart_leg(args.ws_train, args.ws_test, args.ws_epochs, args.ws_restarts)), flush=True)
        return 0
    if args.qaoa_only:
        # the adjoint leg alone in one precision (for profiler runs of its kernels)
        print(json.dumps({"qaoa": [qaoa_leg(Q, args.dtype, args.ps_sets, args.with_copy)]}), flush=True)
        return 0
    n, depth = args.n_qubits, args.depth
    circ, H = W.brick_workload(n, depth)
    main_leg = brick_leg(Q, torch, circ, H, n, args.dtype, args.steps, args.warmup, args.tile, args.with_copy)

    out = {"metric": METRIC, "value": main_leg["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": main_leg["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.dtype == "c64" else "f64",
           "data": "synthetic",
           "config": {"workload": f"brick{n}_depth{depth}_sumZ", "n_qubits": n, "depth": depth,
                      "gates": main_leg["gates"],
                      "amplitude_type": "complex64" if args.dtype == "c64" else "complex128",
                      "state_bytes": main_leg["state_bytes"], "parallelism": "single-gpu"}}
    for k in ("gates_per_s", "expectation", "hbm_frac_of_peak", "ms_per_step_without_events", "kernel_ms_per_step",
              "roofline"):
        out[k] = main_leg[k]
    other = "c64" if args.dtype == "c128" else "c128"
    if not args.no_other_dtype:
        leg = brick_leg(Q, torch, circ, H, n, other, args.steps, args.warmup, args.tile, False)
        out["other_dtype"] = {"dtype": other, **{k: leg[k] for k in ("value", "ms_per_step", "gates_per_s",
                                                                   "expectation", "ms_per_step_without_events",
                                                                   "kernel_ms_per_step", "roofline")}}
    if not args.no_qaoa:
        out["qaoa"] = []
        for dt_ in ([args.dtype] if args.no_other_dtype else [args.dtype, other]):
            try:
                out["qaoa"].append(qaoa_leg(Q, dt_, args.ps_sets))
            except Exception as ex:  # report, do not hide, a failure of the secondary leg
                out["qaoa"].append({"dtype": dt_, "error": repr(ex)})
    if not args.no_hea10:
        try:
            out["hea10"] = hea10_leg(Q, args.hea10_reps)
        except Exception as ex:  # report, do not hide, a failure of the secondary leg
            out["hea10"] = {"error": repr(ex)}
    if not args.no_batch:
        try:
            out["batch"] = batch_leg(Q)
        except Exception as ex:  # report, do not hide, a failure of the secondary leg
            out["batch"] = {"error": repr(ex)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, single thread)")
        out["cpu_baseline"] = run_cpu_baseline(n, depth, args.cpu_seconds)
        if "hea10" in out and "evals_per_s" in out["hea10"] and "hea10_grad_eval_s" in out["cpu_baseline"]:
            out["hea10"]["oracle_s_per_eval"] = out["cpu_baseline"]["hea10_grad_eval_s"]
            out["hea10"]["speedup_vs_oracle"] = out["hea10"]["evals_per_s"] * out["cpu_baseline"]["hea10_grad_eval_s"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
