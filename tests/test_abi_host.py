"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/qsv.h declares, and its planner produces a valid reordering of the
circuit (checked by running the planned order through the CPU oracle)."""

import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2406_17248_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqsv.so is not built (run __graft_entry__.build())")
    return _lib


def test_library_exports_every_declared_symbol():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "qsv.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(qsv_\w+)\s*\(", header, re.M))
    assert len(declared) >= 20
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared <= set(L.EXPORTED)


def test_status_strings_and_version():
    L = _lib()
    assert L.lib().qsv_status_string(0) == b"ok"
    assert L.lib().qsv_status_string(-1) == b"invalid argument"
    assert b"gfx950" in L.lib().qsv_version()


@pytest.mark.parametrize("bad", ["target", "dup", "ctrl_on_target", "ctrl_range", "param_range"])
def test_plan_debug_rejects_invalid_circuits(bad):
    L = _lib()
    g = W.gate("RX", (0,), params=(W.param_angle(0),))
    if bad == "target":
        g = dict(g, targets=(5,))
    elif bad == "dup":
        g = W.gate("RZZ", (1, 2), params=(W.fixed_angle(0.1),))
        g = dict(g, targets=(1, 1))
    elif bad == "ctrl_on_target":
        g = dict(g, ctrls=(0,))
    elif bad == "ctrl_range":
        g = dict(g, ctrls=(9,))
    elif bad == "param_range":
        g = dict(g, params=((-2, 1.0, 0.0),))
    with pytest.raises(L.QsvError) as e:
        L.qsv_plan_debug(W.circuit(3, [g]), 2)
    assert e.value.status == L.QSV_EINVAL


def test_pauli_pair_rotations_lower_to_five_primitives():
    L = _lib()
    circ = W.circuit(4, [W.gate("RXX", (0, 3), params=(W.fixed_angle(0.3),)),
                         W.gate("RYY", (1, 2), ctrls=(0,), params=(W.fixed_angle(0.2),))])
    order, _, _, _ = L.qsv_plan_debug(circ, 4)
    assert sorted(order.tolist()) == [0] * 5 + [1] * 5


@pytest.mark.parametrize("n,m,seed", [(6, 3, 1), (8, 4, 2), (10, 5, 3), (12, 6, 4), (9, 9, 5)])
def test_planned_order_is_equivalent(n, m, seed):
    """Every gate appears once, every pass's non-diagonal targets lie in its tile, and the
    planned execution order gives the same state as the original (oracle on the CPU)."""
    from oracle import statevector as O
    L = _lib()
    kinds = [k for k in W.GATE_KINDS if k not in ("RXX", "RYY")]  # one primitive per gate
    circ = W.random_circuit(n, 120, seed, kinds=kinds, max_ctrls=2)
    order, pass_of, n_passes, masks = L.qsv_plan_debug(circ, m)
    assert sorted(order.tolist()) == list(range(len(circ["gates"])))
    assert np.all(np.diff(pass_of) >= 0) and n_passes == pass_of.max() + 1
    diag_kinds = {"Z", "S", "SDG", "T", "TDG", "RZ", "PS", "RZZ"}
    for gi, p in zip(order, pass_of):
        g = circ["gates"][gi]
        if g["kind"] in diag_kinds:
            continue
        if g["kind"] in ("MAT1", "MAT2") and np.count_nonzero(g["matrix"] - np.diag(np.diag(g["matrix"]))) == 0:
            continue
        for t in g["targets"]:
            assert int(masks[p]) >> t & 1
        assert bin(int(masks[p])).count("1") == min(m, n)
    params = np.random.default_rng(seed).uniform(-3, 3, 8)
    psi0 = W.random_state(n, np.random.default_rng(seed + 7))
    ref = O.simulate(circ, params, psi0)
    reordered = W.circuit(n, [circ["gates"][i] for i in order])
    assert np.allclose(O.simulate(reordered, params, psi0), ref, atol=1e-12)


def test_brick_plan_pass_count():
    """The 30-qubit depth-20 brick circuit (890 gates) fuses into a few tile passes."""
    L = _lib()
    circ, _ = W.brick_workload()
    _, _, n_passes, _ = L.qsv_plan_debug(circ, 13)
    assert n_passes <= 24


def _sanitized_host_program(tmp_path, name):
    """Build tests/host/<name>.cpp against the planner with g++ under AddressSanitizer and
    UndefinedBehaviorSanitizer (any report aborts the program)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    src = os.path.join(ROOT, "tests", "host", name + ".cpp")
    csrc = os.path.join(ROOT, "paper_2406_17248_amd", "csrc")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc, src,
                    os.path.join(csrc, "engine.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


def test_relayout_plans_follow_every_amplitude(tmp_path):
    """The planner's relayouting forward plans, checked on the host through their address
    tables (tests/host/relayout_check.cpp, built with sanitizers against the planner):
    every pass reads each amplitude where the previous pass wrote it, writes a permutation
    of the state, and the last pass leaves the natural layout; for the 30-qubit depth-20
    brick circuit with the library's default options (both amplitude types) the same is
    shown through the single-bit images of each pass's linear address maps."""
    res = _sanitized_host_program(tmp_path, "relayout_check")
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "relayouting plans" in res.stdout
    assert "ok linear brick30 complex128" in res.stdout and "ok linear brick30 complex64" in res.stdout


def test_planner_under_sanitizers(tmp_path):
    """Random circuits of every gate kind planned and bound at every tile width, both
    amplitude types, forward and adjoint (tests/host/planner_fuzz.cpp) with ASan/UBSan."""
    res = _sanitized_host_program(tmp_path, "planner_fuzz")
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "plans checked" in res.stdout and "unitary fused blocks checked" in res.stdout
    assert "split gates checked along their chains" in res.stdout
