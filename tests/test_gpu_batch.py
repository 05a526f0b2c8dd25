"""Batched uneven circuits in one graph replay: energies and adjoint gradients per circuit
against the oracle, repeated replays with other device work in between, the autotuner, and
the 512-circuit workload checked on sampled circuits (oracle) and against the per-circuit
path (every circuit)."""

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    Q.lib()
    return Q


def _scale(terms):
    return max(1.0, sum(abs(c) for c, _ in terms))


def _small_batch(seed):
    circs, hams, params = W.uneven_batch_workload(n_circuits=14, n_min=4, n_max=14, depth_min=1, depth_max=4,
                                                  n_terms=12, seed=seed)
    return circs, hams, params


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_matches_oracle(Q, dtype):
    circs, hams, params = _small_batch(3)
    b = Q.qsv_batch_create(circs, hams, dtype)
    E, g = Q.qsv_batch_expectation_and_grad(b, params)
    for i, (c, h) in enumerate(zip(circs, hams)):
        p = params[b.offsets[i]:b.offsets[i + 1]]
        E_ref, g_ref = O.grad_adjoint(c, h, p)
        tol = TOL[dtype] * _scale(h)
        assert abs(E[i] - E_ref) <= tol, (i, c["n_qubits"])
        assert np.max(np.abs(g[b.offsets[i]:b.offsets[i + 1]] - g_ref)) <= tol, (i, c["n_qubits"])


def test_graph_replays_with_eager_work_between(Q):
    """The captured evaluation replayed several times with new parameters, with other
    kernels and synchronizations of the program in between; every replay against the oracle."""
    circs, hams, params = _small_batch(5)
    b = Q.qsv_batch_create(circs, hams, "c128")
    s = Q.qsv_state_create(12, "c128")
    rng = np.random.default_rng(9)
    for rep in range(3):
        p = params + rng.uniform(-0.5, 0.5, params.size)
        E, g = Q.qsv_batch_expectation_and_grad(b, p)
        Q.qsv_apply_circuit(s, W.random_circuit(12, 40, rep), np.zeros(8))
        Q.qsv_state_synchronize(s)
        for i in (0, 5, len(circs) - 1):
            pi = p[b.offsets[i]:b.offsets[i + 1]]
            E_ref, g_ref = O.grad_adjoint(circs[i], hams[i], pi)
            assert abs(E[i] - E_ref) <= 1e-12 * _scale(hams[i])
            assert np.max(np.abs(g[b.offsets[i]:b.offsets[i + 1]] - g_ref)) <= 1e-12 * _scale(hams[i])


def test_autotune_picks_a_candidate_and_keeps_results(Q):
    circs, hams, params = _small_batch(7)
    b = Q.qsv_batch_create(circs, hams, "c64")
    E0, g0 = Q.qsv_batch_expectation_and_grad(b, params)
    t, low = Q.qsv_batch_autotune(b, params, with_schedule=True)
    assert t in (10, 11, 12, 13) and low in (2, 3, 4)
    assert b.info()["tile_qubits"] == t
    E1, g1 = Q.qsv_batch_expectation_and_grad(b, params)
    S = max(_scale(h) for h in hams)
    assert np.max(np.abs(E1 - E0)) <= 1e-5 * S and np.max(np.abs(g1 - g0)) <= 1e-5 * S


def test_uneven512_workload(Q):
    """512 circuits (8-20 qubits, depth 2-10, 50 Pauli strings each), complex64: every circuit
    against the per-circuit path, and against the oracle the six smallest circuits plus, for
    every qubit count 8..20, its shallowest circuit."""
    circs, hams, params = W.uneven_batch_workload()
    b = Q.qsv_batch_create(circs, hams, "c64")
    E, g = Q.qsv_batch_expectation_and_grad(b, params)
    assert np.all(np.isfinite(E)) and np.all(np.isfinite(g))
    order = list(np.argsort([c["n_qubits"] for c in circs], kind="stable")[:6])
    by_n = {}
    for i, c in enumerate(circs):
        k = c["n_qubits"]
        if k not in by_n or len(c["gates"]) < len(circs[by_n[k]]["gates"]):
            by_n[k] = i
    order += [i for k, i in sorted(by_n.items()) if i not in order]
    checked = 0
    for i in order:
        print(f"uneven512 circuit {i}: n={circs[i]['n_qubits']} gates={len(circs[i]['gates'])}", flush=True)
        p = params[b.offsets[i]:b.offsets[i + 1]]
        E_ref, g_ref = O.grad_adjoint(circs[i], hams[i], p)
        tol = 1e-5 * _scale(hams[i])
        assert abs(E[i] - E_ref) <= tol
        assert np.max(np.abs(g[b.offsets[i]:b.offsets[i + 1]] - g_ref)) <= tol
        checked += 1
    s_by_n = {}
    for i in range(len(circs)):
        n = circs[i]["n_qubits"]
        if n not in s_by_n:
            s_by_n[n] = Q.qsv_state_create(n, "c64")
        p = params[b.offsets[i]:b.offsets[i + 1]]
        Ei, gi = Q.qsv_expectation_and_grad(s_by_n[n], circs[i], hams[i], p)
        tol = 1e-5 * _scale(hams[i])
        assert abs(E[i] - Ei) <= tol, (i, n)
        assert np.max(np.abs(g[b.offsets[i]:b.offsets[i + 1]] - gi)) <= tol, (i, n)
    assert checked == len(order) and len(by_n) == 13
