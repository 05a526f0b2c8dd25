"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on identical seeded
inputs.  Tolerances: amplitudes max |d psi| <= 1e-12 (complex128) / 1e-5 (complex64);
expectations and gradients |d| <= tol * max(1, S), S = sum_k |c_k| of the Hamiltonian."""

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
DTYPES = ["c128", "c64"]


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    Q.lib()
    return Q


def _scale(terms):
    return max(1.0, sum(abs(c) for c, _ in terms))


def _new_state(Q, n, dtype, psi0=None, tile=None, adj_tile=None):
    s = Q.qsv_state_create(n, dtype)
    if psi0 is not None:
        Q.qsv_state_set(s, psi0)
    if tile is not None:
        Q.qsv_state_set_option(s, Q.OPT_TILE_QUBITS, tile)
    if adj_tile is not None:
        Q.qsv_state_set_option(s, Q.OPT_ADJ_TILE_QUBITS, adj_tile)
    return s


# ------------------------------------------------------------------------------------------
# amplitudes
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,tile,seed", [
    (1, None, 1), (2, None, 2), (3, None, 3), (5, None, 4), (8, None, 5), (12, None, 6),
    (14, None, 7), (16, None, 8), (17, 4, 9), (15, 6, 10), (13, 3, 11), (18, 0, 12), (11, 0, 13),
    (19, None, 14), (20, 9, 15), (18, 10, 16), (17, 11, 17), (16, 13, 18),
])
def test_apply_circuit_matches_oracle(Q, dtype, n, tile, seed):
    """Random circuits over every gate kind, target position (0 and n-1 included) and up to
    two controls; fused tile passes of several widths and the unfused per-gate path."""
    print(f"apply_circuit n={n} tile={tile} seed={seed} dtype={dtype}", flush=True)
    circ = W.random_circuit(n, 160 if n > 2 else 40, seed, max_ctrls=2 if n >= 3 else 1)
    params = np.random.default_rng(seed).uniform(-np.pi, np.pi, 8)
    psi0 = W.random_state(n, np.random.default_rng(seed + 1000))
    ref = O.simulate(circ, params, psi0)
    s = _new_state(Q, n, dtype, psi0.astype(np.complex64 if dtype == "c64" else np.complex128), tile=tile)
    Q.qsv_apply_circuit(s, circ, params)
    got = Q.qsv_state_get(s)
    assert np.max(np.abs(got - ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,tile,seed", [(14, None, 41), (16, 9, 42), (15, 11, 43)])
def test_non_unitary_matrices_match_oracle(Q, dtype, n, tile, seed):
    """Brick layers whose one-qubit matrices are Haar unitaries, general complex matrices
    (scaled to spectral norm 1) and unitaries off by 1e-9: only exact unitaries may run as a
    phase and a real matrix, the others stay dense."""
    print(f"non-unitary n={n} tile={tile} seed={seed} dtype={dtype}", flush=True)
    rng = np.random.default_rng(seed)
    gs = []
    for layer in range(8):
        for q in range(n):
            kind = rng.integers(3)
            if kind == 0:
                m = W.haar_unitary_2x2(rng)
            elif kind == 1:
                m = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
                m /= np.linalg.norm(m, 2)
            else:
                m = W.haar_unitary_2x2(rng) * (1.0 + 1e-9)
            gs.append(W.gate("MAT1", (q,), matrix=m))
        for a in range(layer % 2, n - 1, 2):
            gs.append(W.gate("Z", (a + 1,), ctrls=(a,)))
    circ = W.circuit(n, gs)
    psi0 = W.random_state(n, np.random.default_rng(seed + 1000))
    ref = O.simulate(circ, np.zeros(0), psi0)
    s = _new_state(Q, n, dtype, psi0.astype(np.complex64 if dtype == "c64" else np.complex128), tile=tile)
    Q.qsv_apply_circuit(s, circ, np.zeros(0))
    got = Q.qsv_state_get(s)
    assert np.max(np.abs(got - ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,tile,seed", [(20, 9, 31), (19, 10, 32), (21, 11, 33), (18, 9, 34), (22, 12, 35)])
def test_relayout_passes_match_in_place(Q, dtype, n, tile, seed):
    """Fused passes that store each tile in the next pass's bit layout (alternating between
    the state and a scratch buffer; even and odd pass counts) give the same amplitudes, bit
    for bit, as in-place passes, and both match the oracle."""
    print(f"relayout n={n} tile={tile} seed={seed} dtype={dtype}", flush=True)
    circ = W.random_circuit(n, 200, seed, max_ctrls=2)
    params = np.random.default_rng(seed).uniform(-np.pi, np.pi, 8)
    psi0 = W.random_state(n, np.random.default_rng(seed + 1000))
    psi0 = psi0.astype(np.complex64 if dtype == "c64" else np.complex128)
    ref = O.simulate(circ, params, psi0.astype(np.complex128))
    got = {}
    for relayout in (1, 0):
        s = _new_state(Q, n, dtype, psi0, tile=tile)
        Q.qsv_state_set_option(s, Q.OPT_RELAYOUT, relayout)
        Q.qsv_apply_circuit(s, circ, params)
        Q.qsv_apply_circuit(s, circ, params)  # a second call reuses the scratch buffer
        got[relayout] = Q.qsv_state_get(s)
    ref = O.simulate(circ, params, ref)
    assert np.array_equal(got[0], got[1])
    assert np.max(np.abs(got[1] - ref)) <= 2 * TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_apply_from_zero_state_and_reset(Q, dtype):
    n = 6
    gs = [W.gate("H", (0,))] + [W.gate("X", (q + 1,), ctrls=(q,)) for q in range(n - 1)]
    s = Q.qsv_state_create(n, dtype)
    Q.qsv_apply_circuit(s, W.circuit(n, gs))
    got = Q.qsv_state_get(s)
    expect = np.zeros(2 ** n)
    expect[0] = expect[-1] = np.sqrt(0.5)
    assert np.max(np.abs(got - expect)) <= TOL[dtype]
    Q.qsv_state_reset(s)
    e0 = np.zeros(2 ** n)
    e0[0] = 1
    assert np.array_equal(Q.qsv_state_get(s), e0.astype(got.dtype))


def test_paper_examples_on_gpu(Q):
    """Section 2.6 worked examples through the HIP path (complex128)."""
    s = Q.qsv_state_create(2, "c128")
    Q.qsv_apply_circuit(s, W.circuit(2, [W.gate("RX", (0,), params=(W.fixed_angle(2.5),))]))
    e = Q.qsv_expectation(s, [(1.0, ((0, "Z"), (1, "Z")))])
    assert abs(e.real - (-0.8011436155469336)) < 1e-15 and abs(e.imag) < 1e-15
    s2 = Q.qsv_state_create(2, "c128")
    t = Q.qsv_state_create(2, "c128")
    Q.qsv_apply_pauli_sum(t, s2, [(1.0, ((0, "X"), (1, "Y")))])
    Q.qsv_apply_circuit(t, W.circuit(2, [W.gate("H", (0,)), W.gate("X", (1,), ctrls=(0,))]))
    expect = np.zeros(4, complex)
    expect[1], expect[2] = -1j * np.sqrt(0.5), 1j * np.sqrt(0.5)
    assert np.max(np.abs(Q.qsv_state_get(t) - expect)) < 1e-15


# ------------------------------------------------------------------------------------------
# expectations and H psi
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (6, 3), (10, 4), (17, 5)])
def test_expectation_and_hpsi_match_oracle(Q, dtype, n, seed):
    print(f"expectation n={n} seed={seed} dtype={dtype}", flush=True)
    rng = np.random.default_rng(seed)
    terms = W.random_pauli_sum(n, 30, rng)
    psi = W.random_state(n, rng)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    s = _new_state(Q, n, dtype, psi.astype(npdt))
    psi_used = psi.astype(npdt).astype(np.complex128)
    e = Q.qsv_expectation(s, terms)
    ref = O.expectation(psi_used, n, terms)
    tol = TOL[dtype] * _scale(terms)
    assert abs(e - ref) <= tol
    d = Q.qsv_state_create(n, dtype)
    Q.qsv_apply_pauli_sum(d, s, terms)
    lam = Q.qsv_state_get(d)
    assert np.max(np.abs(lam - O.apply_pauli_sum(psi_used, n, terms))) <= tol
    assert np.array_equal(Q.qsv_state_get(s), psi.astype(npdt))  # get_* leaves the state unchanged


def _diagonal_sum(n, n_terms, n_low_patterns, rng):
    """Z-strings whose parts on the 12 low qubits come from a few patterns: the diagonal
    pass evaluates them pattern by pattern (terms sorted by pattern, chunks of 2^12)."""
    lows = [0] + [int(m) for m in rng.integers(1, 1 << 12, n_low_patterns - 1)]
    terms = [(float(rng.standard_normal()), ())]
    for _ in range(n_terms):
        z = int(rng.choice(lows)) | int(rng.integers(0, 1 << (n - 12))) << 12
        terms.append((float(rng.standard_normal()), tuple((q, "Z") for q in range(n) if z >> q & 1)))
    return terms


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,n_terms,n_pats,seed", [(12, 40, 9, 1), (14, 300, 60, 2), (14, 700, 200, 3),
                                                   (13, 513, 255, 4)])
@pytest.mark.parametrize("lead", [False, True])
def test_diagonal_sums_match_oracle(Q, dtype, n, n_terms, n_pats, seed, lead):
    """Diagonal Hamiltonians with term tables below and above the workgroup staging limit
    (512 terms), expectation only and with H psi written; with `lead` an X/Y term comes
    first, so the diagonal group adds its H psi to that of the group before it."""
    print(f"diagonal sum n={n} terms={n_terms} lead={lead} dtype={dtype}", flush=True)
    rng = np.random.default_rng(seed)
    terms = _diagonal_sum(n, n_terms, n_pats, rng)
    if lead:
        terms = [(0.7, ((3, "X"), (n - 1, "Y")))] + terms
    psi = W.random_state(n, rng)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    s = _new_state(Q, n, dtype, psi.astype(npdt))
    psi_used = psi.astype(npdt).astype(np.complex128)
    tol = TOL[dtype] * _scale(terms)
    assert abs(Q.qsv_expectation(s, terms) - O.expectation(psi_used, n, terms)) <= tol
    d = Q.qsv_state_create(n, dtype)
    Q.qsv_apply_pauli_sum(d, s, terms)
    assert np.max(np.abs(Q.qsv_state_get(d) - O.apply_pauli_sum(psi_used, n, terms))) <= tol


# ------------------------------------------------------------------------------------------
# gradients
# ------------------------------------------------------------------------------------------
GRAD_KINDS = ["RX", "RY", "RZ", "PS", "RXX", "RYY", "RZZ", "U3", "H", "S", "T", "X", "Y", "Z",
              "SWAP", "MAT1", "MAT2"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,adj_tile,ctrls,seed", [
    (2, None, 1, 1), (4, None, 2, 2), (7, None, 2, 3), (10, None, 2, 4), (13, None, 2, 5),
    (15, 4, 2, 6), (16, 6, 1, 7), (14, 3, 0, 8), (16, 9, 2, 9), (17, 11, 1, 10), (18, 10, 0, 11),
])
def test_adjoint_gradient_matches_oracle(Q, dtype, n, adj_tile, ctrls, seed):
    """Every parameterized kind (U3 included), shared parameters, controlled rotations."""
    print(f"grad n={n} adj_tile={adj_tile} seed={seed} dtype={dtype}", flush=True)
    circ = W.random_circuit(n, 90, seed, kinds=GRAD_KINDS, max_ctrls=ctrls, n_params=6, param_fraction=0.8)
    rng = np.random.default_rng(seed)
    terms = W.random_pauli_sum(n, 12, rng)
    params = rng.uniform(-np.pi, np.pi, 6)
    psi0 = W.random_state(n, np.random.default_rng(seed + 50))
    npdt = np.complex64 if dtype == "c64" else np.complex128
    psi0 = psi0.astype(npdt)
    E_ref, g_ref = O.grad_adjoint(circ, terms, params, psi0.astype(np.complex128))
    s = _new_state(Q, n, dtype, psi0, adj_tile=adj_tile)
    E, g = Q.qsv_expectation_and_grad(s, circ, terms, params)
    tol = TOL[dtype] * _scale(terms)
    assert abs(E - E_ref) <= tol
    assert np.max(np.abs(g - g_ref)) <= tol
    assert np.array_equal(Q.qsv_state_get(s), psi0)  # start state unchanged


@pytest.mark.parametrize("dtype", DTYPES)
def test_hea10_workload(Q, dtype):
    """10-qubit hardware-efficient ansatz (4 layers, 80 parameters), H = open ZZ chain:
    output state, <H> and the full gradient."""
    circ, terms, params = W.hea10_workload()
    psi_ref = O.simulate(circ, params)
    E_ref, g_ref = O.grad_adjoint(circ, terms, params)
    s = Q.qsv_state_create(10, dtype)
    E, g = Q.qsv_expectation_and_grad(s, circ, terms, params)
    tol = TOL[dtype] * _scale(terms)
    assert abs(E - E_ref) <= tol
    assert np.max(np.abs(g - g_ref)) <= tol
    Q.qsv_apply_circuit(s, circ, params)
    assert np.max(np.abs(Q.qsv_state_get(s) - psi_ref)) <= TOL[dtype]


def test_qupack_qaoa_printed_values_on_gpu(Q, golden_dir):
    """Section 6.2 printed expectation and 20 gradients through the HIP adjoint path."""
    g = json.load(open(os.path.join(golden_dir, "qaoa_k5_depth10.json")))
    n, p = g["n_qubits"], g["depth"]
    edges = W.complete_graph(n)
    circ = W.qaoa_circuit(n, edges, p)
    H = W.zz_sum_hamiltonian(edges)
    params = np.array([g["gamma"]] * p + [g["beta"]] * p)
    s = Q.qsv_state_create(n, "c128")
    E, grad = Q.qsv_expectation_and_grad(s, circ, H, params)
    assert abs(E - g["expectation"]) < 1e-12
    assert np.max(np.abs(grad - np.array(g["grad_gamma"] + g["grad_beta"]))) < 1e-10


@pytest.mark.parametrize("dtype", DTYPES)
def test_qaoa_batch_adjoint_and_param_shift(Q, dtype):
    """Batched QAOA MaxCut (random 3-regular graph): adjoint and GPU parameter-shift
    gradients against the oracle, for several parameter sets."""
    n, p, B = 12, 3, 5
    edges = W.random_regular_graph(3, n, 5)
    circ = W.qaoa_circuit(n, edges, p)
    H = W.maxcut_hamiltonian(edges)
    params = W.uniform_params(2 * p, 3, 0, np.pi, batch=B)
    s = Q.qsv_state_create(n, dtype)
    E, G = Q.qsv_expectation_and_grad_batch(s, circ, H, params)
    Eps, Gps = Q.qsv_param_shift_grad_batch(s, circ, H, params[:2])
    Eb = Q.qsv_expectation_batch(s, circ, H, params)
    tol = TOL[dtype] * _scale(H)
    for b in range(B):
        E_ref, g_ref = O.grad_adjoint(circ, H, params[b])
        assert abs(E[b] - E_ref) <= tol and abs(Eb[b] - E_ref) <= tol
        assert np.max(np.abs(G[b] - g_ref)) <= tol
        if b < 2:
            assert abs(Eps[b] - E_ref) <= tol
            assert np.max(np.abs(Gps[b] - g_ref)) <= tol


# ------------------------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times
# ------------------------------------------------------------------------------------------
def _lightcone_z(circ, q):
    """<Z_q> after a circuit from |0..0>, on the CPU oracle, simulating only the gates in
    the backward light cone of qubit q (gates outside it cancel in U^dag Z_q U)."""
    keep, cone = [], {q}
    for g in reversed(circ["gates"]):
        qs = set(g["targets"]) | set(g["ctrls"])
        if qs & cone:
            cone |= qs
            keep.append(g)
    keep.reverse()
    order = sorted(cone)
    relabel = {old: new for new, old in enumerate(order)}
    gates = [dict(g, targets=tuple(relabel[t] for t in g["targets"]),
                  ctrls=tuple(relabel[c] for c in g["ctrls"])) for g in keep]
    sub = W.circuit(len(order), gates)
    psi = O.simulate(sub)
    return O.expectation(psi, len(order), [(1.0, ((relabel[q], "Z"),))]).real


@pytest.mark.parametrize("dtype", DTYPES)
def test_brick30_sampled_outputs(Q, dtype):
    """30-qubit depth-20 brick circuit (8 / 16 GiB state): <Z_q> for edge qubits against the
    oracle's light-cone simulation, the norm, and <sum Z> = sum of the sampled parts."""
    circ, H = W.brick_workload()
    print(f"brick30 dtype={dtype}", flush=True)
    s = Q.qsv_state_create(30, dtype)
    Q.qsv_apply_circuit(s, circ)
    norm = Q.qsv_expectation(s, [(1.0, ())]).real
    assert abs(norm - 1.0) <= TOL[dtype]
    tol = TOL[dtype]
    for q in (0, 29):
        ref = _lightcone_z(circ, q)
        got = Q.qsv_expectation(s, [(1.0, ((q, "Z"),))]).real
        assert abs(got - ref) <= tol, (q, got, ref)
    total = Q.qsv_expectation(s, H).real
    parts = sum(Q.qsv_expectation(s, [(1.0, ((q, "Z"),))]).real for q in range(30))
    assert abs(total - parts) <= tol


@pytest.mark.parametrize("dtype", DTYPES)
def test_qaoa24_batch64_p1_closed_form(Q, dtype):
    """24-qubit QAOA on the benchmark's random 3-regular graph, batch 64, at p = 1 where the
    energy has a closed form (Wang et al. 2018): energies and gradients (derivative of the
    closed form) for all 64 parameter sets."""
    import networkx as nx
    _, _, _, edges = W.qaoa_workload()
    n = 24
    circ = W.qaoa_circuit(n, edges, 1)
    H = W.maxcut_hamiltonian(edges)
    params = W.uniform_params(2, 99, 0, np.pi, batch=64)
    G = nx.Graph(edges)

    def closed(gp, bp):
        g, b = -2 * gp, bp / 2
        tot = 0.0
        for (u, v) in edges:
            du, dv = G.degree[u] - 1, G.degree[v] - 1
            t = len(set(G[u]) & set(G[v]))
            tot += (0.5 + 0.25 * np.sin(4 * b) * np.sin(g) * (np.cos(g) ** du + np.cos(g) ** dv)
                    - 0.25 * np.sin(2 * b) ** 2 * np.cos(g) ** (du + dv - 2 * t) * (1 - np.cos(2 * g) ** t))
        return tot

    s = Q.qsv_state_create(n, dtype)
    E, Gr = Q.qsv_expectation_and_grad_batch(s, circ, H, params)
    tol = TOL[dtype] * _scale(H)
    h = 1e-30  # complex-step derivative of the closed form: exact to rounding
    for b in range(64):
        gp, bp = params[b]
        assert abs(E[b] - closed(gp, bp)) <= tol
        dg = closed(gp + 1j * h, bp).imag / h
        db = closed(gp, bp + 1j * h).imag / h
        assert abs(Gr[b, 0] - dg) <= tol and abs(Gr[b, 1] - db) <= tol
