"""Pins for the CPU oracle: values the paper prints, closed forms, invariants and brute
force.  Each test names the passage it follows.  None of these values comes from the
HIP path."""

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

RNG_SEEDS = [11, 12, 13]


def _gate(kind, targets, ctrls=(), angles=(), matrix=None):
    return W.gate(kind, targets, ctrls, tuple(W.fixed_angle(a) for a in angles), matrix)


# ------------------------------------------------------------------------------------
# Worked examples printed in the paper
# ------------------------------------------------------------------------------------
def test_hadamard_little_endian_example():
    """Section 2.6: H on qubit 0 of a 2-qubit |00> gives sqrt(2)/2 (|00> + |01>), where the
    ket |01> has qubit 0 in |1> (little endian) -> basis index 1."""
    psi = O.simulate(W.circuit(2, [_gate("H", 0)]))
    expect = np.array([np.sqrt(0.5), np.sqrt(0.5), 0, 0])
    assert np.allclose(psi, expect, atol=1e-15)


def test_apply_hamiltonian_then_circuit_example():
    """Section 2.6 ("apply" method): apply X0 Y1 to |00>, then H(0) and X on 1 controlled
    by 0; the printed state is -sqrt(2)/2 j |01> + sqrt(2)/2 j |10>."""
    psi = O.zero_state(2)
    psi = O.apply_pauli_sum(psi, 2, [(1.0, ((0, "X"), (1, "Y")))])
    psi = O.simulate(W.circuit(2, [_gate("H", 0), _gate("X", 1, ctrls=(0,))]), psi0=psi)
    expect = np.zeros(4, complex)
    expect[0b01] = -1j * np.sqrt(0.5)
    expect[0b10] = 1j * np.sqrt(0.5)
    assert np.allclose(psi, expect, atol=1e-15)


def test_expectation_example():
    """Section 2.6 (get_expectation): <Z0 Z1> after RX(2.5) on qubit 0 is
    -0.8011436155469336."""
    psi = O.simulate(W.circuit(2, [_gate("RX", 0, angles=(2.5,))]))
    e = O.expectation(psi, 2, [(1.0, ((0, "Z"), (1, "Z")))])
    assert abs(e - (-0.8011436155469336)) < 1e-15


def test_inner_product_example():
    """Section 2.6 (get_expectation with H = I): <RY(1.5)00 | RX(2.5)00> is
    0.23071786267161518 - 0.6468646992187576j (fixes the sign of the -i in RX and of RY)."""
    psi = O.simulate(W.circuit(2, [_gate("RX", 0, angles=(2.5,))]))
    phi = O.simulate(W.circuit(2, [_gate("RY", 0, angles=(1.5,))]))
    v = O.inner_product(phi, psi)
    assert abs(v - (0.23071786267161518 - 0.6468646992187576j)) < 1e-15


def test_printed_pauli_operator_matrix(golden_dir):
    """Section 2.5: the printed matrix of 2 X0 Z1 + 2 Y1, reproduced column by column by
    applying the oracle's Pauli action to each basis state, and by the Kronecker form."""
    g = json.load(open(os.path.join(golden_dir, "pauli_2x0z1_plus_2y1.json")))
    M = np.array(g["matrix_re"]) + 1j * np.array(g["matrix_im"])
    terms = [(c, tuple((q, p) for q, p in f)) for c, f in g["terms"]]
    n = g["n_qubits"]
    cols = []
    for b in range(2 ** n):
        e = np.zeros(2 ** n, complex)
        e[b] = 1
        cols.append(O.apply_pauli_sum(e, n, terms))
    assert np.array_equal(np.stack(cols, axis=1), M)
    assert np.array_equal(O.pauli_sum_matrix(terms, n), M)


def test_qupack_qaoa_k5_printed_values(golden_dir):
    """Section 6.2: QuPack QAOA on K5, depth 10, gamma = 1, beta = 2.  Expectation and all
    20 gradients from the adjoint method; parameter-shift and finite differences agree."""
    g = json.load(open(os.path.join(golden_dir, "qaoa_k5_depth10.json")))
    n, p = g["n_qubits"], g["depth"]
    edges = W.complete_graph(n)
    circ = W.qaoa_circuit(n, edges, p)
    H = W.zz_sum_hamiltonian(edges)
    params = np.array([g["gamma"]] * p + [g["beta"]] * p)
    E, grad = O.grad_adjoint(circ, H, params)
    ref = np.array(g["grad_gamma"] + g["grad_beta"])
    assert abs(E - g["expectation"]) < 1e-12
    assert np.max(np.abs(grad - ref)) < 1e-10
    ps = O.grad_param_shift(circ, H, params)
    assert np.max(np.abs(ps - ref)) < 1e-10
    fd = O.grad_finite_diff(circ, H, params, h=1e-5)
    assert np.max(np.abs(fd - ref)) < 1e-6


def test_qaoa_p4_tutorial_optimum():
    """Section 5.2: p = 4 QAOA on the 5-node, 6-edge tutorial graph, trained with Adam
    (learning rate 0.05) from near-zero angles (the printed run starts at cut 3.0001),
    reaches an expected cut of 4.939257.  Gradients from the oracle's adjoint method."""
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (0, 2)]
    p = 4
    circ = W.qaoa_circuit(5, edges, p)
    H = W.maxcut_hamiltonian(edges)
    x = np.random.default_rng(0).normal(0.0, 0.01, 2 * p)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    for t in range(1, 401):
        E, g = O.grad_adjoint(circ, H, x)
        g = -g  # maximize the cut
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        x -= 0.05 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    assert abs(O.energy(circ, H, x) - 4.939257) < 5e-7


def test_rotate_three_states_optimum():
    """Section 4.1 (rotate three states): the maximum of sum_i <Z> over a U3 rotation of
    |0>, |+> and |+i> is sqrt(3) (printed 1.732)."""
    from scipy.optimize import minimize
    encoders = [(), (("RY", np.pi / 2),), (("RX", -np.pi / 2),)]

    def f(x):
        tot, g = 0.0, np.zeros(3)
        for enc in encoders:
            gs = [_gate(k, 0, angles=(a,)) for k, a in enc]
            gs.append(W.gate("U3", (0,), params=tuple(W.param_angle(i) for i in range(3))))
            E, gr = O.grad_adjoint(W.circuit(1, gs), [(1.0, ((0, "Z"),))], x)
            tot += E
            g += gr
        return -tot, -g

    best = max(-minimize(f, x0, jac=True, method="BFGS").fun
               for x0 in np.random.default_rng(1).uniform(-3, 3, (4, 3)))
    assert abs(best - np.sqrt(3)) < 1e-9


# ------------------------------------------------------------------------------------
# Closed forms
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_ghz_closed_form(n):
    """H on qubit 0 then a CNOT ladder gives (|0..0> + |1..1>)/sqrt(2) (section 4.3, GHZ)."""
    gs = [_gate("H", 0)] + [_gate("X", q + 1, ctrls=(q,)) for q in range(n - 1)]
    psi = O.simulate(W.circuit(n, gs))
    expect = np.zeros(2 ** n)
    expect[0] = expect[-1] = np.sqrt(0.5)
    assert np.allclose(psi, expect, atol=1e-15)


def test_bell_pair_with_swap_and_cz():
    """Bell pair: H(0), CNOT(0->1) = (|00>+|11>)/sqrt2; CZ then flips the sign of |11>;
    SWAP leaves it symmetric."""
    gs = [_gate("H", 0), _gate("X", 1, ctrls=(0,)), _gate("Z", 1, ctrls=(0,)), _gate("SWAP", (0, 1))]
    psi = O.simulate(W.circuit(2, gs))
    assert np.allclose(psi, [np.sqrt(.5), 0, 0, -np.sqrt(.5)], atol=1e-15)


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, np.pi, -2.2])
def test_ry_z_expectation_is_cos(theta):
    """<Z> after RY(theta)|0> is cos(theta); <X> is sin(theta); <Y> is 0."""
    psi = O.simulate(W.circuit(1, [_gate("RY", 0, angles=(theta,))]))
    assert abs(O.expectation(psi, 1, [(1.0, ((0, "Z"),))]) - np.cos(theta)) < 1e-15
    assert abs(O.expectation(psi, 1, [(1.0, ((0, "X"),))]) - np.sin(theta)) < 1e-15
    assert abs(O.expectation(psi, 1, [(1.0, ((0, "Y"),))])) < 1e-15


@pytest.mark.parametrize("theta", [0.4, 2.1])
def test_rx_y_expectation_is_minus_sin(theta):
    """<Y> after RX(theta)|0> = -sin(theta) with RX = exp(-i theta X / 2); <Z> = cos(theta)."""
    psi = O.simulate(W.circuit(1, [_gate("RX", 0, angles=(theta,))]))
    assert abs(O.expectation(psi, 1, [(1.0, ((0, "Y"),))]) + np.sin(theta)) < 1e-15
    assert abs(O.expectation(psi, 1, [(1.0, ((0, "Z"),))]) - np.cos(theta)) < 1e-15


@pytest.mark.parametrize("n", [4, 5, 7, 10])
def test_qaoa_p1_ring_closed_form(n):
    """p = 1 QAOA on an n-ring (Wang, Hadfield, Jiang, Rieffel, PRA 97 022304, 2018):
    with U = exp(-i b B) exp(-i g C), <C> = n [1/2 + 1/4 sin(4b) sin(2g)].  In the layer
    convention of section 6.2 (exp(-i g' ZZ), RX(b')) g = -2 g', b = b'/2."""
    edges = W.ring_graph(n)
    circ = W.qaoa_circuit(n, edges, 1)
    H = W.maxcut_hamiltonian(edges)
    for gp, bp in [(0.3, 0.7), (-1.1, 2.5), (0.9, -0.4)]:
        E = O.energy(circ, H, np.array([gp, bp]))
        g, b = -2 * gp, bp / 2
        assert abs(E - n * (0.5 + 0.25 * np.sin(4 * b) * np.sin(2 * g))) < 1e-13


@pytest.mark.parametrize("graph_seed", [3, 4])
def test_qaoa_p1_general_graph_closed_form(graph_seed):
    """p = 1 QAOA on any graph (Wang et al. 2018, theorem for <C_uv> with triangles):
    <C_uv> = 1/2 + 1/4 sin(4b) sin(g) (cos^du g + cos^dv g)
             - 1/4 sin^2(2b) cos^(du+dv-2 t) g (1 - cos^t (2g)),
    du = deg(u) - 1, dv = deg(v) - 1, t = triangles through uv."""
    import networkx as nx
    G = nx.gnp_random_graph(8, 0.5, seed=graph_seed)
    edges = sorted(tuple(sorted(e)) for e in G.edges)
    circ = W.qaoa_circuit(8, edges, 1)
    H = W.maxcut_hamiltonian(edges)
    gp, bp = 0.37, 1.21
    g, b = -2 * gp, bp / 2
    total = 0.0
    for (u, v) in edges:
        du, dv = G.degree[u] - 1, G.degree[v] - 1
        t = len(set(G[u]) & set(G[v]))
        total += (0.5 + 0.25 * np.sin(4 * b) * np.sin(g) * (np.cos(g) ** du + np.cos(g) ** dv)
                  - 0.25 * np.sin(2 * b) ** 2 * np.cos(g) ** (du + dv - 2 * t) * (1 - np.cos(2 * g) ** t))
    assert abs(O.energy(circ, H, np.array([gp, bp])) - total) < 1e-12


# ------------------------------------------------------------------------------------
# Invariants tying the remaining gates to the pinned ones
# ------------------------------------------------------------------------------------
def test_u3_matches_section_4_1_decomposition():
    """Section 4.1 (learning a rotation): U3(a, b, c) = RZ(b) RX(-pi/2) RZ(a) RX(pi/2) RZ(c),
    exactly (the global phase included, which the general form <phi|U_l^dag H U_r|psi>
    sees).  The right side is built from the rotations pinned by the printed section 2.6
    examples; special cases: U3(a, 0, 0) = RY(a), U3(0, b, c) = RZ(b + c)."""
    rng = np.random.default_rng(5)
    for _ in range(5):
        a, b, c = rng.uniform(-np.pi, np.pi, 3)
        gs = [_gate("RZ", 0, angles=(c,)), _gate("RX", 0, angles=(np.pi / 2,)),
              _gate("RZ", 0, angles=(a,)), _gate("RX", 0, angles=(-np.pi / 2,)), _gate("RZ", 0, angles=(b,))]
        V = O.full_circuit_unitary(W.circuit(1, gs))
        U = O.full_circuit_unitary(W.circuit(1, [_gate("U3", 0, angles=(a, b, c))]))
        assert np.allclose(V, U, atol=1e-14)
        RY = O.full_circuit_unitary(W.circuit(1, [_gate("RY", 0, angles=(a,))]))
        assert np.allclose(O.full_circuit_unitary(W.circuit(1, [_gate("U3", 0, angles=(a, 0.0, 0.0))])), RY,
                           atol=1e-15)
        RZ = O.full_circuit_unitary(W.circuit(1, [_gate("RZ", 0, angles=(b + c,))]))
        assert np.allclose(O.full_circuit_unitary(W.circuit(1, [_gate("U3", 0, angles=(0.0, b, c))])), RZ,
                           atol=1e-15)


def test_u3_ansatz_printed_expectation_and_gradient():
    """Section 4.1 (learning a rotation): for the U3 ansatz on |0> and H = X0 the printed
    output is f = -0.04602095 and, in the parameter order (c, a, b) of the listing,
    g = (-1.17e-17, -3.47310364e-02, -7.96875999e-01), at random p0 not printed.  Since
    <X> = sin(a) cos(b) here, the printed numbers fix cos(b) up to sign, sin(a) and cos(a);
    the oracle's E and adjoint gradient at one such point must give all three back."""
    f, gc, ga, gb = -0.04602095, -1.17340357e-17, -3.47310364e-02, -7.96875999e-01
    cb = np.hypot(f, ga)                   # |cos b| from sin a cos b and cos a cos b
    a = np.arctan2(f / cb, ga / cb)
    b = np.arctan2(gb / -np.sin(a), cb)    # dE/db = -sin a sin b
    c = 0.6180339887
    rz = [W.gate("RZ", (0,), params=(W.param_angle(i),)) for i in range(3)]  # c, a, b
    gs = [rz[0], _gate("RX", 0, angles=(np.pi / 2,)), rz[1], _gate("RX", 0, angles=(-np.pi / 2,)), rz[2]]
    H = [(1.0, ((0, "X"),))]
    for circ in (W.circuit(1, gs),
                 W.circuit(1, [W.gate("U3", (0,), params=(W.param_angle(1), W.param_angle(2), W.param_angle(0)))])):
        E, g = O.grad_adjoint(circ, H, np.array([c, a, b]))
        assert abs(E - f) < 1e-8
        assert np.max(np.abs(g - np.array([gc, ga, gb]))) < 1e-8


def test_phase_gates_relations():
    """S^2 = Z, T^2 = S, S SDG = T TDG = I, PS(pi) = Z, PS(pi/2) = S."""
    def U(*gs):
        return O.full_circuit_unitary(W.circuit(1, list(gs)))
    Z = U(_gate("Z", 0))
    S = U(_gate("S", 0))
    assert np.allclose(U(_gate("S", 0), _gate("S", 0)), Z)
    assert np.allclose(U(_gate("T", 0), _gate("T", 0)), S)
    assert np.allclose(U(_gate("S", 0), _gate("SDG", 0)), np.eye(2))
    assert np.allclose(U(_gate("T", 0), _gate("TDG", 0)), np.eye(2))
    assert np.allclose(U(_gate("PS", 0, angles=(np.pi,))), Z)
    assert np.allclose(U(_gate("PS", 0, angles=(np.pi / 2,))), S)


def test_two_qubit_rotations_and_swap_relations():
    """RXX = (H x H) RZZ (H x H); RYY = (RX(pi/2) x RX(pi/2)) RZZ (RX(-pi/2) x RX(-pi/2));
    RZZ(t) = CNOT RZ_1(t) CNOT; SWAP = three alternating CNOTs."""
    def U(*gs):
        return O.full_circuit_unitary(W.circuit(3, list(gs)))
    t = 0.731
    a, b = 0, 2
    hh = [_gate("H", a), _gate("H", b)]
    assert np.allclose(U(_gate("RXX", (a, b), angles=(t,))), U(*hh, _gate("RZZ", (a, b), angles=(t,)), *hh))
    rp = [_gate("RX", a, angles=(np.pi / 2,)), _gate("RX", b, angles=(np.pi / 2,))]
    rm = [_gate("RX", a, angles=(-np.pi / 2,)), _gate("RX", b, angles=(-np.pi / 2,))]
    assert np.allclose(U(_gate("RYY", (a, b), angles=(t,))), U(*rp, _gate("RZZ", (a, b), angles=(t,)), *rm))
    cx = _gate("X", b, ctrls=(a,))
    assert np.allclose(U(_gate("RZZ", (a, b), angles=(t,))), U(cx, _gate("RZ", b, angles=(t,)), cx))
    sw = U(_gate("X", b, ctrls=(a,)), _gate("X", a, ctrls=(b,)), _gate("X", b, ctrls=(a,)))
    assert np.allclose(U(_gate("SWAP", (a, b))), sw)


# ------------------------------------------------------------------------------------
# Brute force against Kronecker products, norms, gradient routes
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", RNG_SEEDS)
@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_gate_application_matches_kronecker_unitary(n, seed):
    """Gate-by-gate tensor application equals the product of full 2^n x 2^n Kronecker
    unitaries, for every gate kind, target position and single/double controls."""
    circ = W.random_circuit(n, 40, seed, max_ctrls=2 if n >= 4 else 1)
    params = np.random.default_rng(seed).uniform(-np.pi, np.pi, 8)
    psi0 = W.random_state(n, np.random.default_rng(seed + 100))
    U = O.full_circuit_unitary(circ, params)
    assert np.allclose(U.conj().T @ U, np.eye(2 ** n), atol=1e-12)
    assert np.allclose(O.simulate(circ, params, psi0), U @ psi0, atol=1e-12)


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_expectation_matches_dense_matrix(seed):
    n = 5
    rng = np.random.default_rng(seed)
    terms = W.random_pauli_sum(n, 20, rng)
    psi = W.random_state(n, rng)
    M = O.pauli_sum_matrix(terms, n)
    assert np.allclose(M, M.conj().T)
    assert abs(O.expectation(psi, n, terms) - np.vdot(psi, M @ psi)) < 1e-12
    assert np.allclose(O.apply_pauli_sum(psi, n, terms), M @ psi, atol=1e-12)


def test_norm_preserved():
    circ = W.random_circuit(9, 300, 7, max_ctrls=2)
    params = np.random.default_rng(7).uniform(-3, 3, 8)
    psi = O.simulate(circ, params, W.random_state(9, np.random.default_rng(8)))
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-13


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_gradient_routes_agree(seed):
    """Adjoint = parameter shift (exact) = central finite differences (O(h^2)) on random
    uncontrolled circuits with every parameterized kind and shared parameters."""
    n = 4
    kinds = ["RX", "RY", "RZ", "PS", "RXX", "RYY", "RZZ", "U3", "H", "S", "MAT1", "MAT2", "X"]
    circ = W.random_circuit(n, 30, seed, kinds=kinds, max_ctrls=0, n_params=5, param_fraction=0.8)
    rng = np.random.default_rng(seed)
    terms = W.random_pauli_sum(n, 8, rng)
    params = rng.uniform(-np.pi, np.pi, 5)
    E, ga = O.grad_adjoint(circ, terms, params)
    gp = O.grad_param_shift(circ, terms, params)
    gf = O.grad_finite_diff(circ, terms, params, h=1e-5)
    assert abs(E - O.energy(circ, terms, params)) < 1e-12
    assert np.max(np.abs(ga - gp)) < 1e-11
    assert np.max(np.abs(ga - gf)) < 1e-7


def test_controlled_gradient_matches_finite_difference():
    n = 4
    kinds = ["RX", "RY", "RZ", "PS", "RZZ", "U3", "H"]
    circ = W.random_circuit(n, 25, 21, kinds=kinds, max_ctrls=2, n_params=4, param_fraction=0.9)
    rng = np.random.default_rng(21)
    terms = W.random_pauli_sum(n, 6, rng)
    params = rng.uniform(-np.pi, np.pi, 4)
    _, ga = O.grad_adjoint(circ, terms, params)
    gf = O.grad_finite_diff(circ, terms, params, h=1e-5)
    assert np.max(np.abs(ga - gf)) < 1e-7


def test_hea_workload_shapes():
    circ, H, params = W.hea10_workload()
    assert circ["n_qubits"] == 10 and len(circ["gates"]) == 4 * 29
    assert params.shape == (80,) and len(H) == 9
    assert np.all((params >= 0) & (params < 2 * np.pi))


def test_brick_and_qaoa_workload_shapes():
    circ, H = W.brick_workload(n_qubits=30, depth=20)
    kinds = [g["kind"] for g in circ["gates"]]
    assert kinds.count("MAT1") == 600 and kinds.count("Z") == 290 and len(H) == 30
    for g in circ["gates"]:
        if g["kind"] == "MAT1":
            assert np.allclose(g["matrix"].conj().T @ g["matrix"], np.eye(2), atol=1e-14)
    circ, H, params, edges = W.qaoa_workload()
    assert len(edges) == 36 and params.shape == (64, 16)
    assert sum(g["kind"] == "RZZ" for g in circ["gates"]) == 288
    assert sum(g["kind"] == "RX" for g in circ["gates"]) == 192


# ------------------------------------------------------------------------------------
# General form <phi| U_l^dag H U_r |psi>
# ------------------------------------------------------------------------------------
def test_general_expectation_printed_inner_product():
    """Section 2.6: with H = I, U_r = RX(2.5), U_l = RY(1.5) on |00> the printed inner
    product is 0.23071786267161518 - 0.6468646992187576j."""
    ur = W.circuit(2, [_gate("RX", 0, angles=(2.5,))])
    ul = W.circuit(2, [_gate("RY", 0, angles=(1.5,))])
    E = O.expectation_general(ur, None, O.zero_state(2), ul, None, O.zero_state(2), [(1.0, ())])
    assert abs(E - (0.23071786267161518 - 0.6468646992187576j)) < 1e-15


def test_general_gradient_matches_finite_differences_and_real_case():
    n = 4
    kinds = ["RX", "RY", "RZ", "PS", "RZZ", "U3", "H", "RXX"]
    cr = W.random_circuit(n, 20, 31, kinds=kinds, max_ctrls=1, n_params=4, param_fraction=0.9)
    cl = W.random_circuit(n, 15, 32, kinds=kinds, max_ctrls=1, n_params=3, param_fraction=0.9)
    rng = np.random.default_rng(33)
    H = W.random_pauli_sum(n, 8, rng)
    psi, phi = W.random_state(n, rng), W.random_state(n, rng)
    pr, pl = rng.uniform(-2, 2, 4), rng.uniform(-2, 2, 3)
    E, gr, gl = O.grad_general(cr, pr, psi, cl, pl, phi, H)
    h = 1e-6
    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        fd = (O.expectation_general(cr, pr + e, psi, cl, pl, phi, H) -
              O.expectation_general(cr, pr - e, psi, cl, pl, phi, H)) / (2 * h)
        assert abs(fd - gr[i]) < 1e-8
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (O.expectation_general(cr, pr, psi, cl, pl + e, phi, H) -
              O.expectation_general(cr, pr, psi, cl, pl - e, phi, H)) / (2 * h)
        assert abs(fd - gl[i]) < 1e-8
    # same circuit and state on both sides: the real gradient is 2 Re of the right part
    Er, gr_same, gl_same = O.grad_general(cr, pr, psi, cr, pr, psi, H)
    _, g_real = O.grad_adjoint(cr, H, pr, psi)
    assert abs(Er.imag) < 1e-12
    assert np.max(np.abs(2 * gr_same.real - g_real)) < 1e-11
    assert np.max(np.abs(gr_same + gl_same - g_real)) < 1e-11
