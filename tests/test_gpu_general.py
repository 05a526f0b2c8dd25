"""The general form <phi|U_l^dag H U_r|psi> with complex gradients of both circuits, and
several Hamiltonians at once, against the oracle."""

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}
KINDS = ["RX", "RY", "RZ", "PS", "RZZ", "RXX", "RYY", "U3", "H", "S", "X", "MAT1", "MAT2", "SWAP"]


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    Q.lib()
    return Q


def _scale(terms):
    return max(1.0, sum(abs(c) for c, _ in terms))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,left,seed", [(3, True, 1), (7, True, 2), (13, True, 3), (15, False, 4)])
def test_general_matches_oracle(Q, dtype, n, left, seed):
    rng = np.random.default_rng(seed)
    cr = W.random_circuit(n, 40, seed, kinds=KINDS, max_ctrls=1, n_params=4, param_fraction=0.8)
    cl = W.random_circuit(n, 30, seed + 100, kinds=KINDS, max_ctrls=1, n_params=3, param_fraction=0.8) if left else None
    H = W.random_pauli_sum(n, 10, rng)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    psi = W.random_state(n, rng).astype(npdt)
    phi = W.random_state(n, rng).astype(npdt)
    pr, pl = rng.uniform(-2, 2, 4), rng.uniform(-2, 2, 3)
    E_ref, gr_ref, gl_ref = O.grad_general(cr, pr, psi.astype(complex), cl, pl if left else None,
                                           phi.astype(complex), H)
    s_psi = Q.qsv_state_create(n, dtype)
    s_phi = Q.qsv_state_create(n, dtype)
    Q.qsv_state_set(s_psi, psi)
    Q.qsv_state_set(s_phi, phi)
    E, gr, gl = Q.qsv_expectation_general(s_psi, cr, pr, s_phi, cl, pl if left else None, H)
    tol = TOL[dtype] * _scale(H)
    assert abs(E - E_ref) <= tol
    assert np.max(np.abs(gr - gr_ref)) <= tol
    if left:
        assert np.max(np.abs(gl - gl_ref)) <= tol
    assert np.array_equal(Q.qsv_state_get(s_psi), psi) and np.array_equal(Q.qsv_state_get(s_phi), phi)


def test_general_with_same_state_reduces_to_expectation(Q):
    """phi = psi and U_l = U_r: E is real and grad_r + grad_l is the ordinary gradient."""
    n = 9
    circ, H, params = W.hea_circuit(n, 2), W.zz_chain_hamiltonian(n), W.uniform_params(36, 4)
    s = Q.qsv_state_create(n, "c128")
    E, gr, gl = Q.qsv_expectation_general(s, circ, params, s, circ, params, H)
    E_ref, g_ref = O.grad_adjoint(circ, H, params)
    assert abs(E - E_ref) < 1e-12 * n and abs(E.imag) < 1e-12 * n
    assert np.max(np.abs((gr + gl) - g_ref)) < 1e-11 * n


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_several_hamiltonians(Q, dtype):
    n = 11
    circ = W.hea_circuit(n, 3)
    params = W.uniform_params(66, 5)
    rng = np.random.default_rng(6)
    hams = [W.random_pauli_sum(n, 15, rng) for _ in range(4)] + [W.zz_chain_hamiltonian(n)]
    s = Q.qsv_state_create(n, dtype)
    E, G = Q.qsv_expectation_and_grad_multi(s, circ, hams, params)
    for k, H in enumerate(hams):
        E_ref, g_ref = O.grad_adjoint(circ, H, params)
        tol = TOL[dtype] * _scale(H)
        assert abs(E[k] - E_ref) <= tol
        assert np.max(np.abs(G[k] - g_ref)) <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_general_u3_in_one_circuit_only(Q, dtype):
    """U3 only in the right circuit (no left circuit, phi != psi): E and the complex
    gradients depend on U3's global phase, which section 4.1's product
    RZ(b) RX(-pi/2) RZ(a) RX(pi/2) RZ(c) fixes; the oracle builds U3 from that product."""
    n = 5
    rng = np.random.default_rng(9)
    gates = []
    for q in range(n):
        gates.append(W.gate("U3", (q,), params=(W.param_angle(0), W.param_angle(1, 0.5), W.param_angle(2, -1.0, 0.3))))
        gates.append(W.gate("X", ((q + 1) % n,), ctrls=(q,)))
    cr = W.circuit(n, gates)
    H = W.random_pauli_sum(n, 8, rng)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    psi = W.random_state(n, rng).astype(npdt)
    phi = W.random_state(n, rng).astype(npdt)
    pr = rng.uniform(-2, 2, 3)
    E_ref, gr_ref, _ = O.grad_general(cr, pr, psi.astype(complex), None, None, phi.astype(complex), H)
    s_psi, s_phi = Q.qsv_state_create(n, dtype), Q.qsv_state_create(n, dtype)
    Q.qsv_state_set(s_psi, psi)
    Q.qsv_state_set(s_phi, phi)
    E, gr, _ = Q.qsv_expectation_general(s_psi, cr, pr, s_phi, None, None, H)
    tol = TOL[dtype] * _scale(H)
    assert abs(E - E_ref) <= tol
    assert np.max(np.abs(gr - gr_ref)) <= tol
    # the standard-matrix U3 (section 4.1's product times e^{i(b+c)/2}) gives another E
    assert abs(E_ref) > 1e-3
