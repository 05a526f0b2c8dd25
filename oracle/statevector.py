"""Plain CPU complex128 state-vector oracle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code with the HIP path: it reads the plain
circuit / Pauli-sum descriptions of ``workloads`` and implements every gate,
expectation and gradient itself, slowly and directly, in numpy complex128.

Conventions (MindSpore Quantum paper, section 2):

* little-endian: bit ``q`` of a basis index is qubit ``q`` (section 2.6, the
  simulator usage example and its remark on endianness);
* fixed gates I, X, Y, Z, H as printed in section 2.3 (fixed gates);
* RX/RY/RZ(theta) = exp(-i theta P / 2) as printed in section 2.3
  (parameterized gates);
* S, T, their inverses, PhaseShift, SWAP and RXX/RYY/RZZ are the standard
  definitions (the paper uses them by name without printing the matrices);
* U3(a, b, c) = RZ(b) RX(-pi/2) RZ(a) RX(pi/2) RZ(c), the decomposition section 4.1
  (learning a rotation) gives for it, taken as its definition;
* expectation E = <psi|H|psi> of a Pauli sum (section 2.6, get_expectation);
* adjoint-method gradient (named in section 7, QAOA task) following Jones &
  Gacon, arXiv:2009.02823; parameter-shift and central finite differences as
  independent routes.

Every function states the passage it follows.  Parity pins for each function
live in ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------------------
# Gate matrices.  Row/column bit b of the matrix index refers to targets[b].
# --------------------------------------------------------------------------------------
_I2 = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)            # section 2.3, fixed gates
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)         # section 2.3, fixed gates
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)           # section 2.3, fixed gates
_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)  # section 2.3
_PAULI = {"I": _I2, "X": _X, "Y": _Y, "Z": _Z}


def _kron2(a_hi, b_lo):
    """Two-qubit operator with ``b_lo`` on targets[0] and ``a_hi`` on targets[1]."""
    return np.kron(a_hi, b_lo)


def _pauli_rotation(P, theta):
    """exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P for P^2 = I (section 2.3)."""
    d = P.shape[0]
    return np.cos(theta / 2.0) * np.eye(d, dtype=np.complex128) - 1j * np.sin(theta / 2.0) * P


def _pauli_rotation_deriv(P, theta):
    """d/dtheta of exp(-i theta P / 2)."""
    d = P.shape[0]
    return -0.5 * np.sin(theta / 2.0) * np.eye(d, dtype=np.complex128) - 0.5j * np.cos(theta / 2.0) * P


def _u3(theta, phi, lam):
    """U3 as section 4.1 defines it: the rotation RZ(phi) RX(-pi/2) RZ(theta) RX(pi/2)
    RZ(lam), in which the middle three factors equal RY(theta), written out in closed form
    (no global phase factor beyond the one this product carries)."""
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    ep, em = np.exp(0.5j * (phi + lam)), np.exp(0.5j * (phi - lam))
    return np.array([[c / ep, -s / em],
                     [em * s, ep * c]], dtype=np.complex128)


def _u3_derivs(theta, phi, lam):
    """Derivatives of the section 4.1 U3 with respect to theta, phi and lam."""
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    ep, em = np.exp(0.5j * (phi + lam)), np.exp(0.5j * (phi - lam))
    d_theta = 0.5 * np.array([[-s / ep, -c / em], [em * c, -ep * s]], dtype=np.complex128)
    d_phi = 0.5j * np.array([[-c / ep, s / em], [em * s, ep * c]], dtype=np.complex128)
    d_lam = 0.5j * np.array([[-c / ep, -s / em], [-em * s, ep * c]], dtype=np.complex128)
    return d_theta, d_phi, d_lam


_FIXED = {
    "X": _X, "Y": _Y, "Z": _Z, "H": _H,
    "S": np.diag([1, 1j]).astype(np.complex128),
    "SDG": np.diag([1, -1j]).astype(np.complex128),
    "T": np.diag([1, np.exp(1j * np.pi / 4)]).astype(np.complex128),
    "TDG": np.diag([1, np.exp(-1j * np.pi / 4)]).astype(np.complex128),
    "SWAP": np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128),
}
_ROT_GENERATOR = {
    "RX": _X, "RY": _Y, "RZ": _Z,
    "RXX": _kron2(_X, _X), "RYY": _kron2(_Y, _Y), "RZZ": _kron2(_Z, _Z),
}


def gate_angles(g, params):
    """Bound angles of a gate: angle = const + coeff * params[index] (section 2.2,
    linear parameter expressions such as RX(0.2a + 0.5b))."""
    out = []
    for (i, coeff, const) in g["params"]:
        out.append(const + (coeff * params[i] if i >= 0 else 0.0))
    return out


def gate_matrix(g, params=None):
    """Unitary of one gate on its targets (controls excluded)."""
    kind = g["kind"]
    if kind in _FIXED:
        return _FIXED[kind]
    if kind in ("MAT1", "MAT2"):
        return np.asarray(g["matrix"], dtype=np.complex128)
    ang = gate_angles(g, params)
    if kind in _ROT_GENERATOR:
        return _pauli_rotation(_ROT_GENERATOR[kind], ang[0])
    if kind == "PS":
        return np.diag([1.0, np.exp(1j * ang[0])]).astype(np.complex128)
    if kind == "U3":
        return _u3(*ang)
    raise ValueError(f"unknown gate {kind}")


def gate_angle_derivs(g, params):
    """d U / d angle_j for each angle of a parameterized gate, from the closed forms."""
    kind = g["kind"]
    ang = gate_angles(g, params)
    if kind in _ROT_GENERATOR:
        return [_pauli_rotation_deriv(_ROT_GENERATOR[kind], ang[0])]
    if kind == "PS":
        return [np.diag([0.0, 1j * np.exp(1j * ang[0])]).astype(np.complex128)]
    if kind == "U3":
        return list(_u3_derivs(*ang))
    return []


# --------------------------------------------------------------------------------------
# Applying gates.  psi is viewed as an n-axis tensor whose axis n-1-q is qubit q
# (little-endian, section 2.6).  A gate on targets T with controls C acts on the
# sub-tensor where every control axis equals 1 (section 2.3, gates with controls via
# on(obj, ctrl)).
# --------------------------------------------------------------------------------------
def apply_matrix(psi, n, U, targets, ctrls=()):
    """psi <- (U on targets, controlled on ctrls) psi, in place; returns psi."""
    k = len(targets)
    t = psi.reshape((2,) * n)
    index = [slice(None)] * n
    for c in ctrls:
        index[n - 1 - c] = 1
    sub = t[tuple(index)]
    # axis of each target inside ``sub`` (control axes were removed by integer indexing)
    remaining = [a for a in range(n) if not (n - 1 - a) in ctrls]
    axis_of = {n - 1 - a: remaining.index(a) for a in remaining}
    # U as a tensor (row bits then column bits), most significant target first
    Ut = np.asarray(U, dtype=np.complex128).reshape((2,) * (2 * k))
    tgt_axes = [axis_of[targets[b]] for b in reversed(range(k))]
    out = np.tensordot(Ut, sub, axes=(list(range(k, 2 * k)), tgt_axes))
    out = np.moveaxis(out, list(range(k)), tgt_axes)
    sub[...] = out
    return psi


def apply_gate(psi, n, g, params=None, dagger=False):
    U = gate_matrix(g, params)
    if dagger:
        U = U.conj().T
    return apply_matrix(psi, n, U, g["targets"], g["ctrls"])


def zero_state(n):
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def simulate(circ, params=None, psi0=None):
    """psi = U_M ... U_1 psi0 (section 2.6, apply_circuit); psi0 defaults to |0...0>."""
    n = circ["n_qubits"]
    psi = zero_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    for g in circ["gates"]:
        apply_gate(psi, n, g, params)
    return psi


# --------------------------------------------------------------------------------------
# Pauli sums (section 2.5, QubitOperator; section 2.6, get_expectation / apply_hamiltonian).
# --------------------------------------------------------------------------------------
def pauli_masks(factors):
    """(x_mask, z_mask) of a Pauli string: X -> x bit, Z -> z bit, Y -> both."""
    xm = zm = 0
    for (q, p) in factors:
        if p in ("X", "Y"):
            xm |= 1 << q
        if p in ("Z", "Y"):
            zm |= 1 << q
    return xm, zm


def _popcount(a):
    a = np.asarray(a, dtype=np.uint64)
    c = np.zeros(a.shape, dtype=np.int64)
    while np.any(a):
        c += (a & np.uint64(1)).astype(np.int64)
        a = a >> np.uint64(1)
    return c


def apply_pauli_string(psi, n, factors):
    """P|psi> for P = prod_q P_q.  With Y = i X Z per qubit:
    P|x> = i^{popcount(xm & zm)} (-1)^{popcount(x & zm)} |x xor xm>."""
    xm, zm = pauli_masks(factors)
    x = np.arange(2 ** n, dtype=np.uint64)
    phase = (1j) ** (bin(xm & zm).count("1"))
    sign = 1.0 - 2.0 * (_popcount(x & np.uint64(zm)) & 1)
    out = np.zeros_like(psi)
    out[(x ^ np.uint64(xm)).astype(np.int64)] = phase * sign * psi
    return out


def apply_pauli_sum(psi, n, terms):
    """lambda = H psi (unnormalized), section 2.6 apply_hamiltonian."""
    out = np.zeros_like(psi)
    for (c, factors) in terms:
        out += c * apply_pauli_string(psi, n, factors)
    return out


def expectation(psi, n, terms):
    """<psi|H|psi> as a complex number (section 2.6, get_expectation)."""
    return np.vdot(psi, apply_pauli_sum(psi, n, terms))


def inner_product(phi, psi):
    """<phi|psi> (section 2.6, get_expectation with H = I)."""
    return np.vdot(phi, psi)


# --------------------------------------------------------------------------------------
# Gradients of E(params) = <psi(params)|H|psi(params)>.
# --------------------------------------------------------------------------------------
def energy(circ, terms, params, psi0=None):
    n = circ["n_qubits"]
    return expectation(simulate(circ, params, psi0), n, terms).real


def grad_adjoint(circ, terms, params, psi0=None):
    """Adjoint method (Jones & Gacon, arXiv:2009.02823): forward psi_M, lambda = H psi_M,
    then for k = M..1: psi_{k-1} = U_k^dag psi_k, g_k = 2 Re <lambda_k | dU_k psi_{k-1}>,
    lambda_{k-1} = U_k^dag lambda_k.  Chain rule over angle = const + coeff * p[idx]."""
    n = circ["n_qubits"]
    params = np.asarray(params, dtype=np.float64)
    psi = simulate(circ, params, psi0)
    lam = apply_pauli_sum(psi, n, terms)
    E = np.vdot(psi, lam).real
    grad = np.zeros_like(params)
    for g in reversed(circ["gates"]):
        apply_gate(psi, n, g, params, dagger=True)
        if any(i >= 0 for (i, _, _) in g["params"]):
            for (i, coeff, _), dU in zip(g["params"], gate_angle_derivs(g, params)):
                if i < 0:
                    continue
                mu = apply_matrix(psi.copy(), n, dU, g["targets"], ()) if not g["ctrls"] else \
                    _apply_controlled_deriv(psi, n, dU, g)
                grad[i] += coeff * 2.0 * np.vdot(lam, mu).real
        apply_gate(lam, n, g, params, dagger=True)
    return E, grad


def _apply_controlled_deriv(psi, n, dU, g):
    """d/dtheta of a controlled gate: dU on the control-satisfied subspace, zero elsewhere."""
    out = np.zeros_like(psi)
    t_out = out.reshape((2,) * n)
    t_in = psi.reshape((2,) * n)
    index = [slice(None)] * n
    for c in g["ctrls"]:
        index[n - 1 - c] = 1
    t_out[tuple(index)] = t_in[tuple(index)]
    return apply_matrix(out, n, dU, g["targets"], ())


def grad_param_shift(circ, terms, params, psi0=None):
    """Two-term parameter-shift rule per gate occurrence (valid for exp(-i theta P/2)
    with P^2 = I, PhaseShift and each U3 angle): dE/dtheta = [E(theta+pi/2) -
    E(theta-pi/2)] / 2; chain rule over the linear parameter binding."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros_like(params)
    gates = circ["gates"]
    for k, g in enumerate(gates):
        for a, (i, coeff, const) in enumerate(g["params"]):
            if i < 0:
                continue
            if g["ctrls"]:
                raise ValueError("two-term shift rule does not hold for controlled rotations")
            vals = []
            for shift in (+np.pi / 2, -np.pi / 2):
                shifted = dict(g)
                ps = list(g["params"])
                ps[a] = (-1, 0.0, const + coeff * params[i] + shift)
                shifted["params"] = tuple(ps)
                c2 = {"n_qubits": circ["n_qubits"], "gates": gates[:k] + [shifted] + gates[k + 1:]}
                vals.append(energy(c2, terms, params, psi0))
            grad[i] += coeff * 0.5 * (vals[0] - vals[1])
    return grad


def grad_finite_diff(circ, terms, params, h=1e-6, psi0=None):
    """Central finite differences of E with step h."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros_like(params)
    for i in range(params.size):
        e = np.zeros_like(params)
        e[i] = h
        grad[i] = (energy(circ, terms, params + e, psi0) - energy(circ, terms, params - e, psi0)) / (2 * h)
    return grad


# --------------------------------------------------------------------------------------
# General form E = <phi| U_l^dag H U_r |psi> (section 2.6, get_expectation with a left
# circuit and state; section 4.1, the gradient operator with circ_left).
# --------------------------------------------------------------------------------------
def expectation_general(circ_r, params_r, psi, circ_l, params_l, phi, terms):
    n = circ_r["n_qubits"]
    psi_r = simulate(circ_r, params_r, psi)
    phi_l = simulate(circ_l, params_l, phi) if circ_l is not None else np.array(phi, dtype=np.complex128)
    return np.vdot(phi_l, apply_pauli_sum(psi_r, n, terms))


def _simulate_replacing(circ, params, psi0, k, a):
    """The circuit with gate k replaced by d(gate)/d(angle a): the derivative matrix on the
    control-satisfied subspace and zero elsewhere."""
    n = circ["n_qubits"]
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for i, g in enumerate(circ["gates"]):
        if i != k:
            apply_gate(psi, n, g, params)
            continue
        dU = gate_angle_derivs(g, params)[a]
        psi = _apply_controlled_deriv(psi, n, dU, g) if g["ctrls"] else apply_matrix(psi, n, dU, g["targets"], ())
    return psi


def grad_general(circ_r, params_r, psi, circ_l, params_l, phi, terms):
    """(E, dE/dparams_r, dE/dparams_l) as complex numbers, by the definition: E is linear in
    every gate of U_r and conjugate-linear in every gate of U_l, so each parameter's
    derivative is the sum over its occurrences of coeff * E with that gate replaced by its
    derivative matrix."""
    n = circ_r["n_qubits"]
    params_r = np.asarray(params_r, dtype=np.float64)
    psi_r = simulate(circ_r, params_r, psi)
    phi_l = simulate(circ_l, params_l, phi) if circ_l is not None else np.array(phi, dtype=np.complex128)
    E = np.vdot(phi_l, apply_pauli_sum(psi_r, n, terms))
    g_r = np.zeros(params_r.size, dtype=np.complex128)
    for k, g in enumerate(circ_r["gates"]):
        for a, (i, coeff, _) in enumerate(g["params"]):
            if i >= 0:
                v = _simulate_replacing(circ_r, params_r, psi, k, a)
                g_r[i] += coeff * np.vdot(phi_l, apply_pauli_sum(v, n, terms))
    g_l = None
    if circ_l is not None:
        params_l = np.asarray(params_l, dtype=np.float64)
        chi = apply_pauli_sum(psi_r, n, terms)
        g_l = np.zeros(params_l.size, dtype=np.complex128)
        for k, g in enumerate(circ_l["gates"]):
            for a, (i, coeff, _) in enumerate(g["params"]):
                if i >= 0:
                    v = _simulate_replacing(circ_l, params_l, phi, k, a)
                    g_l[i] += coeff * np.vdot(v, chi)
    return E, g_r, g_l


# --------------------------------------------------------------------------------------
# Brute force: the full 2^n x 2^n unitary from Kronecker products (small n only).
# --------------------------------------------------------------------------------------
def _kron_chain(ops_by_qubit, n):
    """Kronecker product with qubit n-1 leftmost and qubit 0 rightmost (little-endian)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        out = np.kron(out, ops_by_qubit.get(q, _I2))
    return out


def full_gate_unitary(g, n, params=None):
    """U_full = (I - Pi_C) + sum_{a,b} U[a,b] (x)_q op_q, where op_q = |a_j><b_j| on
    target q = targets[j], |1><1| on controls, I elsewhere; Pi_C projects every
    control on |1>."""
    U = gate_matrix(g, params)
    k = len(g["targets"])
    P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    ctrl_proj = {c: P1 for c in g["ctrls"]}
    full = np.eye(2 ** n, dtype=np.complex128) - _kron_chain(ctrl_proj, n)
    for a in range(2 ** k):
        for b in range(2 ** k):
            if U[a, b] == 0:
                continue
            ops = dict(ctrl_proj)
            for j, t in enumerate(g["targets"]):
                e = np.zeros((2, 2), dtype=np.complex128)
                e[(a >> j) & 1, (b >> j) & 1] = 1.0
                ops[t] = e
            full += U[a, b] * _kron_chain(ops, n)
    return full


def full_circuit_unitary(circ, params=None):
    n = circ["n_qubits"]
    U = np.eye(2 ** n, dtype=np.complex128)
    for g in circ["gates"]:
        U = full_gate_unitary(g, n, params) @ U
    return U


def pauli_sum_matrix(terms, n):
    """Dense matrix of a Pauli sum via Kronecker products (section 2.5, QubitOperator.matrix)."""
    M = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for (c, factors) in terms:
        M += c * _kron_chain({q: _PAULI[p] for (q, p) in factors}, n)
    return M
