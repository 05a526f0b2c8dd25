"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only *describes* circuits, Hamiltonians and parameter sets as plain
data; it contains none of the simulation arithmetic.  Both the oracle (under
``oracle/``) and the product binding read these descriptions, each with its own
code.  Random numbers (Haar single-qubit unitaries, angles, graphs, Pauli
strings) are drawn here from ``numpy.random.default_rng(seed)`` so both sides
see identical bits.

Circuit description (a plain ``dict``)::

    {"n_qubits": n,
     "gates": [ {"kind": "RX", "targets": (q,), "ctrls": (), "params": ((idx, coeff, const),),
                 "matrix": None}, ... ]}

* ``kind`` is one of :data:`GATE_KINDS`.  CNOT is ``X`` with one control, CZ is
  ``Z`` with one control.
* ``params`` holds one ``(param_index, coeff, const)`` triple per angle
  (``angle = const + coeff * params[param_index]``; ``param_index = -1`` means
  the angle is the constant alone).  RX..RZZ and PS take one angle, U3 takes
  three ``(theta, phi, lam)``; fixed gates take none.
* ``matrix`` is a complex128 2x2 (``MAT1``) or 4x4 (``MAT2``) array; row/column
  bit ``b`` of its index refers to ``targets[b]``.

Pauli sum description: a list of ``(coeff, ((qubit, "X"|"Y"|"Z"), ...))``
pairs; an empty string of factors is the identity term.
"""

from __future__ import annotations

import numpy as np

GATE_KINDS = (
    "X", "Y", "Z", "H", "S", "SDG", "T", "TDG",
    "RX", "RY", "RZ", "PS", "RXX", "RYY", "RZZ", "U3",
    "SWAP", "MAT1", "MAT2",
)
N_ANGLES = {k: 0 for k in GATE_KINDS}
N_ANGLES.update({"RX": 1, "RY": 1, "RZ": 1, "PS": 1, "RXX": 1, "RYY": 1, "RZZ": 1, "U3": 3})
N_TARGETS = {k: 1 for k in GATE_KINDS}
N_TARGETS.update({"RXX": 2, "RYY": 2, "RZZ": 2, "SWAP": 2, "MAT2": 2})


def gate(kind, targets, ctrls=(), params=(), matrix=None):
    """Build one gate record.  ``params`` is a tuple of (index, coeff, const)."""
    if kind not in GATE_KINDS:
        raise ValueError(f"unknown gate kind {kind!r}")
    targets = tuple(int(t) for t in np.atleast_1d(targets))
    ctrls = tuple(int(c) for c in np.atleast_1d(ctrls)) if len(np.atleast_1d(ctrls)) else ()
    params = tuple((int(i), float(c), float(k)) for (i, c, k) in params)
    if len(targets) != N_TARGETS[kind]:
        raise ValueError(f"{kind} takes {N_TARGETS[kind]} target(s)")
    if len(params) != N_ANGLES[kind]:
        raise ValueError(f"{kind} takes {N_ANGLES[kind]} angle(s)")
    if matrix is not None:
        matrix = np.ascontiguousarray(matrix, dtype=np.complex128)
    return {"kind": kind, "targets": targets, "ctrls": ctrls, "params": params, "matrix": matrix}


def fixed_angle(theta):
    """Angle triple for a gate whose angle is a constant."""
    return (-1, 0.0, float(theta))


def param_angle(index, coeff=1.0, const=0.0):
    return (int(index), float(coeff), float(const))


def circuit(n_qubits, gates):
    return {"n_qubits": int(n_qubits), "gates": list(gates)}


def n_params_of(circ):
    m = -1
    for g in circ["gates"]:
        for (i, _, _) in g["params"]:
            m = max(m, i)
    return m + 1


# ----------------------------------------------------------------------------------------
# Hardware-efficient ansatz: per layer RY(theta_q) RZ(phi_q) on every qubit, then a CNOT
# ladder q -> q+1 (no wrap).  Parameter layout params[l*2n + q] = theta, params[l*2n+n+q] = phi.
# ----------------------------------------------------------------------------------------
def hea_circuit(n_qubits=10, layers=4):
    gs = []
    n = n_qubits
    for l in range(layers):
        for q in range(n):
            gs.append(gate("RY", (q,), params=(param_angle(l * 2 * n + q),)))
            gs.append(gate("RZ", (q,), params=(param_angle(l * 2 * n + n + q),)))
        for q in range(n - 1):
            gs.append(gate("X", (q + 1,), ctrls=(q,)))
    return circuit(n, gs)


def zz_chain_hamiltonian(n_qubits):
    """H = sum_i Z_i Z_{i+1} over an open chain."""
    return [(1.0, ((i, "Z"), (i + 1, "Z"))) for i in range(n_qubits - 1)]


def uniform_params(n_params, seed, low=0.0, high=2 * np.pi, batch=None):
    rng = np.random.default_rng(seed)
    shape = (n_params,) if batch is None else (batch, n_params)
    return rng.uniform(low, high, size=shape)


# ----------------------------------------------------------------------------------------
# Random brick circuit: each layer a Haar-random 2x2 unitary on every qubit, then CZ on
# (2i, 2i+1) for even layers and on (2i+1, 2i+2) for odd layers.
# ----------------------------------------------------------------------------------------
def haar_unitary_2x2(rng):
    """Haar-distributed U(2): QR of a complex Ginibre matrix with the phases of R's
    diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def brick_circuit(n_qubits=30, depth=20, seed=2406):
    rng = np.random.default_rng(seed)
    gs = []
    n = n_qubits
    for l in range(depth):
        for q in range(n):
            gs.append(gate("MAT1", (q,), matrix=haar_unitary_2x2(rng)))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gs.append(gate("Z", (a + 1,), ctrls=(a,)))
    return circuit(n, gs)


def sum_z_hamiltonian(n_qubits):
    return [(1.0, ((q, "Z"),)) for q in range(n_qubits)]


# ----------------------------------------------------------------------------------------
# QAOA MaxCut.  Start |+>^n (a Hadamard on every qubit), then per layer l:
#   prod_{(i,j) in E} exp(-i gamma_l Z_i Z_j)  (= RZZ with angle 2*gamma_l),
#   prod_q RX(beta_l).
# Parameter layout [gamma_1..gamma_p, beta_1..beta_p].
# ----------------------------------------------------------------------------------------
def qaoa_circuit(n_qubits, edges, p, include_hadamards=True):
    gs = []
    if include_hadamards:
        for q in range(n_qubits):
            gs.append(gate("H", (q,)))
    for l in range(p):
        for (i, j) in edges:
            gs.append(gate("RZZ", (i, j), params=(param_angle(l, 2.0),)))
        for q in range(n_qubits):
            gs.append(gate("RX", (q,), params=(param_angle(p + l, 1.0),)))
    return circuit(n_qubits, gs)


def maxcut_hamiltonian(edges):
    """H = sum_e 1/2 (1 - Z_i Z_j), i.e. the number of cut edges."""
    terms = [(0.5 * len(edges), ())]
    terms += [(-0.5, ((i, "Z"), (j, "Z"))) for (i, j) in edges]
    return terms


def zz_sum_hamiltonian(edges, coeff=1.0):
    return [(coeff, ((i, "Z"), (j, "Z"))) for (i, j) in edges]


def random_regular_graph(degree, n_nodes, seed):
    import networkx as nx
    g = nx.random_regular_graph(degree, n_nodes, seed=seed)
    return sorted(tuple(sorted(e)) for e in g.edges)


def ring_graph(n_nodes):
    return [(i, (i + 1) % n_nodes) if i < (i + 1) % n_nodes else ((i + 1) % n_nodes, i)
            for i in range(n_nodes)]


def complete_graph(n_nodes):
    return [(i, j) for i in range(n_nodes) for j in range(i + 1, n_nodes)]


# ----------------------------------------------------------------------------------------
# Random Pauli sums and random gate sequences (parity tests).
# ----------------------------------------------------------------------------------------
def random_pauli_sum(n_qubits, n_terms, rng, max_locality=4, identity_term=True):
    terms = []
    if identity_term:
        terms.append((float(rng.standard_normal()), ()))
    for _ in range(n_terms):
        k = int(rng.integers(1, min(max_locality, n_qubits) + 1))
        qs = rng.choice(n_qubits, size=k, replace=False)
        ps = rng.choice(["X", "Y", "Z"], size=k)
        terms.append((float(rng.standard_normal()), tuple((int(q), str(p)) for q, p in zip(qs, ps))))
    return terms


def random_circuit(n_qubits, n_gates, seed, kinds=None, max_ctrls=1, n_params=8,
                   param_fraction=0.5):
    """Random gates on random targets (every position, including qubit 0 and n-1)."""
    rng = np.random.default_rng(seed)
    kinds = kinds or GATE_KINDS
    n = n_qubits
    gs = []
    for _ in range(n_gates):
        kind = str(rng.choice(kinds))
        nt = N_TARGETS[kind]
        if nt > n:
            kind, nt = "H", 1
        qs = [int(q) for q in rng.choice(n, size=nt, replace=False)]
        free = [q for q in range(n) if q not in qs]
        nc = int(rng.integers(0, min(max_ctrls, len(free)) + 1)) if max_ctrls else 0
        cs = tuple(int(c) for c in rng.choice(free, size=nc, replace=False)) if nc else ()
        params = []
        for _a in range(N_ANGLES[kind]):
            if n_params > 0 and rng.uniform() < param_fraction:
                params.append(param_angle(int(rng.integers(0, n_params)),
                                          float(rng.choice([1.0, -0.5, 2.0])),
                                          float(rng.uniform(-1, 1))))
            else:
                params.append(fixed_angle(rng.uniform(-np.pi, np.pi)))
        mat = None
        if kind == "MAT1":
            mat = haar_unitary_2x2(rng)
        elif kind == "MAT2":
            z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2.0)
            q, r = np.linalg.qr(z)
            d = np.diagonal(r)
            mat = q * (d / np.abs(d))[None, :]
        gs.append(gate(kind, tuple(qs), ctrls=cs, params=tuple(params), matrix=mat))
    return circuit(n, gs)


def random_state(n_qubits, rng, dtype=np.complex128):
    """A random normalized state (Gaussian amplitudes)."""
    v = rng.standard_normal(2 ** n_qubits) + 1j * rng.standard_normal(2 ** n_qubits)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


# ----------------------------------------------------------------------------------------
# The benchmark workloads, by name.
# ----------------------------------------------------------------------------------------
UNEVEN512 = dict(n_circuits=512, n_min=8, n_max=20, depth_min=2, depth_max=10, n_terms=50, seed=512)
HEA10 = dict(n_qubits=10, layers=4, param_seed=1)
BRICK30 = dict(n_qubits=30, depth=20, seed=2406)
QAOA24 = dict(n_qubits=24, degree=3, graph_seed=17248, p=8, batch=64, param_seed=8)


def hea10_workload(n_qubits=HEA10["n_qubits"], layers=HEA10["layers"], seed=HEA10["param_seed"]):
    circ = hea_circuit(n_qubits, layers)
    ham = zz_chain_hamiltonian(n_qubits)
    params = uniform_params(n_params_of(circ), seed)
    return circ, ham, params


def brick_workload(n_qubits=BRICK30["n_qubits"], depth=BRICK30["depth"], seed=BRICK30["seed"]):
    return brick_circuit(n_qubits, depth, seed), sum_z_hamiltonian(n_qubits)


def qaoa_workload(n_qubits=QAOA24["n_qubits"], p=QAOA24["p"], batch=QAOA24["batch"],
                  graph_seed=QAOA24["graph_seed"], param_seed=QAOA24["param_seed"],
                  degree=QAOA24["degree"]):
    edges = random_regular_graph(degree, n_qubits, graph_seed)
    circ = qaoa_circuit(n_qubits, edges, p)
    ham = maxcut_hamiltonian(edges)
    params = uniform_params(2 * p, param_seed, 0.0, np.pi, batch=batch)
    return circ, ham, params, edges


def uneven_batch_workload(n_circuits=UNEVEN512["n_circuits"], n_min=UNEVEN512["n_min"], n_max=UNEVEN512["n_max"],
                          depth_min=UNEVEN512["depth_min"], depth_max=UNEVEN512["depth_max"],
                          n_terms=UNEVEN512["n_terms"], seed=UNEVEN512["seed"]):
    """Hardware-efficient ansaetze with qubit counts uniform in [n_min, n_max] and depths
    uniform in [depth_min, depth_max]; each with its own Hamiltonian of n_terms random
    1-4-local Pauli strings (qubits without replacement, X/Y/Z uniform, N(0,1)
    coefficients) and its own angles uniform in [0, 2 pi).  Returns (circuits,
    hamiltonians, params) with params concatenated in circuit order."""
    rng = np.random.default_rng(seed)
    circs, hams, params = [], [], []
    for _ in range(n_circuits):
        n = int(rng.integers(n_min, n_max + 1))
        d = int(rng.integers(depth_min, depth_max + 1))
        c = hea_circuit(n, d)
        circs.append(c)
        hams.append(random_pauli_sum(n, n_terms, rng, max_locality=4, identity_term=False))
        params.append(rng.uniform(0.0, 2 * np.pi, n_params_of(c)))
    return circs, hams, np.concatenate(params)


# ----------------------------------------------------------------------------------------
# Learned warm start: 16-node graphs, half random 3-regular, half Erdos-Renyi G(16, 0.3).
# ----------------------------------------------------------------------------------------
WARMSTART = dict(n_nodes=16, p=6, n_train=20000, n_test=1000, seed=616)


def warmstart_graphs(n_graphs, seed, n_nodes=WARMSTART["n_nodes"]):
    """Edge lists: even indices random 3-regular, odd indices G(n, 0.3) (edgeless draws
    are redrawn)."""
    import networkx as nx
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(n_graphs):
        s = int(rng.integers(0, 2**31 - 1))
        if i % 2 == 0:
            g = nx.random_regular_graph(3, n_nodes, seed=s)
        else:
            g = nx.gnp_random_graph(n_nodes, 0.3, seed=s)
            while g.number_of_edges() == 0:
                s += 1
                g = nx.gnp_random_graph(n_nodes, 0.3, seed=s)
        graphs.append(sorted(tuple(sorted(e)) for e in g.edges))
    return graphs


def linear_ramp(p=WARMSTART["p"], d_gamma=1.0, d_beta=0.5):
    """Linear-ramp QAOA schedule gamma_l = d_gamma (l+1)/p, beta_l = d_beta (1 - l/p) for
    U = prod_l exp(-i beta_l B) exp(-i gamma_l C), written in the layer convention of
    qaoa_circuit (exp(-i g' Z Z), RX(b')): g' = -gamma/2, b' = 2 beta."""
    l = np.arange(p)
    return np.concatenate([-0.5 * d_gamma * (l + 1) / p, 2.0 * d_beta * (1 - l / p)])
