"""Learned warm start for QAOA MaxCut on 16-node graphs.

Labels are angles the simulator itself optimized: every graph's p = 6 QAOA circuit is put
in one batch (`qsv_batch`: one HIP graph replay evaluates all energies and adjoint
gradients) and Adam runs on the host over all graphs at once, starting from a linear ramp.
The network (`qsv_mpnn`) is trained on those labels by the library's forward, backward and
Adam kernels; at test time it proposes starting angles, and the same simulator judges the
energy they reach and how many optimizer steps they save.
"""

from __future__ import annotations

import numpy as np

from . import _lib

N_NODES, P_LAYERS = 16, 6


def adjacency_masks(edges, n_nodes=N_NODES):
    m = np.zeros(n_nodes, dtype=np.uint16)
    for (u, v) in edges:
        m[u] |= np.uint16(1 << v)
        m[v] |= np.uint16(1 << u)
    return m


class QaoaBatch:
    """Energies and gradients of p-layer QAOA MaxCut circuits for many graphs (maximize the
    cut = minimize the negated cut Hamiltonian)."""

    def __init__(self, graphs, circuit_fn, hamiltonian_fn, p=P_LAYERS, dtype="c64", n_nodes=N_NODES):
        self.graphs = graphs
        self.p = p
        circs = [circuit_fn(n_nodes, e, p) for e in graphs]
        hams = [[(-c, f) for (c, f) in hamiltonian_fn(e)] for e in graphs]
        self.batch = _lib.qsv_batch_create(circs, hams, dtype)
        self.n_edges = np.array([len(e) for e in graphs], dtype=np.float64)

    def cut_and_grad(self, angles):
        """Expected cut [G] and its gradient [G, 2p] for angles [G, 2p]."""
        E, g = _lib.qsv_batch_expectation_and_grad(self.batch, np.ascontiguousarray(angles).reshape(-1))
        return -E, -g.reshape(angles.shape)


def optimize(qb, init, steps, lr=0.02, target=None):
    """Adam (ascent on the cut) from init [G, 2p]; returns final angles, final cuts, and for
    each graph the first step at which the cut reached target[g] (steps if never)."""
    x = np.array(init, dtype=np.float64, copy=True)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    hit = np.full(x.shape[0], steps, dtype=np.int64)
    cut = None
    for t in range(1, steps + 1):
        cut, g = qb.cut_and_grad(x)
        if target is not None:
            newly = (cut >= target) & (hit == steps)
            hit[newly] = t - 1
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        x += lr * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    cut, _ = qb.cut_and_grad(x)
    if target is not None:
        hit[(cut >= target) & (hit == steps)] = steps
    return x, cut, hit


def init_params(seed, scale=0.1):
    """Initial network parameters: small Gaussian weights, zero biases, zero readout, so the
    untrained network returns the ramp exactly."""
    rng = np.random.default_rng(seed)
    w = np.zeros(_lib.MPNN_PARAMS, dtype=np.float32)
    F, H, O = 3, 64, 12
    offs = [0, F * H, 2 * F * H, 2 * F * H + H, 2 * F * H + H + H * H, 2 * F * H + H + 2 * H * H]
    w[offs[0]:offs[1]] = rng.normal(0, scale, F * H)
    w[offs[1]:offs[2]] = rng.normal(0, scale, F * H)
    w[offs[3]:offs[4]] = rng.normal(0, scale / 4, H * H)
    w[offs[4]:offs[5]] = rng.normal(0, scale / 4, H * H)
    return w


def train(net, masks, labels, ramp, epochs, batch_size=256, lr=3e-3, seed=0):
    """Minibatch Adam on the device; returns the loss of each step."""
    rng = np.random.default_rng(seed)
    n = masks.shape[0]
    losses = []
    for _ in range(epochs):
        order = rng.permutation(n)
        for s in range(0, n, batch_size):
            idx = order[s:s + batch_size]
            losses.append(net.train_step(masks[idx], ramp, labels[idx], lr))
    return np.array(losses)
