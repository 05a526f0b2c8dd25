"""Pins for the warm-start network's CPU reference: autograd gradient against central
finite differences, the zero-weight network returns the ramp plus the output bias, node
features against networkx's degree and triangle counts."""

import numpy as np

import workloads as W
from oracle import mpnn as M


def _masks(graphs):
    out = np.zeros((len(graphs), 16), dtype=np.uint16)
    for i, edges in enumerate(graphs):
        for (u, v) in edges:
            out[i, u] |= 1 << v
            out[i, v] |= 1 << u
    return out


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    masks = _masks(W.warmstart_graphs(4, 1))
    theta = rng.normal(0, 0.2, M.N_PARAMS)
    ramp = W.linear_ramp()
    labels = ramp + rng.normal(0, 0.3, (4, 12))
    _, g = M.loss_and_grad(theta, masks, ramp, labels)
    idx = rng.choice(M.N_PARAMS, 40, replace=False)
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = 1e-6
        fd = (M.loss_and_grad(theta + e, masks, ramp, labels)[0] - M.loss_and_grad(theta - e, masks, ramp, labels)[0]) / 2e-6
        assert abs(fd - g[i]) < 1e-7


def test_zero_weights_return_ramp_plus_bias():
    masks = _masks(W.warmstart_graphs(3, 2))
    theta = np.zeros(M.N_PARAMS)
    theta[-12:] = np.arange(12) * 0.01
    out = M.predict(theta, masks, W.linear_ramp())
    assert np.allclose(out, W.linear_ramp() + np.arange(12) * 0.01)


def test_features_match_networkx():
    import networkx as nx
    graphs = W.warmstart_graphs(6, 3)
    A = M.adjacency(_masks(graphs))
    X = M.features(A).numpy()
    for i, edges in enumerate(graphs):
        G = nx.Graph()
        G.add_nodes_from(range(16))
        G.add_edges_from(edges)
        tri = nx.triangles(G)
        for v in range(16):
            assert X[i, v, 1] == G.degree[v] / 4 and abs(X[i, v, 2] - tri[v] / 3) < 1e-12


def test_warmstart_graph_mix():
    graphs = W.warmstart_graphs(10, 4)
    for i, e in enumerate(graphs):
        deg = np.bincount(np.array(e).ravel(), minlength=16)
        if i % 2 == 0:
            assert np.all(deg == 3)
        assert len(e) > 0
