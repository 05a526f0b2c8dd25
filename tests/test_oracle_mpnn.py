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


def test_forward_by_hand_on_a_fixed_graph():
    """The network's definition (node features, both message-passing layers with the
    neighbour sum scaled by 1/4, ReLU, the mean readout and the output map) worked out by
    hand on a fixed graph with one-hot weights.  Graph: the 4-cycle 0-1-2-3 and the
    triangle 4-5-6; nodes 7..15 are isolated.  Features: nodes 0..6 have degree 2
    ([1, 0.5, t]) with t = 1/3 on the triangle, 0 on the cycle; isolated nodes [1, 0, 0].

    layer 1 (hidden columns 0..4):
      Z1[:,0] = 1 * x0                       -> 1 everywhere
      Z1[:,1] = 2 * x1 - 0.5                 -> 0.5 on nodes 0..6, -0.5 (relu 0) elsewhere
      Z1[:,2] = 4 * (sum of neighbours' x1) / 4 -> 1 on nodes 0..6, 0 elsewhere
      Z1[:,3] = -1 (bias only)               -> relu 0
      Z1[:,4] = 3 * x2                       -> 1 on the triangle, 0 elsewhere
    layer 2:
      Z2[:,0] = 3 * H1[:,0]                  -> 3 everywhere
      Z2[:,1] = H1[:,1] + 4 * (sum of neighbours' H1[:,2]) / 4 -> 0.5 + 2 = 2.5 on 0..6
      Z2[:,2] = -2 * (sum of neighbours' H1[:,0]) / 4 + 0.25 -> -0.75 (relu 0) on 0..6,
                                               0.25 on the 9 isolated nodes
      Z2[:,3] = H1[:,4]                      -> 1 on the triangle
    readout (mean over the 16 nodes): g = (3, 2.5 * 7/16, 0.25 * 9/16, 3/16, 0, ...)
    angles = ramp + (0.1 g0, g1, 4 g2, g3, 0, ...) + bo with bo[5] = -0.5."""
    graph = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 4)]
    masks = _masks([graph])
    A = M.adjacency(masks)
    X = M.features(A).numpy()[0]
    assert np.allclose(X[:4], [1, 0.5, 0]) and np.allclose(X[4:7], [1, 0.5, 1 / 3]) and np.allclose(X[7:], [1, 0, 0])

    P = {name: np.zeros(shape) for name, shape in M.SHAPES}
    P["W1s"][0, 0] = 1.0
    P["W1s"][1, 1] = 2.0
    P["b1"][1] = -0.5
    P["W1n"][1, 2] = 4.0
    P["b1"][3] = -1.0
    P["W1s"][2, 4] = 3.0
    P["W2s"][0, 0] = 3.0
    P["W2s"][1, 1] = 1.0
    P["W2n"][2, 1] = 4.0
    P["W2n"][0, 2] = -2.0
    P["b2"][2] = 0.25
    P["W2s"][4, 3] = 1.0
    P["Wo"][0, 0] = 0.1
    P["Wo"][1, 1] = 1.0
    P["Wo"][2, 2] = 4.0
    P["Wo"][3, 3] = 1.0
    P["bo"][5] = -0.5
    theta = np.concatenate([P[name].ravel() for name, _ in M.SHAPES])
    assert theta.size == M.N_PARAMS

    ramp = W.linear_ramp()
    out = M.predict(theta, masks, ramp)[0]
    g = np.array([3.0, 2.5 * 7 / 16, 0.25 * 9 / 16, 3 / 16])
    expect = ramp.copy()
    expect[0] += 0.1 * g[0]
    expect[1] += g[1]
    expect[2] += 4.0 * g[2]
    expect[3] += g[3]
    expect[5] += -0.5
    assert np.max(np.abs(out - expect)) < 1e-14
