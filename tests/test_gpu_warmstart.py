"""Warm-start network on the GPU: forward and gradient against the CPU reference, and a
small end-to-end run (simulator-optimized labels, device training) showing the trained
network's starting angles beat the linear ramp on held-out graphs."""

import numpy as np
import pytest

import workloads as W
from oracle import mpnn as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    from paper_2406_17248_amd import warmstart as WS
    Q.lib()
    return Q, WS


def test_forward_and_gradient_match_reference(Q):
    Qm, WS = Q
    rng = np.random.default_rng(1)
    graphs = W.warmstart_graphs(48, 5)
    masks = np.stack([WS.adjacency_masks(e) for e in graphs])
    theta = WS.init_params(3, scale=0.3)
    theta[-12 - 64 * 12:-12] = rng.normal(0, 0.1, 64 * 12)
    ramp = W.linear_ramp()
    labels = ramp + rng.normal(0, 0.2, (48, 12))
    net = Qm.Mpnn(theta)
    ang = net.predict(masks, ramp)
    ref_ang = M.predict(theta.astype(np.float64), masks, ramp)
    assert np.max(np.abs(ang - ref_ang)) < 1e-5
    loss, g = net.loss_and_grad(masks, ramp, labels)
    ref_loss, ref_g = M.loss_and_grad(theta.astype(np.float64), masks, ramp, labels)
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, ref_loss)
    assert np.max(np.abs(g - ref_g)) <= 1e-5 * max(1.0, np.max(np.abs(ref_g)))


def test_untrained_network_returns_the_ramp(Q):
    Qm, WS = Q
    masks = np.stack([WS.adjacency_masks(e) for e in W.warmstart_graphs(8, 6)])
    net = Qm.Mpnn(WS.init_params(0))
    assert np.max(np.abs(net.predict(masks, W.linear_ramp()) - W.linear_ramp())) < 1e-6


def test_trained_network_beats_linear_ramp(Q):
    """Labels: angles optimized by the simulator (adjoint gradients in one batch) from the
    linear ramp.  The network, trained on 256 graphs, starts 64 held-out graphs at a higher
    expected cut than the ramp and reaches the ramp-optimized cut in fewer optimizer steps."""
    Qm, WS = Q
    ramp = W.linear_ramp()
    train_g = W.warmstart_graphs(256, 11)
    test_g = W.warmstart_graphs(64, 12)
    qb_train = WS.QaoaBatch(train_g, W.qaoa_circuit, W.maxcut_hamiltonian)
    labels, _, _ = WS.optimize(qb_train, np.tile(ramp, (256, 1)), steps=150)
    masks = np.stack([WS.adjacency_masks(e) for e in train_g])
    net = Qm.Mpnn(WS.init_params(1))
    losses = WS.train(net, masks, labels, ramp, epochs=80, batch_size=64, lr=3e-3)
    assert losses[-10:].mean() < 0.5 * losses[:4].mean()
    qb = WS.QaoaBatch(test_g, W.qaoa_circuit, W.maxcut_hamiltonian)
    tmasks = np.stack([WS.adjacency_masks(e) for e in test_g])
    init_ramp = np.tile(ramp, (64, 1))
    init_net = net.predict(tmasks, ramp)
    cut_ramp, _ = qb.cut_and_grad(init_ramp)
    cut_net, _ = qb.cut_and_grad(init_net)
    assert cut_net.mean() > cut_ramp.mean() + 0.05
    _, best, _ = WS.optimize(qb, init_ramp, steps=150)
    target = best - 1e-3 * qb.n_edges
    _, _, steps_ramp = WS.optimize(qb, init_ramp, steps=150, target=target)
    _, _, steps_net = WS.optimize(qb, init_net, steps=150, target=target)
    assert steps_net.mean() < 0.8 * steps_ramp.mean()
