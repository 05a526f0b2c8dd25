"""CPU reference of the warm-start network (test infrastructure only).

A 2-layer message-passing network on a 16-node graph that outputs p = 6 QAOA angles
(6 gamma then 6 beta) as a correction to a linear-ramp schedule.  Written with plain
PyTorch CPU ops in float64; gradients come from torch autograd (the exact derivative of
this definition).  Only the tests use it; the product's kernels are written separately.

    node features  x_v = [1, deg(v) / 4, triangles(v) / 3]
    layer 1        Z1 = X W1s + (A X) W1n / 4 + b1,   H1 = relu(Z1)
    layer 2        Z2 = H1 W2s + (A H1) W2n / 4 + b2, H2 = relu(Z2)
    readout        g = mean_v H2[v]
    angles         ramp + g Wo + bo
    loss           mean over graphs of sum_k (angles_k - label_k)^2 / 12

Parameter vector layout (float32 on the device): W1s[3,64], W1n[3,64], b1[64], W2s[64,64],
W2n[64,64], b2[64], Wo[64,12], bo[12], row-major, in this order.
"""

from __future__ import annotations

import numpy as np
import torch

N_NODES, N_FEAT, HIDDEN, N_OUT = 16, 3, 64, 12
SHAPES = [("W1s", (N_FEAT, HIDDEN)), ("W1n", (N_FEAT, HIDDEN)), ("b1", (HIDDEN,)),
          ("W2s", (HIDDEN, HIDDEN)), ("W2n", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("Wo", (HIDDEN, N_OUT)), ("bo", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def adjacency(masks):
    """[B, 16] neighbour bit masks -> [B, 16, 16] float64 adjacency."""
    m = np.asarray(masks, dtype=np.int64)
    bits = (m[:, :, None] >> np.arange(N_NODES)[None, None, :]) & 1
    return torch.tensor(bits, dtype=torch.float64)


def features(A):
    deg = A.sum(-1)
    tri = torch.einsum("buv,bvw,bwu->bu", A, A, A) / 2.0
    ones = torch.ones_like(deg)
    return torch.stack([ones, deg / 4.0, tri / 3.0], dim=-1)


def forward(theta, masks, ramp):
    """Angles [B, 12] for parameters theta (torch float64 [N_PARAMS])."""
    P = unpack(theta)
    A = adjacency(masks)
    X = features(A)
    Z1 = X @ P["W1s"] + (A @ X) @ P["W1n"] / 4.0 + P["b1"]
    H1 = torch.relu(Z1)
    Z2 = H1 @ P["W2s"] + (A @ H1) @ P["W2n"] / 4.0 + P["b2"]
    H2 = torch.relu(Z2)
    g = H2.mean(dim=1)
    return torch.as_tensor(ramp, dtype=torch.float64) + g @ P["Wo"] + P["bo"]


def loss_and_grad(theta_np, masks, ramp, labels):
    """(loss, dloss/dtheta) in float64."""
    theta = torch.tensor(np.asarray(theta_np, dtype=np.float64), requires_grad=True)
    ang = forward(theta, masks, ramp)
    lab = torch.tensor(np.asarray(labels, dtype=np.float64))
    loss = ((ang - lab) ** 2).sum(-1).mean() / N_OUT
    loss.backward()
    return float(loss.item()), theta.grad.numpy().copy()


def predict(theta_np, masks, ramp):
    with torch.no_grad():
        return forward(torch.tensor(np.asarray(theta_np, dtype=np.float64)), masks, ramp).numpy()
