"""The adjoint backward behind torch.autograd.Function: gradients against the oracle's
parameter-shift gradient and GPU finite differences, vector-Jacobian products for batched
parameters, call-order robustness, and a training run that reproduces the section 5.2 result."""

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch

    import paper_2406_17248_amd as Q
    from paper_2406_17248_amd import torch_layer
    Q.lib()
    return torch, Q, torch_layer


def test_autograd_gradient_matches_parameter_shift(T):
    torch, Q, TL = T
    circ = W.hea_circuit(8, 3)
    H = W.zz_chain_hamiltonian(8) + [(0.5, ((3, "X"),)), (-0.7, ((1, "Y"), (6, "X")))]
    p0 = W.uniform_params(48, 21)
    s = Q.qsv_state_create(8, "c128")
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    E = TL.expectation(p, s, c, h)
    E.backward()
    ref_E = O.energy(circ, H, p0)
    ref_g = O.grad_param_shift(circ, H, p0)
    scale = sum(abs(x) for x, _ in H)
    assert abs(E.item() - ref_E) <= 1e-12 * scale
    assert np.max(np.abs(p.grad.numpy() - ref_g)) <= 1e-12 * scale


def test_autograd_vjp_for_batched_parameters(T):
    torch, Q, TL = T
    n, p_layers, B = 9, 2, 6
    edges = W.random_regular_graph(3, 10, 4)
    edges = [(u, v) for (u, v) in edges if u < n and v < n]
    circ = W.qaoa_circuit(n, edges, p_layers)
    H = W.maxcut_hamiltonian(edges)
    P = W.uniform_params(2 * p_layers, 5, 0, np.pi, batch=B)
    wts = np.random.default_rng(2).standard_normal(B)
    s = Q.qsv_state_create(n, "c64")
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    p = torch.tensor(P, dtype=torch.float64, requires_grad=True)
    E = TL.expectation(p, s, c, h)
    (E * torch.tensor(wts)).sum().backward()
    scale = sum(abs(x) for x, _ in H)
    for b in range(B):
        E_ref, g_ref = O.grad_adjoint(circ, H, P[b])
        assert abs(E[b].item() - E_ref) <= 1e-5 * scale
        assert np.max(np.abs(p.grad[b].numpy() - wts[b] * g_ref)) <= 1e-5 * scale * max(1, abs(wts[b]))


def test_autograd_matches_gpu_finite_differences(T):
    torch, Q, TL = T
    circ = W.random_circuit(7, 60, 3, kinds=["RX", "RY", "RZ", "RZZ", "U3", "H", "PS"], max_ctrls=1,
                            n_params=5, param_fraction=0.9)
    H = W.random_pauli_sum(7, 10, np.random.default_rng(3))
    s = Q.qsv_state_create(7, "c128")
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    p0 = np.random.default_rng(4).uniform(-2, 2, 5)
    p = torch.tensor(p0, requires_grad=True)
    TL.expectation(p, s, c, h).backward()
    fd = np.zeros(5)
    for i in range(5):
        e = np.zeros(5)
        e[i] = 1e-6
        fd[i] = (Q.qsv_expectation_batch(s, c, h, p0 + e)[0] - Q.qsv_expectation_batch(s, c, h, p0 - e)[0]) / 2e-6
    assert np.max(np.abs(p.grad.numpy() - fd)) < 1e-7


def test_backward_after_an_interleaved_forward(T):
    """Two differentiable evaluations on one state: the first backward finds its kept states
    replaced by the second forward and recomputes them."""
    torch, Q, TL = T
    circ = W.hea_circuit(6, 2)
    H = W.zz_chain_hamiltonian(6)
    s = Q.qsv_state_create(6, "c128")
    c, h = Q.Circuit(circ), Q.PauliSum(H)
    a0, b0 = W.uniform_params(24, 7), W.uniform_params(24, 8)
    a = torch.tensor(a0, requires_grad=True)
    b = torch.tensor(b0, requires_grad=True)
    Ea = TL.expectation(a, s, c, h)
    Eb = TL.expectation(b, s, c, h)
    Ea.backward()
    Eb.backward()
    assert np.max(np.abs(a.grad.numpy() - O.grad_adjoint(circ, H, a0)[1])) < 1e-12 * 5
    assert np.max(np.abs(b.grad.numpy() - O.grad_adjoint(circ, H, b0)[1])) < 1e-12 * 5


def test_training_reproduces_section_5_2_cut(T):
    """Section 5.2: p = 4 QAOA on the 5-node, 6-edge graph trained with Adam (lr 0.05) from
    near-zero angles reaches an expected cut of 4.939257 (here through torch autograd and
    the GPU adjoint sweep)."""
    torch, Q, TL = T
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (0, 2)]
    circ = W.qaoa_circuit(5, edges, 4)
    H = [(-c, f) for c, f in W.maxcut_hamiltonian(edges)]  # minimize -cut
    init = np.random.default_rng(0).normal(0.0, 0.01, 8)
    layer = TL.AnsatzExpectation(circ, H, dtype="c128", init=init, device="cpu")
    opt = torch.optim.Adam(layer.parameters(), lr=0.05)
    for _ in range(400):
        opt.zero_grad()
        loss = layer()
        loss.backward()
        opt.step()
    assert abs(-layer().item() - 4.939257) < 5e-7


def test_torch_memory_and_side_stream_order_with_torch_work(T):
    """torch supplies the state's memory (a wrapped complex128 tensor) and its stream (a
    non-default one): torch work queued before a library call (a delay, then the copy of
    the start state) finishes before the library's kernels read the state, and torch work
    queued after it sees the evolved state, with no host synchronization in between."""
    torch, Q, TL = T
    n = 12
    rng = np.random.default_rng(41)
    circ = W.random_circuit(n, 80, 41, kinds=["RX", "RY", "RZ", "RZZ", "U3", "H", "MAT1"], max_ctrls=1,
                            n_params=5, param_fraction=0.8)
    H = W.random_pauli_sum(n, 10, rng)
    psi0 = W.random_state(n, rng)
    params = rng.uniform(-2, 2, 5)
    src = torch.from_numpy(psi0).to("cuda")
    amps = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    s = TL.state_from_tensor(amps)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)  # keeps the stream busy well past the next host calls
        amps.copy_(src)
        TL.use_current_stream(s)
        assert s.stream_ptr == side.cuda_stream
        Q.qsv_apply_circuit(s, circ, params)  # queued on the side stream, returns at once
        after = amps * 2                       # torch work after the library's passes
    side.synchronize()
    ref = O.simulate(circ, params, psi0)
    assert np.max(np.abs(after.cpu().numpy() / 2 - ref)) <= 1e-12
    # the autograd path on the same wrapped state and stream
    p = torch.tensor(params, requires_grad=True)
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)
        amps.copy_(src)
        E = TL.expectation(p, s, Q.Circuit(circ), Q.PauliSum(H))
        E.backward()
    E_ref, g_ref = O.grad_adjoint(circ, H, params, psi0)
    scale = max(1.0, sum(abs(c) for c, _ in H))
    assert abs(E.item() - E_ref) <= 1e-12 * scale
    assert np.max(np.abs(p.grad.numpy() - g_ref)) <= 1e-12 * scale
    # the state is left unchanged by the gradient evaluation
    side.synchronize()
    assert torch.equal(amps, src)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_encoder_batch_with_shared_ansatz(T, dtype):
    """Section 4.1's quantum neural network form: an encoder whose angles are per-sample data
    and an ansatz whose angles are shared by the batch.  Energies [B], the per-sample encoder
    gradients and the ansatz gradient summed over the batch (weighted by the cotangents)
    against the oracle."""
    torch, Q, TL = T
    n, B, layers = 6, 8, 3
    enc = [W.gate("RY", (q,), params=(W.param_angle(q),)) for q in range(n)]
    ans = W.hea_circuit(n, layers)["gates"]
    ans = [dict(g, params=tuple((i + n if i >= 0 else i, c, k) for (i, c, k) in g["params"])) for g in ans]
    circ = W.circuit(n, enc + ans)
    n_ans = W.n_params_of(circ) - n
    H = W.zz_chain_hamiltonian(n) + [(0.3, ((0, "X"),)), (-0.8, ((2, "Y"), (3, "Y")))]
    rng = np.random.default_rng(17)
    X = rng.uniform(0, np.pi, (B, n))
    theta = rng.uniform(-np.pi, np.pi, n_ans)
    wts = rng.standard_normal(B)
    x = torch.tensor(X, requires_grad=True)
    w = torch.tensor(theta, requires_grad=True)
    P = torch.cat([x, w.unsqueeze(0).expand(B, -1)], dim=1)
    s = Q.qsv_state_create(n, dtype)
    E = TL.expectation(P, s, Q.Circuit(circ), Q.PauliSum(H))
    (E * torch.tensor(wts)).sum().backward()
    tol = (1e-5 if dtype == "c64" else 1e-12) * max(1.0, sum(abs(c) for c, _ in H))
    g_ans = np.zeros(n_ans)
    for b in range(B):
        E_ref, g_ref = O.grad_adjoint(circ, H, np.concatenate([X[b], theta]))
        assert abs(E[b].item() - E_ref) <= tol
        assert np.max(np.abs(x.grad[b].numpy() - wts[b] * g_ref[:n])) <= tol * max(1.0, abs(wts[b]))
        g_ans += wts[b] * g_ref[n:]
    assert np.max(np.abs(w.grad.numpy() - g_ans)) <= tol * max(1.0, np.sum(np.abs(wts)))
