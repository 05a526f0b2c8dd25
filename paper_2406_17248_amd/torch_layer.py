"""PyTorch autograd integration of the adjoint gradient.

The role MindSpore Quantum's MQLayer / MQAnsatzOnlyLayer play (section 4.1 and section 5.2:
a circuit expectation as a trainable network cell): `expectation` is a
``torch.autograd.Function`` whose forward evolves every parameter set on the GPU and returns
the energies, and whose backward runs the library's adjoint reverse sweep (psi and lambda
only) and returns the vector-Jacobian product.  PyTorch supplies the tensors only; both
halves run in the HIP kernels of libqsv.so.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib


class _AdjointExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, state, circuit, hamiltonian):
        p = params.detach().to("cpu", torch.float64).numpy()
        squeeze = p.ndim == 1
        p2 = np.ascontiguousarray(np.atleast_2d(p))
        E = _lib.qsv_forward_batch(state, circuit, hamiltonian, p2)
        ctx.state, ctx.circuit, ctx.hamiltonian = state, circuit, hamiltonian
        ctx.p2, ctx.squeeze = p2, squeeze
        out = torch.as_tensor(E[0] if squeeze else E, dtype=params.dtype)
        return out.to(params.device)

    @staticmethod
    def backward(ctx, grad_E):
        w = grad_E.detach().to("cpu", torch.float64).reshape(-1).numpy()
        g = _lib.qsv_backward_batch(ctx.state, ctx.circuit, ctx.hamiltonian, ctx.p2, w)
        g = g[0] if ctx.squeeze else g
        return torch.as_tensor(g).to(device=grad_E.device, dtype=grad_E.dtype), None, None, None


def expectation(params, state, circuit, hamiltonian):
    """E(params) = <psi0|U(params)^dag H U(params)|psi0> for params of shape [P] or [B, P],
    differentiable with respect to params (adjoint method on the GPU)."""
    return _AdjointExpectation.apply(params, state, circuit, hamiltonian)


class AnsatzExpectation(torch.nn.Module):
    """A trainable ansatz: owns its parameters, a device state (start state |0...0>, or set
    with `set_initial_state`) and the marshalled circuit / Hamiltonian.  forward() returns
    the energy; backward goes through the adjoint sweep."""

    def __init__(self, circuit, hamiltonian, dtype="c128", init=None, device="cuda"):
        super().__init__()
        self.circuit = _lib.Circuit(circuit)
        self.hamiltonian = _lib.PauliSum(hamiltonian)
        self.state = _lib.qsv_state_create(self.circuit.n_qubits, dtype)
        n = max(self.circuit.n_params, 1)
        w = torch.zeros(n, dtype=torch.float64) if init is None else torch.as_tensor(init, dtype=torch.float64)
        self.weight = torch.nn.Parameter(w.to(device))

    def set_initial_state(self, amplitudes):
        _lib.qsv_state_set(self.state, amplitudes)

    def forward(self):
        return expectation(self.weight, self.state, self.circuit, self.hamiltonian)
