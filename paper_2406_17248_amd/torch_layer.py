"""PyTorch autograd integration of the adjoint gradient.

The role MindSpore Quantum's MQLayer / MQAnsatzOnlyLayer play (section 4.1 and section 5.2:
a circuit expectation as a trainable network cell): `expectation` is a
``torch.autograd.Function`` whose forward evolves every parameter set on the GPU and returns
the energies, and whose backward runs the library's adjoint reverse sweep (psi and lambda
only) and returns the vector-Jacobian product.  PyTorch supplies device memory and streams
only: `state_from_tensor` wraps a torch tensor's memory as the library's state, and every
call queues its kernels on torch's current stream of the state's device, so torch work
before and after a call is ordered with it.  Both halves run in the HIP kernels of
libqsv.so.

Parameters and cotangents cross to the host: the library binds angles to gate matrices
on the host (a few doubles per gate), and its energies and gradients come back as host
arrays.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib

_TORCH_DTYPE = {_lib.QSV_C64: torch.complex64, _lib.QSV_C128: torch.complex128}


def state_from_tensor(t):
    """The library state over a torch tensor's memory: a contiguous complex64 / complex128
    CUDA tensor of 2^n elements, interleaved (re, im) like the library's layout.  The state
    keeps the tensor alive; the tensor's contents are the state's amplitudes (no copy)."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dim() == 1):
        raise ValueError("state_from_tensor needs a contiguous 1-d CUDA tensor")
    if t.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("state_from_tensor needs a complex64 or complex128 tensor")
    n = int(t.numel()).bit_length() - 1
    if t.numel() != 1 << n or n < 1:
        raise ValueError("the tensor must hold 2^n amplitudes, n >= 1")
    dt = _lib.QSV_C64 if t.dtype == torch.complex64 else _lib.QSV_C128
    s = _lib.qsv_state_wrap(t.data_ptr(), n, dt, keepalive=t)
    s.device_index = t.device.index if t.device.index is not None else torch.cuda.current_device()
    return s


def use_current_stream(state):
    """Queue the state's further work on torch's current stream of its device.  When that
    stream differs from the one the state used so far, the state's queued work is waited
    for first, so nothing runs out of order across the switch."""
    dev = getattr(state, "device_index", None)
    stream = torch.cuda.current_stream(dev) if dev is not None else torch.cuda.current_stream()
    ptr = stream.cuda_stream
    if getattr(state, "stream_ptr", 0) != ptr:
        _lib.qsv_state_synchronize(state)
        _lib.qsv_state_set_stream(state, ptr)
        state.stream_ptr = ptr
    return state


class _AdjointExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, state, circuit, hamiltonian):
        p = params.detach().to("cpu", torch.float64).numpy()
        squeeze = p.ndim == 1
        p2 = np.ascontiguousarray(np.atleast_2d(p))
        if torch.cuda.is_available():
            use_current_stream(state)
        E = _lib.qsv_forward_batch(state, circuit, hamiltonian, p2)
        ctx.state, ctx.circuit, ctx.hamiltonian = state, circuit, hamiltonian
        ctx.p2, ctx.squeeze = p2, squeeze
        out = torch.as_tensor(E[0] if squeeze else E, dtype=params.dtype)
        return out.to(params.device)

    @staticmethod
    def backward(ctx, grad_E):
        w = grad_E.detach().to("cpu", torch.float64).reshape(-1).numpy()
        if torch.cuda.is_available():
            use_current_stream(ctx.state)
        g = _lib.qsv_backward_batch(ctx.state, ctx.circuit, ctx.hamiltonian, ctx.p2, w)
        g = g[0] if ctx.squeeze else g
        return torch.as_tensor(g).to(device=grad_E.device, dtype=grad_E.dtype), None, None, None


def expectation(params, state, circuit, hamiltonian):
    """E(params) = <psi0|U(params)^dag H U(params)|psi0> for params of shape [P] or [B, P],
    differentiable with respect to params (adjoint method on the GPU).  A batch can mix
    per-sample and shared parameters (section 4.1's encoder data and ansatz weights): pass
    the shared ones expanded over the batch and autograd sums their gradient."""
    return _AdjointExpectation.apply(params, state, circuit, hamiltonian)


class AnsatzExpectation(torch.nn.Module):
    """A trainable ansatz: owns its parameters, a device state held in a torch tensor (start
    state |0...0>, or set with `set_initial_state`) and the marshalled circuit /
    Hamiltonian.  forward() returns the energy; backward goes through the adjoint sweep."""

    def __init__(self, circuit, hamiltonian, dtype="c128", init=None, device="cuda", state_device=None):
        super().__init__()
        self.circuit = _lib.Circuit(circuit)
        self.hamiltonian = _lib.PauliSum(hamiltonian)
        n_q = self.circuit.n_qubits
        # the amplitudes live in a torch tensor (not a registered buffer: moving the module
        # must not move memory the library holds a pointer to)
        sdev = torch.device(state_device if state_device is not None else "cuda")
        self.amplitudes = torch.zeros(1 << n_q, dtype=_TORCH_DTYPE[_lib._dt(dtype)], device=sdev)
        self.amplitudes[0] = 1
        self.state = state_from_tensor(self.amplitudes)
        n = max(self.circuit.n_params, 1)
        w = torch.zeros(n, dtype=torch.float64) if init is None else torch.as_tensor(init, dtype=torch.float64)
        self.weight = torch.nn.Parameter(w.to(device))

    def set_initial_state(self, amplitudes):
        a = torch.as_tensor(amplitudes, dtype=self.amplitudes.dtype)
        with torch.no_grad():
            self.amplitudes.copy_(a.to(self.amplitudes.device))

    def forward(self):
        return expectation(self.weight, self.state, self.circuit, self.hamiltonian)
