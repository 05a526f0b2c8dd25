"""Status codes of the GPU entry points for invalid calls, through the raw C ABI: dtype
mismatches, NULL handles and outputs, size and qubit-count mismatches, out-of-range
parameters.  Every invalid call is rejected before device work is queued and leaves the
state unchanged."""

import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

EINVAL, EDTYPE, ERANGE = -1, -3, -5


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    Q.lib()
    return Q


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def test_invalid_calls_return_status_codes(Q):
    L = Q.lib()
    n = 6
    rng = np.random.default_rng(3)
    psi0 = W.random_state(n, rng)
    s = Q.qsv_state_create(n, "c128")
    s64 = Q.qsv_state_create(n, "c64")
    s7 = Q.qsv_state_create(n + 1, "c128")
    Q.qsv_state_set(s, psi0)
    circ = Q.Circuit(W.hea_circuit(n, 2))
    circ7 = Q.Circuit(W.hea_circuit(n + 1, 2))
    H = Q.PauliSum(W.zz_chain_hamiltonian(n))
    P = W.n_params_of(W.hea_circuit(n, 2))
    params = np.linspace(0.1, 1.0, P)
    E = C.c_double()
    g = np.zeros(P)

    # dtype mismatches between two states
    assert L.qsv_state_copy(s64.handle, s.handle) == EDTYPE
    assert L.qsv_apply_pauli_sum(s64.handle, s.handle, H.ptr) == EDTYPE
    # qubit-count mismatches
    assert L.qsv_state_copy(s7.handle, s.handle) == EINVAL
    assert L.qsv_apply_circuit(s.handle, circ7.ptr, _dp(params), P) == EINVAL
    assert L.qsv_expectation_and_grad(s.handle, circ7.ptr, H.ptr, _dp(params), P, C.byref(E), _dp(g)) == EINVAL
    H7 = Q.PauliSum([(1.0, ((n, "Z"),))])  # acts on qubit n of an n-qubit state
    assert L.qsv_expectation(s.handle, H7.ptr, None, None) == EINVAL
    # parameter index beyond n_params
    assert L.qsv_apply_circuit(s.handle, circ.ptr, _dp(params), P - 1) == EINVAL
    # NULL handles and outputs
    assert L.qsv_apply_circuit(None, circ.ptr, _dp(params), P) == EINVAL
    assert L.qsv_apply_circuit(s.handle, None, _dp(params), P) == EINVAL
    assert L.qsv_expectation(s.handle, None, None, None) == EINVAL
    assert L.qsv_expectation_and_grad(s.handle, circ.ptr, H.ptr, _dp(params), P, None, _dp(g)) == EINVAL
    assert L.qsv_expectation_and_grad(s.handle, circ.ptr, H.ptr, _dp(params), P, C.byref(E), None) == EINVAL
    assert L.qsv_expectation_and_grad(s.handle, circ.ptr, H.ptr, None, P, C.byref(E), _dp(g)) == EINVAL
    assert L.qsv_expectation_and_grad_batch(s.handle, circ.ptr, H.ptr, _dp(params), 0, P, C.byref(E), _dp(g)) == ERANGE
    assert L.qsv_state_wrap(None, n, 1, C.byref(C.c_void_p())) == EINVAL
    # sizes and dtypes
    buf = np.zeros(1 << n, dtype=np.complex128)
    assert L.qsv_state_get(s.handle, buf.ctypes.data_as(C.c_void_p), (1 << n) - 1) == EINVAL
    assert L.qsv_state_set(s.handle, buf.ctypes.data_as(C.c_void_p), (1 << n) + 1) == EINVAL
    assert L.qsv_state_create(n, 7, C.byref(C.c_void_p())) == EDTYPE
    assert L.qsv_state_create(35, 1, C.byref(C.c_void_p())) == ERANGE
    assert L.qsv_state_set_option(s.handle, Q.OPT_TILE_QUBITS, 14) == EINVAL
    # a message for the failed call, and the state untouched by all of the above
    assert L.qsv_state_set_option(s.handle, 99, 1) == EINVAL
    assert L.qsv_last_error().decode()
    assert np.array_equal(Q.qsv_state_get(s), psi0)
