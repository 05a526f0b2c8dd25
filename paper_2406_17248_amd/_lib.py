"""ctypes binding of libqsv.so (the HIP state-vector engine).

Argument marshalling only: every step of the hot path runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

QSV_OK, QSV_EINVAL, QSV_ENOMEM, QSV_EDTYPE, QSV_EHIP, QSV_ERANGE, QSV_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
QSV_C64, QSV_C128 = 0, 1
OPT_TILE_QUBITS, OPT_ADJ_TILE_QUBITS, OPT_THREADS, OPT_PROFILE, OPT_RELAYOUT = 0, 1, 2, 3, 4
K_TILE_FORWARD, K_TILE_ADJOINT, K_PAULI, K_GATE_STREAM, K_OTHER = 0, 1, 2, 3, 4

GATE_KIND = {
    "X": 0, "Y": 1, "Z": 2, "H": 3, "S": 4, "SDG": 5, "T": 6, "TDG": 7,
    "RX": 8, "RY": 9, "RZ": 10, "PS": 11, "RXX": 12, "RYY": 13, "RZZ": 14, "U3": 15,
    "SWAP": 16, "MAT1": 17, "MAT2": 18,
}

EXPORTED = (
    "qsv_status_string", "qsv_last_error", "qsv_version",
    "qsv_state_create", "qsv_state_wrap", "qsv_state_destroy", "qsv_state_set_stream",
    "qsv_state_release_workspace",
    "qsv_state_synchronize", "qsv_state_info", "qsv_state_reset", "qsv_state_set", "qsv_state_get",
    "qsv_state_copy", "qsv_state_set_option", "qsv_state_get_option",
    "qsv_apply_circuit", "qsv_expectation", "qsv_apply_pauli_sum",
    "qsv_expectation_and_grad", "qsv_expectation_and_grad_batch", "qsv_expectation_batch",
    "qsv_param_shift_grad_batch", "qsv_plan_debug", "qsv_profile_read",
    "qsv_forward_batch", "qsv_backward_batch",
    "qsv_batch_create", "qsv_batch_destroy", "qsv_batch_info", "qsv_batch_set_tile", "qsv_batch_autotune",
    "qsv_batch_expectation_and_grad",
    "qsv_mpnn_create", "qsv_mpnn_destroy", "qsv_mpnn_get_params", "qsv_mpnn_predict", "qsv_mpnn_loss_and_grad",
    "qsv_mpnn_train_step", "qsv_expectation_general", "qsv_expectation_and_grad_multi",
    "qsv_expectation_noalloc",
)
MPNN_PARAMS, MPNN_NODES, MPNN_OUTPUTS = 9484, 16, 12


class qsv_gate(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("targets", C.c_int32 * 2),
        ("param_index", C.c_int32 * 3),
        ("ctrl_mask", C.c_uint64),
        ("param_coeff", C.c_double * 3),
        ("angle_const", C.c_double * 3),
        ("matrix_offset", C.c_int64),
    ]


class qsv_circuit(C.Structure):
    _fields_ = [
        ("n_qubits", C.c_int32),
        ("reserved", C.c_int32),
        ("gates", C.POINTER(qsv_gate)),
        ("n_gates", C.c_size_t),
        ("matrices", C.POINTER(C.c_double)),
        ("n_matrix_doubles", C.c_size_t),
    ]


class qsv_pauli_sum(C.Structure):
    _fields_ = [
        ("n_terms", C.c_size_t),
        ("coeffs", C.POINTER(C.c_double)),
        ("x_masks", C.POINTER(C.c_uint64)),
        ("z_masks", C.POINTER(C.c_uint64)),
    ]


assert C.sizeof(qsv_gate) == 88, "qsv_gate layout must match include/qsv.h"


class QsvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qsv error {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libqsv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2406_17248_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.POINTER(C.c_double)
        sigs = {
            "qsv_status_string": ([C.c_int], C.c_char_p),
            "qsv_last_error": ([], C.c_char_p),
            "qsv_version": ([], C.c_char_p),
            "qsv_state_create": ([i32, i32, C.POINTER(vp)], C.c_int),
            "qsv_state_wrap": ([vp, i32, i32, C.POINTER(vp)], C.c_int),
            "qsv_state_destroy": ([vp], C.c_int),
            "qsv_state_set_stream": ([vp, vp], C.c_int),
            "qsv_state_release_workspace": ([vp], C.c_int),
            "qsv_state_synchronize": ([vp], C.c_int),
            "qsv_state_info": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(vp)], C.c_int),
            "qsv_state_reset": ([vp], C.c_int),
            "qsv_state_set": ([vp, vp, sz], C.c_int),
            "qsv_state_get": ([vp, vp, sz], C.c_int),
            "qsv_state_copy": ([vp, vp], C.c_int),
            "qsv_state_set_option": ([vp, i32, i64], C.c_int),
            "qsv_state_get_option": ([vp, i32, C.POINTER(i64)], C.c_int),
            "qsv_apply_circuit": ([vp, C.POINTER(qsv_circuit), dp, sz], C.c_int),
            "qsv_expectation": ([vp, C.POINTER(qsv_pauli_sum), dp, dp], C.c_int),
            "qsv_expectation_noalloc": ([vp, C.POINTER(qsv_pauli_sum), dp, dp], C.c_int),
            "qsv_apply_pauli_sum": ([vp, vp, C.POINTER(qsv_pauli_sum)], C.c_int),
            "qsv_expectation_and_grad": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, dp, dp],
                                         C.c_int),
            "qsv_expectation_and_grad_batch": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, sz,
                                                dp, dp], C.c_int),
            "qsv_expectation_batch": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, sz, dp],
                                      C.c_int),
            "qsv_param_shift_grad_batch": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, sz,
                                            dp, dp], C.c_int),
            "qsv_profile_read": ([vp, i32, dp, C.POINTER(i64), dp], C.c_int),
            "qsv_batch_create": ([i32, sz, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), C.POINTER(vp)],
                                 C.c_int),
            "qsv_batch_destroy": ([vp], C.c_int),
            "qsv_batch_info": ([vp, C.POINTER(sz), C.POINTER(i64), dp, C.POINTER(i32)], C.c_int),
            "qsv_batch_set_tile": ([vp, i32], C.c_int),
            "qsv_batch_autotune": ([vp, dp, C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "qsv_batch_expectation_and_grad": ([vp, dp, dp, dp], C.c_int),
            "qsv_mpnn_create": ([C.POINTER(C.c_float), C.POINTER(vp)], C.c_int),
            "qsv_mpnn_destroy": ([vp], C.c_int),
            "qsv_mpnn_get_params": ([vp, C.POINTER(C.c_float)], C.c_int),
            "qsv_mpnn_predict": ([vp, C.POINTER(C.c_uint16), sz, dp, dp], C.c_int),
            "qsv_mpnn_loss_and_grad": ([vp, C.POINTER(C.c_uint16), sz, dp, dp, dp, C.POINTER(C.c_float)], C.c_int),
            "qsv_mpnn_train_step": ([vp, C.POINTER(C.c_uint16), sz, dp, dp, C.c_double, dp], C.c_int),
            "qsv_expectation_general": ([vp, C.POINTER(qsv_circuit), dp, sz, vp, C.POINTER(qsv_circuit), dp, sz,
                                         C.POINTER(qsv_pauli_sum), dp, dp, dp], C.c_int),
            "qsv_expectation_and_grad_multi": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), sz, dp, sz,
                                                dp, dp], C.c_int),
            "qsv_forward_batch": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, sz, dp],
                                  C.c_int),
            "qsv_backward_batch": ([vp, C.POINTER(qsv_circuit), C.POINTER(qsv_pauli_sum), dp, sz, sz, dp, dp],
                                   C.c_int),
            "qsv_plan_debug": ([C.POINTER(qsv_circuit), i32, C.POINTER(i32), C.POINTER(i32), i32, C.POINTER(i32),
                                C.POINTER(i32), C.POINTER(C.c_uint64), i32], C.c_int),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status):
    if status != QSV_OK:
        msg = lib().qsv_last_error().decode()
        raise QsvError(status, msg or lib().qsv_status_string(status).decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None and a.size else None


# ------------------------------------------------------------------------------------------
# Marshalling of circuit / Pauli-sum descriptions
# ------------------------------------------------------------------------------------------
class Circuit:
    """A circuit description (dict with n_qubits and gates) as qsv_gate records."""

    def __init__(self, circ):
        self.n_qubits = int(circ["n_qubits"])
        gates = circ["gates"]
        self._gates = (qsv_gate * max(1, len(gates)))()
        mats = []
        n_params = 0
        for i, g in enumerate(gates):
            rec = self._gates[i]
            rec.kind = GATE_KIND[g["kind"]]
            t = list(g["targets"]) + [-1]
            rec.targets[0], rec.targets[1] = int(t[0]), int(t[1])
            cm = 0
            for c in g["ctrls"]:
                cm |= 1 << int(c)
            rec.ctrl_mask = cm
            for a in range(3):
                rec.param_index[a] = -1
                rec.param_coeff[a] = 0.0
                rec.angle_const[a] = 0.0
            for a, (idx, coeff, const) in enumerate(g["params"]):
                rec.param_index[a] = int(idx)
                rec.param_coeff[a] = float(coeff)
                rec.angle_const[a] = float(const)
                n_params = max(n_params, int(idx) + 1)
            rec.matrix_offset = -1
            if g["kind"] in ("MAT1", "MAT2"):
                m = np.ascontiguousarray(g["matrix"], dtype=np.complex128).reshape(-1)
                rec.matrix_offset = sum(len(x) for x in mats)
                mats.append(m)
        self._mats = (np.ascontiguousarray(np.concatenate(mats)).view(np.float64) if mats
                      else np.zeros(0, np.float64))
        self.n_params = n_params
        self.c = qsv_circuit(self.n_qubits, 0, self._gates, len(gates), _dp(self._mats), self._mats.size)

    @property
    def ptr(self):
        return C.byref(self.c)


class PauliSum:
    """Pauli sum [(coeff, ((qubit, 'X'|'Y'|'Z'), ...)), ...] as coefficient / mask arrays."""

    def __init__(self, terms):
        coeffs, xs, zs = [], [], []
        for c, factors in terms:
            xm = zm = 0
            for q, p in factors:
                if p in ("X", "Y"):
                    xm |= 1 << int(q)
                if p in ("Z", "Y"):
                    zm |= 1 << int(q)
            coeffs.append(float(c))
            xs.append(xm)
            zs.append(zm)
        self._c = np.ascontiguousarray(coeffs, dtype=np.float64)
        self._x = np.ascontiguousarray(xs, dtype=np.uint64)
        self._z = np.ascontiguousarray(zs, dtype=np.uint64)
        self.h = qsv_pauli_sum(len(coeffs), _dp(self._c),
                               self._x.ctypes.data_as(C.POINTER(C.c_uint64)) if len(xs) else None,
                               self._z.ctypes.data_as(C.POINTER(C.c_uint64)) if len(zs) else None)

    @property
    def ptr(self):
        return C.byref(self.h)


def _circuit(c):
    return c if isinstance(c, Circuit) else Circuit(c)


def _pauli(h):
    return h if isinstance(h, PauliSum) else PauliSum(h)


def _params(p):
    return np.ascontiguousarray(np.zeros(0) if p is None else p, dtype=np.float64)


# ------------------------------------------------------------------------------------------
# States and the hot-path calls (same names as the C ABI, without the qsv_ prefix object)
# ------------------------------------------------------------------------------------------
class State:
    """A device state vector (qsv_state*)."""

    def __init__(self, handle, n_qubits, dtype, keepalive=None):
        self.handle = C.c_void_p(handle)
        self.n_qubits = n_qubits
        self.dtype = dtype
        self._keepalive = keepalive
        self.stream_ptr = 0        # hipStream_t the state's work is queued on (0: null stream)
        self.device_index = None   # device of wrapped memory, when known

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.qsv_state_destroy(self.handle)
                self.handle = C.c_void_p(None)
        except Exception:
            pass

    @property
    def np_dtype(self):
        return np.complex64 if self.dtype == QSV_C64 else np.complex128


def _dt(dtype):
    if dtype in (QSV_C64, "c64", "complex64", np.complex64):
        return QSV_C64
    if dtype in (QSV_C128, "c128", "complex128", np.complex128):
        return QSV_C128
    raise ValueError(f"unknown dtype {dtype!r}")


def qsv_state_create(n_qubits, dtype="c128"):
    h = C.c_void_p()
    dt = _dt(dtype)
    check(lib().qsv_state_create(int(n_qubits), dt, C.byref(h)))
    return State(h.value, int(n_qubits), dt)


def qsv_state_wrap(device_ptr, n_qubits, dtype, keepalive=None):
    h = C.c_void_p()
    dt = _dt(dtype)
    check(lib().qsv_state_wrap(C.c_void_p(device_ptr), int(n_qubits), dt, C.byref(h)))
    return State(h.value, int(n_qubits), dt, keepalive)


def qsv_state_destroy(s):
    if s.handle:
        check(lib().qsv_state_destroy(s.handle))
        s.handle = C.c_void_p(None)


def qsv_state_set_stream(s, stream_ptr):
    check(lib().qsv_state_set_stream(s.handle, C.c_void_p(stream_ptr)))
    s.stream_ptr = int(stream_ptr or 0)


def qsv_state_release_workspace(s):
    check(lib().qsv_state_release_workspace(s.handle))


def qsv_state_synchronize(s):
    check(lib().qsv_state_synchronize(s.handle))


def qsv_state_reset(s):
    check(lib().qsv_state_reset(s.handle))


def qsv_state_set(s, amps):
    a = np.ascontiguousarray(amps, dtype=s.np_dtype)
    check(lib().qsv_state_set(s.handle, a.ctypes.data_as(C.c_void_p), a.size))


def qsv_state_get(s):
    out = np.empty(1 << s.n_qubits, dtype=s.np_dtype)
    check(lib().qsv_state_get(s.handle, out.ctypes.data_as(C.c_void_p), out.size))
    return out


def qsv_state_copy(dst, src):
    check(lib().qsv_state_copy(dst.handle, src.handle))


def qsv_state_set_option(s, option, value):
    check(lib().qsv_state_set_option(s.handle, int(option), int(value)))


def qsv_state_get_option(s, option):
    v = C.c_int64()
    check(lib().qsv_state_get_option(s.handle, int(option), C.byref(v)))
    return v.value


def qsv_apply_circuit(s, circuit, params=None):
    c = _circuit(circuit)
    p = _params(params)
    check(lib().qsv_apply_circuit(s.handle, c.ptr, _dp(p), p.size))


def qsv_expectation(s, hamiltonian):
    h = _pauli(hamiltonian)
    re, im = C.c_double(), C.c_double()
    check(lib().qsv_expectation(s.handle, h.ptr, C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


def qsv_expectation_noalloc(s, hamiltonian):
    h = _pauli(hamiltonian)
    re, im = C.c_double(), C.c_double()
    check(lib().qsv_expectation_noalloc(s.handle, h.ptr, C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


def qsv_apply_pauli_sum(dst, src, hamiltonian):
    h = _pauli(hamiltonian)
    check(lib().qsv_apply_pauli_sum(dst.handle, src.handle, h.ptr))


def qsv_expectation_and_grad(s, circuit, hamiltonian, params):
    c, h, p = _circuit(circuit), _pauli(hamiltonian), _params(params)
    E = C.c_double()
    g = np.zeros(p.size, dtype=np.float64)
    check(lib().qsv_expectation_and_grad(s.handle, c.ptr, h.ptr, _dp(p), p.size, C.byref(E), _dp(g)))
    return E.value, g


def _batch_params(params):
    p = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    return p, p.shape[0], p.shape[1]


def qsv_expectation_and_grad_batch(s, circuit, hamiltonian, params):
    c, h = _circuit(circuit), _pauli(hamiltonian)
    p, B, P = _batch_params(params)
    E = np.zeros(B)
    g = np.zeros((B, P))
    check(lib().qsv_expectation_and_grad_batch(s.handle, c.ptr, h.ptr, _dp(p), B, P, _dp(E), _dp(g)))
    return E, g


def qsv_expectation_batch(s, circuit, hamiltonian, params):
    c, h = _circuit(circuit), _pauli(hamiltonian)
    p, B, P = _batch_params(params)
    E = np.zeros(B)
    check(lib().qsv_expectation_batch(s.handle, c.ptr, h.ptr, _dp(p), B, P, _dp(E)))
    return E


def qsv_expectation_general(psi, circuit_r, params_r, phi, circuit_l, params_l, hamiltonian, grads=True):
    """E = <phi|U_l^dag H U_r|psi> (complex) and complex gradients for both circuits
    (circuit_l None: U_l = I)."""
    cr, h = _circuit(circuit_r), _pauli(hamiltonian)
    cl = _circuit(circuit_l) if circuit_l is not None else None
    pr, pl = _params(params_r), _params(params_l)
    E = np.zeros(2)
    gr = np.zeros(2 * max(pr.size, 1))
    gl = np.zeros(2 * max(pl.size, 1))
    check(lib().qsv_expectation_general(psi.handle, cr.ptr, _dp(pr), pr.size, phi.handle,
                                        cl.ptr if cl is not None else None, _dp(pl), pl.size, h.ptr, _dp(E),
                                        _dp(gr) if grads else None, _dp(gl) if grads and cl is not None else None))
    g_r = gr[:2 * pr.size].view(np.complex128) if grads else None
    g_l = gl[:2 * pl.size].view(np.complex128) if grads and cl is not None else None
    return complex(E[0], E[1]), g_r, g_l


def qsv_expectation_and_grad_multi(s, circuit, hamiltonians, params):
    c = _circuit(circuit)
    hs = [_pauli(h) for h in hamiltonians]
    arr = (qsv_pauli_sum * len(hs))(*[h.h for h in hs])
    p = _params(params)
    E = np.zeros(len(hs))
    g = np.zeros((len(hs), max(p.size, 1)))
    check(lib().qsv_expectation_and_grad_multi(s.handle, c.ptr, arr, len(hs), _dp(p), p.size, _dp(E), _dp(g)))
    return E, g[:, :p.size]


def qsv_forward_batch(s, circuit, hamiltonian, params):
    c, h = _circuit(circuit), _pauli(hamiltonian)
    p, B, P = _batch_params(params)
    E = np.zeros(B)
    check(lib().qsv_forward_batch(s.handle, c.ptr, h.ptr, _dp(p), B, P, _dp(E)))
    return E


def qsv_backward_batch(s, circuit, hamiltonian, params, dE_weights):
    c, h = _circuit(circuit), _pauli(hamiltonian)
    p, B, P = _batch_params(params)
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(dE_weights, dtype=np.float64), (B,)))
    g = np.zeros((B, P))
    check(lib().qsv_backward_batch(s.handle, c.ptr, h.ptr, _dp(p), B, P, _dp(w), _dp(g)))
    return g


def qsv_param_shift_grad_batch(s, circuit, hamiltonian, params):
    c, h = _circuit(circuit), _pauli(hamiltonian)
    p, B, P = _batch_params(params)
    E = np.zeros(B)
    g = np.zeros((B, P))
    check(lib().qsv_param_shift_grad_batch(s.handle, c.ptr, h.ptr, _dp(p), B, P, _dp(E), _dp(g)))
    return E, g


def qsv_profile_read(s, kernel_class):
    """(total_ms, launches, algorithmic_bytes) of one kernel class since the last read."""
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    check(lib().qsv_profile_read(s.handle, int(kernel_class), C.byref(ms), C.byref(n), C.byref(b)))
    return ms.value, n.value, b.value


def qsv_plan_debug(circuit, tile_qubits):
    """(gate index per executed primitive, pass of each, number of passes, tile masks)."""
    c = _circuit(circuit)
    cap = max(5 * int(c.c.n_gates), 1)
    order = (C.c_int32 * cap)()
    pass_of = (C.c_int32 * cap)()
    n_entries, n_passes = C.c_int32(), C.c_int32()
    masks = (C.c_uint64 * cap)()
    check(lib().qsv_plan_debug(c.ptr, int(tile_qubits), order, pass_of, cap, C.byref(n_entries),
                               C.byref(n_passes), masks, cap))
    k = n_entries.value
    return (np.array(order[:k]), np.array(pass_of[:k]), int(n_passes.value),
            np.array(masks[:n_passes.value], dtype=np.uint64))


# ------------------------------------------------------------------------------------------
# Batches of uneven circuits
# ------------------------------------------------------------------------------------------
class Batch:
    """Many independent circuits with their own Hamiltonians (qsv_batch*)."""

    def __init__(self, circuits, hamiltonians, dtype="c64"):
        self._circs = [_circuit(c) for c in circuits]
        self._hams = [_pauli(h) for h in hamiltonians]
        carr = (qsv_circuit * len(self._circs))(*[c.c for c in self._circs])
        harr = (qsv_pauli_sum * len(self._hams))(*[h.h for h in self._hams])
        h = C.c_void_p()
        check(lib().qsv_batch_create(_dt(dtype), len(self._circs), carr, harr, C.byref(h)))
        self.handle = h
        self.n = len(self._circs)
        total = C.c_size_t()
        offs = (C.c_int64 * (self.n + 1))()
        check(lib().qsv_batch_info(self.handle, C.byref(total), offs, None, None))
        self.total_params = total.value
        self.offsets = np.array(offs[:], dtype=np.int64)

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.qsv_batch_destroy(self.handle)
                self.handle = C.c_void_p(None)
        except Exception:
            pass

    def info(self):
        ms, tile = C.c_double(), C.c_int32()
        check(lib().qsv_batch_info(self.handle, None, None, C.byref(ms), C.byref(tile)))
        return {"last_ms": ms.value, "tile_qubits": tile.value}


def qsv_batch_create(circuits, hamiltonians, dtype="c64"):
    return Batch(circuits, hamiltonians, dtype)


def qsv_batch_set_tile(b, tile_qubits):
    check(lib().qsv_batch_set_tile(b.handle, int(tile_qubits)))


def qsv_batch_autotune(b, params, with_schedule=False):
    """The fastest tile width (and, with_schedule, (width, low qubits kept per tile))."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    t, low = C.c_int32(), C.c_int32()
    check(lib().qsv_batch_autotune(b.handle, _dp(p), C.byref(t), C.byref(low)))
    return (t.value, low.value) if with_schedule else t.value


def qsv_batch_expectation_and_grad(b, params):
    """(E[n_circuits], grad with the layout of params)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.size != b.total_params:
        raise ValueError(f"expected {b.total_params} parameters, got {p.size}")
    E = np.zeros(b.n)
    g = np.zeros(max(p.size, 1))
    check(lib().qsv_batch_expectation_and_grad(b.handle, _dp(p), _dp(E), _dp(g)))
    return E, g[:p.size]


# ------------------------------------------------------------------------------------------
# Warm-start network
# ------------------------------------------------------------------------------------------
def _u16(a):
    a = np.ascontiguousarray(a, dtype=np.uint16)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint16))


class Mpnn:
    """The warm-start network on the device (qsv_mpnn*)."""

    def __init__(self, init_params):
        w = np.ascontiguousarray(init_params, dtype=np.float32)
        if w.size != MPNN_PARAMS:
            raise ValueError(f"expected {MPNN_PARAMS} parameters")
        h = C.c_void_p()
        check(lib().qsv_mpnn_create(w.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self.handle = h

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.qsv_mpnn_destroy(self.handle)
                self.handle = C.c_void_p(None)
        except Exception:
            pass

    def params(self):
        out = np.zeros(MPNN_PARAMS, dtype=np.float32)
        check(lib().qsv_mpnn_get_params(self.handle, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def predict(self, adjacency, ramp):
        a, ap = _u16(adjacency)
        n = a.shape[0]
        r = np.ascontiguousarray(ramp, dtype=np.float64)
        out = np.zeros((n, MPNN_OUTPUTS))
        check(lib().qsv_mpnn_predict(self.handle, ap, n, _dp(r), _dp(out)))
        return out

    def loss_and_grad(self, adjacency, ramp, labels):
        a, ap = _u16(adjacency)
        r = np.ascontiguousarray(ramp, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.float64)
        loss = C.c_double()
        g = np.zeros(MPNN_PARAMS, dtype=np.float32)
        check(lib().qsv_mpnn_loss_and_grad(self.handle, ap, a.shape[0], _dp(r), _dp(lab), C.byref(loss),
                                           g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def train_step(self, adjacency, ramp, labels, lr):
        a, ap = _u16(adjacency)
        r = np.ascontiguousarray(ramp, dtype=np.float64)
        lab = np.ascontiguousarray(labels, dtype=np.float64)
        loss = C.c_double()
        check(lib().qsv_mpnn_train_step(self.handle, ap, a.shape[0], _dp(r), _dp(lab), float(lr), C.byref(loss)))
        return loss.value
