"""The allocation-free expectation entry point (fixed per-device scratch) against
qsv_expectation, through the C ABI: two calls in a row, the second on a smaller state and a
smaller Pauli sum, both precisions; and its size limit."""

import numpy as np
import pytest

import workloads as W
from oracle import statevector as O

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def Q():
    import paper_2406_17248_amd as Q
    Q.lib()
    return Q


def _scale(terms):
    return max(1.0, sum(abs(c) for c, _ in terms))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_expectation_matches_expectation(Q, dtype):
    cdt = np.complex64 if dtype == "c64" else np.complex128
    # each call is smaller than the one before in both the state and the sum, so stale
    # scratch contents of an earlier call would show; the first sum has more groups of terms
    # than share the scratch's partial sums at once
    for k, (n, n_terms, seed) in enumerate(((20, 300, 31), (16, 60, 32), (12, 9, 33))):
        print(f"noalloc call {k}: n={n} terms={n_terms} dtype={dtype}", flush=True)
        rng = np.random.default_rng(seed)
        psi0 = W.random_state(n, rng)
        H = W.random_pauli_sum(n, n_terms, rng)
        s = Q.qsv_state_create(n, dtype)
        Q.qsv_state_set(s, psi0.astype(cdt))
        e_ref = Q.qsv_expectation(s, H)
        e_na = Q.qsv_expectation_noalloc(s, H)
        tol = TOL[dtype] * _scale(H)
        assert abs(e_na - e_ref) <= tol, (k, e_na, e_ref)
        e_or = O.expectation(psi0.astype(cdt).astype(np.complex128), n, H)
        assert abs(e_na.real - e_or.real) <= tol, (k, e_na, e_or)
        # the state is unchanged
        assert np.array_equal(Q.qsv_state_get(s), psi0.astype(cdt))
        del s


def test_noalloc_expectation_rejects_sums_beyond_its_scratch(Q):
    n = 14
    s = Q.qsv_state_create(n, "c128")
    rng = np.random.default_rng(7)
    # one term more than the fixed scratch's tables hold
    H = W.random_pauli_sum(n, 8193, rng)
    with pytest.raises(Q.QsvError) as ei:
        Q.qsv_expectation_noalloc(s, H)
    assert ei.value.status == -5
    # the limit itself is accepted, and the regular entry point agrees
    H = H[:8192]
    e_na = Q.qsv_expectation_noalloc(s, H)
    e_ref = Q.qsv_expectation(s, H)
    assert abs(e_na - e_ref) <= 1e-12 * _scale(H)
