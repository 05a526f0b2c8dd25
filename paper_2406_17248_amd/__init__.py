"""MI355X (gfx950) state-vector engine for parameterized circuits (arXiv 2406.17248 hot path).

The compute runs in hand-written HIP kernels inside ``libqsv.so``; this package is a thin
ctypes binding with the C ABI's names (see ``include/qsv.h``).  Importing it does not
touch the GPU; the first call that needs the library loads it and raises if it has not
been built (``paper_2406_17248_amd.build.build()``).
"""

from ._lib import (  # noqa: F401
    Batch, GATE_KIND, Mpnn, qsv_batch_autotune, qsv_batch_create, qsv_batch_expectation_and_grad,
    qsv_batch_set_tile, K_GATE_STREAM, K_OTHER, K_PAULI, K_TILE_ADJOINT, K_TILE_FORWARD, OPT_ADJ_TILE_QUBITS,
    OPT_PROFILE, OPT_RELAYOUT, OPT_THREADS, OPT_TILE_QUBITS, QSV_C64, QSV_C128, Circuit,
    PauliSum, QsvError, State, lib, qsv_apply_circuit, qsv_apply_pauli_sum, qsv_expectation,
    qsv_backward_batch, qsv_expectation_and_grad, qsv_expectation_and_grad_batch, qsv_expectation_batch,
    qsv_forward_batch, qsv_expectation_general, qsv_expectation_and_grad_multi, qsv_expectation_noalloc,
    qsv_param_shift_grad_batch, qsv_plan_debug, qsv_profile_read, qsv_state_copy, qsv_state_create, qsv_state_destroy,
    qsv_state_get, qsv_state_get_option, qsv_state_reset, qsv_state_set, qsv_state_set_option,
    qsv_state_set_stream, qsv_state_synchronize, qsv_state_wrap, qsv_state_release_workspace,
)
