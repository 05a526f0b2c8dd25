/*
 * qsv.h - C ABI of the MI355X (gfx950) state-vector engine for parameterized circuits.
 *
 * The engine holds a 2^n complex amplitude vector in device memory (HBM), applies
 * 1- and 2-qubit gates and fused gate blocks to it, reduces Pauli-sum expectations,
 * and computes adjoint-method gradients of those expectations with respect to the
 * circuit parameters (MindSpore Quantum, arXiv 2406.17248: section 2.3 for the gates,
 * section 2.5 for Pauli-sum observables, section 2.6 for the simulator's apply / get
 * semantics, section 4.1 for the gradient API, section 7 (QAOA task) for the adjoint
 * method).
 *
 * Conventions
 *  - Little-endian basis order: bit q of an amplitude's index is qubit q (section 2.6).
 *  - Amplitudes are interleaved (re, im): float2 for QSV_C64, double2 for QSV_C128.
 *  - Every number crossing the ABI (angles, matrices, coefficients, expectations,
 *    gradients) is fp64.  For QSV_C64 the library forms gate matrices in fp64 and rounds
 *    them to fp32 once per call; all reductions accumulate in fp64 in a fixed order, so
 *    results are bitwise repeatable for the same inputs and options.
 *  - Return value: QSV_OK (0) on success, a negative QSV_E* code otherwise.  On error
 *    qsv_last_error() returns a message for the calling thread.  No C++ exception
 *    crosses the ABI.  Arguments are validated before any device work is queued; an
 *    invalid call leaves the state unchanged.
 *  - Ownership: every host array passed in is owned by the caller and may be freed when
 *    the call returns (the library copies what it needs).  A state from
 *    qsv_state_create owns its device buffer; a wrapped state does not.
 *  - Threading: a qsv_state is not thread-safe; calls on one state must not overlap.
 *    Work is queued on the state's stream (default: the null stream); calls that
 *    return host values (expectations, gradients, qsv_state_get) synchronize it.
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define QSV_OK       0
#define QSV_EINVAL  -1  /* bad argument: qubit out of range, duplicate targets, control on a
                           target, parameter index >= n_params, size mismatch, null pointer */
#define QSV_ENOMEM  -2  /* device or host allocation failed */
#define QSV_EDTYPE  -3  /* unknown dtype, or dtype mismatch between two states */
#define QSV_EHIP    -4  /* a HIP runtime call failed (message in qsv_last_error) */
#define QSV_ERANGE  -5  /* size beyond the supported maximum (n_qubits > 34, too many params) */
#define QSV_ENOTSUP -6  /* valid request the engine does not implement (e.g. the two-term
                           parameter shift of a controlled rotation) */

/* ---- amplitude types --------------------------------------------------------------- */
typedef enum { QSV_C64 = 0, QSV_C128 = 1 } qsv_dtype;

/* ---- gate kinds (section 2.3) ---------------------------------------------------------
 * Fixed: X, Y, Z, H as printed in section 2.3; S = diag(1, i), SDG = S^dag,
 * T = diag(1, e^{i pi/4}), TDG = T^dag, SWAP.
 * Rotations (one angle): RX, RY, RZ = exp(-i theta P / 2) (section 2.3);
 * RXX, RYY, RZZ = exp(-i theta P(x)P / 2) on targets[0], targets[1];
 * PS (phase shift) = diag(1, e^{i theta}).
 * U3 (three angles theta, phi, lambda) = RZ(phi) RX(-pi/2) RZ(theta) RX(pi/2) RZ(lambda)
 *   = RZ(phi) RY(theta) RZ(lambda) as section 4.1 defines it, global phase included:
 *   [[e^{-i(p+l)/2} cos t/2, -e^{-i(p-l)/2} sin t/2], [e^{i(p-l)/2} sin t/2, e^{i(p+l)/2} cos t/2]].
 * MAT1 / MAT2: explicit 2x2 / 4x4 complex matrix (section 2.3, custom gates).
 * Any kind may carry controls (ctrl_mask); CNOT is X with one control, CZ is Z with one
 * control.  For 2-qubit kinds, bit b of a matrix row/column index refers to targets[b]. */
enum qsv_gate_kind {
  QSV_GATE_X = 0, QSV_GATE_Y = 1, QSV_GATE_Z = 2, QSV_GATE_H = 3,
  QSV_GATE_S = 4, QSV_GATE_SDG = 5, QSV_GATE_T = 6, QSV_GATE_TDG = 7,
  QSV_GATE_RX = 8, QSV_GATE_RY = 9, QSV_GATE_RZ = 10, QSV_GATE_PS = 11,
  QSV_GATE_RXX = 12, QSV_GATE_RYY = 13, QSV_GATE_RZZ = 14, QSV_GATE_U3 = 15,
  QSV_GATE_SWAP = 16, QSV_GATE_MAT1 = 17, QSV_GATE_MAT2 = 18,
  QSV_GATE_KIND_COUNT = 19
};

/* One gate record.  Angle a of the gate is bound as
 *     angle_a = angle_const[a] + param_coeff[a] * params[param_index[a]]
 * (param_index[a] = -1: the constant alone), the linear parameter expressions of
 * section 2.2.  Unused angle slots must have param_index = -1.  For 1-qubit kinds
 * targets[1] is ignored.  matrix_offset indexes, in complex elements, the circuit's
 * matrix array (MAT1: 4 row-major entries, MAT2: 16); ignored for other kinds.
 * Layout (88 bytes): int32 kind; int32 targets[2]; int32 param_index[3];
 * uint64 ctrl_mask; double param_coeff[3]; double angle_const[3]; int64 matrix_offset. */
typedef struct qsv_gate {
  int32_t  kind;
  int32_t  targets[2];
  int32_t  param_index[3];
  uint64_t ctrl_mask;
  double   param_coeff[3];
  double   angle_const[3];
  int64_t  matrix_offset;
} qsv_gate;

/* A circuit: gates applied in array order (section 2.4).  matrices: interleaved
 * (re, im) fp64, n_matrix_doubles entries (may be NULL when no MAT gate is used). */
typedef struct qsv_circuit {
  int32_t          n_qubits;
  int32_t          reserved;
  const qsv_gate*  gates;
  size_t           n_gates;
  const double*    matrices;
  size_t           n_matrix_doubles;
} qsv_circuit;

/* A Pauli sum H = sum_k coeffs[k] P_k (section 2.5).  P_k is the tensor product with X
 * on qubits set only in x_masks[k], Z on qubits set only in z_masks[k], Y on qubits set
 * in both, identity elsewhere; so P_k|x> = i^{popcount(x_k & z_k)} (-1)^{popcount(x & z_k)}
 * |x xor x_k>.  Coefficients are real, so H is Hermitian. */
typedef struct qsv_pauli_sum {
  size_t          n_terms;
  const double*   coeffs;
  const uint64_t* x_masks;
  const uint64_t* z_masks;
} qsv_pauli_sum;

typedef struct qsv_state qsv_state;

/* ---- errors -------------------------------------------------------------------------- */
const char* qsv_status_string(int status);
/* Message of the last failed call on this thread ("" if none). */
const char* qsv_last_error(void);
/* Library version string. */
const char* qsv_version(void);

/* ---- states (section 2.6: Simulator('mqvector', n), get_qs / set_qs / reset) --------- */
/* Allocate a 2^n_qubits state on the current HIP device, set to |0...0>.
 * 1 <= n_qubits <= 34.  *out receives the handle (QSV_ENOMEM if HBM is short). */
int qsv_state_create(int32_t n_qubits, int32_t dtype, qsv_state** out);
/* Wrap caller-owned device memory holding 2^n_qubits amplitudes of the given dtype
 * (e.g. a torch tensor).  Contents are used as they are; the caller keeps the memory
 * alive until qsv_state_destroy. */
int qsv_state_wrap(void* device_ptr, int32_t n_qubits, int32_t dtype, qsv_state** out);
/* Free the state, its workspaces and (if owned) its amplitude buffer.  NULL is a no-op. */
int qsv_state_destroy(qsv_state* s);
/* Queue all further work of this state on the given hipStream_t (NULL: null stream).
 * Work already queued on the previous stream is not waited for: order it first (e.g.
 * qsv_state_synchronize) when switching streams. */
int qsv_state_set_stream(qsv_state* s, void* hip_stream);
/* Free the state's device workspaces (batch states, costates, partial sums, the relayout
 * buffer; not the amplitudes).  They are allocated again, grow-only, by later calls that need
 * them.  Waits for the state's stream first. */
int qsv_state_release_workspace(qsv_state* s);
/* Wait for all queued work of this state. */
int qsv_state_synchronize(qsv_state* s);
/* Basic queries. */
int qsv_state_info(const qsv_state* s, int32_t* n_qubits, int32_t* dtype, void** device_ptr);
/* Set the state to |0...0> (section 2.6, reset). */
int qsv_state_reset(qsv_state* s);
/* Copy n_amps = 2^n host amplitudes of the state's dtype into the state (set_qs). */
int qsv_state_set(qsv_state* s, const void* host_amps, size_t n_amps);
/* Copy the state to n_amps = 2^n host amplitudes of its dtype (get_qs). */
int qsv_state_get(qsv_state* s, void* host_amps, size_t n_amps);
/* Copy the amplitudes of src into dst (same n and dtype) with one plain copy kernel on
   dst's stream (reads and writes 2^n amplitudes once each); work on src's stream, if it
   differs, must be ordered before the call by the caller. */
int qsv_state_copy(qsv_state* dst, const qsv_state* src);

/* Execution options (integers).  Defaults are chosen per dtype and n. */
enum qsv_option {
  QSV_OPT_TILE_QUBITS = 0,   /* qubits per fused LDS tile pass (0: per-gate kernels only);
                                default 12 (c64) / 11 (c128); clamped to n */
  QSV_OPT_ADJ_TILE_QUBITS = 1, /* tile width of the adjoint reverse sweep (psi and lambda
                                  share LDS); default 10 (c64) / 11 (c128);
                                  complex128 is capped at 12 */
  QSV_OPT_THREADS = 2,       /* reserved (threads per tile workgroup follow the tile width) */
  QSV_OPT_PROFILE = 3,       /* 1: time every kernel launch with HIP events on the state's
                                stream (read with qsv_profile_read); 0: off (default) */
  QSV_OPT_RELAYOUT = 4,      /* 1 (default): qsv_apply_circuit runs fused passes out of place
                                between the state and a scratch buffer of the same size as the
                                state (2^n amplitudes: 16 GiB for 30 qubits in complex128),
                                storing each pass in a bit layout whose low bits are the next
                                pass's tile so that every pass after the first reads contiguous
                                blocks; the state is back in the natural layout when the call
                                returns.  The buffer is allocated with hipMalloc on the first
                                multi-pass call (also for wrapped states: outside the caller's
                                allocator) and kept until qsv_state_release_workspace or
                                qsv_state_destroy.  It is allocated only while at least 1/8 of
                                its size plus 256 MiB of device memory would stay free; otherwise,
                                or if the allocation fails, the passes run in place (same
                                results).  0: always in place, no buffer */
  QSV_OPT_COUNT = 5
};
int qsv_state_set_option(qsv_state* s, int32_t option, int64_t value);
int qsv_state_get_option(const qsv_state* s, int32_t option, int64_t* value);

/* ---- hot path ------------------------------------------------------------------------ */
/* psi <- U(params) psi (section 2.6, apply_circuit).  n_params must cover every
 * param_index used.  The circuit's n_qubits must equal the state's. */
int qsv_apply_circuit(qsv_state* s, const qsv_circuit* c, const double* params, size_t n_params);

/* <psi|H|psi> (section 2.6, get_expectation with U_l = U_r = I); the state is unchanged.
 * *out_im is the rounding-level imaginary part (H is Hermitian); either pointer may be NULL. */
int qsv_expectation(qsv_state* s, const qsv_pauli_sum* h, double* out_re, double* out_im);

/* qsv_expectation for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same result from the same kernels,
 * bit for bit, but every device buffer beyond the state (term tables, per-workgroup partial
 * sums, reduced columns) is one fixed 4 MiB array compiled into the library, one copy per
 * GPU, kept until the process ends.  The call allocates no device or pinned host memory
 * (qsv_expectation grows the state's workspaces and a pinned staging buffer) and records
 * no profiling events.  Limits: at most 8192 terms and 48 distinct x masks (groups of terms
 * sharing their X/Y qubits); larger sums return QSV_ERANGE before any device work.  Every
 * call on one GPU uses that GPU's single array: calls that overlap on one GPU (other host
 * threads, or states on different streams with work in flight) race and may return wrong
 * values.  The call synchronizes the state's stream before it returns, so calls made one
 * after another from one thread are safe. */
int qsv_expectation_noalloc(qsv_state* s, const qsv_pauli_sum* h, double* out_re, double* out_im);

/* dst <- H src, unnormalized (section 2.6, apply_hamiltonian); dst != src, same n/dtype. */
int qsv_apply_pauli_sum(qsv_state* dst, const qsv_state* src, const qsv_pauli_sum* h);

/* E(params) = <psi0|U^dag H U|psi0> and dE/dparams by the adjoint method (section 4.1,
 * get_expectation_with_grad; section 7, adjoint method), starting from the state's
 * current contents psi0, which are left unchanged.  out_grad has n_params entries;
 * parameters not used by the circuit get 0.  Every parameterized gate kind is
 * supported, with or without controls. */
int qsv_expectation_and_grad(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                             const double* params, size_t n_params,
                             double* out_E, double* out_grad);

/* The same for a batch of parameter sets sharing the start state and circuit structure
 * (section 4.1: outputs [n_batch] and [n_batch][n_params] with one Hamiltonian).
 * params is row-major [batch][n_params]; out_E[batch]; out_grad[batch][n_params]. */
int qsv_expectation_and_grad_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                                   const double* params, size_t batch, size_t n_params,
                                   double* out_E, double* out_grad);

/* Differentiable evaluation in two halves (the forward and backward of an autograd
 * function).  qsv_forward_batch computes out_E[b] like qsv_expectation_batch and keeps the
 * evolved states in the state's workspace.  qsv_backward_batch then runs lambda = H psi and
 * the adjoint reverse sweep over those states, holding only psi and lambda per batch item,
 * and returns out_grad[b][p] = dE_weights[b] * dE_b / dparams[b][p] (a vector-Jacobian
 * product).  If the kept states do not match the call (different circuit, Hamiltonian,
 * parameters or batch, another call used the workspace in between, or an entry point of
 * this library wrote the start state since: qsv_state_set / reset / copy, qsv_apply_circuit,
 * qsv_apply_pauli_sum) the forward sweep is recomputed first, so the result does not depend
 * on call order.  Writes to a wrapped state's memory made outside this library are not
 * seen: after such a write, call qsv_forward_batch again before qsv_backward_batch. */
int qsv_forward_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                      const double* params, size_t batch, size_t n_params, double* out_E);
int qsv_backward_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                       const double* params, size_t batch, size_t n_params,
                       const double* dE_weights, double* out_grad);

/* Energies only, for a batch of parameter sets: out_E[batch] (no gradient). */
int qsv_expectation_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                          const double* params, size_t batch, size_t n_params, double* out_E);

/* General form E = <phi| U_l^dag H U_r |psi> (section 2.6, get_expectation with a left
 * circuit and state; section 4.1, get_expectation_with_grad with circ_left), complex, with
 * its complex derivatives: grad_r[2k], grad_r[2k+1] = Re, Im of dE/dparams_r[k] and grad_l
 * likewise for params_l (E is conjugate-linear in U_l phi).  c_l NULL means U_l = I.  phi may
 * be psi; both states are left unchanged.  out_E receives (Re E, Im E).  grad_r / grad_l may
 * be NULL.  Uses four state-sized workspaces of two amplitudes vectors each. */
int qsv_expectation_general(qsv_state* psi, const qsv_circuit* c_r, const double* params_r, size_t n_r,
                            const qsv_state* phi, const qsv_circuit* c_l, const double* params_l, size_t n_l,
                            const qsv_pauli_sum* h, double* out_E, double* grad_r, double* grad_l);

/* Several Hamiltonians of one circuit at once (section 4.1: outputs [n_ham] and
 * [n_ham][n_params]): one forward sweep, then lambda_k = H_k psi and the adjoint sweep for
 * all Hamiltonians as batch items.  The state is unchanged. */
int qsv_expectation_and_grad_multi(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* hams, size_t n_hams,
                                   const double* params, size_t n_params, double* out_E, double* out_grad);

/* Gradient by the two-term parameter-shift rule, evaluated on the GPU with the same
 * kernels (2 energies per parameterized angle occurrence).  Comparator for the adjoint
 * method.  QSV_ENOTSUP if a parameterized gate has controls. */
int qsv_param_shift_grad_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                               const double* params, size_t batch, size_t n_params,
                               double* out_E, double* out_grad);

/* ---- batches of uneven circuits --------------------------------------------------------
 * Many independent circuits, each with its own Pauli-sum Hamiltonian and parameters
 * (section 4.1's batch mode, with circuits of different sizes and depths), evaluated
 * together from |0...0>: pass round r of every circuit runs in one launch, lambda = H psi of
 * every circuit in one gather-form launch, and the whole evaluation is captured once into
 * a HIP graph that each call replays.  Circuits have 1..28 qubits.  The library copies the
 * circuits and Hamiltonians at creation.  Circuit i's parameters are params[off[i] ..
 * off[i+1]) with off from qsv_batch_info (n_params of a circuit = largest param_index + 1). */
typedef struct qsv_batch qsv_batch;
int qsv_batch_create(int32_t dtype, size_t n_circuits, const qsv_circuit* circuits,
                     const qsv_pauli_sum* hams, qsv_batch** out);
int qsv_batch_destroy(qsv_batch* b);
/* total parameter count, offsets (n_circuits + 1 entries, or NULL), device time of the last
 * graph replay in ms, current tile width; any pointer may be NULL. */
int qsv_batch_info(const qsv_batch* b, size_t* total_params, int64_t* param_offsets, double* last_ms,
                   int32_t* tile_qubits);
/* Fix the tile (fusion) width of every fused pass, in [9, 13]; rebuilds plans and graph. */
int qsv_batch_set_tile(qsv_batch* b, int32_t tile_qubits);
/* Autotuner: time the whole evaluation with these parameters on the device for each tile
 * width (10..13) and tile schedule (2, 3 or 4 low qubits kept by every tile for dense global
 * accesses: fewer mean fewer passes), keep the fastest and return its width in *out_tile and
 * its low-qubit count in *out_low_qubits (either may be NULL).  Rebuilds plans and graph. */
int qsv_batch_autotune(qsv_batch* b, const double* params, int32_t* out_tile, int32_t* out_low_qubits);
/* out_E[i] = <H_i> of circuit i; out_grad (may be NULL) has the layout of params. */
int qsv_batch_expectation_and_grad(qsv_batch* b, const double* params, double* out_E, double* out_grad);

/* ---- learned warm start for QAOA MaxCut -------------------------------------------------
 * A 2-layer message-passing network (hidden 64, fp32) mapping a 16-node graph to p = 6
 * QAOA angles (6 gamma then 6 beta in the layer convention of section 6.2), as a correction
 * to a given ramp schedule: angles = ramp + readout(graph).  Node features are
 * [1, degree / 4, triangles / 3]; layer l: Z = H Ws + (A H) Wn / 4 + b, H' = relu(Z);
 * readout: mean over nodes, then a linear map to 12 outputs.  Parameters (float32, row
 * major, in this order): W1s[3][64], W1n[3][64], b1[64], W2s[64][64], W2n[64][64], b2[64],
 * Wo[64][12], bo[12].  Graphs are given as 16 neighbour bit masks each (uint16, no self
 * loops).  Training minimizes the mean over graphs of |angles - labels|^2 / 12 with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8), all on the device. */
#define QSV_MPNN_NODES 16
#define QSV_MPNN_FEATURES 3
#define QSV_MPNN_HIDDEN 64
#define QSV_MPNN_OUTPUTS 12
#define QSV_MPNN_PARAMS 9484
typedef struct qsv_mpnn qsv_mpnn;
int qsv_mpnn_create(const float* init_params, qsv_mpnn** out);
int qsv_mpnn_destroy(qsv_mpnn* m);
int qsv_mpnn_get_params(const qsv_mpnn* m, float* out_params);
/* out_angles[n_graphs][12] */
int qsv_mpnn_predict(qsv_mpnn* m, const uint16_t* adjacency, size_t n_graphs, const double* ramp,
                     double* out_angles);
/* loss and its gradient with respect to the parameters (no update) */
int qsv_mpnn_loss_and_grad(qsv_mpnn* m, const uint16_t* adjacency, size_t n_graphs, const double* ramp,
                           const double* labels, double* out_loss, float* out_grad);
/* one Adam step on this minibatch; *out_loss (may be NULL) is the loss before the step */
int qsv_mpnn_train_step(qsv_mpnn* m, const uint16_t* adjacency, size_t n_graphs, const double* ramp,
                        const double* labels, double lr, double* out_loss);

/* ---- profiling ----------------------------------------------------------------------- */
/* Kernel classes timed when QSV_OPT_PROFILE is 1. */
enum qsv_kernel_class {
  QSV_K_TILE_FORWARD = 0,   /* fused forward tile passes */
  QSV_K_TILE_ADJOINT = 1,   /* fused adjoint reverse-sweep passes (psi and lambda) */
  QSV_K_PAULI = 2,          /* Pauli-sum passes (expectation, lambda = H psi) */
  QSV_K_GATE_STREAM = 3,    /* unfused per-gate passes */
  QSV_K_OTHER = 4,          /* state init, broadcast, reductions */
  QSV_K_COUNT = 5
};
/* Synchronize the state's stream and return, for one kernel class, the summed device
 * time (ms) of the launches recorded since the last read, their number, and the
 * algorithmic HBM bytes they move (each amplitude a launch must read or write, once).
 * Reading clears the class's record.  Any output pointer may be NULL. */
int qsv_profile_read(qsv_state* s, int32_t kernel_class, double* total_ms, int64_t* launches,
                     double* algorithmic_bytes);

/* ---- host-only diagnostics (no device work; usable without a GPU) ------------------- */
/* Plan the fused execution of a circuit with tile width tile_qubits.  The circuit is
 * first lowered into primitives (one per gate, except RXX and RYY, which become two
 * basis changes on each side of a diagonal RZZ: five primitives).  On return, for
 * i < *n_entries, order[i] is the gate index of the i-th primitive executed and
 * pass_of[i] its tile pass; *n_passes is the number of passes.  order and pass_of hold
 * max_entries entries (5 * n_gates always suffices; QSV_ERANGE if too small).  tile_masks,
 * when not NULL, receives up to max_passes 64-bit masks of each pass's tile qubits. */
int qsv_plan_debug(const qsv_circuit* c, int32_t tile_qubits, int32_t* order, int32_t* pass_of,
                   int32_t max_entries, int32_t* n_entries, int32_t* n_passes, uint64_t* tile_masks,
                   int32_t max_passes);

#ifdef __cplusplus
}
#endif

#endif /* QSV_H */
