// Host-side launchers of the HIP kernels (defined in qsv_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "qsv_ops.h"

namespace qsv {

hipError_t launch_tile_pass(int dtype, bool adj, int maxm, const PassArgs& A, uint64_t n_tiles,
                            int batch, hipStream_t s);
// Register-blocked tile pass (reg_bits = 3, or 4 for complex64 forward passes; 2^(maxm -
// reg_bits) threads, a 2^maxm-amplitude LDS exchange buffer, plus dynamic LDS for the ctab
// window and deferred gradient sums); maxm in [9, 13] and equal to A.m.
hipError_t launch_tile_pass_rb(int dtype, bool adj, int reg_bits, int maxm, const PassArgs& A, uint64_t n_tiles,
                               int batch, hipStream_t s);
// Multi-circuit variants (batched uneven circuits).
constexpr int kPauliChunk = 4096;  // amplitudes per workgroup of the multi-circuit Pauli pass
// max_win / max_pslots: the largest win_n / pass_pslots of the items (they size the
// dynamic LDS of every workgroup).
hipError_t launch_tile_pass_rb_multi(int dtype, bool adj, int maxm, const PassArgs* items, const uint32_t* prefix,
                                     int n_items, uint32_t n_wg, int max_win, int max_pslots, hipStream_t s);
hipError_t launch_pauli_apply_multi(int dtype, const PauliJob* jobs, const uint32_t* prefix, int n_jobs, uint32_t n_wg,
                                    hipStream_t s);
hipError_t launch_reduce_segments(const double* in, const int64_t* offs, const int32_t* lens, const int32_t* strides,
                                  double* out, int ncols, hipStream_t s);
hipError_t launch_set_zero_multi(int dtype, void* const* ptrs, const int32_t* nq, const uint32_t* prefix, int n_jobs,
                                 uint32_t n_wg, hipStream_t s);
// dst = (ar + i ai) src for one 2^n state; inner product partials (re: [0, blocks),
// im: [blocks, 2 blocks)) of conj(a) b.
hipError_t launch_scale_copy(int dtype, void* dst, const void* src, int n, double ar, double ai, hipStream_t s);
unsigned inner_blocks(int n);
hipError_t launch_inner_product(int dtype, const void* a, const void* b, int n, double* partials, hipStream_t s);
hipError_t launch_gate1(int dtype, void* psi, int64_t bstride, int batch, int n, int t, uint64_t cmask,
                        const void* ctab, int64_t ctab_bstride, int mat, hipStream_t s);
hipError_t launch_gate2(int dtype, void* psi, int64_t bstride, int batch, int n, int ta, int tb,
                        uint64_t cmask, const void* ctab, int64_t ctab_bstride, int mat, hipStream_t s);
hipError_t launch_diag(int dtype, void* psi, int64_t bstride, int batch, int n, const DiagEntry* diag,
                       int first, int count, const void* ctab, int64_t ctab_bstride, hipStream_t s);
unsigned pauli_blocks(int n);
hipError_t launch_pauli_group(int dtype, const PauliGroupArgs& A, int batch, hipStream_t s);
hipError_t launch_reduce_columns(const double* in, int64_t len, int64_t ncols, double* out, hipStream_t s);
hipError_t launch_set_basis(int dtype, void* psi, int64_t bstride, int batch, int n, uint64_t index,
                            hipStream_t s);
hipError_t launch_broadcast_state(int dtype, void* dst, int64_t bstride, int batch, const void* src, int n,
                                  hipStream_t s);

}  // namespace qsv
