/*
 * tsk_test.h -- host-side inspection entry points of libtsk.so for test
 * suites and kernel-level checks.  They are not part of the library's
 * public interface (tsk.h) and carry no compatibility promise.
 *
 * The plan self-checks never touch a GPU: they plan a call against
 * synthetic, widely separated buffer addresses and verify that every
 * address any planned launch can read or write lies inside the buffer it is
 * allowed to touch (the caller's inputs and outputs or the workspace).
 * Return value: 0 when every access is in bounds, a tsk_status when the
 * problem is rejected by validation, 98 for an out-of-bounds access and 99
 * when the workspace size differs between the size query and the call; a
 * one-line explanation (NUL-terminated, at most msglen bytes) goes to msg.
 */
#ifndef TSK_TEST_H_
#define TSK_TEST_H_

#include <stddef.h>
#include <stdint.h>

#include "tsk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Self-check of tucker_sum_sketch (sketch_only != 0) or
 * tucker_sum_recompress (with R_out when with_r != 0); out_dtype is a
 * tsk_dtype value. */
int tsk_plan_selfcheck(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec, int out_dtype,
                       int sketch_only, int with_r, char* msg, size_t msglen);

/* Self-check of tucker_sum_recompress_batched over `batch` sums. */
int tsk_plan_selfcheck_batched(int32_t batch, const tsk_tucker_sum* sums,
                               const tsk_sketch_spec* specs, int out_dtype, char* msg,
                               size_t msglen);

/* Self-check of tucker_sum_recompress_backward (with a Q_bar argument when
 * with_qbar != 0). */
int tsk_plan_selfcheck_backward(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                                int out_dtype, int with_qbar, char* msg, size_t msglen);

/* Self-check of tucker_sum_project (basis_dtype, out_dtype: tsk_dtype
 * values; project_prec: a tsk_precision value). */
int tsk_plan_selfcheck_project(const tsk_tucker_sum* sum, const int64_t* widths, int basis_dtype,
                               int project_prec, int out_dtype, char* msg, size_t msglen);

/* Self-check of tucker_truncate with the mode ranks the device would
 * report (ranks: host [order], 1 <= ranks[k] <= widths[k]). */
int tsk_plan_selfcheck_truncate(int32_t order, const int64_t* dims, const int64_t* widths,
                                const int32_t* ranks, char* msg, size_t msglen);

/* The same for tucker_truncate_batched over `batch` jobs of one order:
 * dims, widths and ranks hold order entries per job, job after job. */
int tsk_plan_selfcheck_truncate_batched(int32_t batch, int32_t order, const int64_t* dims,
                                        const int64_t* widths, const int32_t* ranks, char* msg,
                                        size_t msglen);

/* Parses a tuning cache (the JSON of tsk_autotune_save) for GPU
 * architecture `arch` and writes the table back as JSON to `out`, or the
 * parse error; TSK_OK or TSK_ERR_INVALID_ARG. */
int tsk_tune_json_check(const char* json, const char* arch, char* out, size_t outlen);

/* Self-check of tucker_sum_subranks. */
int tsk_plan_selfcheck_subranks(const tsk_tucker_sum* sum, char* msg, size_t msglen);

/* Self-check of tucker_sum_subranks_batched. */
int tsk_plan_selfcheck_subranks_batched(int32_t batch, const tsk_tucker_sum* sums, char* msg,
                                        size_t msglen);

/* Self-check of the first launch sequence of tucker_sum_round_deterministic
 * (concatenation, QR, dense core, TTM chain; the truncation that follows is
 * covered by tsk_plan_selfcheck_truncate). */
int tsk_plan_selfcheck_deterministic(const tsk_tucker_sum* sum, char* msg, size_t msglen);

/* The batched self-check, then one line per planned launch in msg: kernel,
 * descriptors, workgroups, largest K-split and segment count; a last line
 * gives the workspace and descriptor-blob sizes in bytes. */
int tsk_plan_describe(int32_t batch, const tsk_tucker_sum* sums, const tsk_sketch_spec* specs,
                      int out_dtype, char* msg, size_t msglen);

/* One GEMM through the library's grouped MFMA kernel, on `stream`:
 * C (M x N, column-major, ld ldc, FP64 if c_f64 else FP32) = op(A) op(B) with
 * op(A)[m][k] = A[m*a_sx + k*a_sk] and op(B)[k][n] = B[n*b_sx + k*b_sk] in
 * arithmetic `prec` (a tsk_precision value), K split `splits` ways.  A and B
 * hold FP64 when prec is TSK_PREC_FP64 and FP32 otherwise.  ws: device
 * workspace, 256-byte aligned, large enough for the split partial tiles and
 * the descriptor upload (TSK_ERR_WORKSPACE_TOO_SMALL otherwise). */
int tsk_debug_gemm(tsk_handle handle, int prec, int M, int N, int K, const void* A, int64_t a_sx,
                   int64_t a_sk, const void* B, int64_t b_sx, int64_t b_sk, void* C, int64_t ldc,
                   int c_f64, int splits, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TSK_TEST_H_ */
