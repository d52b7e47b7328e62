/*
 * tsk.h -- C ABI of the MI355X (gfx950) library for recompressing a sum of
 * Tucker tensors by structured Gaussian sketching.
 *
 * Problem (Section 3, "Sketching-Based Summation of Tucker Tensors"): given
 *     X = sum_{i=1}^{s} c_i [[G^(i); U_1^(i), ..., U_d^(i)]]
 * with cores G^(i) of size r_1^(i) x ... x r_d^(i) and factors U_k^(i) of
 * size n_k x r_k^(i), a sketch kind and sketch sizes, compute, without ever
 * forming X:
 *   Y_n = X_(n) S_n    for every mode n                    (Stage 2 sketch)
 *   Q_n                thin QR basis of Y_n, diag(R_n) >= 0  (Stage 2 QR)
 *   H   = sum_i c_i G^(i) x_1 Q_1^T U_1^(i) ... x_d Q_d^T U_d^(i)  (Stage 3)
 * so that X ~ [[H; Q_1, ..., Q_d]].  S_n is the Khatri-Rao product
 * Omega_d (.) ... (.) Omega_1 (skipping n, Section 3.1.1) or the Kronecker
 * product Omega_d (x) ... (x) Omega_1 (skipping n, Section 3.1.2) of one
 * Gaussian test matrix Omega_k per mode, reused by every S_n with n != k.
 *
 * Layout.  Every matrix and tensor is column-major: mode 1 fastest, the
 * mode-n unfolding orders the remaining modes first-mode-fastest (Section
 * 2.1, unfolding index equation).  U_k^(i) has leading dimension n_k.
 * Omega_k is n_k x m (KRP) or n_k x q_k (Kron).  Y_n is n_n x W_n with
 * W_n = m (KRP) or prod_{k != n} q_k (Kron).  Q_n is n_n x w_n with
 * w_n = min(n_n, W_n) (economy QR).  H is w_1 x ... x w_d.
 *
 * Ownership.  The caller allocates and owns every input, output and
 * workspace buffer; the library never frees them and keeps no pointer past
 * the call.  A handle owns only its device, a small device counter block,
 * pinned staging memory for launch descriptors, and its last error text.
 *
 * Asynchrony.  Calls validate on the host, enqueue on `stream` (a
 * hipStream_t passed as void*, NULL = default stream) and return without
 * synchronising.  Outputs are valid once the stream reaches that point.
 *
 * Errors.  Every function returns a tsk_status.  On any host-side error
 * nothing is enqueued and no output is written; tsk_last_error_detail()
 * describes it.  Device-side faults surface as TSK_ERR_DEVICE from a later
 * call that checks the runtime.  The library never aborts and never prints.
 *
 * Threads.  One handle per host thread; distinct handles are independent.
 */
#ifndef TSK_H_
#define TSK_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSK_OK = 0,
  TSK_ERR_INVALID_ARG = 1,         /* NULL pointer, size < 1, bad enum, ...      */
  TSK_ERR_UNSUPPORTED = 2,         /* valid but outside what the kernels handle  */
  TSK_ERR_OUT_OF_MEMORY = 3,       /* pinned staging or handle memory            */
  TSK_ERR_WORKSPACE_TOO_SMALL = 4, /* ws_bytes < tucker_sum_workspace_size()     */
  TSK_ERR_DEVICE = 5,              /* HIP runtime error                          */
  TSK_ERR_RANK_DEFICIENT = 6       /* Cholesky QR broke down under qr_policy 2   */
} tsk_status;

typedef enum { TSK_F64 = 0, TSK_F32 = 1 } tsk_dtype;

typedef enum { TSK_SKETCH_KRP = 0, TSK_SKETCH_KRON = 1 } tsk_sketch_kind;

/* Arithmetic of a stage.  FP64 and FP32 run on the matching MFMA units.
 * BF16X1/X3/X6 split each FP32 operand into 1, 2 or 3 bfloat16 parts and
 * keep 1, 3 or 6 of the cross products on BF16 MFMA with FP32 accumulation.
 * The QR of Y_n is always FP64. */
typedef enum {
  TSK_PREC_FP64 = 0,
  TSK_PREC_FP32 = 1,
  TSK_PREC_BF16X1 = 2,
  TSK_PREC_BF16X3 = 3,
  TSK_PREC_BF16X6 = 4
} tsk_precision;

typedef struct tsk_handle_* tsk_handle;

/* X = sum_i coeffs[i] * [[G_i; U_1^(i) .. U_d^(i)]]  (Section 2.2 Tucker
 * format; the coefficients are those of the RoundSum({X_i},{c_i}) call of
 * Algorithm 6 and the alpha, beta of Algorithm 1). */
typedef struct {
  int32_t order;               /* d >= 2                                            */
  int32_t num_terms;           /* s >= 1                                            */
  const int64_t* dims;         /* host [d], n_k >= 1                                */
  const int32_t* ranks;        /* host [s*d], ranks[i*d + k] = r_k^(i) >= 1          */
  const void* const* cores;    /* host [s] device pointers, core i column-major     */
  const void* const* factors;  /* host [s*d] device pointers, factors[i*d + k] is
                                  n_k x r_k^(i) column-major, ld = n_k              */
  const double* coeffs;        /* host [s], or NULL for all ones                    */
  tsk_dtype dtype;             /* element type of cores and factors                 */
} tsk_tucker_sum;

typedef struct {
  tsk_sketch_kind kind;
  const int32_t* sizes;        /* host; KRP: sizes[0] = m; Kron: sizes[k] = q_k, [d] */
  uint64_t seed;               /* Omega_k generated on the device from (seed, k)    */
  const void* const* omega;    /* optional host [d] device pointers to caller-made
                                  Omega_k (sum dtype, n_k x width_k column-major);
                                  NULL = generate from seed                        */
  tsk_precision sketch_prec;   /* factor sketch, core sketch, term expansion        */
  tsk_precision project_prec;  /* Q^T U and the multi-TTM of the core projection    */
  int32_t qr_policy;           /* 0: Cholesky QR2, Householder on breakdown (device
                                  side), and directly for a mode whose total rank
                                  sum_i r_n^(i) is below its sketch width (Y_n is
                                  then rank deficient); 1: Householder always;
                                  2: Cholesky QR2, breakdown reported as
                                  TSK_ERR_RANK_DEFICIENT                            */
} tsk_sketch_spec;

/* Handle on HIP device `device`.  Allocates the handle's counter block and
 * nothing else on the device, and creates a second stream of default
 * priority: a call forks independent launches onto it from the caller's
 * stream and joins them back before it returns (the caller's stream waits
 * for them, so stream order is kept and a captured graph holds both
 * branches).
 *
 * Graph capture: a call made while `stream` is being captured (relaxed
 * mode) allocates a device copy of its launch descriptors, which the handle
 * holds until tsk_destroy, and records a device-to-device copy of them into
 * the workspace; every replay therefore rewrites what it needs, and other
 * calls may use the same workspace between replays.  The capture itself
 * waits on the handle's second stream while filling that copy. */
tsk_status tsk_create(tsk_handle* handle, int device);
tsk_status tsk_destroy(tsk_handle handle);
const char* tsk_status_string(tsk_status status);
/* Text of the last error on this handle ("" if none).  Owned by the handle. */
const char* tsk_last_error_detail(tsk_handle handle);

/* Sketch sizes of Section 3.2.  KRP width m = max_k ell_k.  Kron sizes
 * q_k = ceil((prod_j ell_j)^(1/(d-1)) / ell_k) (heuristic sketch-dimension
 * equation), computed exactly in integers as the least q with
 * (q ell_k)^(d-1) >= prod_j ell_j.  ell: host [d]; out: host [1] or [d]. */
tsk_status tsk_krp_width(int32_t order, const int32_t* ell, int32_t* m_out);
tsk_status tsk_kron_sizes(int32_t order, const int32_t* ell, int32_t* q_out);

/* Per-mode widths: sketch_width[n] = W_n (columns of Y_n), basis_width[n] =
 * w_n = min(n_n, W_n) (columns of Q_n and mode-n size of H).  Host arrays [d]. */
tsk_status tsk_sketch_widths(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                             int64_t* sketch_width, int64_t* basis_width);

/* Omega_k for 0-based `mode` (Section 3.1: a standard Gaussian n_k x width
 * matrix per mode).  Entry e = i + n_k t uses Philox4x32-10 (Salmon et al.,
 * SC'11) block e/2 with counter (lo32(e/2), hi32(e/2), mode, 0) and key
 * (lo32(seed), hi32(seed)); a Box-Muller pair in FP64 from the two 53-bit
 * uniforms u1 = (w0 >> 11) + 1, u2 = w1 >> 11 (scaled by 2^-53; w0 = words
 * 1:0, w1 = words 3:2); even entries take rho cos, odd take rho sin; the value
 * is rounded to 8 significant bits (nearest even), so it is exact in BF16,
 * FP32 and FP64.  `out` is a device buffer of rows*cols elements of out_dtype. */
tsk_status tsk_sketch_omega(tsk_handle handle, uint64_t seed, int32_t mode, int64_t rows,
                            int64_t cols, void* out, tsk_dtype out_dtype, void* stream);

/* Bytes of device workspace that tucker_sum_sketch / tucker_sum_recompress
 * need for this problem (the same figure covers both). */
tsk_status tucker_sum_workspace_size(tsk_handle handle, const tsk_tucker_sum* sum,
                                     const tsk_sketch_spec* spec, size_t* bytes);

/* Stage 2 sketch only (eqs. for the KRP and Kronecker sketched unfoldings of
 * a sum): Y_out[n] is a device n_n x W_n FP64 buffer.  `ws` is device
 * workspace of at least tucker_sum_workspace_size() bytes, 256-byte aligned. */
tsk_status tucker_sum_sketch(tsk_handle handle, const tsk_tucker_sum* sum,
                             const tsk_sketch_spec* spec, double* const* Y_out, void* ws,
                             size_t ws_bytes, void* stream);

/* Stages 2 and 3 (Algorithms 4/5 without Stage 1 and Stage 4): Q_out[n] is a
 * device n_n x w_n buffer, H_out a device w_1 x ... x w_d buffer, both of
 * out_dtype.  Optional R_out (NULL or host [d] of device pointers, FP64
 * w_n x W_n upper triangular) receives the R factors. */
tsk_status tucker_sum_recompress(tsk_handle handle, const tsk_tucker_sum* sum,
                                 const tsk_sketch_spec* spec, void* const* Q_out, void* H_out,
                                 tsk_dtype out_dtype, double* const* R_out, void* ws,
                                 size_t ws_bytes, void* stream);

/* Stage 3 alone (Section 3.3, projection of each summand by linearity):
 *   H = sum_i c_i G^(i) x_1 B_1^T U_1^(i) ... x_d B_d^T U_d^(i)
 * for caller-given bases B_k (bases[k]: device n_k x widths[k], column-major,
 * ld n_k, element type basis_dtype; orthonormal columns are what makes
 * [[H; B]] the projection of the sum, but any matrices are accepted), in the
 * arithmetic project_prec.  H_out is a device widths[0] x ... x widths[d-1]
 * buffer of out_dtype.  The core projection of tucker_sum_recompress is this
 * computation on its Q_n; with the Stage 4 factors it gives the truncated
 * core.  Workspace as for tucker_sum_recompress. */
tsk_status tucker_sum_project_workspace_size(tsk_handle handle, const tsk_tucker_sum* sum,
                                             const int64_t* widths, tsk_dtype basis_dtype,
                                             tsk_precision project_prec, size_t* bytes);
tsk_status tucker_sum_project(tsk_handle handle, const tsk_tucker_sum* sum,
                              const void* const* bases, const int64_t* widths,
                              tsk_dtype basis_dtype, tsk_precision project_prec, void* H_out,
                              tsk_dtype out_dtype, void* ws, size_t ws_bytes, void* stream);

/* Stage 1 of Algorithms 4/5: phase 1 of Algorithm 3 (effective subranks
 * from the weighted Gram matrix, Section 3.2).  For every mode n:
 * V_n = [w_1 U_n^(1), ..., w_s U_n^(s)] with w_i = |c_i| ||G^(i)||_F, the
 * eigenvalues lambda_1 >= lambda_2 >= ... of V_n^T V_n clipped at zero, the
 * rank r_n = the smallest r >= 1 with sum_{j > r} lambda_j <= (eps^2 / d)
 * sum_j lambda_j, and ell_out[n] = r_n + p[n] (p: host [d] oversampling,
 * >= 0).  Sketch sizes then follow from tsk_krp_width / tsk_kron_sizes
 * (phase 2).  FP64 throughout; requires sum_i r_n^(i) <= 4096 per mode.
 * Synchronises `stream` to return the sizes on the host. */
tsk_status tucker_sum_subranks_workspace_size(tsk_handle handle, const tsk_tucker_sum* sum,
                                              size_t* bytes);
tsk_status tucker_sum_subranks(tsk_handle handle, const tsk_tucker_sum* sum, double eps,
                               const int32_t* p, int32_t* ell_out, void* ws, size_t ws_bytes,
                               void* stream);

/* Stage 1 for many independent sums at once (the per-node sums of a
 * time step, Section 5.3): each launch of tucker_sum_subranks runs once for
 * every sum of the batch.  sums: host [batch]; p and ell_out: host arrays of
 * sum_j order_j entries, sum j's modes after those of sums 0..j-1.
 * Synchronises `stream` once. */
tsk_status tucker_sum_subranks_batched_workspace_size(tsk_handle handle, int32_t batch,
                                                      const tsk_tucker_sum* sums, size_t* bytes);
tsk_status tucker_sum_subranks_batched(tsk_handle handle, int32_t batch,
                                       const tsk_tucker_sum* sums, double eps, const int32_t* p,
                                       int32_t* ell_out, void* ws, size_t ws_bytes, void* stream);

/* Stage 4 of Algorithms 4/5: ST-HOSVD of the projected core with relative
 * tolerance eps and the rank rule of Algorithm 2, phase 2.  With
 * theta = eps^2 ||H||_F^2 / d, for n = 1..d in order: the eigenvalues
 * lambda_1 >= lambda_2 >= ... of G_(n) G_(n)^T (G the current core, first
 * H), the rank r_n = the smallest r >= 1 with sum_{i > r} lambda_i <= theta,
 * V_n = the r_n leading eigenvectors, G <- G x_n V_n^T; then the factors
 * U_n = Q_n V_n.  Everything in FP64.
 *   dims, widths: host [order]; widths[k] = w_k <= min(dims[k], 1024) (above
 *     96 the eigensolver keeps its matrices in the workspace, not in LDS).
 *   Q[k]: device n_k x w_k (ld n_k); H: device w_1 x ... x w_d (the outputs
 *     of tucker_sum_recompress with out_dtype TSK_F64).
 *   U_out[k]: device n_k x w_k buffers, of which the first r_k columns
 *     (ld n_k) are written; G_out: device buffer of prod_k w_k doubles that
 *     receives the r_1 x ... x r_d core; ranks_out: host [order].
 * The ranks decide the shapes of later launches, so the call synchronises
 * `stream` once per mode and returns after the work is enqueued (the last
 * launches may still be running).  The result [[G; U_1..U_d]] is within
 * eps ||H|| of [[H; Q]] when the Q_k have orthonormal columns. */
tsk_status tucker_truncate_workspace_size(tsk_handle handle, int32_t order, const int64_t* dims,
                                          const int64_t* widths, double eps, size_t* bytes);
tsk_status tucker_truncate(tsk_handle handle, int32_t order, const int64_t* dims,
                           const int64_t* widths, const double* const* Q, const double* H,
                           double eps, double* const* U_out, double* G_out, int32_t* ranks_out,
                           void* ws, size_t ws_bytes, void* stream);

/* One Stage 4 truncation of a batch (tucker_truncate_batched): the
 * arguments of tucker_truncate for one core.  The workspace query reads only
 * order, dims, widths and eps. */
typedef struct {
  int32_t order;               /* d >= 2                                             */
  const int64_t* dims;         /* host [d]                                           */
  const int64_t* widths;       /* host [d], w_k <= min(n_k, 1024)                    */
  const double* const* Q;      /* host array of d device ptrs, n_k x w_k              */
  const double* H;             /* device w_1 x ... x w_d                             */
  double eps;                  /* relative tolerance in [0, 1]                       */
  double* const* U_out;        /* host array of d device ptrs, n_k x w_k capacity     */
  double* G_out;               /* device, prod_k w_k doubles                         */
  int32_t* ranks_out;          /* host [d]                                           */
} tsk_truncation;

/* Stage 4 for many independent cores at once: tucker_truncate on every job,
 * mode by mode, with each kind of launch (TTM, Gram, eigensolver, the final
 * U_n = Q_n V_n) grouped over the jobs, and one synchronisation of `stream`
 * per mode that reads every job's rank of that mode.  Jobs may differ in
 * order and sizes; their outputs must not overlap each other or any input. */
tsk_status tucker_truncate_batched_workspace_size(tsk_handle handle, int32_t batch,
                                                  const tsk_truncation* jobs, size_t* bytes);
tsk_status tucker_truncate_batched(tsk_handle handle, int32_t batch, const tsk_truncation* jobs,
                                   void* ws, size_t ws_bytes, void* stream);

/* The paper's deterministic baseline for the same sum: Algorithm 1
 * (TuckerAxby) over all terms, i.e. the concatenated factors
 * W_n = [U_n^(1), ..., U_n^(s)] (n_n x R_n, R_n = sum_i r_n^(i)) and the
 * dense R_1 x ... x R_d core holding c_i G^(i) in disjoint blocks along the
 * super-diagonal, followed by Algorithm 2 (TuckerRounding): the thin QR
 * W_n = Q_n R_n with R_n absorbed into the core, then ST-HOSVD of that core
 * with relative tolerance tau (theta = tau^2 ||core||^2 / d, the rank rule
 * of tucker_truncate).  FP64 throughout.  Outputs as for tucker_truncate,
 * with widths w_n = min(n_n, R_n): U_out[k] device n_k x w_k capacity (the
 * first r_k columns written), G_out device prod_k w_k capacity, ranks_out
 * host [d].  The dense core has prod_n R_n entries (the memory growth the
 * sketched sum avoids); requires w_n <= 1024.  Synchronises `stream` once
 * per mode. */
tsk_status tucker_sum_round_deterministic_workspace_size(tsk_handle handle,
                                                        const tsk_tucker_sum* sum, double tau,
                                                        size_t* bytes);
tsk_status tucker_sum_round_deterministic(tsk_handle handle, const tsk_tucker_sum* sum,
                                          double tau, double* const* U_out, double* G_out,
                                          int32_t* ranks_out, void* ws, size_t ws_bytes,
                                          void* stream);

/* tucker_sum_recompress for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and the same kernels, with no workspace
 * argument.  Intermediates live in a static device array of
 * TSK_NOALLOC_SCRATCH_BYTES that every device the library runs on holds
 * until the process ends; launch descriptors are uploaded from pinned host
 * memory that tsk_create set aside (at most TSK_NOALLOC_DESCRIPTOR_BYTES).
 * The call performs no device or pinned-host allocation and no free.
 * Returns TSK_ERR_WORKSPACE_TOO_SMALL (nothing enqueued) when the problem
 * needs more scratch than the array holds (tucker_sum_workspace_size gives
 * the need), TSK_ERR_UNSUPPORTED when its descriptors exceed the staging.
 * All calls on one device share the array, which keeps the last call's
 * contents: calls whose executions overlap on one device (different streams,
 * threads or handles) race and must be serialised by the caller.  Before
 * reusing the staging the call waits for the previous no-allocation call's
 * descriptor upload on the same handle.  Under graph capture the recorded
 * upload reads the handle's staging again on every replay, so a replay
 * uploads the descriptors of the last no-allocation call made on that
 * handle: while such a graph is in use, its handle must make no other
 * no-allocation call (give each captured no-allocation call a handle of its
 * own; handles are cheap, and the scratch array is shared by all of them). */
#define TSK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define TSK_NOALLOC_DESCRIPTOR_BYTES ((size_t)1 << 20)
tsk_status tucker_sum_recompress_noalloc(tsk_handle handle, const tsk_tucker_sum* sum,
                                         const tsk_sketch_spec* spec, void* const* Q_out,
                                         void* H_out, tsk_dtype out_dtype, double* const* R_out,
                                         void* stream);

/* Per-launch timing.  While enabled, every kernel a call enqueues is
 * bracketed by two HIP events on the call's stream (not inside stream
 * capture).  tsk_profile_report() waits for the recorded events, writes a
 * JSON object {"<kernel symbol> <step>": {"launches": n, "ms": total,
 * "flops": algorithmic flops, "bytes": algorithmic bytes}, ...} into `buf`
 * (NUL-terminated; *needed receives the size including the NUL; buf may be
 * NULL to query the size) and clears the records. */
tsk_status tsk_profile_enable(tsk_handle handle, int32_t on);
tsk_status tsk_profile_report(tsk_handle handle, char* buf, size_t buf_len, size_t* needed);

/* Batched form: `batch` independent sums (sums[b], specs[b]) recompressed by
 * one launch sequence, every stage of every sum in the same grouped kernel
 * launches (the many independent sums of Section 5.3's time step, or the
 * repeated RoundSum calls of Algorithm 6).  All sums share order, sketch kind
 * and precisions; mode sizes, term counts, ranks, widths and seeds may
 * differ.  Q_out[b][n] and H_out[b] as in tucker_sum_recompress. */
tsk_status tucker_sum_batched_workspace_size(tsk_handle handle, int32_t batch,
                                             const tsk_tucker_sum* sums,
                                             const tsk_sketch_spec* specs, size_t* bytes);
tsk_status tucker_sum_recompress_batched(tsk_handle handle, int32_t batch,
                                         const tsk_tucker_sum* sums, const tsk_sketch_spec* specs,
                                         void* const* const* Q_out, void* const* H_out,
                                         tsk_dtype out_dtype, void* ws, size_t ws_bytes,
                                         void* stream);

/* Reverse mode of tucker_sum_recompress for the Khatri-Rao sketch (the paper
 * gives no gradients; the rules are derived from the Stage 2-3 definitions of
 * Algorithm 5): given the forward outputs Q[n] (n_n x w_n) and R[n] (FP64,
 * w_n x w_n, from R_out), and the gradients H_bar (w_1 x ... x w_d) and
 * Q_bar[n] (NULL = zero) of a scalar loss, write the gradients with respect
 * to every core (core_bar[i], core-shaped) and factor (factor_bar[i*d+k],
 * n_k x r_k^(i)), in the sum's dtype.  Q, H_bar and Q_bar are of out_dtype.
 * The thin-QR adjoint
 *   Y_bar = (Q_bar + Q copyltu(-Q_bar^T Q)) R^-T
 * runs in FP64 and needs full column rank (w_n = W_n <= n_n, R invertible);
 * the contractions run in spec->sketch_prec.  Intermediates (P, V, W) are
 * recomputed from the inputs and Omega (regenerated from the seed).
 * Returns TSK_ERR_UNSUPPORTED for the Kronecker sketch, oversketched modes or
 * widths above 96.  The solve checks each R_n on the device: a mode with
 * some |R_jj| <= 64 w_n u max_i |R_ii| (u = 2^-53; e.g. the Householder result
 * of a rank-deficient Y_n) is counted, and the next tsk_qr_fallback_count
 * returns TSK_ERR_RANK_DEFICIENT; that call's gradients are then not
 * meaningful. */
tsk_status tucker_sum_backward_workspace_size(tsk_handle handle, const tsk_tucker_sum* sum,
                                              const tsk_sketch_spec* spec, size_t* bytes);
tsk_status tucker_sum_recompress_backward(tsk_handle handle, const tsk_tucker_sum* sum,
                                          const tsk_sketch_spec* spec, const void* const* Q,
                                          const double* const* R, const void* H_bar,
                                          const void* const* Q_bar, tsk_dtype out_dtype,
                                          void* const* core_bar, void* const* factor_bar,
                                          void* ws, size_t ws_bytes, void* stream);

/* Autotuning of the planner's launch parameters for the batched and
 * single-sum calls (the autotuned tiles of the batching form): the K-split
 * target of every grouped GEMM class (factor sketch, term expansion,
 * projection W and final TTM) and of the Khatri-Rao core sketch, and how many
 * waves may share one 32 x 32 output quadrant in the core sketch.  A class
 * is (kernel, precision, log2 of the launch's output tiles before
 * splitting, log2 of its K-tiles).  tsk_autotune plans and runs the batch
 * (the arguments of tucker_sum_recompress_batched, which it overwrites)
 * under every candidate value, times each launch with HIP events over
 * `reps` runs after a warm-up, and keeps per class the value whose launches
 * were fastest; it allocates and frees its own workspace and synchronises
 * `stream`.  The table lives in the handle and shapes every plan made
 * after it changes (workspace sizes included: query them again).  Results
 * of tuned plans differ from untuned ones only in the order of
 * floating-point summation.
 * tsk_autotune_save writes the table as JSON ({"arch": ..., "entries":
 * [{"kernel", "param", "prec", "tiles_log2", "ktiles_log2", "value",
 * "us"}, ...]}); tsk_autotune_load replaces the table with a file's, and
 * rejects a file written for another GPU architecture. */
tsk_status tsk_autotune(tsk_handle handle, int32_t batch, const tsk_tucker_sum* sums,
                        const tsk_sketch_spec* specs, void* const* const* Q_out,
                        void* const* H_out, tsk_dtype out_dtype, int32_t reps, void* stream);
tsk_status tsk_autotune_save(tsk_handle handle, const char* path);
tsk_status tsk_autotune_load(tsk_handle handle, const char* path);
tsk_status tsk_autotune_clear(tsk_handle handle);

/* Number of mode QRs that took the Householder path since the handle was
 * created (Cholesky breakdown, a total rank below the sketch width under
 * qr_policy 0, or qr_policy 1).  Synchronises `stream`.
 * Returns TSK_ERR_RANK_DEFICIENT (count still written) if, since the last
 * call, a Cholesky QR broke down under qr_policy 2 (the outputs of that call
 * are still the Householder result) or a backward call met a numerically
 * singular R_n.  Each condition is reported once. */
tsk_status tsk_qr_fallback_count(tsk_handle handle, void* stream, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* TSK_H_ */
