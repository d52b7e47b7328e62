// Internal declarations shared by the device kernels and the host planner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsk {

// Arithmetic of a contraction stage (mirrors tsk_precision in tsk.h).
enum Prec : int32_t { P_FP64 = 0, P_FP32 = 1, P_BF16X1 = 2, P_BF16X3 = 3, P_BF16X6 = 4 };

constexpr int kMaxOrder = 8;

// Step of the method a GEMM launch serves (names the kernel symbol only).
enum Role : int32_t {
  R_FACTOR_SKETCH = 0,  // P_k^(i) = U_k^(i)T Omega_k
  R_KRON_TTM = 1,       // Kronecker core sketch TTM chain
  R_TERM_EXPAND = 2,    // Y_n = sum_i c_i U_n^(i) V^(i)_(n)
  R_QR_GRAM = 3,        // Y^T Y (Cholesky QR)
  R_QR_BASIS = 4,       // Y R^-1 (Cholesky QR)
  R_PROJ_W = 5,         // W_k^(i) = Q_k^T U_k^(i)
  R_PROJ_TTM = 6,       // leading TTMs of the core projection
  R_PROJ_FINAL = 7,     // last TTM, K-concatenated over terms, writes H
  R_OTHER = 8
};

// ---------------------------------------------------------------------------
// Grouped, batched, K-segmented GEMM descriptors (device-resident).
//
// For one descriptor and batch instance b:
//   C_b = beta * C_b + sum_seg alpha_seg * op(A_seg,b) op(B_seg,b)
// where C_b is M x N column-major (ldc) at C + b*strideC, op(A) is M x K and
// op(B) is K x N of the segment.  Operands are read through two strides:
//   op(A)[m][k] = A[m*a_sx + k*a_sk],  op(B)[k][n] = B[n*b_sx + k*b_sk],
// one of which is 1.  A K-split s of `splits` covers K-tiles s, s+splits, ...
// of the concatenated segment K range and writes its 64 x 64 partial tile to
// `part`; the last split to arrive at a tile (arrival counter) adds the
// partials in split order, applies beta and writes C, then re-arms the
// counter, so the result does not depend on arrival order.
struct GemmSeg {
  const void* A;
  const void* B;
  int64_t a_sx, a_sk, strideA;
  int64_t b_sx, b_sk, strideB;
  int32_t K;
  int32_t pad_;
  double alpha;
};

static_assert(sizeof(GemmSeg) % 8 == 0, "segments are copied as 8-byte words");

struct GemmDesc {
  void* C;
  void* part;          // splits > 1: per-tile partial blocks (64 x 64, accumulator type)
  int64_t ldc, strideC;
  int32_t bpw;         // batch elements per workgroup (one-tile elements, splits == 1)
  int32_t pad_;
  int32_t M, N, batch, splits;
  int32_t seg_begin, seg_count;
  int32_t tiles_m, tiles_n;
  int32_t beta;   // 1: accumulate into C (only when splits == 1)
  int32_t c_f64;  // 1: C is double, 0: C is float
  int64_t tile_begin;  // first linear tile id of this descriptor
};

// ---------------------------------------------------------------------------
// KRP core sketch descriptor: V[a][t] = sum_c G_(n)[a][c] * prod_{k != n}
// P_k[j_k(c)][t] for one term i and mode n (Algorithm 5, core sketch line).
struct KrpDesc {
  const void* G;                 // core, column-major
  const void* P[kMaxOrder];      // P_k = U_k^T Omega_k, r_k x m column-major (P[n] unused)
  void* V;                       // r_n x m, column-major, ld r_n
  void* part;                    // splits > 1: per-tile partial blocks
  int32_t r[kMaxOrder];
  int32_t order, mode, m, splits;
  int32_t kw_max;                // most waves that may share one 32x32 quadrant (1, 2 or 4)
  int32_t pad_kw;
  int64_t Kc;                    // prod_{k != n} r_k
  int32_t tiles_m, tiles_n;
  int64_t tile_begin;
  double alpha;
};

// ---------------------------------------------------------------------------
// Adjoint of the KRP core sketch with respect to the core, for one term and
// mode n: G_bar_(n) += Vbar (r_n x m) * KR_n^T, written through the mode-n
// unfolding into a core-shaped (column-major) output.
struct KrpAdjDesc {
  const void* Vbar;              // r_n x m, ld r_n
  const void* P[kMaxOrder];      // r_k x m (P[n] unused)
  void* Gout;                    // core-shaped output
  int32_t r[kMaxOrder];
  int32_t order, mode, m, pad_;
  int64_t Nc;                    // prod_{k != n} r_k
  int32_t tiles_m, tiles_n;
  int64_t tile_begin;
  double alpha;
};

// Y_bar = Z R^-T for one mode (rows of Z are independent back substitutions).
struct TrsmJob {
  const double* Z;      // n x w, ld n
  const double* R;      // w x w upper triangular, ld w
  double* X;            // n x w, ld n (may alias Z)
  int64_t n, w;
  int64_t row0;         // first row of this job's chunk
  int32_t rows, pad_;
  // counted once per mode (by the chunk at row 0) when some |R_jj| is at most
  // 64 w u max_i |R_ii| (u = 2^-53): R is numerically singular and the
  // solve meaningless
  unsigned long long* singular;
};

// S = copyltu(M): lower triangle of M mirrored to the upper one.
struct SymJob {
  const double* M;
  double* S;
  int64_t w;
};

// ---------------------------------------------------------------------------
// Per-mode QR bookkeeping (Cholesky QR2 with Householder fallback).
struct QrDesc {
  const double* Y;      // n x W input sketch
  double* Q;            // n x w output basis (FP64)
  double* R;            // w x W (nullable): R factor
  double* gram_part;    // splits x W x W partial Gram blocks
  double* rinv;         // W x W upper triangular inverse of the current R
  double* r1;           // W x W first-pass R (kept for the product R2 R1)
  double* q1;           // n x W first-pass Q
  double* hh;           // n x W Householder scratch
  double* tau;          // W Householder scalars
  int32_t* flag;        // 1: use Householder for this mode
  int64_t n, W, w;
  int32_t gram_splits;
  int32_t hh_direct;    // 1: Householder without trying Cholesky QR (W > n, W too wide, policy)
  int32_t report_only;  // 1: a Cholesky breakdown is also counted as a rank-deficiency report
  int32_t pad_;
};

}  // namespace tsk
