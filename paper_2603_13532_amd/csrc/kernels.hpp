// Launch functions of the device kernels (host-callable, stream-ordered).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace tsk {

// Omega_k (rows x cols, column-major) from (seed, mode); FP64 or FP32 output.
hipError_t launch_omega(uint64_t seed, int mode, int64_t rows, int64_t cols, void* out, bool f64,
                        hipStream_t stream);

// Many Omega_k in one launch.
struct OmegaJobDev {
  void* out;
  int64_t count;
  uint64_t seed;
  int32_t mode, f64;
};
hipError_t launch_omega_jobs(const OmegaJobDev* jobs, int count, int64_t max_count,
                             hipStream_t stream);

// Grouped GEMM over `ndesc` device descriptors covering `total_tiles` tiles.
// a32: the A operands are FP32 in an FP64 product (factor sketch and term
// expansion only).  grouped: some descriptors give a workgroup several
// one-tile batch elements (bpw > 1; projection TTMs only).
hipError_t launch_gemm(int prec, int role, const GemmDesc* descs, int ndesc, const GemmSeg* segs,
                       int64_t total_tiles, hipStream_t stream, bool a32 = false,
                       bool grouped = false);

// KRP core sketches over `ndesc` device descriptors covering `total_tiles` tiles.
// Elements of P slices a KRP workgroup may keep in LDS (the block's 64
// columns of every P_k, k != n); launches size their LDS by the largest
// such slice set among their descriptors (`lds_elems`, <= kKrpLds).
constexpr int kKrpLds = 6144;
// g32: FP32 cores in an FP64 core sketch.
hipError_t launch_krp(int prec, const KrpDesc* descs, int ndesc, int64_t total_tiles,
                      int lds_elems, hipStream_t stream, bool g32 = false);

// Core adjoint of the KRP sketch (core-shaped outputs).
hipError_t launch_krp_adj(int prec, const KrpAdjDesc* descs, int ndesc, int64_t total_tiles,
                          hipStream_t stream);
// Adjoint of the thin QR: copyltu and the R^-T substitution.
hipError_t launch_sym(const SymJob* jobs, int count, hipStream_t stream);
hipError_t launch_trsm_rt(const TrsmJob* jobs, int count, hipStream_t stream);

// out[j] (rows x cols, ld_out) = beta * out + sum_{s < parts} part[s] (rows x
// cols, ld_part, part stride `stride_part`), for `count` independent jobs.
struct ReduceJob {
  void* out;
  const void* part;
  int64_t rows, cols, ld_out, ld_part, stride_part;
  int32_t parts, beta;
  int32_t out_f64, part_f64;
};
hipError_t launch_reduce(const ReduceJob* jobs, int count, hipStream_t stream);
// Same jobs, each a <= 64 x 64 tile whose parts are 64 x 64 blocks (ld 64).
hipError_t launch_tile_reduce(const ReduceJob* jobs, int count, hipStream_t stream);

// Fill `count` int32 words with `value` (used instead of hipMemsetAsync so
// that captured graphs hold no memset nodes).
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t stream);

// Typed copies with conversion of contiguous rows x cols matrices
// (ld_dst == ld_src == rows): dst[e] = src[e]. A launch splits every job into
// chunks of kCopyChunk elements; chunk_begin is the job's first chunk in the
// launch (a prefix sum over the jobs before it), and one workgroup copies one
// chunk.
constexpr int kCopyChunk = 2048;
// With norm2 set, every element is also multiplied by mul * sqrt(*norm2)
// (a scale known only on the device).
struct CopyJob {
  void* dst;
  const void* src;
  int64_t rows, cols, ld_dst, ld_src;
  int32_t dst_f64, src_f64;
  int64_t chunk_begin;
  const double* norm2;
  double mul;
};
hipError_t launch_copy(const CopyJob* jobs, int count, int64_t chunks, hipStream_t stream);

// Dense placement of one scaled core into a larger tensor (the
// super-diagonal core of Algorithm 1): dst[(i_k + off_k)_k] = alpha *
// src[(i_k)_k] over the r_1 x ... x r_d source (column-major), dst of
// extents ext (column-major).  One workgroup per kCopyChunk source
// elements; chunk_begin as for CopyJob.
struct BlockJob {
  double* dst;
  const void* src;
  int64_t r[kMaxOrder], off[kMaxOrder], ext[kMaxOrder];
  int32_t order, src_f64;
  double alpha;
  int64_t count;
  int64_t chunk_begin;
};
hipError_t launch_block_scatter(const BlockJob* jobs, int count, int64_t chunks,
                                hipStream_t stream);

// Cholesky QR passes and the Householder fallback over `count` modes.
// wmax: widest Gram (W) among the descriptors; sizes the dynamic LDS.
hipError_t launch_chol(const QrDesc* qr, int count, int pass, double tol, int wmax,
                       hipStream_t stream);
// max_elems: largest (n+1)*W + 2W among the descriptors (sizes the in-LDS panel).
// Panels the eight-wave register kernel takes (the others go to the
// general Householder kernel).  A launch factors the modes `sel` names (bit
// 0: planned for Householder directly, or all under `force`; bit 1: broken
// down in the first Cholesky pass), workgroup b taking the b-th such mode of
// its kernel's kind; grid[0] / grid[1] workgroups of the register / general
// kernel (at least the number of such modes; 0 skips that kernel).
constexpr int kHhWideCols = 64;
constexpr int kHhWideRows = 384;
__host__ __device__ inline bool hh_wide_panel(int64_t n, int64_t W) { return W <= kHhWideCols && n <= kHhWideRows; }
hipError_t launch_householder(const QrDesc* qr, int count, int force, int64_t* fallback_counter,
                              int64_t max_elems, int sel, const int* grid, hipStream_t stream);

// Symmetric eigendecomposition of a W x W matrix (W <= kEigMaxW) by one
// workgroup: eigenvalues in decreasing order into lam[0..W), their
// eigenvectors as the columns of V (ld ldv), eigenvalues clipped at zero
// when clip != 0.  With rank != null, the rank rule: theta = theta_scale *
// trace(C) is computed and stored when set_theta != 0, else read from
// *theta, and *rank = the smallest r >= 1 with sum_{i >= r} lam_i <= theta.
// Widths above kEigMaxW (up to kEigMaxWGlobal) keep the matrix and its
// eigenvectors in `work` (2 Wp^2 doubles, Wp = W rounded up to even).
constexpr int kEigMaxW = 96;
constexpr int kEigMaxWGlobal = 1024;
struct EigJob {
  const double* C;
  double* V;
  double* lam;
  double* theta;
  int32_t* rank;
  double* work;
  int64_t ldc, ldv;
  double tol, theta_scale;
  int32_t W, set_theta, clip;
  int32_t values_only;  // Jacobi: skip the eigenvectors (V neither formed nor written)
};
hipError_t launch_jacobi_eig(const EigJob* jobs, int count, int wmax, hipStream_t stream);
// Eigenvalues only (lam, decreasing; no eigenvectors) of larger matrices,
// W <= kTriMaxW: V is a W x W workspace (ld ldv) that the reduction to
// tridiagonal form overwrites.  Same rank rule.
constexpr int kTriMaxW = 4096;
hipError_t launch_tridiag_eig(const EigJob* jobs, int count, int wmax, hipStream_t stream);

}  // namespace tsk
