// Thin QR of the sketches Y_n in FP64 (the economy QR of Stage 2 of
// Algorithms 4/5), with diag(R) >= 0.
//
// Default path: Cholesky QR2.  The Gram matrix Y^T Y is formed by the MFMA
// GEMM (K-split over rows, partial blocks summed here in a fixed order); one
// workgroup per mode factors it in LDS, G = L L^T with R = L^T, and forms
// L^-1 = R^-T, so that Q1 = Y R^-1 is one more GEMM.  The second pass
// repeats this on Q1 and multiplies R = R2 R1.  A pivot that is not positive,
// or smaller than tol times the original diagonal entry, marks the mode as
// breaking down.
//
// Fallback: Householder QR by one workgroup per flagged mode, panel in
// global memory, reflectors applied column by column; chosen on the device
// from the breakdown flag, so the launch sequence never depends on data.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace tsk {

namespace {

constexpr int kCholMax = 96;  // widest Gram handled in LDS
constexpr int kCholBs = 16;   // column block of the factorization

// The Gram is padded with an identity block to a multiple of 16 columns, so
// every panel is full and no step needs a bounds test; the padding does not
// change the leading W x W block of L or of L^-1.  Leading dimension: even
// (16-byte aligned row pairs) and two rows past the padded width.
__host__ __device__ constexpr int chol_pad(int W) { return (W + kCholBs - 1) & ~(kCholBs - 1); }
__host__ __device__ constexpr int chol_ld(int W) { return chol_pad(W) + 2; }

// Dynamic LDS of a launch whose widest Gram is Wmax: L, L^-1, 1/diag, diag
// and the breakdown word.
__host__ __device__ constexpr size_t chol_lds_bytes(int Wmax) {
  return (2 * (size_t)chol_pad(Wmax) * chol_ld(Wmax) + 2 * kCholMax) * sizeof(double) + 16;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Cholesky G = L L^T and X = L^-1 of one W x W Gram (W <= 96), one
// workgroup.  Latency bounds this kernel, not arithmetic, so the design
// keeps the column-to-column chain short and free of branches:
//   * the Gram's lower triangle is summed from the split partials with the
//     loads of eight elements times eight splits in flight together;
//   * a 16-column panel (diagonal block and all rows below it) is factored
//     by one wave in registers, lane l holding rows k0 + l and k0 + 64 + l;
//     the pivot and the multipliers of later panel columns come from their
//     lanes by readlane, 1/sqrt of the pivot from the hardware reciprocal
//     square root and one Newton step; a bad pivot is recorded and replaced
//     by 1 so that the panel finishes without a branch;
//   * L^-1 is formed alongside by block forward substitution on the
//     identity: X_K = L_KK^-1 B_K (thread per column), then
//     B_{>K} -= L_{>K,K} X_K, next to the trailing update of the Gram
//     A_{>K} -= L_{>K,K} L_{>K,K}^T; both updates use 2 x 2 register blocks
//     over the 16 panel columns;
//   * look-ahead: the next panel's columns are updated first, so that wave 0
//     factors the next panel while the other waves finish block K.
// LDS is sized by the widest Gram of the launch, so narrow Grams leave room
// for several workgroups per CU.
// One 16-column panel of the Cholesky factorization by one wave: lane l
// holds row k0 + l (and k0 + 64 + l when TWO) of the panel in registers.
template <bool TWO>
__device__ __forceinline__ void chol_panel(double* sA, int ld, double* dinv, const double* diag0,
                                           int* s_bad, int k0, int Wp, int lane, double tol) {
  const int r0 = k0 + lane, r1 = k0 + 64 + lane;
  double p0[kCholBs], p1[kCholBs], g0[kCholBs];
#pragma unroll
  for (int c = 0; c < kCholBs; ++c) {
    p0[c] = (c <= lane && r0 < Wp) ? sA[r0 + (k0 + c) * ld] : 0.0;
    if (TWO) p1[c] = (r1 < Wp) ? sA[r1 + (k0 + c) * ld] : 0.0;
    g0[c] = diag0[k0 + c];
  }
  bool bad = false;
  double yc = 0.0;  // lane c: 1 / L(k0 + c, k0 + c)
#pragma unroll
  for (int c = 0; c < kCholBs; ++c) {
    const double piv = readlane_d(p0[c], c);
    const bool badc = !(piv > tol * g0[c]) || !(g0[c] > 0.0);
    bad = bad || badc;
    const double x = badc ? 1.0 : piv;
    double y = __builtin_amdgcn_rsq(x);
    double t = x * y;
    const double e = fma(-t, 0.5 * y, 0.5);
    y = fma(y, e, y);  // 1 / sqrt(x)
    t = fma(t, e, t);  // sqrt(x)
    yc = (lane == c) ? y : yc;
    p0[c] = (lane == c) ? t : p0[c] * y;
    if (TWO) p1[c] *= y;
#pragma unroll
    for (int c2 = c + 1; c2 < kCholBs; ++c2) {
      const double l = readlane_d(p0[c], c2);  // L(k0 + c2, k0 + c)
      p0[c2] = fma(-p0[c], l, p0[c2]);
      if (TWO) p1[c2] = fma(-p1[c], l, p1[c2]);
    }
  }
#pragma unroll
  for (int c = 0; c < kCholBs; ++c) {
    if (c <= lane && r0 < Wp) sA[r0 + (k0 + c) * ld] = p0[c];
    if (TWO && r1 < Wp) sA[r1 + (k0 + c) * ld] = p1[c];
  }
  if (lane < kCholBs) dinv[k0 + lane] = yc;
  if (bad && lane == 0) *s_bad = 1;
}

__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ qrs, int pass,
                                                   double tol) {
  extern __shared__ __align__(16) double smem[];
  const QrDesc& D = qrs[blockIdx.x];
  const int W = (int)D.W;
  if (D.hh_direct) return;
  // The first pass initialises the mode's breakdown flag (no clearing launch
  // is needed before the program); the second skips modes that broke down.
  const bool fits = W <= kCholMax && D.W <= D.n;
  if (pass == 1) {
    if (threadIdx.x == 0) *D.flag = fits ? 0 : 1;
  } else if (*D.flag != 0) {
    return;
  }
  if (!fits) return;
  const int Wp = chol_pad(W), ld = chol_ld(W);
  double* sA = smem;            // Gram, then L (lower triangle), column-major
  double* sX = smem + Wp * ld;  // identity, then L^-1 (lower triangle)
  double* dinv = sX + Wp * ld;  // 1 / L(c, c)
  double* diag0 = dinv + kCholMax;
  int& s_bad = *reinterpret_cast<int*>(diag0 + kCholMax);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---- identity in X, identity padding of the Gram
  for (int j = wave; j < Wp; j += 4)
    for (int i = lane; i < Wp; i += 64) {
      const double id = (i == j) ? 1.0 : 0.0;
      sX[i + j * ld] = id;
      if (i >= W || j >= W) sA[i + j * ld] = id;
    }
  for (int i = W + tid; i < Wp; i += 256) diag0[i] = 1.0;
  if (tid == 0) s_bad = 0;

  // ---- Gram lower triangle = partial blocks summed in split order.  The
  // packed lower triangle (row-major: e = i (i + 1) / 2 + j, j <= i) is
  // spread evenly over the threads, eight elements per thread and round,
  // each with the loads of eight splits in flight together.  The partial
  // blocks are full W x W Gram matrices, so G(i, j) is read at its mirror
  // (j, i): consecutive j are then consecutive addresses.
  {
    const int splits = max(1, (int)D.gram_splits);
    const int64_t WW = (int64_t)W * W;
    const double* part = D.gram_part;
    const int npk = W * (W + 1) / 2;
    for (int e0 = 0; e0 < npk; e0 += 8 * 256) {
      int off[8], ii[8], jj[8];
      bool ok[8];
      double acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + tid + 256 * u;
        int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
        if ((i + 1) * (i + 2) / 2 <= e) ++i;
        if (i * (i + 1) / 2 > e) --i;
        const int j = e - i * (i + 1) / 2;
        ok[u] = e < npk;
        ii[u] = i;
        jj[u] = j;
        off[u] = ok[u] ? j + i * W : 0;
        acc[u] = 0.0;
      }
      for (int s0 = 0; s0 < splits; s0 += 8) {
        double v[8][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const double* p = part + (int64_t)min(s0 + s, splits - 1) * WW;
#pragma unroll
          for (int u = 0; u < 8; ++u) v[s][u] = p[off[u]];
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
          if (s0 + s < splits)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += v[s][u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (ok[u]) {
          sA[ii[u] + jj[u] * ld] = acc[u];
          if (ii[u] == jj[u]) diag0[ii[u]] = acc[u];
        }
    }
  }
  __syncthreads();

  // Blocks of 16 columns with look-ahead: phase 1 (all threads) solves X_K
  // and applies block K to the next panel's 16 columns; phase 2 factors that
  // panel on wave 0 while the other waves apply block K to the rest of the
  // trailing Gram and to B.  Each phase touches disjoint parts of LDS.
  const int nb = Wp / kCholBs;
  auto panel = [&](int K) {
    const int k0 = K * kCholBs;
    if (Wp - k0 > 64)
      chol_panel<true>(sA, ld, dinv, diag0, &s_bad, k0, Wp, lane, tol);
    else
      chol_panel<false>(sA, ld, dinv, diag0, &s_bad, k0, Wp, lane, tol);
  };
  // A(i0..i0+1, j0..j0+1) -= L(i0.., K) L(j0.., K)^T over the 16 columns of block K
  auto sub22 = [&](int k0, int i0, int j0) {
    double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
#pragma unroll
    for (int c = 0; c < kCholBs; ++c) {
      const double2 li = *reinterpret_cast<const double2*>(&sA[i0 + (k0 + c) * ld]);
      const double2 lj = *reinterpret_cast<const double2*>(&sA[j0 + (k0 + c) * ld]);
      a00 = fma(li.x, lj.x, a00);
      a01 = fma(li.x, lj.y, a01);
      a10 = fma(li.y, lj.x, a10);
      a11 = fma(li.y, lj.y, a11);
    }
    sA[i0 + j0 * ld] -= a00;
    sA[i0 + 1 + j0 * ld] -= a10;
    if (i0 > j0) sA[i0 + (j0 + 1) * ld] -= a01;
    sA[i0 + 1 + (j0 + 1) * ld] -= a11;
  };
  if (wave == 0) panel(0);
  __syncthreads();
  for (int K = 0; K < nb; ++K) {
    const int k0 = K * kCholBs, k1 = k0 + kCholBs, k2 = k1 + kCholBs;
    if (s_bad) {  // panel K broke down
      if (tid == 0) *D.flag = 1;
      return;
    }
    const bool ahead = K + 1 < nb;
    // ---- phase 1a: X_K = L_KK^-1 B_K for the columns col < k1 (thread per column)
    if (tid < k1) {
      const int col = tid;
      double b[kCholBs];
#pragma unroll
      for (int r = 0; r < kCholBs; ++r) b[r] = sX[(k0 + r) + col * ld];
#pragma unroll
      for (int r = 0; r < kCholBs; ++r) {
        const double x = b[r] * dinv[k0 + r];
        b[r] = x;
#pragma unroll
        for (int r2 = r + 1; r2 < kCholBs; ++r2)
          b[r2] = fma(-sA[(k0 + r2) + (k0 + r) * ld], x, b[r2]);
      }
#pragma unroll
      for (int r = 0; r < kCholBs; ++r) sX[(k0 + r) + col * ld] = b[r];
    }
    // ---- phase 1b: block K applied to the next panel's columns [k1, k2):
    // 2 x 2 blocks (bi, bj), bj < 8, bi >= bj, rows k1 + 2 bi
    const int nbk = (Wp - k1) >> 1;
    if (ahead)
      for (int e = tid; e < nbk * (kCholBs / 2); e += 256) {
        const int bi = e / (kCholBs / 2), bj = e % (kCholBs / 2);
        if (bi >= bj) sub22(k0, k1 + 2 * bi, k1 + 2 * bj);
      }
    __syncthreads();
    // ---- phase 2: panel K + 1 on wave 0; block K applied to the trailing
    // Gram beyond the next panel (rows, columns >= k2) and to B by the others
    // (by every wave after the last panel)
    const int wb = ahead ? 64 : 0, nw = 256 - wb, wt = tid - wb;
    if (ahead && wave == 0) {
      panel(K + 1);
    } else {
      const int T2 = Wp - k2, nbk2 = T2 > 0 ? T2 >> 1 : 0;
      const int nblk = nbk2 * (nbk2 + 1) / 2;
      for (int e = wt; e < nblk; e += nw) {
        // packed lower-triangle block index -> (bi, bj), bi >= bj
        int bi = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
        if ((bi + 1) * (bi + 2) / 2 <= e) ++bi;
        if (bi * (bi + 1) / 2 > e) --bi;
        const int bj = e - bi * (bi + 1) / 2;
        sub22(k0, k2 + 2 * bi, k2 + 2 * bj);
      }
      // B(i, col) -= sum_c L(i, k0 + c) X(k0 + c, col), i >= k1 > col
      const int ncb = k1 >> 1, nblkb = nbk * ncb;
      for (int e = wt; e < nblkb; e += nw) {
        const int bi = e / ncb, bj = e - bi * ncb;
        const int i0 = k1 + 2 * bi, j0 = 2 * bj;
        double b00 = 0.0, b01 = 0.0, b10 = 0.0, b11 = 0.0;
#pragma unroll
        for (int c = 0; c < kCholBs; ++c) {
          const double2 li = *reinterpret_cast<const double2*>(&sA[i0 + (k0 + c) * ld]);
          const double x0 = sX[(k0 + c) + j0 * ld], x1 = sX[(k0 + c) + (j0 + 1) * ld];
          b00 = fma(li.x, x0, b00);
          b01 = fma(li.x, x1, b01);
          b10 = fma(li.y, x0, b10);
          b11 = fma(li.y, x1, b11);
        }
        sX[i0 + j0 * ld] -= b00;
        sX[i0 + 1 + j0 * ld] -= b10;
        sX[i0 + (j0 + 1) * ld] -= b01;
        sX[i0 + 1 + (j0 + 1) * ld] -= b11;
      }
    }
    __syncthreads();
  }

  // ---- outputs: R^-1 = X^T, R = L^T (upper triangular, zeros below); the
  // LDS reads of eight elements per thread are in flight together
  for (int e0 = 0; e0 < W * W; e0 += 8 * 256) {
    double x[8], l[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + tid + 256 * u, W * W - 1), i = e % W, k = e / W;
      x[u] = (i <= k) ? sX[k + i * ld] : 0.0;
      l[u] = (i <= k) ? sA[k + i * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + tid + 256 * u;
      if (e < W * W) {
        D.rinv[e] = x[u];
        if (pass == 1) D.r1[e] = l[u];
      }
    }
  }
  if (pass == 2 && D.R != nullptr) {
    // R = R2 R1 with R2(i, l) = L2(l, i); w == W on this path.  R1 is staged
    // in LDS (X is no longer needed).
    __syncthreads();
    for (int k = wave; k < W; k += 4)
      for (int i = lane; i < W; i += 64) sX[i + k * ld] = D.r1[i + (int64_t)k * W];
    __syncthreads();
    for (int k = wave; k < W; k += 4)
      for (int i = lane; i < W; i += 64) {
        // four independent partial sums, so that the LDS reads and FMAs of
        // consecutive l overlap
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int l = i;
        for (; l + 3 <= k; l += 4) {
          a0 = fma(sA[l + i * ld], sX[l + k * ld], a0);
          a1 = fma(sA[l + 1 + i * ld], sX[l + 1 + k * ld], a1);
          a2 = fma(sA[l + 2 + i * ld], sX[l + 2 + k * ld], a2);
          a3 = fma(sA[l + 3 + i * ld], sX[l + 3 + k * ld], a3);
        }
        for (; l <= k; ++l) a0 = fma(sA[l + i * ld], sX[l + k * ld], a0);
        D.R[i + (int64_t)k * W] = (i <= k) ? (a0 + a1) + (a2 + a3) : 0.0;
      }
  }
}

constexpr int64_t kHhLdsMax = 19456;  // doubles of LDS for an in-LDS Householder panel (152 KB)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Householder QR with the whole n x W panel in LDS (column-major, ld n),
// used when it fits.  Reflector j: norm of the subdiagonal part by a block
// reduction, then each wave applies it to every fourth trailing column, two
// columns per pass so that their two reductions overlap.  Q is formed in
// place from the stored reflectors, last to first (the LAPACK org2r order),
// after R has been written out; signs then make diag(R) >= 0.
typedef __attribute__((address_space(3))) double lds_f64;

// Householder QR of the n x W matrix Ysrc (leading dimension ldy) in the
// panel A (leading dimension lda).  Writes R (w x W, ld ldr; null to skip)
// and Q (n x w, ld ldq); with fix_signs, rows of R and columns of Q are
// negated where needed so that diag(R) >= 0.  A, tau, sgn: LDS or global
// (the same algorithm for both); red, part: LDS.
//
// Reflector j: a block reduction gives the norm below the diagonal, and
// every thread then derives tau, beta and the scale of the reflector.  The
// trailing columns are updated with lane = column and wave = every fourth
// row: partial dot products, one exchange through LDS, then the rank-one
// update, so each reflector costs three barriers and no per-column
// reductions.  The reflector's column is scaled one step later, while the
// next norm is formed.  Q is then formed in place, last reflector first
// (LAPACK org2r order), with the same column-parallel update.
template <typename PA, typename PV>
__device__ __forceinline__ void hh_core(const double* Ysrc, int64_t ldy, double* Qdst,
                                        int64_t ldq, double* Rdst, int64_t ldr, bool fix_signs,
                                        PA A, int64_t lda, PV tau, PV sgn, lds_f64* red,
                                        lds_f64* part, int64_t n64, int64_t W64, int64_t w64) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = (int)n64, W = (int)W64, w = (int)w64;
  // column k of the panel
  auto col_of = [&](int k) { return A + (int64_t)k * lda; };
  for (int k = wave; k < W; k += 4) {
    auto ak = col_of(k);
    const double* yk = Ysrc + (int64_t)k * ldy;
    for (int i = lane; i < n; i += 64) ak[i] = yk[i];
  }
  __syncthreads();
  double scal_prev = 1.0;
  for (int j = 0; j < w; ++j) {
    auto aj = col_of(j);
    double pn = 0.0;
#pragma unroll 4
    for (int i = j + 1 + tid; i < n; i += 256) pn += aj[i] * aj[i];
    if (j > 0) {
      auto ap = col_of(j - 1);
      for (int i = j + tid; i < n; i += 256) ap[i] *= scal_prev;
    }
    const double alpha = aj[j];
    pn = wave_sum(pn);
    if (lane == 0) red[wave] = pn;
    __syncthreads();
    const double sigma = red[0] + red[1] + red[2] + red[3];
    double t = 0.0, scal = 1.0, beta = alpha;
    if (sigma > 0.0) {
      const double mu = sqrt(alpha * alpha + sigma);
      beta = (alpha <= 0.0) ? mu : -mu;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      aj[j] = beta;
      tau[j] = t;
    }
    if (t != 0.0) {
      for (int cb = j + 1; cb < W; cb += 64) {
        const int col = cb + lane;
        const bool ok = col < W;
        auto ac = col_of(ok ? col : j);
        double d = 0.0, arow = 0.0;
        if (ok) {
#pragma unroll 4
          for (int i = j + 1 + wave; i < n; i += 4) d += aj[i] * ac[i];
          arow = ac[j];
        }
        part[wave * 64 + lane] = d;
        __syncthreads();
        const double S = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
        const double f = t * (arow + scal * S), fs = f * scal;
        if (ok) {
#pragma unroll 4
          for (int i = j + 1 + wave; i < n; i += 4) ac[i] -= fs * aj[i];
          if (wave == 0) ac[j] = arow - f;
        }
        __syncthreads();
      }
    } else {
      __syncthreads();
    }
    scal_prev = scal;
  }
  __syncthreads();
  if (w > 0) {
    auto al = col_of(w - 1);
    for (int i = w + tid; i < n; i += 256) al[i] *= scal_prev;
  }
  for (int i = tid; i < w; i += 256) sgn[i] = (fix_signs && col_of(i)[i] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  if (Rdst != nullptr) {
    for (int k = wave; k < W; k += 4) {
      auto ak = col_of(k);
      for (int i = lane; i < w; i += 64) Rdst[i + (int64_t)k * ldr] = (i <= k) ? sgn[i] * ak[i] : 0.0;
    }
  }
  __syncthreads();
  // Q = H_0 ... H_{w-1} [I_w; 0], formed in place in columns 0 .. w-1
  for (int j = w - 1; j >= 0; --j) {
    auto aj = col_of(j);
    const double t = tau[j];
    if (t != 0.0) {
      for (int cb = j + 1; cb < w; cb += 64) {
        const int col = cb + lane;
        const bool ok = col < w;
        auto ac = col_of(ok ? col : j);
        double d = 0.0, arow = 0.0;
        if (ok) {
#pragma unroll 4
          for (int i = j + 1 + wave; i < n; i += 4) d += aj[i] * ac[i];
          arow = ac[j];
        }
        part[wave * 64 + lane] = d;
        __syncthreads();
        const double S = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
        const double f = t * (arow + S);
        if (ok) {
#pragma unroll 4
          for (int i = j + 1 + wave; i < n; i += 4) ac[i] -= f * aj[i];
          if (wave == 0) ac[j] = arow - f;
        }
        __syncthreads();
      }
    }
    for (int i = tid; i < n; i += 256) {
      if (i > j) aj[i] *= -t;
      else if (i == j) aj[i] = 1.0 - t;
      else aj[i] = 0.0;
    }
    __syncthreads();
  }
  for (int k = wave; k < w; k += 4) {
    auto ak = col_of(k);
    double* qk = Qdst + (int64_t)k * ldq;
    for (int i = lane; i < n; i += 64) qk[i] = sgn[k] * ak[i];
  }
  __syncthreads();
}

// Register-resident Householder QR for n <= 4 NR rows and W <= 64 columns:
// lane c holds column c, wave w holds rows w, w + 4, ...  The reflector
// column is broadcast from its lane with readlane (a scalar operand of the
// FMAs, read where it is used so that it never stays live); the norm and
// the partial dot products of all trailing columns come from one pass over
// the registers, four partial sums per column are exchanged through LDS
// (double-buffered by step parity), and one more pass applies the update:
// one barrier per reflector and no LDS traffic proportional to the panel.
// Registers are shifted by one row block every four reflectors, so that row
// j always sits in register 0 of wave j % 4 (static register indexing);
// rows leaving the window are parked in the LDS panel A (ld lda), which
// also stages the coalesced input and output.  Q is formed backwards (org2r
// order) with the window shifted back.  Same arithmetic as hh_core.
template <int NR>
__device__ __forceinline__ void hh_regs(const double* Ysrc, int64_t ldy, double* Qdst,
                                        int64_t ldq, double* Rdst, int64_t ldr, bool fix_signs,
                                        lds_f64* A, int lda, lds_f64* tau, lds_f64* sgn,
                                        lds_f64* red, lds_f64* part, int n, int W, int w) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c = lane;
  for (int k = wave; k < W; k += 4)
    for (int i = lane; i < n; i += 64) A[i + k * lda] = Ysrc[i + (int64_t)k * ldy];
  __syncthreads();
  double a[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = wave + 4 * r;
    a[r] = (i < n && c < W) ? A[i + c * lda] : 0.0;
  }
  __syncthreads();
  const int nq = (w + 3) / 4;
  for (int q = 0; q < nq; ++q) {
#pragma unroll
    for (int jw = 0; jw < 4; ++jw) {
      const int j = 4 * q + jw;
      if (j < w) {
        const bool first_below = wave > jw;  // register 0 holds a row below j
        lds_f64* rd = red + 8 * jw;           // step parity buffers (jw & 1 would do;
        lds_f64* pt = part + 320 * (jw & 1);  // red is indexed by jw for clarity)
        double p = 0.0, d = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double v = readlane_d(a[r], j);
          if (r > 0 || first_below) {
            p += v * v;
            d += v * a[r];
          }
        }
        const double a0j = readlane_d(a[0], j);
        if (lane == 0) rd[wave] = p;
        if (wave == jw && lane == 0) rd[4] = a0j;  // alpha = A(j, j)
        pt[wave * 64 + lane] = d;
        if (wave == jw) pt[256 + lane] = a[0];  // row j
        __syncthreads();
        const double sigma = rd[0] + rd[1] + rd[2] + rd[3], alpha = rd[4];
        double t = 0.0, scal = 1.0, beta = alpha;
        if (sigma > 0.0) {
          const double mu = sqrt(alpha * alpha + sigma);
          beta = (alpha <= 0.0) ? mu : -mu;
          t = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        const double S = pt[lane] + pt[64 + lane] + pt[128 + lane] + pt[192 + lane];
        const double arow = pt[256 + lane];
        const double f = t * (arow + scal * S), fs = f * scal;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double v = readlane_d(a[r], j);
          if (r > 0 || first_below)
            a[r] = (c > j) ? a[r] - fs * v : ((c == j) ? a[r] * scal : a[r]);
        }
        if (wave == jw) a[0] = (c > j) ? arow - f : ((c == j) ? beta : a[0]);
        if (tid == 0) tau[j] = t;
      }
    }
    // park row 4q + wave and shift the window down by one row block
    {
      const int i = 4 * q + wave;
      if (i < n && c < W) A[i + c * lda] = a[0];
    }
#pragma unroll
    for (int r = 0; r < NR - 1; ++r) a[r] = a[r + 1];
    a[NR - 1] = 0.0;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = 4 * nq + wave + 4 * r;
    if (i < n && c < W) A[i + c * lda] = a[r];
  }
  __syncthreads();
  for (int i = tid; i < w; i += 256) sgn[i] = (fix_signs && A[i + i * lda] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  if (Rdst != nullptr)
    for (int k = wave; k < W; k += 4)
      for (int i = lane; i < w; i += 64)
        Rdst[i + (int64_t)k * ldr] = (i <= k) ? sgn[i] * A[i + k * lda] : 0.0;
  // Q = H_0 ... H_{w-1} [I_w; 0]: window at the last row block, entries on
  // or above the diagonal cleared (formed columns are zero above their index)
  const int q0 = nq > 0 ? nq - 1 : 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = 4 * q0 + wave + 4 * r;
    a[r] = (i < n && c < w && c < i) ? A[i + c * lda] : 0.0;
  }
  for (int q = nq - 1; q >= 0; --q) {
#pragma unroll
    for (int jw = 3; jw >= 0; --jw) {
      const int j = 4 * q + jw;
      if (j < w) {
        const bool first_below = wave > jw;
        lds_f64* pt = part + 320 * (jw & 1);
        const double t = tau[j];
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double v = readlane_d(a[r], j);
          if (r > 0 || first_below) d += v * a[r];
        }
        pt[wave * 64 + lane] = d;
        if (wave == jw) pt[256 + lane] = a[0];
        __syncthreads();
        const double S = pt[lane] + pt[64 + lane] + pt[128 + lane] + pt[192 + lane];
        const double arow = pt[256 + lane];
        const double f = t * (arow + S);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double v = readlane_d(a[r], j);
          if (r > 0 || first_below)
            a[r] = (c > j) ? a[r] - f * v : ((c == j) ? -t * a[r] : a[r]);
        }
        if (wave == jw) a[0] = (c > j) ? arow - f : ((c == j) ? 1.0 - t : a[0]);
      }
    }
    if (q > 0) {
#pragma unroll
      for (int r = NR - 1; r > 0; --r) a[r] = a[r - 1];
      const int i = 4 * (q - 1) + wave;
      a[0] = (i < n && c < w && c < i) ? A[i + c * lda] : 0.0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = wave + 4 * r;
    if (i < n && c < w) A[i + c * lda] = sgn[c] * a[r];
  }
  __syncthreads();
  for (int k = wave; k < w; k += 4)
    for (int i = lane; i < n; i += 64) Qdst[i + (int64_t)k * ldq] = A[i + k * lda];
  __syncthreads();
}

// Register path when the panel fits it (n <= 256, W <= 64), else hh_core.
__device__ __forceinline__ void hh_any(const double* Ysrc, int64_t ldy, double* Qdst, int64_t ldq,
                                       double* Rdst, int64_t ldr, bool fix_signs, lds_f64* A,
                                       int64_t lda, lds_f64* tau, lds_f64* sgn, lds_f64* red,
                                       lds_f64* part, int64_t n, int64_t W, int64_t w) {
  if (W <= 64 && n <= 256) {
    const int ni = (int)n, Wi = (int)W, wi = (int)w, li = (int)lda;
    if (n <= 64)
      hh_regs<16>(Ysrc, ldy, Qdst, ldq, Rdst, ldr, fix_signs, A, li, tau, sgn, red, part, ni, Wi, wi);
    else if (n <= 128)
      hh_regs<32>(Ysrc, ldy, Qdst, ldq, Rdst, ldr, fix_signs, A, li, tau, sgn, red, part, ni, Wi, wi);
    else if (n <= 192)
      hh_regs<48>(Ysrc, ldy, Qdst, ldq, Rdst, ldr, fix_signs, A, li, tau, sgn, red, part, ni, Wi, wi);
    else
      hh_regs<64>(Ysrc, ldy, Qdst, ldq, Rdst, ldr, fix_signs, A, li, tau, sgn, red, part, ni, Wi, wi);
  } else {
    hh_core(Ysrc, ldy, Qdst, ldq, Rdst, ldr, fix_signs, A, lda, tau, sgn, red, part, n, W, w);
  }
}

// Tall panels that do not fit LDS whole (n >= 4 W): one level of TSQR.
// The two row halves are factored in LDS, their R factors stacked, the
// stack factored (with the sign fix), and Q = diag(Q1, Q2) Q3 formed from
// LDS copies of Q3 and of each half's Q.  Workspace: the stack S (m3 x W)
// and Q3 (m3 x w) in the panel scratch, Q1 and Q2 in place in Q.
__device__ __forceinline__ void hh_tsqr(const QrDesc& D, lds_f64* base, lds_f64* red,
                                        lds_f64* part, int64_t n, int64_t W, int64_t w) {
  const int tid = threadIdx.x;
  const int64_t n1 = (n + 1) / 2, n2 = n - n1;
  const int64_t w1 = n1 < W ? n1 : W, w2 = n2 < W ? n2 : W, m3 = w1 + w2;
  double* S = D.hh;             // m3 x W, ld m3
  double* Q3 = D.hh + m3 * W;   // m3 x w, ld m3
  lds_f64* A = base;
  const int64_t l1 = n1 + 1, l2 = n2 + 1, l3 = m3 + 1;  // odd leading dimensions
  hh_any(D.Y, n, D.Q, n, S, m3, false, A, l1, A + l1 * W, A + l1 * W + W, red, part, n1, W, w1);
  hh_any(D.Y + n1, n, D.Q + n1, n, S + w1, m3, false, A, l2, A + l2 * W, A + l2 * W + W, red, part,
         n2, W, w2);
  hh_any(S, m3, Q3, m3, D.R, w, true, A, l3, A + l3 * W, A + l3 * W + W, red, part, m3, W, w);
  // Q rows of half h: Q_h (rows x wh, in place in D.Q) times Q3 rows [off, off + wh)
  lds_f64* sQ3 = base;          // m3 x w
  lds_f64* sQh = base + m3 * w; // rows x wh
  for (int64_t e = tid; e < m3 * w; e += 256) sQ3[e] = Q3[e];
  for (int h = 0; h < 2; ++h) {
    const int64_t r0 = h ? n1 : 0, rows = h ? n2 : n1, wh = h ? w2 : w1, off = h ? w1 : 0;
    __syncthreads();
    for (int64_t e = tid; e < rows * wh; e += 256) {
      const int64_t i = e % rows, k = e / rows;
      sQh[e] = D.Q[r0 + i + k * n];
    }
    __syncthreads();
    for (int64_t e = tid; e < rows * w; e += 256) {
      const int64_t i = e % rows, c = e / rows;
      double acc = 0.0;
      for (int64_t k = 0; k < wh; ++k) acc += sQh[i + k * rows] * sQ3[off + k + c * m3];
      D.Q[r0 + i + c * n] = acc;
    }
  }
}

// Register-resident Householder QR of one n x W panel (n <= NW * NR,
// W <= kWideCols) with NW waves: lane c holds column c, wave v holds rows
// v, v + NW, ...; the arithmetic is that of hh_regs (and hh_core).  With
// more waves each wave walks fewer rows per reflector and the waves sharing
// a SIMD hide each other's latencies.  Per reflector j every lane needs the
// entries of column j in its wave's rows: lane j writes them to a per-wave
// LDS row and all lanes read it (LDS operations of one wave complete in
// order; a broadcast through readlane measured no faster and spills SGPRs).
// Every lane forms its column's partial dot product, and one barrier
// exchanges the NW partials; lane j's partial is the squared norm below the
// diagonal, so the norm needs no separate reduction.  The update is a
// multiply and an FMA per element.  Registers shift by one row block every
// NW reflectors (row j sits in register 0 of wave j % NW); rows leaving the
// window are parked in LDS, which is all the LDS the panel needs, so tall
// panels do not have to fit it whole.
constexpr int kWideWaves = 8;
constexpr int kWideCols = kHhWideCols;
constexpr int kWideRows = kHhWideRows;  // 48 rows per wave: 225 VGPRs; 64 per wave spills
constexpr int kWidePark = kWideCols + kWideWaves;  // parked rows: w rounded up to NW
constexpr int kWideLdp = kWideCols + 1;

// sum over the wave's rows below the reflector (register 0 only when fb) of
// v_r a_r, v = column j read from the wave's broadcast row in batches of
// eight (one batch in flight: the reads of a batch overlap, and the window
// does not spill)
template <int NR>
__device__ __forceinline__ double hh_wide_dot(const lds_f64* cb, const double (&a)[NR], bool fb) {
  static_assert(NR % 8 == 0, "rows per wave come in batches of eight");
  double d = 0.0;
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = cb[r0 + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) d = fma(v[k], (r0 + k > 0 || fb) ? a[r0 + k] : 0.0, d);
    __builtin_amdgcn_sched_barrier(0);
  }
  return d;
}
// a_r = a_r m + coef v_r over the same rows (m = 1 and coef = 0 leave a
// column unchanged; a column is scaled by m exactly, not through v = a)
template <int NR>
__device__ __forceinline__ void hh_wide_update(const lds_f64* cb, double (&a)[NR], bool fb,
                                               double m, double coef) {
  const double m0 = fb ? m : 1.0, c0 = fb ? coef : 0.0;
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = cb[r0 + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool z = r0 + k == 0;
      a[r0 + k] = fma(v[k], z ? c0 : coef, a[r0 + k] * (z ? m0 : m));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NW, int NR>
__device__ __forceinline__ void hh_wide(const QrDesc& D, lds_f64* park, lds_f64* colb,
                                        lds_f64* part, lds_f64* tau, lds_f64* sgn, int n, int W,
                                        int w) {
  const int tid = threadIdx.x, lane = tid & 63, c = lane;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* Y = D.Y;
  const int64_t ldy = n;
  lds_f64* cb = colb + wave * NR;  // this wave's broadcast row
  double a[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = wave + NW * r;
    a[r] = (i < n && c < W) ? Y[i + (int64_t)c * ldy] : 0.0;
  }
  const int nq = (w + NW - 1) / NW;
  int step = 0;  // parity of the exchange buffer
  for (int q = 0; q < nq; ++q) {
    for (int jw = 0; jw < NW; ++jw) {
      const int j = NW * q + jw;
      if (j >= w) break;
      const bool fb = wave > jw;  // register 0 holds a row below j
      lds_f64* pt = part + (NW + 1) * 64 * (step & 1);
      ++step;
      if (lane == j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) cb[r] = a[r];
      }
      // the other lanes read what lane j wrote: the fence keeps the compiler
      // from forwarding or reusing earlier values of the row
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const double d = hh_wide_dot<NR>(cb, a, fb);
      pt[wave * 64 + lane] = d;
      if (wave == jw) pt[NW * 64 + lane] = a[0];  // row j
      __syncthreads();
      double S = 0.0, sigma = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        S += pt[v * 64 + lane];
        sigma += pt[v * 64 + j];
      }
      const double arow = pt[NW * 64 + lane], alpha = pt[NW * 64 + j];
      double t = 0.0, scal = 1.0, beta = alpha;
      if (sigma > 0.0) {
        const double mu = sqrt(alpha * alpha + sigma);
        beta = (alpha <= 0.0) ? mu : -mu;
        t = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      const double f = t * (arow + scal * S), fs = f * scal;
      // rows below j: a -= fs v right of column j, a *= scal in column j
      hh_wide_update<NR>(cb, a, fb, (c == j) ? scal : 1.0, (c > j) ? -fs : 0.0);
      if (wave == jw) a[0] = (c > j) ? arow - f : ((c == j) ? beta : a[0]);
      if (tid == 0) tau[j] = t;
      __builtin_amdgcn_wave_barrier();
    }
    // park row NW q + wave and shift the window down by one row block
    park[(NW * q + wave) * kWideLdp + c] = a[0];
#pragma unroll
    for (int r = 0; r < NR - 1; ++r) a[r] = a[r + 1];
    a[NR - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < w; i += NW * 64)
    sgn[i] = (park[i * kWideLdp + i] < 0.0) ? -1.0 : 1.0;  // R with a non-negative diagonal
  __syncthreads();
  if (D.R != nullptr)
    for (int e = tid; e < w * W; e += NW * 64) {
      const int i = e % w, k = e / w;
      D.R[i + (int64_t)k * w] = (i <= k) ? sgn[i] * park[i * kWideLdp + k] : 0.0;
    }
  // Q = H_0 ... H_{w-1} [I_w; 0], formed backwards: the window goes back to
  // block nq - 1 and keeps only reflector entries (columns below w and left
  // of the diagonal; rows in registers are all below the diagonal).
#pragma unroll
  for (int r = NR - 1; r > 0; --r) a[r] = (c < w) ? a[r - 1] : 0.0;
  {
    const int i = NW * (nq - 1) + wave;
    a[0] = (i < n && c < w && c < i) ? park[i * kWideLdp + c] : 0.0;
  }
  for (int q = nq - 1; q >= 0; --q) {
    for (int jw = NW - 1; jw >= 0; --jw) {
      const int j = NW * q + jw;
      if (j >= w) continue;
      const bool fb = wave > jw;
      lds_f64* pt = part + (NW + 1) * 64 * (step & 1);
      ++step;
      const double t = tau[j];
      if (lane == j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) cb[r] = a[r];
      }
      // the other lanes read what lane j wrote: the fence keeps the compiler
      // from forwarding or reusing earlier values of the row
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const double d = hh_wide_dot<NR>(cb, a, fb);
      pt[wave * 64 + lane] = d;
      if (wave == jw) pt[NW * 64 + lane] = a[0];
      __syncthreads();
      double S = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) S += pt[v * 64 + lane];
      const double arow = pt[NW * 64 + lane];
      const double f = t * (arow + S);
      // rows below j: a -= f v right of column j, a *= -t in column j
      hh_wide_update<NR>(cb, a, fb, (c == j) ? -t : 1.0, (c > j) ? -f : 0.0);
      if (wave == jw) a[0] = (c > j) ? arow - f : ((c == j) ? 1.0 - t : a[0]);
      __builtin_amdgcn_wave_barrier();
    }
    if (q > 0) {
#pragma unroll
      for (int r = NR - 1; r > 0; --r) a[r] = a[r - 1];
      const int i = NW * (q - 1) + wave;
      a[0] = (i < n && c < w && c < i) ? park[i * kWideLdp + c] : 0.0;
    }
  }
  double* Q = D.Q;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = wave + NW * r;
    if (i < n && c < w) Q[i + (int64_t)c * n] = sgn[c] * a[r];
  }
}

// Whether descriptor D needs the Householder path of the given kind (the
// eight-wave register kernel when `wide`, the general kernel otherwise) in
// a launch that takes the modes `sel` names: bit 0 the modes planned for
// Householder directly (or every mode under `force`), bit 1 the modes whose
// Cholesky pass broke down.
__device__ __forceinline__ bool hh_needed(const QrDesc& D, int force, bool wide, int sel) {
  if (hh_wide_panel(D.n, D.W) != wide) return false;
  if (force || D.hh_direct) return (sel & 1) != 0;
  return (sel & 2) != 0 && *D.flag != 0;  // flag written by the first chol pass
}

// Index of the b-th descriptor (in descriptor order) that needs this
// kernel, or -1: the launch covers every mode, but whether a mode breaks
// down is known only on the device, so workgroup b takes the b-th mode that
// does.  The modes that run then sit on consecutive workgroups, which the
// dispatcher spreads over distinct CUs, instead of wherever their
// descriptors fall.  Block-wide: every thread returns the same index.
template <int T>
__device__ int hh_nth_job(const QrDesc* __restrict__ qrs, int count, int force, bool wide,
                          int sel, int b) {
  constexpr int NWV = T / 64;
  __shared__ int s_cnt[NWV];
  __shared__ int s_found;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) s_found = -1;
  int base = 0;
  for (int c0 = 0; c0 < count; c0 += T) {
    const int i = c0 + t;
    const bool need = i < count && hh_needed(qrs[i], force, wide, sel);
    const unsigned long long m = __ballot(need);
    if (lane == 0) s_cnt[wv] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int v = 0; v < NWV; ++v) {
      if (v < wv) before += s_cnt[v];
      total += s_cnt[v];
    }
    const int rank = base + before + __popcll(m & ((1ull << lane) - 1ull));
    if (need && rank == b) s_found = i;
    base += total;
    __syncthreads();
    if (s_found >= 0 || base > b) break;
  }
  const int r = s_found;
  __syncthreads();
  return r;
}

// Panels with W <= kWideCols and n <= kWideRows go here (one workgroup of
// kWideWaves waves each); householder_kernel takes the others.
__global__ __launch_bounds__(kWideWaves * 64) void householder_wide_kernel(
    const QrDesc* __restrict__ qrs, int count, int force, int sel, unsigned long long* counter) {
  const int job = hh_nth_job<kWideWaves * 64>(qrs, count, force, true, sel, blockIdx.x);
  if (job < 0) return;
  const QrDesc& D = qrs[job];
  const bool broke = !D.hh_direct && *D.flag != 0;
  const int64_t n = D.n, W = D.W;
  const int64_t w = n < W ? n : W;
  if (threadIdx.x == 0 && counter != nullptr) {
    atomicAdd(counter, 1ull);                              // QRs done by Householder
    if (broke && D.report_only) atomicAdd(counter + 1, 1ull);  // reported breakdowns
  }
  constexpr int NW = kWideWaves;
  __shared__ double park_s[kWidePark * kWideLdp];
  __shared__ double colb_s[NW * (kWideRows / NW)];
  __shared__ double part_s[2 * (NW + 1) * 64];
  __shared__ double tau_s[kWideCols], sgn_s[kWideCols];
  lds_f64* park = (lds_f64*)park_s;
  lds_f64* colb = (lds_f64*)colb_s;
  lds_f64* part = (lds_f64*)part_s;
  lds_f64* tau = (lds_f64*)tau_s;
  lds_f64* sgn = (lds_f64*)sgn_s;
  const int ni = (int)n, Wi = (int)W, wi = (int)w;
  if (n <= 8 * NW)
    hh_wide<NW, 8>(D, park, colb, part, tau, sgn, ni, Wi, wi);
  else if (n <= 16 * NW)
    hh_wide<NW, 16>(D, park, colb, part, tau, sgn, ni, Wi, wi);
  else if (n <= 32 * NW)
    hh_wide<NW, 32>(D, park, colb, part, tau, sgn, ni, Wi, wi);
  else
    hh_wide<NW, 48>(D, park, colb, part, tau, sgn, ni, Wi, wi);
}
static_assert(kWideRows <= 48 * kWideWaves, "register window of the wide Householder path");

__global__ __launch_bounds__(256) void householder_kernel(const QrDesc* __restrict__ qrs,
                                                          int count, int force, int sel,
                                                          unsigned long long* counter,
                                                          int64_t lds_elems) {
  extern __shared__ __align__(16) double hsm[];
  const int job = hh_nth_job<256>(qrs, count, force, false, sel, blockIdx.x);
  if (job < 0) return;
  const QrDesc& D = qrs[job];
  const bool broke = !D.hh_direct && *D.flag != 0;
  const int64_t n = D.n, W = D.W;
  const int64_t w = n < W ? n : W;
  const int tid = threadIdx.x;
  if (tid == 0 && counter != nullptr) {
    atomicAdd(counter, 1ull);                              // QRs done by Householder
    if (broke && D.report_only) atomicAdd(counter + 1, 1ull);  // reported breakdowns
  }
  __shared__ double red_s[32];
  __shared__ double part_s[640];
  lds_f64* red = (lds_f64*)red_s;
  lds_f64* part = (lds_f64*)part_s;
  lds_f64* base = (lds_f64*)hsm;
  const int64_t n1 = (n + 1) / 2, w1 = n1 < W ? n1 : W;
  if ((n + 1) * W + 2 * W <= lds_elems) {
    const int64_t la = n + 1;  // odd: lanes on different columns hit different banks
    hh_any(D.Y, n, D.Q, n, D.R, w, true, base, la, base + la * W, base + la * W + W, red, part, n,
           W, w);
  } else if (n >= 4 * W && (n1 + 1) * W + 2 * W <= lds_elems &&
             (2 * w1 + 1) * W + 2 * W <= lds_elems && 2 * w1 * w + n1 * w1 <= lds_elems) {
    hh_tsqr(D, base, red, part, n, W, w);
  } else {
    // panel in global memory (workspace: n x W panel, then W signs)
    hh_core(D.Y, n, D.Q, n, D.R, w, true, D.hh, n, D.tau, D.hh + n * W, red, part, n, W, w);
  }
}

// copyltu(M): S(i, j) = M(max(i,j), min(i,j)).
__global__ __launch_bounds__(256) void sym_kernel(const SymJob* __restrict__ jobs) {
  const SymJob J = jobs[blockIdx.x];
  const int64_t w = J.w;
  for (int64_t e = threadIdx.x; e < w * w; e += 256) {
    const int64_t i = e % w, j = e / w;
    J.S[e] = (i >= j) ? J.M[i + j * w] : J.M[j + i * w];
  }
}

// X = Z R^-T: thread per row, x R^T = z, i.e. back substitution with the
// rows of R.  R and the running solutions live in LDS (one wave per job).
constexpr int kTrsmMax = 96;
__global__ __launch_bounds__(64) void trsm_rt_kernel(const TrsmJob* __restrict__ jobs) {
  const TrsmJob J = jobs[blockIdx.x];
  const int w = (int)J.w, t = threadIdx.x;
  __shared__ double sR[kTrsmMax * kTrsmMax];
  __shared__ double sx[kTrsmMax][64];
  for (int e = t; e < w * w; e += 64) sR[e] = J.R[e];
  __syncthreads();
  if (t == 0 && J.row0 == 0 && J.singular != nullptr) {
    double dmax = 0.0, dmin = INFINITY;
    for (int j = 0; j < w; ++j) {
      const double a = fabs(sR[j + j * w]);
      dmax = fmax(dmax, a);
      dmin = fmin(dmin, a);
    }
    if (!(dmin > 64.0 * w * 0x1p-53 * dmax)) atomicAdd(J.singular, 1ull);
  }
  const int64_t row = J.row0 + t;
  const bool active = t < J.rows && row < J.n;
  if (active) {
    for (int j = w - 1; j >= 0; --j) {
      double acc = J.Z[row + (int64_t)j * J.n];
      for (int l = j + 1; l < w; ++l) acc -= sR[j + l * w] * sx[l][t];
      sx[j][t] = acc / sR[j + j * w];
    }
    for (int j = 0; j < w; ++j) J.X[row + (int64_t)j * J.n] = sx[j][t];
  }
}

}  // namespace

hipError_t launch_sym(const SymJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  sym_kernel<<<dim3((unsigned)count), dim3(256), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_trsm_rt(const TrsmJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  trsm_rt_kernel<<<dim3((unsigned)count), dim3(64), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_chol(const QrDesc* qr, int count, int pass, double tol, int wmax,
                       hipStream_t stream) {
  if (count <= 0 || wmax <= 0) return hipSuccess;
  if (wmax > kCholMax) wmax = kCholMax;  // wider Grams skip the kernel
  const size_t lds = chol_lds_bytes(wmax);
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)chol_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)chol_lds_bytes(kCholMax));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  chol_kernel<<<dim3((unsigned)count), dim3(256), lds, stream>>>(qr, pass, tol);
  return hipGetLastError();
}

hipError_t launch_householder(const QrDesc* qr, int count, int force, int64_t* fallback_counter,
                              int64_t max_elems, int sel, const int* grid, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  // LDS for the largest panel (plus tau, signs and reduction slots), capped
  int64_t elems = max_elems < kHhLdsMax ? max_elems : kHhLdsMax;
  if (elems < 0) elems = 0;
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)householder_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(kHhLdsMax * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (grid[0] > 0) {
    householder_wide_kernel<<<dim3((unsigned)grid[0]), dim3(kWideWaves * 64), 0, stream>>>(
        qr, count, force, sel, (unsigned long long*)fallback_counter);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (grid[1] > 0) {
    householder_kernel<<<dim3((unsigned)grid[1]), dim3(256), (size_t)elems * sizeof(double), stream>>>(
        qr, count, force, sel, (unsigned long long*)fallback_counter, elems);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace tsk
