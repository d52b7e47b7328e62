// Thin QR of the sketches Y_n in FP64 (the "qr(Y_n, 'econ')" step of
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
//     over the 16 panel columns.
// LDS is sized by the widest Gram of the launch, so narrow Grams leave room
// for several workgroups per CU.
__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ qrs, int pass,
                                                   double tol) {
  extern __shared__ __align__(16) double smem[];
  const QrDesc& D = qrs[blockIdx.x];
  const int W = (int)D.W;
  if (D.hh_direct || *D.flag != 0 || W > kCholMax || D.W > D.n) return;
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

  // ---- Gram lower triangle = partial blocks summed in split order
  {
    const int splits = max(1, (int)D.gram_splits);
    const int64_t WW = (int64_t)W * W;
    const double* part = D.gram_part;
    for (int j0 = wave; j0 < W; j0 += 16) {
      // elements u: column j0 + 4 (u >> 1), rows lane + 64 (u & 1)
      int off[8];
      bool ok[8];
      double acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + 4 * (u >> 1), i = lane + 64 * (u & 1);
        ok[u] = j < W && i < W && i >= j;
        off[u] = ok[u] ? i + j * W : 0;
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
          const int j = j0 + 4 * (u >> 1), i = lane + 64 * (u & 1);
          sA[i + j * ld] = acc[u];
          if (i == j) diag0[i] = acc[u];
        }
    }
  }
  __syncthreads();

  const int nb = Wp / kCholBs;
  for (int K = 0; K < nb; ++K) {
    const int k0 = K * kCholBs, k1 = k0 + kCholBs;
    // ---- panel factorization, wave 0
    if (wave == 0) {
      const int r0 = k0 + lane, r1 = k0 + 64 + lane;
      const bool two = Wp - k0 > 64;
      double p0[kCholBs], p1[kCholBs], g0[kCholBs];
#pragma unroll
      for (int c = 0; c < kCholBs; ++c) {
        p0[c] = (c <= lane && r0 < Wp) ? sA[r0 + (k0 + c) * ld] : 0.0;
        p1[c] = (two && r1 < Wp) ? sA[r1 + (k0 + c) * ld] : 0.0;
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
        p1[c] *= y;
#pragma unroll
        for (int c2 = c + 1; c2 < kCholBs; ++c2) {
          const double l = readlane_d(p0[c], c2);  // L(k0 + c2, k0 + c)
          p0[c2] = fma(-p0[c], l, p0[c2]);
          p1[c2] = fma(-p1[c], l, p1[c2]);
        }
      }
#pragma unroll
      for (int c = 0; c < kCholBs; ++c) {
        if (c <= lane && r0 < Wp) sA[r0 + (k0 + c) * ld] = p0[c];
        if (two && r1 < Wp) sA[r1 + (k0 + c) * ld] = p1[c];
      }
      if (lane < kCholBs) dinv[k0 + lane] = yc;
      if (bad && lane == 0) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
      if (tid == 0) *D.flag = 1;
      return;
    }
    // ---- X_K = L_KK^-1 B_K for the columns col < k1 (thread per column)
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
    // ---- trailing Gram: A(i, j) -= sum_c L(i, k0 + c) L(j, k0 + c), i >= j >= k1
    const int T = Wp - k1, nbk = T >> 1;
    if (T > 0) {
      const int nblk = nbk * (nbk + 1) / 2;
      for (int e = tid; e < nblk; e += 256) {
        // packed lower-triangle block index -> (bi, bj), bi >= bj
        int bi = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
        if ((bi + 1) * (bi + 2) / 2 <= e) ++bi;
        if (bi * (bi + 1) / 2 > e) --bi;
        const int bj = e - bi * (bi + 1) / 2;
        const int i0 = k1 + 2 * bi, j0 = k1 + 2 * bj;
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
      }
    }
    __syncthreads();
    // ---- B(i, col) -= sum_c L(i, k0 + c) X(k0 + c, col), i >= k1 > col
    if (T > 0) {
      const int ncb = k1 >> 1, nblk = nbk * ncb;
      for (int e = tid; e < nblk; e += 256) {
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
      __syncthreads();
    }
  }

  // ---- outputs: R^-1 = X^T, R = L^T (upper triangular, zeros below)
  for (int k = wave; k < W; k += 4)
    for (int i = lane; i < W; i += 64) {
      D.rinv[i + (int64_t)k * W] = (i <= k) ? sX[k + i * ld] : 0.0;
      if (pass == 1) D.r1[i + (int64_t)k * W] = (i <= k) ? sA[k + i * ld] : 0.0;
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
        double acc = 0.0;
        for (int l = i; l <= k; ++l) acc = fma(sA[l + i * ld], sX[l + k * ld], acc);
        D.R[i + (int64_t)k * W] = (i <= k) ? acc : 0.0;
      }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void householder_kernel(const QrDesc* __restrict__ qrs,
                                                          int force,
                                                          unsigned long long* counter) {
  const QrDesc& D = qrs[blockIdx.x];
  const bool broke = *D.flag != 0;
  if (!force && !broke && !D.hh_direct) return;
  const int64_t n = D.n, W = D.W;
  const int64_t w = n < W ? n : W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0 && counter != nullptr) {
    atomicAdd(counter, 1ull);                              // QRs done by Householder
    if (broke && D.report_only) atomicAdd(counter + 1, 1ull);  // reported breakdowns
  }
  double* A = D.hh;
  for (int64_t e = tid; e < n * W; e += 256) A[e] = D.Y[e];
  __shared__ double red[4];
  __shared__ double s_tau, s_scal;
  __syncthreads();

  for (int64_t j = 0; j < w; ++j) {
    double part = 0.0;
    for (int64_t i = j + 1 + tid; i < n; i += 256) {
      const double x = A[i + j * n];
      part += x * x;
    }
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      const double sigma = red[0] + red[1] + red[2] + red[3];
      const double alpha = A[j + j * n];
      double tau = 0.0, scal = 0.0, beta = alpha;
      if (sigma > 0.0) {
        const double mu = sqrt(alpha * alpha + sigma);
        beta = (alpha <= 0.0) ? mu : -mu;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      A[j + j * n] = beta;
      D.tau[j] = tau;
      s_tau = tau;
      s_scal = scal;
    }
    __syncthreads();
    const double tau = s_tau;
    if (tau != 0.0) {
      const double scal = s_scal;
      for (int64_t i = j + 1 + tid; i < n; i += 256) A[i + j * n] *= scal;
      __syncthreads();
      for (int64_t c = j + 1 + wave; c < W; c += 4) {
        double dot = 0.0;
        for (int64_t i = j + 1 + lane; i < n; i += 64) dot += A[i + j * n] * A[i + c * n];
        dot = wave_sum(dot) + A[j + c * n];
        const double f = tau * dot;
        for (int64_t i = j + 1 + lane; i < n; i += 64) A[i + c * n] -= f * A[i + j * n];
        if (lane == 0) A[j + c * n] -= f;
      }
    }
    __syncthreads();
  }

  // R (w x W, ld w) with signs making diag(R) >= 0
  if (D.R != nullptr) {
    for (int64_t e = tid; e < w * W; e += 256) {
      const int64_t i = e % w, k = e / w;
      const double sgn = (A[i + i * n] < 0.0) ? -1.0 : 1.0;
      D.R[e] = (i <= k) ? sgn * A[i + k * n] : 0.0;
    }
  }
  // Q = H_0 H_1 ... H_{w-1} [I_w; 0]
  double* Q = D.Q;
  for (int64_t e = tid; e < n * w; e += 256) {
    const int64_t i = e % n, c = e / n;
    Q[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int64_t j = w - 1; j >= 0; --j) {
    const double tau = D.tau[j];
    if (tau != 0.0) {
      for (int64_t c = j + wave; c < w; c += 4) {
        double dot = 0.0;
        for (int64_t i = j + 1 + lane; i < n; i += 64) dot += A[i + j * n] * Q[i + c * n];
        dot = wave_sum(dot) + Q[j + c * n];
        const double f = tau * dot;
        for (int64_t i = j + 1 + lane; i < n; i += 64) Q[i + c * n] -= f * A[i + j * n];
        if (lane == 0) Q[j + c * n] -= f;
      }
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < n * w; e += 256) {
    const int64_t c = e / n;
    if (A[c + c * n] < 0.0) Q[e] = -Q[e];
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
                              hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  householder_kernel<<<dim3((unsigned)count), dim3(256), 0, stream>>>(
      qr, force, (unsigned long long*)fallback_counter);
  return hipGetLastError();
}

}  // namespace tsk
