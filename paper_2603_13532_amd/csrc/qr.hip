// Thin QR of the sketches Y_n in FP64 (the "qr(Y_n, 'econ')" step of
// Algorithms 4/5), with diag(R) >= 0.
//
// Default path: Cholesky QR2.  The Gram matrix Y^T Y is formed by the MFMA
// GEMM (K-split over rows, partial blocks summed here in a fixed order); one
// workgroup per mode factors it in LDS, G = R^T R, while applying the same
// row operations to the identity to get L^-1 = R^-T, so that Q1 = Y R^-1 is
// one more GEMM.  The second pass repeats this on Q1 and multiplies
// R = R2 R1.  A pivot that is not positive, or smaller than tol times the
// original diagonal entry, marks the mode as breaking down.
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

// Blocked Cholesky G = L L^T (L = R^T) and L^-1, one workgroup per mode,
// both W x W matrices in LDS (leading dimension kLd).  Block size 16:
//   1. wave 0 factors the 16 x 16 diagonal block in registers, exchanging
//      columns with lane shuffles (no barrier inside the block);
//   2. each row below the block solves its 16 unknowns by substitution;
//   3. the trailing lower triangle is updated by 16-term dot products.
// L^-1 follows blockwise: diagonal blocks inverted by substitution, then
// block row I from X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ.  About 5
// barriers per block instead of one per column.
constexpr int kLd = kCholMax + 1;

__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ qrs, int pass,
                                                   double tol) {
  const QrDesc& D = qrs[blockIdx.x];
  const int W = (int)D.W;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  if (D.hh_direct || *D.flag != 0 || W > kCholMax || D.W > D.n) return;

  __shared__ double sA[kCholMax * kLd];  // Gram, then L in the lower triangle
  __shared__ double sX[kCholMax * kLd];  // L^-1 (lower triangle)
  __shared__ double diag0[kCholMax];
  __shared__ int s_broke;

  // ---- Gram = sum of the K-split partial blocks (split loop outside so that
  // each thread has many independent loads in flight)
  const int WW = W * W;
  constexpr int kPer = (kCholMax * kCholMax + 255) / 256;
  {
    double acc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
    for (int s = 0; s < D.gram_splits; ++s) {
      const double* ps = D.gram_part + (int64_t)s * WW;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int e = tid + 256 * q;
        if (e < WW) acc[q] += ps[e];
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + 256 * q;
      if (e < WW) {
        const int i = e % W, k = e / W;
        sA[i + k * kLd] = acc[q];
        sX[i + k * kLd] = 0.0;
        if (i == k) diag0[i] = acc[q];
      }
    }
  }
  if (tid == 0) s_broke = 0;
  __syncthreads();

  const int nb = (W + 15) >> 4;
  for (int K = 0; K < nb; ++K) {
    const int k0 = K * 16;
    const int bs = min(16, W - k0);
    // ---- 1. diagonal block, wave 0: lane = r + 16 qq holds A(k0+r, k0+qq+4e)
    if (tid < 64) {
      const int r = tid & 15, qq = tid >> 4;
      double a[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = qq + 4 * e;
        a[e] = (r < bs && q < bs) ? sA[(k0 + r) + (k0 + q) * kLd] : 0.0;
      }
      bool broke = false;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c < bs && !broke) {
          const int ec = c >> 2, src = 16 * (c & 3);
          const double piv = __shfl(a[ec], c + src, 64);
          if (!(piv > tol * diag0[k0 + c]) || !(diag0[k0 + c] > 0.0)) {
            broke = true;
          } else {
            const double lcc = sqrt(piv);
            const double inv = 1.0 / lcc;
            if (qq == (c & 3)) {
              if (r == c) a[ec] = lcc;
              else if (r > c) a[ec] *= inv;
            }
            const double lrc = __shfl(a[ec], r + src, 64);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int q = qq + 4 * e;
              const double lqc = __shfl(a[ec], q + src, 64);
              if (q > c && q <= r) a[e] -= lrc * lqc;
            }
          }
        }
      }
      if (broke) {
        if (tid == 0) s_broke = 1;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = qq + 4 * e;
          if (r < bs && q < bs && q <= r) sA[(k0 + r) + (k0 + q) * kLd] = a[e];
        }
      }
    }
    __syncthreads();
    if (s_broke) {
      if (tid == 0) *D.flag = 1;
      return;
    }
    // ---- 2. panel: rows below the block, x L_KK^T = a by substitution
    const int i0 = k0 + bs;
    for (int i = i0 + tid; i < W; i += 256) {
      double x[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c < bs) {
          double v = sA[i + (k0 + c) * kLd];
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (q < c) v -= x[q] * sA[(k0 + c) + (k0 + q) * kLd];
          x[c] = v / sA[(k0 + c) + (k0 + c) * kLd];
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < bs) sA[i + (k0 + c) * kLd] = x[c];
    }
    __syncthreads();
    // ---- 3. trailing lower triangle: A(i,j) -= sum_c L(i,k0+c) L(j,k0+c), i >= j >= i0
    for (int j = i0 + ty; j < W; j += 16)
      for (int i = j + tx; i < W; i += 16) {
        double v = sA[i + j * kLd];
        for (int c = 0; c < bs; ++c) v -= sA[i + (k0 + c) * kLd] * sA[j + (k0 + c) * kLd];
        sA[i + j * kLd] = v;
      }
    __syncthreads();
  }

  // ---- L^-1: diagonal blocks by substitution, thread per (block, column)
  if (tid < nb * 16) {
    const int I = tid >> 4, c = tid & 15;
    const int k0 = I * 16, bs = min(16, W - k0);
    if (c < bs) {
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double v = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q >= c && q < r) v -= sA[(k0 + r) + (k0 + q) * kLd] * x[q];
        x[r] = (r >= c && r < bs) ? v / sA[(k0 + r) + (k0 + r) * kLd] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (r < bs) sX[(k0 + r) + (k0 + c) * kLd] = x[r];
    }
  }
  __syncthreads();
  // ---- off-diagonal blocks, block row by block row
  for (int I = 1; I < nb; ++I) {
    const int r0 = I * 16, bsI = min(16, W - r0);
    // T_IJ = sum_{K=J}^{I-1} L_IK X_KJ for every J < I, stored in X_IJ's place
    for (int e = tid; e < I * 256; e += 256) {
      const int J = e >> 8, rc = e & 255, r = rc & 15, c = rc >> 4;
      if (r >= bsI) continue;
      const int col = J * 16 + c;
      double v = 0.0;
      for (int q = J * 16; q < r0; ++q) v += sA[(r0 + r) + q * kLd] * sX[q + col * kLd];
      sX[(r0 + r) + col * kLd] = v;
    }
    __syncthreads();
    // X_IJ = -X_II T_IJ, thread per column of the block row
    for (int col = tid; col < r0; col += 256) {
      double tcol[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) tcol[q] = (q < bsI) ? sX[(r0 + q) + col * kLd] : 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r < bsI) {
          double v = 0.0;
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (q <= r) v += sX[(r0 + r) + (r0 + q) * kLd] * tcol[q];
          sX[(r0 + r) + col * kLd] = -v;
        }
      }
    }
    __syncthreads();
  }

  // ---- outputs: R^-1 = X^T, R = L^T (upper triangular, zeros below)
  for (int e = tid; e < WW; e += 256) {
    const int i = e % W, k = e / W;
    D.rinv[e] = (i <= k) ? sX[k + i * kLd] : 0.0;
    if (pass == 1) D.r1[e] = (i <= k) ? sA[k + i * kLd] : 0.0;
  }
  if (pass == 2 && D.R != nullptr) {
    // R = R2 R1 with R2(i,l) = L2(l,i); w == W on this path
    for (int e = tid; e < WW; e += 256) {
      const int i = e % W, k = e / W;
      double acc = 0.0;
      for (int l = i; l <= k; ++l) acc += sA[l + i * kLd] * D.r1[l + (int64_t)k * W];
      D.R[e] = (i <= k) ? acc : 0.0;
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

hipError_t launch_chol(const QrDesc* qr, int count, int pass, double tol, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  chol_kernel<<<dim3((unsigned)count), dim3(256), 0, stream>>>(qr, pass, tol);
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
