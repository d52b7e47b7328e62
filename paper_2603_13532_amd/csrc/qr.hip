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

__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ qrs, int pass,
                                                   double tol) {
  const QrDesc& D = qrs[blockIdx.x];
  const int W = (int)D.W;
  const int tid = threadIdx.x;
  if (*D.flag != 0 || W > kCholMax || D.W > D.n) return;

  __shared__ double sG[kCholMax * kCholMax];
  __shared__ double sX[kCholMax * kCholMax];
  __shared__ double diag0[kCholMax];

  const int WW = W * W;
  for (int e = tid; e < WW; e += 256) {
    double acc = 0.0;
    for (int s = 0; s < D.gram_splits; ++s) acc += D.gram_part[(int64_t)s * WW + e];
    sG[e] = acc;
    const int r = e % W, c = e / W;
    sX[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = tid; i < W; i += 256) diag0[i] = sG[i + i * W];
  __syncthreads();

  bool broke = false;
  for (int j = 0; j < W; ++j) {
    const double piv = sG[j + j * W];
    if (!(piv > tol * diag0[j]) || !(diag0[j] > 0.0)) {
      broke = true;
      break;
    }
    const double rjj = sqrt(piv);
    const double inv = 1.0 / rjj;
    __syncthreads();
    // row j of R (upper storage) and row j of X = L^-1
    for (int k = j + tid; k < W; k += 256) sG[j + k * W] = (k == j) ? rjj : sG[j + k * W] * inv;
    for (int c = tid; c <= j; c += 256) sX[j + c * W] *= inv;
    __syncthreads();
    const int L = W - 1 - j;
    // trailing update of the Gram (upper triangle) and of X's rows below j
    for (int e = tid; e < L * L; e += 256) {
      const int i = j + 1 + e % L, k = j + 1 + e / L;
      if (i <= k) sG[i + k * W] -= sG[j + i * W] * sG[j + k * W];
    }
    for (int e = tid; e < L * (j + 1); e += 256) {
      const int i = j + 1 + e % L, c = e / L;
      sX[i + c * W] -= sG[j + i * W] * sX[j + c * W];
    }
    __syncthreads();
  }
  if (broke) {
    if (tid == 0) *D.flag = 1;
    return;
  }
  // R^-1 = X^T (upper triangular), zeros below the diagonal.
  for (int e = tid; e < WW; e += 256) {
    const int i = e % W, k = e / W;
    D.rinv[e] = (i <= k) ? sX[k + i * W] : 0.0;
  }
  if (pass == 1) {
    for (int e = tid; e < WW; e += 256) {
      const int i = e % W, k = e / W;
      D.r1[e] = (i <= k) ? sG[e] : 0.0;
    }
  } else if (D.R != nullptr) {
    // R = R2 R1, both upper triangular; R is w x W with w == W on this path.
    for (int e = tid; e < WW; e += 256) {
      const int i = e % W, k = e / W;
      double acc = 0.0;
      for (int l = i; l <= k; ++l) acc += sG[i + l * W] * D.r1[l + (int64_t)k * W];
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
  if (!force && *D.flag == 0) return;
  const int64_t n = D.n, W = D.W;
  const int64_t w = n < W ? n : W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0 && counter != nullptr) atomicAdd(counter, 1ull);
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

}  // namespace

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
