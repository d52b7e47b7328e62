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

// One workgroup per mode, 256 threads as a 16 x 16 grid.  Thread (ty, tx)
// keeps in registers the Gram entries G(i, k) and the entries X(i, k) of
// X = L^-1 = R^-T for i = ty (mod 16), k = tx (mod 16): at most 6 x 6 of
// each for W <= 96.  Elimination step j needs only row j of G and of X:
// its owners publish it to an LDS buffer (double-buffered by the parity of
// j), one barrier, then every thread updates its own entries.  X is built
// by applying each elimination step to the identity.
constexpr int kOwn = kCholMax / 16;

__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ qrs, int pass,
                                                   double tol) {
  const QrDesc& D = qrs[blockIdx.x];
  const int W = (int)D.W;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  if (*D.flag != 0 || W > kCholMax || D.W > D.n) return;

  __shared__ double rowG[2][kCholMax];
  __shared__ double rowX[2][kCholMax];
  __shared__ double diag0[kCholMax];
  __shared__ double sR2[kCholMax * kCholMax];  // pass 2: R2 for the product R2 R1

  double g[kOwn][kOwn], x[kOwn][kOwn];
  const int WW = W * W;
  const double* part = D.gram_part;
  const int ns = D.gram_splits;
#pragma unroll
  for (int a = 0; a < kOwn; ++a)
#pragma unroll
    for (int b = 0; b < kOwn; ++b) g[a][b] = 0.0;
  // split loop outside, owned entries inside: 36 independent loads per split
  for (int s = 0; s < ns; ++s) {
    const double* ps = part + (int64_t)s * WW;
#pragma unroll
    for (int a = 0; a < kOwn; ++a)
#pragma unroll
      for (int b = 0; b < kOwn; ++b) {
        const int i = ty + 16 * a, k = tx + 16 * b;
        if (i < W && k < W) g[a][b] += ps[i + k * W];
      }
  }
#pragma unroll
  for (int a = 0; a < kOwn; ++a)
#pragma unroll
    for (int b = 0; b < kOwn; ++b) {
      const int i = ty + 16 * a, k = tx + 16 * b;
      x[a][b] = (i == k && i < W) ? 1.0 : 0.0;
      if (i == k && i < W) diag0[i] = g[a][b];
    }
  __syncthreads();
  bool broke = false;
  for (int j = 0; j < W; ++j) {
    const int buf = j & 1;
    const int aj = j >> 4;  // slot of row j among its owners' rows
    if (ty == (j & 15)) {
#pragma unroll
      for (int a = 0; a < kOwn; ++a)
        if (a == aj) {
#pragma unroll
          for (int b = 0; b < kOwn; ++b) {
            const int k = tx + 16 * b;
            if (k < W) {
              rowG[buf][k] = g[a][b];
              rowX[buf][k] = x[a][b];
            }
          }
        }
    }
    __syncthreads();
    const double piv = rowG[buf][j];
    if (!(piv > tol * diag0[j]) || !(diag0[j] > 0.0)) {
      broke = true;
      break;
    }
    const double inv = 1.0 / sqrt(piv);
    const double ipiv = inv * inv;
    double gi[kOwn], gk[kOwn], xk[kOwn];
#pragma unroll
    for (int a = 0; a < kOwn; ++a) {
      const int i = ty + 16 * a;
      gi[a] = (i < W) ? rowG[buf][i] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < kOwn; ++b) {
      const int k = tx + 16 * b;
      gk[b] = (k < W) ? rowG[buf][k] : 0.0;
      // X(j, c) for c = k: Z(j, c) * inv for c < j, inv for c == j, 0 beyond
      xk[b] = (k < j) ? rowX[buf][k] * inv : ((k == j) ? inv : 0.0);
    }
#pragma unroll
    for (int a = 0; a < kOwn; ++a) {
      const int i = ty + 16 * a;
#pragma unroll
      for (int b = 0; b < kOwn; ++b) {
        const int k = tx + 16 * b;
        if (i > j && k >= i) g[a][b] -= gi[a] * gk[b] * ipiv;   // trailing update, upper part
        if (i > j && k <= j) x[a][b] -= gi[a] * inv * xk[b];     // X rows below j
        if (i == j) {
          if (k >= j) g[a][b] *= inv;                           // row j of R
          if (k <= j) x[a][b] = xk[b];                          // row j of X final
        }
      }
    }
  }
  if (broke) {
    if (tid == 0) *D.flag = 1;
    return;
  }
  // R^-1 = X^T (upper triangular); R in the upper triangle of g
#pragma unroll
  for (int a = 0; a < kOwn; ++a)
#pragma unroll
    for (int b = 0; b < kOwn; ++b) {
      const int i = ty + 16 * a, k = tx + 16 * b;
      if (i < W && k < W) {
        D.rinv[k + (int64_t)i * W] = (k <= i) ? x[a][b] : 0.0;
        const double r = (i <= k) ? g[a][b] : 0.0;
        if (pass == 1) D.r1[i + (int64_t)k * W] = r;
        else sR2[i + k * W] = r;
      }
    }
  if (pass == 2 && D.R != nullptr) {
    __syncthreads();
    // R = R2 R1 (w == W on this path)
    for (int e = tid; e < WW; e += 256) {
      const int i = e % W, k = e / W;
      double acc = 0.0;
      for (int l = i; l <= k; ++l) acc += sR2[i + l * W] * D.r1[l + (int64_t)k * W];
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
