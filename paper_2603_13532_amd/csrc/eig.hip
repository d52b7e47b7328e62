// Symmetric eigendecomposition of the mode Gram matrices of Stage 4
// (ST-HOSVD of the projected core, Algorithms 4/5 Stage 4, with the rank rule
// of Algorithm 2 phase 2), and of the weighted Gram matrices of Stage 1
// (Algorithm 3): one workgroup per matrix, the matrix and its eigenvectors
// in LDS.
//
// Cyclic two-sided Jacobi with the round-robin parallel ordering: a sweep is
// Wp - 1 rounds, each round pairs every index with another (Wp = W rounded
// up to even; the extra index is an identity row/column), so the W/2
// rotations of a round touch disjoint rows and columns.  A round computes
// the rotations (one lane per pair, Golub and Van Loan's symmetric 2 x 2
// Schur form), then every 2 x 2 block (row pair, column pair) of A is
// replaced by J1^T A J2 and every row of V by its row times J, in one pass.
// A pair is left alone once |a_pq| <= tol sqrt(|a_pp a_qq|), or once both
// of its diagonal entries and a_pq are at the rounding level of the largest
// diagonal entry d (|a_pq| <= tol d and a_pp, a_qq <= 64 tol d); the
// decomposition has converged when a sweep rotates no pair.  The relative
// test gives a positive semidefinite matrix's small eigenvalues (and their
// eigenvectors) relative accuracy; the second test stops the rotations
// inside a rank-deficient Gram's near-null block, whose entries are the
// rounding noise of the Gram's formation and would otherwise keep sweeps
// going, while every pair with a diagonal entry above that level (a kept
// direction) is still rotated.  Eigenvalues are then sorted in decreasing order (rank of each
// by counting), with their eigenvectors, and the rank rule is applied:
// r = the smallest r >= 1 whose discarded eigenvalue sum is <= theta.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace tsk {

namespace {

constexpr int kEigThreads = 512;
constexpr int kEigMaxSweeps = 40;

// Position of round-robin slot i in round r (slot 0 stays put, the others
// rotate): slot k is paired with slot Wp - 1 - k.
__device__ __forceinline__ int rr_index(int i, int r, int Wp) {
  return i == 0 ? 0 : 1 + (i - 1 + r) % (Wp - 1);
}

// GLOBAL: the matrix and its eigenvectors live in the job's workspace (A at
// J.work, Wp x Wp each) instead of LDS, for widths above kEigMaxW; the
// rotation parameters stay in LDS.
// NT threads (64 for widths up to 16, whose rounds hold at most 64 block
// updates: one wave, so the barriers cost nothing; else 512).
template <bool GLOBAL, int NT>
__global__ __launch_bounds__(NT) void jacobi_eig_kernel(const EigJob* __restrict__ jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int W = J.W;
  const int Wp = W + (W & 1);
  const int half = Wp / 2;
  const int t = threadIdx.x;
  extern __shared__ __align__(16) unsigned char eig_dyn[];
  double* A = GLOBAL ? J.work : (double*)eig_dyn;  // Wp x Wp, column-major (ld Wp)
  double* V = A + (size_t)Wp * Wp;                 // Wp x Wp
  double* cs = GLOBAL ? (double*)eig_dyn : V + (size_t)Wp * Wp;  // c, s per pair
  int* pr = (int*)(cs + 2 * half);  // p, q per pair
  __shared__ int s_rotated;

  __shared__ double s_dmax[NT / 64];
  for (int e = t; e < Wp * Wp; e += NT) {
    const int i = e % Wp, j = e / Wp;
    A[e] = (i < W && j < W) ? J.C[i + (int64_t)J.ldc * j] : 0.0;
    if (!J.values_only) V[e] = i == j ? 1.0 : 0.0;
  }
  // the largest diagonal entry (>= every |a_pq| of a positive semidefinite
  // matrix), the scale of the Gram's rounding noise
  double dm = 0.0;
  for (int i = t; i < W; i += NT) dm = fmax(dm, fabs(J.C[i + (int64_t)J.ldc * i]));
  for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off));
  if ((t & 63) == 0) s_dmax[t >> 6] = dm;
  __syncthreads();
  double floor_apq = 0.0;
  for (int w = 0; w < NT / 64; ++w) floor_apq = fmax(floor_apq, s_dmax[w]);
  floor_apq *= J.tol;

  for (int sweep = 0; sweep < kEigMaxSweeps; ++sweep) {
    if (t == 0) s_rotated = 0;
    __syncthreads();
    for (int r = 0; r < Wp - 1; ++r) {
      if (t < half) {
        int p = rr_index(t, r, Wp), q = rr_index(Wp - 1 - t, r, Wp);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        if (q < W) {
          const double app = A[p + Wp * p], aqq = A[q + Wp * q], apq = A[p + Wp * q];
          if (fabs(apq) > J.tol * sqrt(fabs(app * aqq)) &&
              (fabs(apq) > floor_apq || fmax(fabs(app), fabs(aqq)) > 64.0 * floor_apq) &&
              fabs(apq) > 1e-300) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            s_rotated = 1;
          }
        }
        cs[2 * t] = c;
        cs[2 * t + 1] = s;
        pr[2 * t] = p;
        pr[2 * t + 1] = q;
      }
      __syncthreads();
      // A <- J^T A J, one 2 x 2 block (row pair k1, column pair k2) per item
      for (int e = t; e < half * half; e += NT) {
        const int k1 = e % half, k2 = e / half;
        const int p1 = pr[2 * k1], q1 = pr[2 * k1 + 1], p2 = pr[2 * k2], q2 = pr[2 * k2 + 1];
        const double c1 = cs[2 * k1], s1 = cs[2 * k1 + 1], c2 = cs[2 * k2], s2 = cs[2 * k2 + 1];
        const double a = A[p1 + Wp * p2], b = A[p1 + Wp * q2];
        const double c = A[q1 + Wp * p2], d = A[q1 + Wp * q2];
        // rows: (p, q) <- (c1 p - s1 q, s1 p + c1 q)
        const double ra = c1 * a - s1 * c, rb = c1 * b - s1 * d;
        const double rc = s1 * a + c1 * c, rd = s1 * b + c1 * d;
        // columns: (p, q) <- (c2 p - s2 q, s2 p + c2 q)
        // a diagonal block's off-diagonal pair is what the rotation annihilates
        const bool diag = k1 == k2 && s1 != 0.0;
        A[p1 + Wp * p2] = c2 * ra - s2 * rb;
        A[p1 + Wp * q2] = diag ? 0.0 : s2 * ra + c2 * rb;
        A[q1 + Wp * p2] = diag ? 0.0 : c2 * rc - s2 * rd;
        A[q1 + Wp * q2] = s2 * rc + c2 * rd;
      }
      // V <- V J: row i, pair k
      for (int e = t; e < (J.values_only ? 0 : Wp * half); e += NT) {
        const int i = e % Wp, k = e / Wp;
        const int p = pr[2 * k], q = pr[2 * k + 1];
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double vp = V[i + Wp * p], vq = V[i + Wp * q];
        V[i + Wp * p] = c * vp - s * vq;
        V[i + Wp * q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (s_rotated == 0) break;
    __syncthreads();
  }

  // eigenvalues (clipped at zero when asked), their order, and the rank
  // rule; sorted eigenvalues go to the (now free) rotation scratch (Wp
  // doubles), every thread handling the eigenvalues t, t + NT, ...
  double* sorted = cs;
  __syncthreads();
  for (int i = t; i < W; i += NT) {
    double lam = A[i + Wp * i];
    if (J.clip) lam = fmax(lam, 0.0);
    int pos = 0;
    for (int j = 0; j < W; ++j) {
      double lj = A[j + Wp * j];
      if (J.clip) lj = fmax(lj, 0.0);
      pos += (lj > lam || (lj == lam && j < i)) ? 1 : 0;
    }
    sorted[pos] = lam;
    J.lam[pos] = lam;
  }
  for (int e = t; e < (J.values_only ? 0 : W * W); e += NT) {
    const int i = e % W, j = e / W;  // row i of eigenvector j
    int pj = 0;
    double lj = A[j + Wp * j];
    if (J.clip) lj = fmax(lj, 0.0);
    for (int k = 0; k < W; ++k) {
      double lk = A[k + Wp * k];
      if (J.clip) lk = fmax(lk, 0.0);
      pj += (lk > lj || (lk == lj && k < j)) ? 1 : 0;
    }
    J.V[i + (int64_t)J.ldv * pj] = V[i + Wp * j];
  }
  __syncthreads();
  if (J.rank != nullptr && t == 0) {
    double theta;
    if (J.set_theta) {
      double tr = 0.0;
      for (int j = 0; j < W; ++j) tr += sorted[j];
      theta = J.theta_scale * tr;
      *J.theta = theta;
    } else {
      theta = *J.theta;
    }
    // smallest r >= 1 with sum_{i >= r} lam_i <= theta (i 0-based) 
    double tail = 0.0;
    int r = W;
    for (int i = W - 1; i >= 1; --i) {
      tail += sorted[i];
      if (tail <= theta) r = i;
      else break;
    }
    *J.rank = r;
  }
}

// Eigenvalues only, for matrices too large for the LDS Jacobi: one
// workgroup reduces the symmetric W x W matrix (a workspace copy, lower
// triangle used and updated) to tridiagonal form by Householder reflectors,
// A <- H A H with H = I - tau v v^T: the reflector from the column below the
// diagonal, p = tau A v from the lower triangle (each wave walks columns,
// lanes rows, so loads coalesce; the transposed half of the product is a
// wave reduction per column), w = p - (tau/2)(p^T v) v, and A -= v w^T +
// w v^T on the lower triangle.  The eigenvalues of the tridiagonal matrix
// are then found by bisection on Sturm counts, one thread per eigenvalue
// (the k-th largest directly, so no sort is needed), and the rank rule is
// applied as in the Jacobi kernel.
constexpr int kTriThreads = 1024;

__device__ double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += red[i];
  return tot;
}

// number of eigenvalues of the tridiagonal (d, e) below x
__device__ int sturm_below(const double* d, const double* e, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__global__ __launch_bounds__(kTriThreads) void tridiag_eig_kernel(const EigJob* __restrict__ jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int W = J.W;
  double* A = J.V;  // W x W workspace, ld ldv
  const int64_t ld = J.ldv;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = kTriThreads / 64;
  extern __shared__ __align__(16) unsigned char tri_dyn[];
  double* v = (double*)tri_dyn;  // W
  double* p = v + W;             // W
  double* dg = p + W;            // W
  double* of = dg + W;           // W
  __shared__ double red[kTriThreads / 64];

  // working copy of the lower triangle
  for (int j = wave; j < W; j += nw)
    for (int i = j + lane; i < W; i += 64) A[i + ld * j] = J.C[i + J.ldc * j];
  __syncthreads();

  for (int k = 0; k + 2 < W; ++k) {
    const int m = W - k - 1;  // length of the column below the diagonal
    double part = 0.0;
    for (int i = t; i < m; i += kTriThreads) {
      const double x = A[(k + 1 + i) + ld * k];
      v[i] = x;
      part += x * x;
    }
    const double nrm2 = block_sum(part, red);
    const double x0 = v[0];
    double tau = 0.0, alpha = x0;
    if (nrm2 > 0.0) {
      alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
      const double v0 = x0 - alpha;
      const double vn2 = nrm2 - x0 * x0 + v0 * v0;
      tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      if (tau == 0.0) alpha = x0;
    }
    if (t == 0) {
      dg[k] = A[k + ld * k];
      of[k] = tau == 0.0 ? x0 : alpha;
    }
    __syncthreads();
    if (t == 0 && tau != 0.0) v[0] = x0 - alpha;
    for (int i = t; i < m; i += kTriThreads) p[i] = 0.0;
    __syncthreads();
    if (tau != 0.0) {
      // p = tau * A22 v, A22 = A[k+1:, k+1:] from its lower triangle: wave
      // `wave` takes columns j = wave, wave + nw, ...; the column's entries
      // below the diagonal add A_ij v_j to p_i (LDS atomics) and their
      // transposes A_ij v_i to p_j (wave reduction)
      for (int j = wave; j < m; j += nw) {
        const double vj = v[j];
        double colsum = 0.0;
        for (int i = j + lane; i < m; i += 64) {
          const double a = A[(k + 1 + i) + ld * (k + 1 + j)];
          if (i != j) {
            atomicAdd(&p[i], a * vj);
            colsum += a * v[i];
          } else {
            colsum += a * vj;
          }
        }
        for (int o = 32; o > 0; o >>= 1) colsum += __shfl_xor(colsum, o);
        if (lane == 0) atomicAdd(&p[j], colsum);
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = t; i < m; i += kTriThreads) {
        p[i] *= tau;
        pv += p[i] * v[i];
      }
      const double K = 0.5 * tau * block_sum(pv, red);
      for (int i = t; i < m; i += kTriThreads) p[i] -= K * v[i];
      __syncthreads();
      // A22 -= v w^T + w v^T on the lower triangle
      for (int j = wave; j < m; j += nw) {
        const double vj = v[j], wj = p[j];
        for (int i = j + lane; i < m; i += 64)
          A[(k + 1 + i) + ld * (k + 1 + j)] -= v[i] * wj + p[i] * vj;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (W >= 2) {
      dg[W - 2] = A[(W - 2) + ld * (W - 2)];
      of[W - 2] = A[(W - 1) + ld * (W - 2)];
    }
    dg[W - 1] = A[(W - 1) + ld * (W - 1)];
  }
  __syncthreads();
  // Gershgorin interval and the pivot floor
  // (pivots below the LAPACK floor safmin * max(1, max e_i^2) count as
  // negative)
  double lo = 1e300, hi = -1e300, e2 = 1.0;
  for (int i = 0; i < W; ++i) {
    const double r = (i > 0 ? fabs(of[i - 1]) : 0.0) + (i + 1 < W ? fabs(of[i]) : 0.0);
    lo = fmin(lo, dg[i] - r);
    hi = fmax(hi, dg[i] + r);
    if (i + 1 < W) e2 = fmax(e2, of[i] * of[i]);
  }
  const double pivmin = 2.2250738585072014e-308 * e2;
  const double span = fmax(hi - lo, 1e-300);
  lo -= 1e-14 * span + 1e-300;
  hi += 1e-14 * span + 1e-300;
  // the k-th largest eigenvalue: the smallest x with at least W - k below it
  double* sorted = v;  // v is free now
  __syncthreads();
  for (int kk = t; kk < W; kk += kTriThreads) {
    const int need = W - kk;
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (sturm_below(dg, of, W, mid, pivmin) >= need) b = mid; else a = mid;
    }
    double lam = 0.5 * (a + b);
    if (J.clip) lam = fmax(lam, 0.0);
    sorted[kk] = lam;
    J.lam[kk] = lam;
  }
  __syncthreads();
  if (J.rank != nullptr && t == 0) {
    double theta;
    if (J.set_theta) {
      double tr = 0.0;
      for (int j = 0; j < W; ++j) tr += sorted[j];
      theta = J.theta_scale * tr;
      *J.theta = theta;
    } else {
      theta = *J.theta;
    }
    double tail = 0.0;
    int r = W;
    for (int i = W - 1; i >= 1; --i) {
      tail += sorted[i];
      if (tail <= theta) r = i;
      else break;
    }
    *J.rank = r;
  }
}

}  // namespace

hipError_t launch_tridiag_eig(const EigJob* jobs, int count, int wmax, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (wmax < 1 || wmax > kTriMaxW) return hipErrorInvalidValue;
  const size_t lds = (size_t)4 * wmax * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)tridiag_eig_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(4 * kTriMaxW * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  tridiag_eig_kernel<<<dim3((unsigned)count), dim3(kTriThreads), lds, stream>>>(jobs);
  return hipGetLastError();
}

size_t jacobi_eig_lds(int wmax) {
  const int Wp = wmax + (wmax & 1);
  return (size_t)(2 * Wp * Wp + Wp) * sizeof(double) + (size_t)Wp * sizeof(int);
}

hipError_t launch_jacobi_eig(const EigJob* jobs, int count, int wmax, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (wmax < 1 || wmax > kEigMaxWGlobal) return hipErrorInvalidValue;
  if (wmax > kEigMaxW) {
    const int Wp = wmax + (wmax & 1);
    const size_t lds = (size_t)Wp * sizeof(double) + (size_t)Wp * sizeof(int);
    jacobi_eig_kernel<true, kEigThreads><<<dim3((unsigned)count), dim3(kEigThreads), lds, stream>>>(jobs);
    return hipGetLastError();
  }
  const size_t lds = jacobi_eig_lds(wmax);
  if (wmax <= 16) {
    jacobi_eig_kernel<false, 64><<<dim3((unsigned)count), dim3(64), lds, stream>>>(jobs);
    return hipGetLastError();
  }
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)jacobi_eig_kernel<false, kEigThreads>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)jacobi_eig_lds(kEigMaxW));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  jacobi_eig_kernel<false, kEigThreads><<<dim3((unsigned)count), dim3(kEigThreads), lds, stream>>>(jobs);
  return hipGetLastError();
}

}  // namespace tsk
