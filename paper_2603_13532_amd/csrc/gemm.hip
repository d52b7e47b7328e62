// Contraction kernels of the hot path, all on the MFMA tile engine:
//   * gemm_kernel: grouped, batched, K-segmented GEMM.  Serves the factor
//     sketches P = U^T Omega (Algorithms 4/5, M_j lines), the term expansion
//     Y_n = sum_i c_i U_n^(i) V^(i)_(n) with the term sum as the K dimension,
//     the Kronecker-sketch TTM chains, the Gram and basis products of the
//     Cholesky QR, W = Q^T U and the TTMs of the core projection (Section 3.3).
//   * krp_kernel: the KRP core sketch V_(n) = G_(n) (M_d (.) ... (.) M_1
//     skipping n) (eq. for the KRP sketched unfolding), with the Khatri-Rao
//     rows generated on the fly from the small M_k = U_k^T Omega_k and staged
//     through LDS, so neither the KRP nor the unfolding is ever stored.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "mfma_engine.hpp"

namespace tsk {

namespace {

template <typename D>
__device__ __forceinline__ int find_desc(const D* __restrict__ descs, int ndesc, int64_t tile) {
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int P, typename OutT>
__device__ __forceinline__ void store_tile(typename PT<P>::acc_t (&acc)[2][2], OutT* __restrict__ C,
                                           int64_t ldc, int M, int N, int m0, int n0, bool accum,
                                           int lane, int wm, int wn) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + acc_col(wn, j, lane);
      if (col >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + acc_row<P>(wm, i, lane, v);
        if (row < M) {
          OutT* p = C + (int64_t)row + (int64_t)col * ldc;
          if (accum) *p = (OutT)((double)*p + (double)acc[i][j][v]);
          else *p = (OutT)acc[i][j][v];
        }
      }
    }
}

// ROLE only names the launch (one symbol per step of the method, so that
// kernel traces separate them); the code is the same for every role.
template <int P, int ROLE>
__global__ __launch_bounds__(NTHREADS) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                        int ndesc,
                                                        const GemmSeg* __restrict__ segs) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  constexpr int BK = PT<P>::BK;
  constexpr int PER = Stage<P>::PER_THREAD;
  __shared__ typename Lds<P>::type s;

  const int64_t tile = blockIdx.x;
  const GemmDesc& D = descs[find_desc(descs, ndesc, tile)];
  int64_t local = tile - D.tile_begin;
  const int splits = D.splits;
  const int split = (int)(local % splits);
  local /= splits;
  const int tm = (int)(local % D.tiles_m);
  local /= D.tiles_m;
  const int tn = (int)(local % D.tiles_n);
  const int64_t b = local / D.tiles_n;
  const int M = D.M, N = D.N;
  const int m0 = tm * TILE, n0 = tn * TILE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;

  acc_t acc[2][2];
  acc_zero<P>(acc);
  in_t ra[PER], rb[PER];
  int g = 0;
  for (int si = 0; si < D.seg_count; ++si) {
    const GemmSeg& S = segs[D.seg_begin + si];
    const in_t* __restrict__ A = (const in_t*)S.A + b * S.strideA;
    const in_t* __restrict__ B = (const in_t*)S.B + b * S.strideB;
    const bool a_xc = (S.a_sx == 1), b_xc = (S.b_sx == 1);
    const int K = S.K;
    const in_t alpha = (in_t)S.alpha;
    const int nkt = (K + BK - 1) / BK;
    for (int kt = 0; kt < nkt; ++kt, ++g) {
      if (g % splits != split) continue;
      const int k0 = kt * BK;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        int x, k;
        PanelMap<P>::xk(a_xc, t, j, x, k);
        const int mm = m0 + x, kk = k0 + k;
        ra[j] = (mm < M && kk < K) ? A[(int64_t)mm * S.a_sx + (int64_t)kk * S.a_sk] * alpha
                                   : (in_t)0;
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        int x, k;
        PanelMap<P>::xk(b_xc, t, j, x, k);
        const int nn = n0 + x, kk = k0 + k;
        rb[j] = (nn < N && kk < K) ? B[(int64_t)nn * S.b_sx + (int64_t)kk * S.b_sk] : (in_t)0;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        int x, k;
        PanelMap<P>::xk(a_xc, t, j, x, k);
        lds_put<P>(s, 0, x, k, ra[j]);
        PanelMap<P>::xk(b_xc, t, j, x, k);
        lds_put<P>(s, 1, x, k, rb[j]);
      }
      __syncthreads();
      mma_tile<P>(s, acc, lane, wm, wn);
    }
  }

  const bool accum = (splits == 1) && D.beta;
  const int64_t off = b * D.strideC + (int64_t)split * D.strideSplit;
  if (D.c_f64)
    store_tile<P, double>(acc, (double*)D.C + off, D.ldc, M, N, m0, n0, accum, lane, wm, wn);
  else
    store_tile<P, float>(acc, (float*)D.C + off, D.ldc, M, N, m0, n0, accum, lane, wm, wn);
}

// KRP core sketch: rows a of G_(n) against Khatri-Rao columns t, K = c over
// the other modes, first remaining mode fastest (unfolding index equation).
template <int P>
__global__ __launch_bounds__(NTHREADS) void krp_kernel(const KrpDesc* __restrict__ descs,
                                                       int ndesc) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  constexpr int BK = PT<P>::BK;
  constexpr int PER = Stage<P>::PER_THREAD;
  __shared__ typename Lds<P>::type s;

  const int64_t tile = blockIdx.x;
  const KrpDesc& D = descs[find_desc(descs, ndesc, tile)];
  int64_t local = tile - D.tile_begin;
  const int splits = D.splits;
  const int split = (int)(local % splits);
  local /= splits;
  const int tm = (int)(local % D.tiles_m);
  const int tn = (int)(local / D.tiles_m);
  const int order = D.order, n = D.mode, m = D.m;
  const int rn = D.r[n];
  const int m0 = tm * TILE, n0 = tn * TILE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;
  const in_t* __restrict__ G = (const in_t*)D.G;
  const in_t alpha = (in_t)D.alpha;

  int64_t st[kMaxOrder];
  int rk[kMaxOrder];
  const in_t* Pk[kMaxOrder];
  {
    int64_t acc_st = 1;
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k) {
      rk[k] = (k < order) ? D.r[k] : 1;
      st[k] = acc_st;
      acc_st *= rk[k];
      Pk[k] = (const in_t*)D.P[k];
    }
  }
  const int64_t stn = st[n];

  acc_t acc[2][2];
  acc_zero<P>(acc);
  in_t ra[PER], rb[PER];
  const int64_t Kc = D.Kc;
  const int64_t nkt = (Kc + BK - 1) / BK;
  const int kq = t % BK;
  for (int64_t kt = split; kt < nkt; kt += splits) {
    const int64_t c = kt * BK + kq;
    const bool valid = c < Kc;
    int dig[kMaxOrder];
    int64_t offg = 0;
    {
      int64_t rem = valid ? c : 0;
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) {
        dig[k] = 0;
        if (k < order && k != n) {
          const int64_t q = rem / rk[k];
          dig[k] = (int)(rem - q * rk[k]);
          rem = q;
          offg += (int64_t)dig[k] * st[k];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int x = t / BK + (NTHREADS / BK) * j;
      const int a = m0 + x;
      ra[j] = (valid && a < rn) ? G[(int64_t)a * stn + offg] * alpha : (in_t)0;
      const int tt = n0 + x;
      in_t prod = (in_t)0;
      if (valid && tt < m) {
        prod = (in_t)1;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k)
          if (k < order && k != n) prod *= Pk[k][dig[k] + (int64_t)tt * rk[k]];
      }
      rb[j] = prod;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int x = t / BK + (NTHREADS / BK) * j;
      lds_put<P>(s, 0, x, kq, ra[j]);
      lds_put<P>(s, 1, x, kq, rb[j]);
    }
    __syncthreads();
    mma_tile<P>(s, acc, lane, wm, wn);
  }
  const int64_t off = (int64_t)split * D.strideSplit;
  if constexpr (P == P_FP64)
    store_tile<P, double>(acc, (double*)D.V + off, rn, rn, m, m0, n0, false, lane, wm, wn);
  else
    store_tile<P, float>(acc, (float*)D.V + off, rn, rn, m, m0, n0, false, lane, wm, wn);
}

__global__ __launch_bounds__(256) void reduce_kernel(const ReduceJob* __restrict__ jobs) {
  const ReduceJob& J = jobs[blockIdx.y];
  const int64_t total = J.rows * J.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % J.rows, c = e / J.rows;
    double acc = 0.0;
    for (int s = 0; s < J.parts; ++s) {
      const int64_t idx = (int64_t)s * J.stride_part + r + c * J.ld_part;
      acc += J.part_f64 ? ((const double*)J.part)[idx] : (double)((const float*)J.part)[idx];
    }
    const int64_t o = r + c * J.ld_out;
    if (J.out_f64) {
      double* p = (double*)J.out;
      p[o] = J.beta ? p[o] + acc : acc;
    } else {
      float* p = (float*)J.out;
      p[o] = (float)(J.beta ? (double)p[o] + acc : acc);
    }
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const CopyJob* __restrict__ jobs) {
  const CopyJob& J = jobs[blockIdx.y];
  const int64_t total = J.rows * J.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % J.rows, c = e / J.rows;
    const int64_t is = r + c * J.ld_src, id = r + c * J.ld_dst;
    const double v = J.src_f64 ? ((const double*)J.src)[is] : (double)((const float*)J.src)[is];
    if (J.dst_f64) ((double*)J.dst)[id] = v;
    else ((float*)J.dst)[id] = (float)v;
  }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t count, int32_t value) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = value;
}

}  // namespace

template <int P>
hipError_t launch_gemm_p(int role, dim3 grid, const GemmDesc* descs, int ndesc,
                         const GemmSeg* segs, hipStream_t stream) {
  const dim3 block(NTHREADS);
  switch (role) {
    case R_FACTOR_SKETCH: gemm_kernel<P, R_FACTOR_SKETCH><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    case R_KRON_TTM: gemm_kernel<P, R_KRON_TTM><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    case R_TERM_EXPAND: gemm_kernel<P, R_TERM_EXPAND><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    case R_PROJ_W: gemm_kernel<P, R_PROJ_W><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    case R_PROJ_TTM: gemm_kernel<P, R_PROJ_TTM><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    case R_PROJ_FINAL: gemm_kernel<P, R_PROJ_FINAL><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
    default: gemm_kernel<P, R_OTHER><<<grid, block, 0, stream>>>(descs, ndesc, segs); break;
  }
  return hipGetLastError();
}

hipError_t launch_gemm(int prec, int role, const GemmDesc* descs, int ndesc, const GemmSeg* segs,
                       int64_t total_tiles, hipStream_t stream) {
  if (ndesc <= 0 || total_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_tiles), block(NTHREADS);
  switch (prec) {
    case P_FP64:
      // the QR products are FP64 only
      if (role == R_QR_GRAM) {
        gemm_kernel<P_FP64, R_QR_GRAM><<<grid, block, 0, stream>>>(descs, ndesc, segs);
        return hipGetLastError();
      }
      if (role == R_QR_BASIS) {
        gemm_kernel<P_FP64, R_QR_BASIS><<<grid, block, 0, stream>>>(descs, ndesc, segs);
        return hipGetLastError();
      }
      return launch_gemm_p<P_FP64>(role, grid, descs, ndesc, segs, stream);
    case P_FP32: return launch_gemm_p<P_FP32>(role, grid, descs, ndesc, segs, stream);
    case P_BF16X1: return launch_gemm_p<P_BF16X1>(role, grid, descs, ndesc, segs, stream);
    case P_BF16X3: return launch_gemm_p<P_BF16X3>(role, grid, descs, ndesc, segs, stream);
    case P_BF16X6: return launch_gemm_p<P_BF16X6>(role, grid, descs, ndesc, segs, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_krp(int prec, const KrpDesc* descs, int ndesc, int64_t total_tiles,
                      hipStream_t stream) {
  if (ndesc <= 0 || total_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_tiles), block(NTHREADS);
  switch (prec) {
    case P_FP64: krp_kernel<P_FP64><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_FP32: krp_kernel<P_FP32><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X1: krp_kernel<P_BF16X1><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X3: krp_kernel<P_BF16X3><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X6: krp_kernel<P_BF16X6><<<grid, block, 0, stream>>>(descs, ndesc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  reduce_kernel<<<dim3(64, (unsigned)count), dim3(256), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_copy(const CopyJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  copy_kernel<<<dim3(64, (unsigned)count), dim3(256), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  fill_i32_kernel<<<dim3(8), dim3(256), 0, stream>>>(p, count, value);
  return hipGetLastError();
}

}  // namespace tsk
