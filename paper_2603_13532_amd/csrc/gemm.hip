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

#include <type_traits>

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

// Accumulator element type of a precision form.
template <int P> struct AccElem { typedef float type; };
template <> struct AccElem<P_FP64> { typedef double type; };

// Split-K: every split writes its 64 x 64 partial tile (accumulator type,
// column-major, ld 64); a reduce launch then adds the partials in split order,
// applies beta and writes C, so the result does not depend on timing.
template <int P>
__device__ __forceinline__ void store_partial(typename PT<P>::acc_t (&acc)[2][2], void* part_tile,
                                              int lane, int wm, int wn) {
  typedef typename AccElem<P>::type ae;
  ae* mine = (ae*)part_tile;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        mine[acc_row<P>(wm, i, lane, v) + TILE * acc_col(wn, j, lane)] = (ae)acc[i][j][v];
}

// Stage one K-tile held in registers into an LDS buffer.
template <int P>
__device__ __forceinline__ void stage(typename Lds<P>::type& s, bool a_xc, bool b_xc, int t,
                                     const typename PT<P>::in_t (&ra)[Stage<P>::PER_THREAD],
                                     const typename PT<P>::in_t (&rb)[Stage<P>::PER_THREAD]) {
#pragma unroll
  for (int j = 0; j < Stage<P>::PER_THREAD; ++j) {
    int x, k;
    PanelMap<P>::xk(a_xc, t, j, x, k);
    lds_put<P>(s, 0, x, k, ra[j]);
    PanelMap<P>::xk(b_xc, t, j, x, k);
    lds_put<P>(s, 1, x, k, rb[j]);
  }
}

// Position in the concatenated K range of a descriptor's segments, with the
// per-thread element offsets of the current segment kept in registers.
template <int P>
struct SegCursor {
  typedef typename PT<P>::in_t in_t;
  static constexpr int BK = PT<P>::BK;
  static constexpr int PER = Stage<P>::PER_THREAD;
  const GemmSeg* segs;
  int si, seg_end, kt, nkt, K;
  const in_t* A;
  const in_t* B;
  int64_t a_step, b_step;  // element step of one K-tile
  in_t alpha;
  bool a_xc, b_xc;
  int64_t offA[PER], offB[PER];
  int kA[PER], kB[PER];
  bool okA[PER], okB[PER];

  __device__ __forceinline__ void load(int64_t b, int m0, int n0, int M, int N, int t) {
    const GemmSeg S = segs[si];
    A = (const in_t*)S.A + b * S.strideA;
    B = (const in_t*)S.B + b * S.strideB;
    a_step = (int64_t)BK * S.a_sk;
    b_step = (int64_t)BK * S.b_sk;
    K = S.K;
    nkt = (K + BK - 1) / BK;
    alpha = (in_t)S.alpha;
    a_xc = S.a_sx == 1;
    b_xc = S.b_sx == 1;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int x, k;
      PanelMap<P>::xk(a_xc, t, j, x, k);
      okA[j] = m0 + x < M;
      offA[j] = (int64_t)(m0 + x) * S.a_sx + (int64_t)k * S.a_sk;
      kA[j] = k;
      PanelMap<P>::xk(b_xc, t, j, x, k);
      okB[j] = n0 + x < N;
      offB[j] = (int64_t)(n0 + x) * S.b_sx + (int64_t)k * S.b_sk;
      kB[j] = k;
    }
  }
  // Move `step` K-tiles forward; false once past the last segment.
  __device__ __forceinline__ bool advance(int step, int64_t b, int m0, int n0, int M, int N, int t) {
    kt += step;
    while (kt >= nkt) {
      kt -= nkt;
      if (++si >= seg_end) return false;
      load(b, m0, n0, M, N, t);
    }
    return true;
  }
  __device__ __forceinline__ void fetch(in_t (&ra)[PER], in_t (&rb)[PER]) const {
    const int k0 = kt * BK;
    const in_t* Ak = A + (int64_t)kt * a_step;
    const in_t* Bk = B + (int64_t)kt * b_step;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      ra[j] = (okA[j] && k0 + kA[j] < K) ? Ak[offA[j]] * alpha : (in_t)0;
      rb[j] = (okB[j] && k0 + kB[j] < K) ? Bk[offB[j]] : (in_t)0;
    }
  }
};

// ROLE only names the launch (one symbol per step of the method, so that
// kernel traces separate them); the code is the same for every role.
template <int P, int ROLE>
__global__ __launch_bounds__(NTHREADS) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                        int ndesc,
                                                        const GemmSeg* __restrict__ segs) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  constexpr int PER = Stage<P>::PER_THREAD;
  __shared__ typename Lds<P>::type s[2];

  const int64_t tile = blockIdx.x;
  const int di = find_desc(descs, ndesc, tile);
  const GemmDesc D = descs[di];
  int64_t local = tile - D.tile_begin;
  const int splits = D.splits;
  const int split = (int)(local % splits);
  local /= splits;
  const int64_t tile_ns = local;  // tile index without the split
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

  SegCursor<P> cur;
  cur.segs = segs;
  cur.si = D.seg_begin;
  cur.seg_end = D.seg_begin + D.seg_count;
  cur.kt = 0;
  cur.nkt = 0;
  bool have = false;
  if (D.seg_count > 0) {
    cur.load(b, m0, n0, M, N, t);
    have = cur.advance(split, b, m0, n0, M, N, t);
  }
  // Double-buffered LDS: the next K-tile's global loads are in flight while
  // the current one feeds the MFMAs; one barrier per K-tile.
  int buf = 0;
  if (have) {
    cur.fetch(ra, rb);
    stage<P>(s[0], cur.a_xc, cur.b_xc, t, ra, rb);
  }
  __syncthreads();
  while (have) {
    const bool next = cur.advance(splits, b, m0, n0, M, N, t);
    if (next) cur.fetch(ra, rb);
    mma_tile<P>(s[buf], acc, lane, wm, wn);
    if (next) stage<P>(s[buf ^ 1], cur.a_xc, cur.b_xc, t, ra, rb);
    __syncthreads();
    buf ^= 1;
    have = next;
  }

  const int64_t off = b * D.strideC;
  if (splits == 1) {
    if (D.c_f64)
      store_tile<P, double>(acc, (double*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane, wm, wn);
    else
      store_tile<P, float>(acc, (float*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane, wm, wn);
  } else {
    typedef typename AccElem<P>::type ae;
    store_partial<P>(acc, (ae*)D.part + (tile_ns * splits + split) * (TILE * TILE), lane, wm, wn);
  }
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
  __shared__ typename Lds<P>::type s[2];

  const int64_t tile = blockIdx.x;
  const KrpDesc& D = descs[find_desc(descs, ndesc, tile)];
  int64_t local = tile - D.tile_begin;
  const int splits = D.splits;
  const int split = (int)(local % splits);
  local /= splits;
  const int64_t tile_ns = local;
  const int tm = (int)(local % D.tiles_m);
  const int tn = (int)(local / D.tiles_m);
  const int order = D.order, n = D.mode, m = D.m;
  const int m0 = tm * TILE, n0 = tn * TILE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;
  const in_t* __restrict__ G = (const in_t*)D.G;
  const in_t alpha = (in_t)D.alpha;
  void* part_base = D.part;
  void* Vout = D.V;
  const int64_t Kc = D.Kc;

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
  const int rn = rk[n];
  const int64_t stn = st[n];

  acc_t acc[2][2];
  acc_zero<P>(acc);
  in_t ra[PER], rb[PER];
  const int64_t nkt = (Kc + BK - 1) / BK;
  const int kq = t % BK;
  // gather one K-tile: row a of G_(n) and the Khatri-Rao entry
  // prod_{k != n} P_k[j_k(c)][t] for this thread's depth c = kt*BK + kq
#define TSK_KRP_FETCH(KT)                                                          \
  {                                                                                \
    const int64_t c = (KT) * BK + kq;                                              \
    const bool valid = c < Kc;                                                     \
    int dig[kMaxOrder];                                                            \
    int64_t offg = 0;                                                              \
    int64_t rem = valid ? c : 0;                                                   \
    _Pragma("unroll") for (int k = 0; k < kMaxOrder; ++k) {                        \
      dig[k] = 0;                                                                  \
      if (k < order && k != n) {                                                   \
        const int64_t q = rem / rk[k];                                             \
        dig[k] = (int)(rem - q * rk[k]);                                           \
        rem = q;                                                                   \
        offg += (int64_t)dig[k] * st[k];                                           \
      }                                                                            \
    }                                                                              \
    _Pragma("unroll") for (int j = 0; j < PER; ++j) {                              \
      const int x = t / BK + (NTHREADS / BK) * j;                                  \
      const int a = m0 + x;                                                        \
      ra[j] = (valid && a < rn) ? G[(int64_t)a * stn + offg] * alpha : (in_t)0;    \
      const int tt = n0 + x;                                                       \
      in_t prod = (in_t)0;                                                         \
      if (valid && tt < m) {                                                       \
        prod = (in_t)1;                                                            \
        _Pragma("unroll") for (int k = 0; k < kMaxOrder; ++k) if (k < order &&     \
                                                                  k != n) prod *=  \
            Pk[k][dig[k] + (int64_t)tt * rk[k]];                                   \
      }                                                                            \
      rb[j] = prod;                                                                \
    }                                                                              \
  }
  int64_t kt = split;
  int buf = 0;
  if (kt < nkt) {
    TSK_KRP_FETCH(kt);
    stage<P>(s[0], false, false, t, ra, rb);
  }
  __syncthreads();
  while (kt < nkt) {
    const int64_t kn = kt + splits;
    if (kn < nkt) TSK_KRP_FETCH(kn);
    mma_tile<P>(s[buf], acc, lane, wm, wn);
    if (kn < nkt) stage<P>(s[buf ^ 1], false, false, t, ra, rb);
    __syncthreads();
    buf ^= 1;
    kt = kn;
  }
#undef TSK_KRP_FETCH
  typedef typename std::conditional<P == P_FP64, double, float>::type vt;
  if (splits == 1) {
    store_tile<P, vt>(acc, (vt*)Vout, rn, rn, m, m0, n0, false, lane, wm, wn);
  } else {
    typedef typename AccElem<P>::type ae;
    store_partial<P>(acc, (ae*)part_base + (tile_ns * splits + split) * (TILE * TILE), lane, wm, wn);
  }
}

// Adjoint of the KRP core sketch with respect to the core: rows a (mode n
// of the core) against columns c (the other modes, first remaining mode
// fastest), K = t over the sketch width.  The Khatri-Rao row of column c is
// generated from the P_k; its mixed-radix digits are computed once per
// thread because a thread's columns do not change along K.  The result is
// scattered through the mode-n unfolding into the core layout.
template <int P>
__global__ __launch_bounds__(NTHREADS) void krp_adj_kernel(const KrpAdjDesc* __restrict__ descs,
                                                           int ndesc) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  constexpr int BK = PT<P>::BK;
  constexpr int PER = Stage<P>::PER_THREAD;
  __shared__ typename Lds<P>::type s[2];

  const int64_t tile = blockIdx.x;
  const KrpAdjDesc& D = descs[find_desc(descs, ndesc, tile)];
  const int64_t local = tile - D.tile_begin;
  const int tm = (int)(local % D.tiles_m);
  const int64_t tn = local / D.tiles_m;
  const int order = D.order, n = D.mode, m = D.m;
  const int64_t Nc = D.Nc;
  const int64_t m0 = (int64_t)tm * TILE, n0 = tn * TILE;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w & 1, wn = w >> 1;
  const in_t* __restrict__ Vb = (const in_t*)D.Vbar;
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
  const int rn = rk[n];
  // this thread's B columns (k-contiguous mapping: depth kq, rows x_j)
  const int kq = t % BK;
  int dig[PER][kMaxOrder];
  bool colok[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t c = n0 + t / BK + (NTHREADS / BK) * j;
    colok[j] = c < Nc;
    int64_t rem = colok[j] ? c : 0;
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k) {
      dig[j][k] = 0;
      if (k < order && k != n) {
        const int64_t q = rem / rk[k];
        dig[j][k] = (int)(rem - q * rk[k]);
        rem = q;
      }
    }
  }
  acc_t acc[2][2];
  acc_zero<P>(acc);
  in_t ra[PER], rb[PER];
  const int nkt = (m + BK - 1) / BK;
#define TSK_ADJ_FETCH(KT)                                                           \
  {                                                                                 \
    const int k0 = (KT) * BK;                                                       \
    _Pragma("unroll") for (int j = 0; j < PER; ++j) {                               \
      int x, k;                                                                     \
      PanelMap<P>::xk(true, t, j, x, k);                                            \
      const int64_t a = m0 + x;                                                     \
      ra[j] = (a < rn && k0 + k < m) ? Vb[a + (int64_t)(k0 + k) * rn] * alpha : (in_t)0; \
      const int tt = k0 + kq;                                                       \
      in_t prod = (in_t)0;                                                          \
      if (colok[j] && tt < m) {                                                     \
        prod = (in_t)1;                                                             \
        _Pragma("unroll") for (int q = 0; q < kMaxOrder; ++q) if (q < order &&      \
                                                                 q != n) prod *=    \
            Pk[q][dig[j][q] + (int64_t)tt * rk[q]];                                 \
      }                                                                             \
      rb[j] = prod;                                                                 \
    }                                                                               \
  }
  int kt = 0, buf = 0;
  if (kt < nkt) {
    TSK_ADJ_FETCH(kt);
    stage<P>(s[0], true, false, t, ra, rb);
  }
  __syncthreads();
  while (kt < nkt) {
    const int kn = kt + 1;
    if (kn < nkt) TSK_ADJ_FETCH(kn);
    mma_tile<P>(s[buf], acc, lane, wm, wn);
    if (kn < nkt) stage<P>(s[buf ^ 1], true, false, t, ra, rb);
    __syncthreads();
    buf ^= 1;
    kt = kn;
  }
#undef TSK_ADJ_FETCH
  // scatter through the unfolding: (a, c) -> a*st_n + sum_k dig_k(c) st_k
  typedef typename std::conditional<P == P_FP64, double, float>::type vt;
  vt* __restrict__ Gout = (vt*)D.Gout;
#pragma unroll
  for (int jj = 0; jj < 2; ++jj) {
    const int64_t c = n0 + acc_col(wn, jj, lane);
    if (c >= Nc) continue;
    int64_t rem = c, off = 0;
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k)
      if (k < order && k != n) {
        const int64_t q = rem / rk[k];
        off += (rem - q * rk[k]) * st[k];
        rem = q;
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t a = m0 + acc_row<P>(wm, i, lane, v);
        if (a < rn) Gout[a * st[n] + off] = (vt)acc[i][jj][v];
      }
  }
}

// One job per blockIdx.y; blocks stride over columns, threads over rows.
// Parts are summed four at a time so that several loads are in flight.
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceJob* __restrict__ jobs) {
  const ReduceJob& J = jobs[blockIdx.y];
  const int64_t rows = J.rows, cols = J.cols, sp = J.stride_part;
  const int parts = J.parts;
  for (int64_t c = blockIdx.x; c < cols; c += gridDim.x) {
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
      double acc = 0.0;
      const int64_t base = r + c * J.ld_part;
      int s = 0;
      if (J.part_f64) {
        const double* p = (const double*)J.part + base;
        for (; s + 4 <= parts; s += 4) {
          const double v0 = p[s * sp], v1 = p[(s + 1) * sp], v2 = p[(s + 2) * sp], v3 = p[(s + 3) * sp];
          acc += v0;
          acc += v1;
          acc += v2;
          acc += v3;
        }
        for (; s < parts; ++s) acc += p[s * sp];
      } else {
        const float* p = (const float*)J.part + base;
        for (; s + 4 <= parts; s += 4) {
          const float v0 = p[s * sp], v1 = p[(s + 1) * sp], v2 = p[(s + 2) * sp], v3 = p[(s + 3) * sp];
          acc += (double)v0;
          acc += (double)v1;
          acc += (double)v2;
          acc += (double)v3;
        }
        for (; s < parts; ++s) acc += (double)p[s * sp];
      }
      const int64_t o = r + c * J.ld_out;
      if (J.out_f64) {
        double* q = (double*)J.out;
        q[o] = J.beta ? q[o] + acc : acc;
      } else {
        float* q = (float*)J.out;
        q[o] = (float)(J.beta ? (double)q[o] + acc : acc);
      }
    }
  }
}

// Split-K tile reduction: one workgroup per 64 x 64 output tile, 16
// elements per thread, one batch of 16 independent loads per split.
__global__ __launch_bounds__(256) void tile_reduce_kernel(const ReduceJob* __restrict__ jobs) {
  const ReduceJob J = jobs[blockIdx.x];
  constexpr int EPT = 64 * 64 / 256;
  const int t = threadIdx.x;
  double sum[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) sum[i] = 0.0;
  for (int s = 0; s < J.parts; ++s) {
    if (J.part_f64) {
      const double* p = (const double*)J.part + (int64_t)s * J.stride_part + t;
      double v[EPT];
#pragma unroll
      for (int i = 0; i < EPT; ++i) v[i] = p[256 * i];
#pragma unroll
      for (int i = 0; i < EPT; ++i) sum[i] += v[i];
    } else {
      const float* p = (const float*)J.part + (int64_t)s * J.stride_part + t;
      float v[EPT];
#pragma unroll
      for (int i = 0; i < EPT; ++i) v[i] = p[256 * i];
#pragma unroll
      for (int i = 0; i < EPT; ++i) sum[i] += (double)v[i];
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = t + 256 * i;
    const int r = e & 63, c = e >> 6;
    if (r >= J.rows || c >= J.cols) continue;
    const int64_t o = r + (int64_t)c * J.ld_out;
    if (J.out_f64) {
      double* q = (double*)J.out;
      q[o] = J.beta ? q[o] + sum[i] : sum[i];
    } else {
      float* q = (float*)J.out;
      q[o] = (float)(J.beta ? (double)q[o] + sum[i] : sum[i]);
    }
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const CopyJob* __restrict__ jobs) {
  const CopyJob& J = jobs[blockIdx.y];
  for (int64_t c = blockIdx.x; c < J.cols; c += gridDim.x) {
    for (int64_t r = threadIdx.x; r < J.rows; r += blockDim.x) {
      const int64_t is = r + c * J.ld_src, id = r + c * J.ld_dst;
      const double v = J.src_f64 ? ((const double*)J.src)[is] : (double)((const float*)J.src)[is];
      if (J.dst_f64) ((double*)J.dst)[id] = v;
      else ((float*)J.dst)[id] = (float)v;
    }
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

hipError_t launch_krp_adj(int prec, const KrpAdjDesc* descs, int ndesc, int64_t total_tiles,
                          hipStream_t stream) {
  if (ndesc <= 0 || total_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_tiles), block(NTHREADS);
  switch (prec) {
    case P_FP64: krp_adj_kernel<P_FP64><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_FP32: krp_adj_kernel<P_FP32><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X1: krp_adj_kernel<P_BF16X1><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X3: krp_adj_kernel<P_BF16X3><<<grid, block, 0, stream>>>(descs, ndesc); break;
    case P_BF16X6: krp_adj_kernel<P_BF16X6><<<grid, block, 0, stream>>>(descs, ndesc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  reduce_kernel<<<dim3(64, (unsigned)count), dim3(256), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_tile_reduce(const ReduceJob* jobs, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  tile_reduce_kernel<<<dim3((unsigned)count), dim3(256), 0, stream>>>(jobs);
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
