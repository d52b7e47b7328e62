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

// Index of the last of n entries whose begin(i) <= key (begin(0) = 0 <=
// key, and begin never decreases), for a 256-thread block in uniform
// control flow.  Up to 256 entries every thread tests one and the block
// counts; up to 65536, a coarse pass over every stride-th entry finds the
// block of `stride` entries that holds the key and a second pass counts
// within it: two memory round trips instead of a binary search's chain of
// dependent loads.
template <typename F>
__device__ __forceinline__ int find_last_le(int n, int64_t key, F begin) {
  const int t = threadIdx.x;
  if (n <= NTHREADS) {
    const bool le = t < n && begin(t) <= key;
    return uni(__syncthreads_count(le) - 1);
  }
  if (n <= NTHREADS * NTHREADS) {
    const int stride = (n + NTHREADS - 1) / NTHREADS;
    const int i1 = t * stride;
    const bool le1 = i1 < n && begin(i1) <= key;
    const int base = uni(__syncthreads_count(le1) - 1) * stride;
    const int i2 = base + t;
    const bool le2 = t < stride && i2 < n && begin(i2) <= key;
    return base + uni(__syncthreads_count(le2) - 1);
  }
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin(mid) <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Descriptor of a linear tile id: the last one whose tile_begin <= tile.
template <typename D>
__device__ __forceinline__ int find_desc(const D* __restrict__ descs, int ndesc, int64_t tile) {
  return find_last_le(ndesc, tile, [&](int i) { return (int64_t)descs[i].tile_begin; });
}

// GEMM descriptor lookup that also returns the descriptor's segment range
// (read in the same pass for up to 256 descriptors, so that the segment
// table can be fetched while the descriptor itself is still in flight).
__device__ __forceinline__ int find_gemm_desc(const GemmDesc* __restrict__ descs, int ndesc,
                                              int64_t tile, int& seg_begin, int& seg_count) {
  __shared__ int s_sb[NTHREADS], s_sc[NTHREADS];
  if (ndesc <= NTHREADS) {
    const int t = threadIdx.x;
    bool le = false;
    if (t < ndesc) {
      le = descs[t].tile_begin <= tile;
      s_sb[t] = descs[t].seg_begin;
      s_sc[t] = descs[t].seg_count;
    }
    const int di = uni(__syncthreads_count(le) - 1);
    seg_begin = uni(s_sb[di]);
    seg_count = uni(s_sc[di]);
    return di;
  }
  const int di = find_desc(descs, ndesc, tile);
  seg_begin = descs[di].seg_begin;
  seg_count = descs[di].seg_count;
  return di;
}

// Accumulator element type of a precision form.
template <int P> struct AccElem { typedef float type; };
template <> struct AccElem<P_FP64> { typedef double type; };

// Epilogue through LDS: the accumulators go to a 64 x 64 tile in the K-loop's
// LDS buffers (free once the loop's last barrier has passed), and every store
// instruction then writes 64 consecutive rows of one column, coalesced,
// instead of the MFMA layout's 16 columns x 4 scattered rows.
constexpr int kEpiLd = TILE + 1;
// With kw waves per quadrant (K split among them), the waves of phase 0
// write their quadrant and those of each later phase add theirs, in phase
// order (the sum does not depend on timing).
template <int P>
__device__ __forceinline__ typename AccElem<P>::type* epi_stage(
    typename PT<P>::acc_t (&acc)[2][2], void* lds, int lane, int wm, int wn, int phase = 0,
    int kw = 1) {
  typedef typename AccElem<P>::type ae;
  static_assert(sizeof(typename Lds<P>::type) * 2 >= sizeof(ae) * TILE * kEpiLd,
                "the epilogue tile fits the K-loop buffers");
  ae* T = (ae*)lds;
  __syncthreads();
  for (int ph = 0; ph < kw; ++ph) {
    if (phase == ph) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            ae& cell = T[acc_row<P>(wm, i, lane, v) + kEpiLd * acc_col(wn, j, lane)];
            cell = (ph == 0) ? (ae)acc[i][j][v] : cell + (ae)acc[i][j][v];
          }
    }
    __syncthreads();
  }
  return T;
}

// C(m0 + r, n0 + c) (=|+=) tile(r, c) for r < M - m0, c < N - n0 (column-major C).
template <int P, typename OutT>
__device__ __forceinline__ void store_tile(typename PT<P>::acc_t (&acc)[2][2], OutT* __restrict__ C,
                                           int64_t ldc, int M, int N, int m0, int n0, bool accum,
                                           int lane, int wm, int wn, void* lds, int t, int phase = 0,
                                           int kw = 1) {
  const typename AccElem<P>::type* T = epi_stage<P>(acc, lds, lane, wm, wn, phase, kw);
  const int r = t & (TILE - 1), row = m0 + r;
  if (row >= M) return;
#pragma unroll 4
  for (int c = t / TILE; c < TILE; c += NTHREADS / TILE) {
    const int col = n0 + c;
    if (col >= N) break;
    OutT* p = C + (int64_t)row + (int64_t)col * ldc;
    const double v = (double)T[r + kEpiLd * c];
    if (accum) *p = (OutT)((double)*p + v);
    else *p = (OutT)v;
  }
}

// Split-K: every split writes its 64 x 64 partial tile (accumulator type,
// column-major, ld 64); a reduce launch then adds the partials in split order,
// applies beta and writes C, so the result does not depend on timing.
template <int P>
__device__ __forceinline__ void store_partial(typename PT<P>::acc_t (&acc)[2][2], void* part_tile,
                                              int lane, int wm, int wn, void* lds, int t,
                                              int phase = 0, int kw = 1) {
  typedef typename AccElem<P>::type ae;
  const ae* T = epi_stage<P>(acc, lds, lane, wm, wn, phase, kw);
  ae* mine = (ae*)part_tile;
  const int r = t & (TILE - 1);
#pragma unroll 4
  for (int c = t / TILE; c < TILE; c += NTHREADS / TILE) mine[r + TILE * c] = T[r + kEpiLd * c];
}

// Stage one K-tile held in registers into an LDS buffer.
// LDS element offsets of a thread's staged elements for both thread maps
// (x-contiguous and k-contiguous operands); fixed for the whole kernel.
template <int P>
struct StageMap {
  static constexpr int PER = Stage<P>::PER_THREAD;
  int lx[PER], lk[PER];
  __device__ __forceinline__ explicit StageMap(int t) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int x, k;
      PanelMap<P>::xk(true, t, j, x, k);
      lx[j] = k * (TILE + 2) + x;
      PanelMap<P>::xk(false, t, j, x, k);
      lk[j] = k * (TILE + 2) + x;
    }
  }
};

// Stage one K-tile held in registers into an LDS buffer; the A operand is
// scaled by its segment coefficient here, after the loads have landed.
template <int P>
__device__ __forceinline__ void stage(typename Lds<P>::type& s, const StageMap<P>& map, bool a_xc,
                                     bool b_xc, int t,
                                     const typename PT<P>::in_t (&ra)[Stage<P>::PER_THREAD],
                                     const typename PT<P>::in_t (&rb)[Stage<P>::PER_THREAD],
                                     typename PT<P>::in_t alpha) {
  if constexpr (P == P_FP64 || P == P_FP32) {
    typedef typename PT<P>::in_t in_t;
    in_t* sa = &s.a[0][0];
    in_t* sb = &s.b[0][0];
#pragma unroll
    for (int j = 0; j < Stage<P>::PER_THREAD; ++j) {
      sa[a_xc ? map.lx[j] : map.lk[j]] = ra[j] * alpha;
      sb[b_xc ? map.lx[j] : map.lk[j]] = rb[j];
    }
  } else {
    stage_bf<P>(s.a, t, ra, alpha);
    stage_bf<P>(s.b, t, rb, 1.0f);
  }
}

// Position in the concatenated K range of a descriptor's segments, with the
// per-thread byte offsets of the current segment kept in registers.  The
// segment table is read through an LDS window of kSegCache entries, refilled
// by the whole block when the cursor leaves it, so a segment change costs no
// global round trip.
constexpr int kSegCache = 32;  // small enough for four FP64 workgroups per CU
typedef __attribute__((address_space(3))) GemmSeg lds_seg_t;
typedef __attribute__((address_space(3))) uint64_t lds_u64_t;

// A32: the A operands are stored in FP32 while the product runs in P (FP64):
// they are converted as they are loaded, so no FP64 copy is made.
template <int P, bool A32 = false>
struct SegCursor {
  typedef typename PT<P>::in_t in_t;
  typedef typename std::conditional<A32, float, in_t>::type a_src_t;
  static constexpr int BK = PT<P>::BK;
  static constexpr int PER = Stage<P>::PER_THREAD;
  const GemmSeg* segs;  // global table, from the descriptor's first segment
  lds_seg_t* cache;     // LDS window [c0, c0 + kSegCache)
  int c0;
  int si, seg_end, kt, nkt, K;
  const char* A;  // byte address of the tile origin (row m0 / column n0, k = 0)
  const char* B;
  int64_t a_step, b_step;  // bytes per K-tile
  in_t alpha;
  bool a_xc, b_xc;
  uint32_t offA[PER], offB[PER];  // byte offsets from the origin (kOob outside M / N)
  int kA[PER], kB[PER];
  // launch context: batch index, tile origin, bounds, thread, K-tile stride
  int64_t b;
  int m0, n0, M, N, t, step;

  // Copy segments [first, first + kSegCache) into the window (block-wide,
  // called in uniform control flow).
  __device__ __forceinline__ void fill(int first) {
    constexpr int kw = sizeof(GemmSeg) / 8;
    const int n = min(kSegCache, seg_end - first);
    const uint64_t* src = (const uint64_t*)(segs + first);
    lds_u64_t* dst = (lds_u64_t*)cache;
    __syncthreads();
    for (int e = t; e < n * kw; e += NTHREADS) dst[e] = src[e];
    __syncthreads();
    c0 = first;
  }
  __device__ __forceinline__ void load() {
    if (si - c0 >= kSegCache) fill(si);
    lds_seg_t& S = cache[si - c0];
    constexpr int64_t es = sizeof(in_t), ea = sizeof(a_src_t);
    const char* sA = uni((const char*)S.A);
    const char* sB = uni((const char*)S.B);
    const int64_t a_sx = uni((int64_t)S.a_sx), a_sk = uni((int64_t)S.a_sk);
    const int64_t b_sx = uni((int64_t)S.b_sx), b_sk = uni((int64_t)S.b_sk);
    A = sA + (b * uni((int64_t)S.strideA) + (int64_t)m0 * a_sx) * ea;
    B = sB + (b * uni((int64_t)S.strideB) + (int64_t)n0 * b_sx) * es;
    a_step = (int64_t)BK * a_sk * ea;
    b_step = (int64_t)BK * b_sk * es;
    K = uni((int)S.K);
    nkt = (K + BK - 1) / BK;
    alpha = (in_t)uni(S.alpha);
    a_xc = a_sx == 1;
    b_xc = b_sx == 1;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int x, k;
      PanelMap<P>::xk(a_xc, t, j, x, k);
      offA[j] = m0 + x < M ? (uint32_t)(((int64_t)x * a_sx + (int64_t)k * a_sk) * ea) : kOob;
      kA[j] = k;
      PanelMap<P>::xk(b_xc, t, j, x, k);
      offB[j] = n0 + x < N ? (uint32_t)(((int64_t)x * b_sx + (int64_t)k * b_sk) * es) : kOob;
      kB[j] = k;
    }
  }
  // Move `n` K-tiles forward; false once past the last segment.
  __device__ __forceinline__ bool skip(int n) {
    kt += n;
    while (kt >= nkt) {
      kt -= nkt;
      if (++si >= seg_end) return false;
      load();
    }
    return true;
  }
  __device__ __forceinline__ bool advance() { return skip(step); }
  // Loads of the current K-tile; with live == false every offset is out of
  // range, so the same number of loads issue and all of them read zero.
  // One straight-line sequence for full and ragged tiles alike: a branch
  // between the two makes the compiler wait for every load in flight before
  // the ragged variant overwrites the registers.
  __device__ __forceinline__ void fetch(in_t (&ra)[PER], in_t (&rb)[PER], bool live) const {
    const int left = live ? K - kt * BK : 0;  // depths of this tile inside K
    const rsrc_t rA = make_rsrc(A + (int64_t)kt * a_step);
    const rsrc_t rB = make_rsrc(B + (int64_t)kt * b_step);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      ra[j] = (in_t)bload<a_src_t>(rA, kA[j] < left ? offA[j] : kOob);
      rb[j] = bload<in_t>(rB, kB[j] < left ? offB[j] : kOob);
    }
  }
};

// Register ring depth of the K-loop: K-tiles whose global loads are in
// flight while one tile feeds the MFMAs.  Two for every precision: deeper
// rings measured slower on the method's launches (their K-loops are short
// and the extra registers cost occupancy), and the loop needs two slots
// (the slot staged next is never the one just fetched).
template <int P> struct Depth { static constexpr int value = 2; };

// K-loop shared by the contraction kernels.  Most launches of the method put
// one or two workgroups on a CU, so global latency (first touches after the
// producing kernel, about a microsecond) is hidden by depth rather than by
// occupancy: D K-tiles are fetched ahead into registers, and each iteration
// stages the next one into the idle half of the double-buffered LDS while
// the MFMAs consume the other half.  `Cur` supplies fetch(ra, rb, live) for
// its current K-tile (zeros when not live), advance() to its next one, and
// the operand orientations.
//
// MMA = false is the copy run by a wave whose 32 x 32 quadrant lies wholly
// outside the output tile: it fetches and stages its share and meets every
// barrier, but issues no MFMAs (the choice is made once, outside the loop,
// so the loop body stays one basic block).
template <int P, int D, bool MMA, class Cur, int KW = 1, int MB = 2>
__device__ __forceinline__ void kloop(Cur& cur, bool have, typename Lds<P>::type (&s)[2],
                                      typename PT<P>::acc_t (&acc)[2][2], int t, int lane, int wm,
                                      int wn, int phase = 0) {
  static_assert(D >= 2, "the slot staged next must differ from the one just fetched");
  typedef typename PT<P>::in_t in_t;
  constexpr int PER = Stage<P>::PER_THREAD;
  const StageMap<P> map(t);
  in_t ra[D][PER], rb[D][PER], al[D];
  bool ax[D], bx[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    al[d] = (in_t)0;
    ax[d] = bx[d] = false;
  }
  int inflight = 0;
  // Every slot issues its loads and is staged whether or not it holds a
  // K-tile (a dead slot stages zeros into the buffer nobody reads next).
  // With a conditional stage the compiler sinks each fetch down to its only
  // use, D - 1 barriers later, and the ring degenerates into one load, one
  // wait per K-tile; unconditional use keeps the fetches where they are and
  // the wait before staging leaves the D - 1 younger slots in flight.
#pragma unroll
  for (int d = 0; d < D; ++d) {
    cur.fetch(ra[d], rb[d], have);
    if (have) {
      ax[d] = cur.a_xc;
      bx[d] = cur.b_xc;
      al[d] = cur.alpha;
      ++inflight;
      have = cur.advance();
    }
  }
  if (inflight == 0) return;
  stage<P>(s[0], map, ax[0], bx[0], t, ra[0], rb[0], al[0]);
  __syncthreads();
  int buf = 0;
  while (true) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      // s[buf] holds slot d's tile; its registers take the next fetch.  The
      // fetch, the MFMAs and the staging of the next slot form one basic
      // block (the cursor steps after them), so their instructions can be
      // interleaved.
      cur.fetch(ra[d], rb[d], have);
      const bool fa = cur.a_xc, fb = cur.b_xc;
      const in_t fal = cur.alpha;
      if constexpr (MMA) mma_tile<P, KW, MB>(s[buf], acc, lane, wm, wn, phase);
      const int nx = (d + 1) % D;
      stage<P>(s[buf ^ 1], map, ax[nx], bx[nx], t, ra[nx], rb[nx], al[nx]);
      --inflight;
      if (have) {
        ax[d] = fa;
        bx[d] = fb;
        al[d] = fal;
        ++inflight;
        have = cur.advance();
      }
      __syncthreads();
      buf ^= 1;
      if (inflight == 0) return;
    }
  }
}

// Which quadrant each wave computes, and over which K-steps.  A tile whose
// valid region (rows [0, mr), columns [0, nc) of the 64 x 64 tile) covers
// all four 32 x 32 quadrants gives one to each wave (kw = 1).  A smaller one
// covers one or two quadrants: with the 4-deep FP64/FP32 instructions its
// waves share them, kw = 4 or 2 waves per quadrant each taking every kw-th
// step of the K-tile, so no SIMD idles; BF16 K-tiles are a single step, and
// their waves outside the region skip the MFMAs (kw = 1, `active` false).
// kw_max (a tuning choice of the launch) caps the sharing: below 4 a
// one-quadrant tile, below 2 a two-quadrant tile, keeps kw = 1.  mb: the
// 16-row blocks of the wave's quadrant that hold valid rows (FP64/FP32: 1
// when they all lie in the first block, whose MFMAs are then the only ones
// issued; otherwise 2).
struct WaveRole {
  int kw, wm, wn, phase;
  bool active;
  int mb;
};
template <int P>
__device__ __forceinline__ WaveRole wave_role(int w, int mr, int nc, int kw_max) {
  auto blocks = [&](int wm) { return (P == P_FP64 || P == P_FP32) && mr - 32 * wm <= 16 ? 1 : 2; };
  if constexpr (P == P_FP64 || P == P_FP32) {
    const int qm = mr > 32 ? 2 : 1, qn = nc > 32 ? 2 : 1;
    if (qm * qn == 1 && kw_max >= 4) return WaveRole{4, 0, 0, w, true, blocks(0)};
    if (qm * qn == 2 && kw_max >= 2) {
      const int q = w & 1, wm = qm == 2 ? q : 0;
      return WaveRole{2, wm, qm == 2 ? 0 : q, w >> 1, true, blocks(wm)};
    }
  }
  const int wm = w & 1, wn = w >> 1;
  return WaveRole{1, wm, wn, 0, wm * 32 < mr && wn * 32 < nc, blocks(wm)};
}

// K-loop with the wave role chosen per tile (one branch, outside the loop).
template <int P, class Cur>
__device__ __forceinline__ void kloop_role(Cur& cur, bool have, typename Lds<P>::type (&s)[2],
                                           typename PT<P>::acc_t (&acc)[2][2], int t, int lane,
                                           const WaveRole& role) {
  constexpr int D = Depth<P>::value;
  if constexpr (P == P_FP64 || P == P_FP32) {
    if (role.kw == 4) {
      if (role.mb == 1) kloop<P, D, true, Cur, 4, 1>(cur, have, s, acc, t, lane, role.wm, role.wn, role.phase);
      else kloop<P, D, true, Cur, 4>(cur, have, s, acc, t, lane, role.wm, role.wn, role.phase);
      return;
    }
    if (role.kw == 2) {
      if (role.mb == 1) kloop<P, D, true, Cur, 2, 1>(cur, have, s, acc, t, lane, role.wm, role.wn, role.phase);
      else kloop<P, D, true, Cur, 2>(cur, have, s, acc, t, lane, role.wm, role.wn, role.phase);
      return;
    }
    if (role.active && role.mb == 1) {
      kloop<P, D, true, Cur, 1, 1>(cur, have, s, acc, t, lane, role.wm, role.wn);
      return;
    }
  }
  if (role.active)
    kloop<P, D, true, Cur>(cur, have, s, acc, t, lane, role.wm, role.wn);
  else
    kloop<P, D, false, Cur>(cur, have, s, acc, t, lane, role.wm, role.wn);
}

// ROLE only names the launch (one symbol per step of the method, so that
// kernel traces separate them); the code is the same for every role.
// At least four waves per SIMD (<= 128 VGPRs): with the LDS of one
// workgroup under 40 KB, four workgroups share a CU.
// GROUPED: the variant whose workgroups take several consecutive one-tile
// batch elements (the descriptors' bpw); launched only for launches that
// group, so that every other launch runs the one-tile body alone.
template <int P, int ROLE, bool A32 = false, bool GROUPED = false>
__global__ __launch_bounds__(NTHREADS, 4) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                        int ndesc,
                                                        const GemmSeg* __restrict__ segs) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  __shared__ typename Lds<P>::type s[2];

  const int64_t tile = blockIdx.x;
  int seg_begin, seg_count;
  const int di = find_gemm_desc(descs, ndesc, tile, seg_begin, seg_count);
  __shared__ GemmSeg sseg[kSegCache];
  SegCursor<P, A32> cur;
  cur.segs = segs + seg_begin;
  cur.cache = (lds_seg_t*)sseg;
  cur.seg_end = seg_count;
  cur.t = threadIdx.x;
  const GemmDesc D = descs[di];  // scalar loads, in flight with the segment copy
  if (seg_count > 0) cur.fill(0);
  int64_t local = tile - D.tile_begin;
  const int splits = D.splits;
  const int split = (int)(local % splits);
  local /= splits;
  const int64_t tile_ns = local;  // tile index without the split
  const int tm = (int)(local % D.tiles_m);
  local /= D.tiles_m;
  const int tn = (int)(local % D.tiles_n);
  if constexpr (GROUPED) {
    // a workgroup takes bpw consecutive batch elements (one tile each, no
    // K-split) or one tile of one element
    const int bpw = D.bpw > 1 ? D.bpw : 1;
    const int64_t b0 = (local / D.tiles_n) * bpw;
    const int nb = (int)min((int64_t)bpw, (int64_t)D.batch - b0);
    const int M = D.M, N = D.N;
    const int m0 = tm * TILE, n0 = tn * TILE;
    // the wave index goes through readfirstlane so that the compiler sees it as
    // uniform: branches on it stay scalar and the accumulators stay in place
    const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6);
    // one quadrant per wave here: the shared-quadrant variants of the K-loop
    // push this kernel past its 128-register budget (it spills), and at two
    // workgroups per CU the lost occupancy costs what the shared quadrants save
    const WaveRole role{1, w & 1, w >> 1, 0, (w & 1) * 32 < M - m0 && (w >> 1) * 32 < N - n0, 2};

    for (int e = 0; e < nb; ++e) {
      const int64_t b = b0 + e;
      if (e > 0) {
        // the previous element's epilogue reads its tile from the K-loop's
        // LDS buffers, which this element's first staging overwrites
        __syncthreads();
        if (cur.c0 != 0) cur.fill(0);
      }
      acc_t acc[2][2];
      acc_zero<P>(acc);

      cur.si = 0;
      cur.kt = 0;
      cur.nkt = 0;
      cur.b = b;
      cur.m0 = m0;
      cur.n0 = n0;
      cur.M = M;
      cur.N = N;
      cur.t = t;
      cur.step = splits;
      bool have = false;
      if (seg_count > 0) {
        cur.load();
        have = cur.skip(split);
      }
      if (have) {
        if (role.active) kloop<P, Depth<P>::value, true>(cur, have, s, acc, t, lane, role.wm, role.wn);
        else kloop<P, Depth<P>::value, false>(cur, have, s, acc, t, lane, role.wm, role.wn);
      }

      const int64_t off = b * D.strideC;
      if (splits == 1) {
        if (D.c_f64)
          store_tile<P, double>(acc, (double*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane,
                                role.wm, role.wn, s, t, role.phase, role.kw);
        else
          store_tile<P, float>(acc, (float*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane,
                               role.wm, role.wn, s, t, role.phase, role.kw);
      } else {
        typedef typename AccElem<P>::type ae;
        store_partial<P>(acc, (ae*)D.part + (tile_ns * splits + split) * (TILE * TILE), lane,
                         role.wm, role.wn, s, t, role.phase, role.kw);
      }
    }
  } else {
    const int64_t b = local / D.tiles_n;
    const int M = D.M, N = D.N;
    const int m0 = tm * TILE, n0 = tn * TILE;
    // the wave index goes through readfirstlane so that the compiler sees it as
    // uniform: branches on it stay scalar and the accumulators stay in place
    const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6);

    acc_t acc[2][2];
    acc_zero<P>(acc);

    cur.si = 0;
    cur.kt = 0;
    cur.nkt = 0;
    cur.b = b;
    cur.m0 = m0;
    cur.n0 = n0;
    cur.M = M;
    cur.N = N;
    cur.t = t;
    cur.step = splits;
    bool have = false;
    if (seg_count > 0) {
      cur.load();
      have = cur.skip(split);
    }
    // one quadrant per wave here: the shared-quadrant variants of the K-loop
    // push this kernel past its 128-register budget (it spills), and at two
    // workgroups per CU the lost occupancy costs what the shared quadrants save
    const WaveRole role{1, w & 1, w >> 1, 0, (w & 1) * 32 < M - m0 && (w >> 1) * 32 < N - n0, 2};
    if (have) {
      if (role.active) kloop<P, Depth<P>::value, true>(cur, have, s, acc, t, lane, role.wm, role.wn);
      else kloop<P, Depth<P>::value, false>(cur, have, s, acc, t, lane, role.wm, role.wn);
    }

    const int64_t off = b * D.strideC;
    if (splits == 1) {
      if (D.c_f64)
        store_tile<P, double>(acc, (double*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane,
                              role.wm, role.wn, s, t, role.phase, role.kw);
      else
        store_tile<P, float>(acc, (float*)D.C + off, D.ldc, M, N, m0, n0, D.beta != 0, lane,
                             role.wm, role.wn, s, t, role.phase, role.kw);
    } else {
      typedef typename AccElem<P>::type ae;
      store_partial<P>(acc, (ae*)D.part + (tile_ns * splits + split) * (TILE * TILE), lane,
                       role.wm, role.wn, s, t, role.phase, role.kw);
    }
  }
}

// K-tiles of the KRP core sketch: row a of G_(n) and the Khatri-Rao entry
// prod_{k != n} P_k[j_k(c)][t] for depth c.  FP64/FP32: one depth per thread
// and four rows x_j (the k-contiguous staging map); BF16: one row x = t % 64
// and eight consecutive depths, whose mixed-radix digits are stepped
// incrementally (they wrap, so they stay inside their ranges past the end of
// K).  With LDS_P the block's 64 columns of every P_k sit in LDS (slice k at
// soff[k], column x at x * r_k), so the Khatri-Rao products wait only on LDS;
// the core loads are buffer loads that nothing waits for before staging.
typedef __attribute__((address_space(3))) const float lds_cf32;
typedef __attribute__((address_space(3))) const double lds_cf64;

// The Khatri-Rao entry is computed for every depth and column and then
// selected (zero past K or past the sketch width): its LDS reads stay in
// range because the digits wrap, and the select discards what lies past the
// loaded columns.  Pinning the product in a register keeps the compiler from
// sinking its reads and products under a per-element divergent branch.
template <typename T>
__device__ __forceinline__ T krp_select(bool keep, T prod) {
  asm volatile("" : "+v"(prod));
  return keep ? prod : (T)0;
}

template <int P, bool LDS_P, bool G32 = false>
struct KrpCursor {
  typedef typename PT<P>::in_t in_t;
  typedef typename std::conditional<G32, float, in_t>::type g_src_t;  // core elements
  typedef typename std::conditional<P == P_FP64, lds_cf64, lds_cf32>::type lds_in_t;
  static constexpr int BK = PT<P>::BK;
  static constexpr int PER = Stage<P>::PER_THREAD;
  const void* G;  // core, g_src_t elements
  in_t alpha;
  const in_t* Pk[kMaxOrder];
  lds_in_t* sP;
  int soff[kMaxOrder];
  int rk[kMaxOrder];
  int64_t st[kMaxOrder];
  int order, n, m, m0, n0, t, rn;
  int64_t stn, Kc, kt, nkt, step;
  bool a_xc = false, b_xc = false;

  __device__ __forceinline__ bool advance() {
    kt += step;
    return kt < nkt;
  }
  // P_k[dg][n0 + x]
  __device__ __forceinline__ in_t pval(int k, int x, int dg) const {
    if constexpr (LDS_P) return sP[soff[k] + x * rk[k] + dg];
    else return Pk[k][dg + (int64_t)(n0 + x) * rk[k]];
  }
  __device__ __forceinline__ void fetch(in_t (&ra)[PER], in_t (&rb)[PER], bool live) const {
    constexpr int64_t es = sizeof(g_src_t);
    const rsrc_t rG = make_rsrc(G);
    const int64_t Kc = live ? this->Kc : 0;
    if constexpr (P != P_FP64 && P != P_FP32) {
      const int x = t & (TILE - 1);
      const int a = m0 + x, tt = n0 + x;
      const int64_t c0 = kt * BK + 8 * (t >> 6);
      int dg[kMaxOrder];
      int64_t offg = 0;
      {
        uint32_t rem = c0 < Kc ? (uint32_t)c0 : 0u;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k) {
          dg[k] = 0;
          if (k < order && k != n) {
            const uint32_t q = rem / (uint32_t)rk[k];
            dg[k] = (int)(rem - q * (uint32_t)rk[k]);
            rem = q;
            offg += (int64_t)dg[k] * st[k];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const bool valid = c0 + j < Kc;
        ra[j] = (in_t)bload<g_src_t>(rG, (valid && a < rn) ? (uint32_t)(((int64_t)a * stn + offg) * es) : kOob);
        in_t prod = (in_t)1;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k)
          if (k < order && k != n) prod *= pval(k, x, dg[k]);
        rb[j] = krp_select(valid && tt < m, prod);
        // next depth: add one to the mixed-radix digits, branch-free
        bool carry = true;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k) {
          if (k < order && k != n) {
            const int nd = dg[k] + (carry ? 1 : 0);
            const bool wrap = nd == rk[k];
            offg += carry ? (wrap ? (int64_t)(1 - rk[k]) * st[k] : st[k]) : 0;
            dg[k] = wrap ? 0 : nd;
            carry = carry && wrap;
          }
        }
      }
    } else {
      const int64_t c = kt * BK + t % BK;
      const bool valid = c < Kc;
      int dig[kMaxOrder];
      int64_t offg = 0;
      uint32_t rem = valid ? (uint32_t)c : 0u;
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) {
        dig[k] = 0;
        if (k < order && k != n) {
          const uint32_t q = rem / (uint32_t)rk[k];
          dig[k] = (int)(rem - q * (uint32_t)rk[k]);
          rem = q;
          offg += (int64_t)dig[k] * st[k];
        }
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int x = t / BK + (NTHREADS / BK) * j;
        const int a = m0 + x, tt = n0 + x;
        ra[j] = (in_t)bload<g_src_t>(rG, (valid && a < rn) ? (uint32_t)(((int64_t)a * stn + offg) * es) : kOob);
        in_t prod = (in_t)1;
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k)
          if (k < order && k != n) prod *= pval(k, x, dig[k]);
        rb[j] = krp_select(valid && tt < m, prod);
      }
    }
  }
};

// The same K-tiles for a sketch whose other modes number NO (2 or 3: cores
// of order 3 or 4) with their P slices in LDS.  The other modes are listed
// compactly (radix, core stride, LDS column base), the thread's mixed-radix
// digits advance from tile to tile by adding the digits of the tile step
// with one carry each (no division after setup), and the Khatri-Rao entry
// is NO LDS reads with no branch, so the whole K-loop iteration stays one
// basic block.  Digits past the end of K wrap and stay inside their ranges;
// those depths read zeros.
template <int P, int NO, bool G32 = false>
struct KrpFixed {
  typedef typename PT<P>::in_t in_t;
  typedef typename std::conditional<G32, float, in_t>::type g_src_t;  // core elements
  typedef typename std::conditional<P == P_FP64, lds_cf64, lds_cf32>::type lds_in_t;
  static constexpr int BK = PT<P>::BK;
  static constexpr int PER = Stage<P>::PER_THREAD;
  static constexpr bool FPK = (P == P_FP64 || P == P_FP32);  // one depth, PER rows per thread
  static constexpr int NX = FPK ? PER : 1;                   // rows (and columns) per thread
  const void* G;  // core, g_src_t elements
  in_t alpha;
  lds_in_t* sP;
  int rk[NO], inc[NO];  // radices of the other modes and the digits of one tile step
  int st[NO];           // core strides of the other modes (in elements)
  int pb[NX][NO];       // LDS index of P_k[.][n0 + x] without the digit
  uint32_t rowoff[NX];  // byte offset of core row m0 + x (kOob outside)
  bool tok[NX];         // column n0 + x inside the sketch width
  int dg[NO];           // digits of the thread's first depth in the current tile
  int64_t c, Kc, kt, nkt, step;
  bool a_xc = false, b_xc = false;

  // digits of v in the radices rk (the part beyond their product dropped)
  __device__ __forceinline__ void digits(int64_t v, int (&d)[NO]) const {
    uint64_t rem = (uint64_t)v;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const uint64_t q = rem / (uint64_t)rk[j];
      d[j] = (int)(rem - q * (uint64_t)rk[j]);
      rem = q;
    }
  }
  __device__ __forceinline__ bool advance() {
    kt += step;
    c += (int64_t)BK * step;
    int carry = 0;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int d = dg[j] + inc[j] + carry;
      carry = d >= rk[j] ? 1 : 0;
      dg[j] = carry ? d - rk[j] : d;
    }
    return kt < nkt;
  }
  __device__ __forceinline__ void fetch(in_t (&ra)[PER], in_t (&rb)[PER], bool live) const {
    constexpr uint32_t es = sizeof(g_src_t);
    const rsrc_t rG = make_rsrc(G);
    if constexpr (FPK) {
      const bool valid = live && c < Kc;
      uint32_t offg = 0;
#pragma unroll
      for (int j = 0; j < NO; ++j) offg += (uint32_t)(dg[j] * st[j]) * es;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        ra[i] = (in_t)bload<g_src_t>(rG, (valid && rowoff[i] != kOob) ? rowoff[i] + offg : kOob);
        in_t prod = sP[pb[i][0] + dg[0]];
#pragma unroll
        for (int j = 1; j < NO; ++j) prod *= sP[pb[i][j] + dg[j]];
        rb[i] = krp_select(valid && tok[i], prod);
      }
    } else {
      int d[NO];
      uint32_t offg = 0;
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        d[j] = dg[j];
        offg += (uint32_t)(d[j] * st[j]) * es;
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const bool valid = live && c + i < Kc;
        ra[i] = (in_t)bload<g_src_t>(rG, (valid && rowoff[0] != kOob) ? rowoff[0] + offg : kOob);
        in_t prod = sP[pb[0][0] + d[0]];
#pragma unroll
        for (int j = 1; j < NO; ++j) prod *= sP[pb[0][j] + d[j]];
        rb[i] = krp_select(valid && tok[0], prod);
        // next depth: add one to the digits, branch-free
        bool carry = true;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          const int nd = d[j] + (carry ? 1 : 0);
          const bool wrap = nd == rk[j];
          offg += carry ? (wrap ? (uint32_t)((1 - rk[j]) * st[j]) * es : (uint32_t)st[j] * es) : 0u;
          d[j] = wrap ? 0 : nd;
          carry = carry && wrap;
        }
      }
    }
  }
};

// KRP core sketch: rows a of G_(n) against Khatri-Rao columns t, K = c over
// the other modes, first remaining mode fastest (unfolding index equation).
template <int P, bool G32 = false>
__global__ __launch_bounds__(NTHREADS) void krp_kernel(const KrpDesc* __restrict__ descs,
                                                       int ndesc, int lds_cap) {
  typedef typename PT<P>::in_t in_t;
  typedef typename PT<P>::acc_t acc_t;
  constexpr int BK = PT<P>::BK;
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
  // the wave index goes through readfirstlane so that the compiler sees it as
  // uniform: branches on it stay scalar and the accumulators stay in place
  const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6), wm = w & 1, wn = w >> 1;
  const void* G = D.G;  // FP32 elements when G32
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

  const WaveRole role = wave_role<P>(w, rn - m0, m - n0, D.kw_max);
  acc_t acc[2][2];
  acc_zero<P>(acc);
  // the block's 64 columns of every P_k (k != n) into LDS when they fit the
  // launch's dynamic LDS (sized for its largest slice set)
  extern __shared__ __align__(16) unsigned char krp_dyn[];
  in_t* sP = reinterpret_cast<in_t*>(krp_dyn);
  int soff[kMaxOrder];
  int total = 0;
#pragma unroll
  for (int k = 0; k < kMaxOrder; ++k) {
    soff[k] = total;
    if (k < order && k != n) total += TILE * rk[k];
  }
  const bool lds_p = total <= lds_cap;
  if (lds_p) {
    const int cols = min(TILE, m - n0);
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k) {
      if (k < order && k != n) {
        const in_t* src = Pk[k] + (int64_t)n0 * rk[k];
        const int cnt = cols * rk[k];
        for (int e = t; e < cnt; e += NTHREADS) sP[soff[k] + e] = src[e];
      }
    }
    __syncthreads();
  }
#define TSK_KRP_CURSOR(CUR)          \
  CUR.G = G;                         \
  CUR.alpha = alpha;                 \
  _Pragma("unroll") for (int k = 0; k < kMaxOrder; ++k) { \
    CUR.Pk[k] = Pk[k];               \
    CUR.soff[k] = soff[k];           \
    CUR.rk[k] = rk[k];               \
    CUR.st[k] = st[k];               \
  }                                  \
  CUR.order = order;                 \
  CUR.n = n;                         \
  CUR.m = m;                         \
  CUR.m0 = m0;                       \
  CUR.n0 = n0;                       \
  CUR.t = t;                         \
  CUR.rn = rn;                       \
  CUR.stn = stn;                     \
  CUR.Kc = Kc;                       \
  CUR.kt = split;                    \
  CUR.nkt = (Kc + BK - 1) / BK;      \
  CUR.step = splits;
  // NO other modes listed compactly: radix, core stride and LDS base
  auto fixed = [&](auto& cur, auto no) {
    constexpr int NO = decltype(no)::value;
    typedef typename std::remove_reference<decltype(cur)>::type Cur;
    cur.G = G;
    cur.alpha = alpha;
    cur.sP = (typename Cur::lds_in_t*)sP;
    // the j-th other mode is j below n, j + 1 from n on; its entries are
    // picked by selects over statically indexed arrays (a runtime index into
    // a register array would put the cursor in scratch memory)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int kj = j < n ? j : j + 1;
      int r = 1, so = 0;
      int64_t sk = 1;
#pragma unroll
      for (int k = 0; k < kMaxOrder; ++k) {
        if (k == kj) {
          r = rk[k];
          sk = st[k];
          so = soff[k];
        }
      }
      cur.rk[j] = r;
      cur.st[j] = (int)sk;
#pragma unroll
      for (int i = 0; i < Cur::NX; ++i) {
        const int x = Cur::FPK ? t / BK + (NTHREADS / BK) * i : (t & (TILE - 1));
        cur.pb[i][j] = so + x * r;
      }
    }
#pragma unroll
    for (int i = 0; i < Cur::NX; ++i) {
      const int x = Cur::FPK ? t / BK + (NTHREADS / BK) * i : (t & (TILE - 1));
      cur.rowoff[i] = m0 + x < rn ? (uint32_t)((int64_t)(m0 + x) * stn *
                                               (int64_t)sizeof(typename Cur::g_src_t))
                                  : kOob;
      cur.tok[i] = n0 + x < m;
    }
    cur.Kc = Kc;
    cur.kt = split;
    cur.nkt = (Kc + BK - 1) / BK;
    cur.step = splits;
    cur.c = (int64_t)split * BK + (Cur::FPK ? t % BK : 8 * (t >> 6));
    cur.digits(cur.c, cur.dg);
    cur.digits((int64_t)BK * splits, cur.inc);
    kloop_role<P>(cur, cur.kt < cur.nkt, s, acc, t, lane, role);
  };
  if (lds_p && order == 3) {
    KrpFixed<P, 2, G32> cur;
    fixed(cur, std::integral_constant<int, 2>());
  } else if (lds_p && order == 4) {
    KrpFixed<P, 3, G32> cur;
    fixed(cur, std::integral_constant<int, 3>());
  } else if (lds_p) {
    KrpCursor<P, true, G32> cur;
    TSK_KRP_CURSOR(cur)
    cur.sP = (typename KrpCursor<P, true, G32>::lds_in_t*)sP;
    kloop_role<P>(cur, cur.kt < cur.nkt, s, acc, t, lane, role);
  } else {
    KrpCursor<P, false, G32> cur;
    TSK_KRP_CURSOR(cur)
    cur.sP = nullptr;
    kloop_role<P>(cur, cur.kt < cur.nkt, s, acc, t, lane, role);
  }
#undef TSK_KRP_CURSOR
  typedef typename std::conditional<P == P_FP64, double, float>::type vt;
  if (splits == 1) {
    store_tile<P, vt>(acc, (vt*)Vout, rn, rn, m, m0, n0, false, lane, role.wm, role.wn, s, t,
                      role.phase, role.kw);
  } else {
    typedef typename AccElem<P>::type ae;
    store_partial<P>(acc, (ae*)part_base + (tile_ns * splits + split) * (TILE * TILE), lane,
                     role.wm, role.wn, s, t, role.phase, role.kw);
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
  // the wave index goes through readfirstlane so that the compiler sees it as
  // uniform: branches on it stay scalar and the accumulators stay in place
  const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6), wm = w & 1, wn = w >> 1;
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
  // this thread's B columns: FP64/FP32 stage k-contiguous (depth kq, columns
  // x_j); the BF16 forms give each thread one column and eight depths.
  constexpr bool BF = P != P_FP64 && P != P_FP32;
  constexpr int NCOL = BF ? 1 : PER;
  const int kq = t % BK;
  int dig[NCOL][kMaxOrder];
  bool colok[NCOL];
#pragma unroll
  for (int j = 0; j < NCOL; ++j) {
    const int64_t c = BF ? n0 + (t & (TILE - 1)) : n0 + t / BK + (NTHREADS / BK) * j;
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
      const int jc = BF ? 0 : j;                                                    \
      const int tt = k0 + (BF ? 8 * (t >> 6) + j : kq);                             \
      in_t prod = (in_t)0;                                                          \
      if (colok[jc] && tt < m) {                                                    \
        prod = (in_t)1;                                                             \
        _Pragma("unroll") for (int q = 0; q < kMaxOrder; ++q) if (q < order &&      \
                                                                 q != n) prod *=    \
            Pk[q][dig[jc][q] + (int64_t)tt * rk[q]];                                \
      }                                                                             \
      rb[j] = prod;                                                                 \
    }                                                                               \
  }
  const StageMap<P> smap(t);
  int kt = 0, buf = 0;
  if (kt < nkt) {
    TSK_ADJ_FETCH(kt);
    stage<P>(s[0], smap, true, false, t, ra, rb, (in_t)1);
  }
  __syncthreads();
  while (kt < nkt) {
    const int kn = kt + 1;
    if (kn < nkt) TSK_ADJ_FETCH(kn);
    mma_tile<P>(s[buf], acc, lane, wm, wn);
    if (kn < nkt) stage<P>(s[buf ^ 1], smap, true, false, t, ra, rb, (in_t)1);
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

// Split-K tile reduction: each 64 x 64 output tile is spread over
// kReduceChunks workgroups (more of the chip's memory pipes busy) and every
// thread loads its elements for eight splits at a time, so one round trip
// covers eight partials (splits past the count read zeros through
// out-of-range buffer offsets, which leaves the sums unchanged).  Partials
// are added in split order, so the result does not depend on timing.
constexpr int kReduceChunks = 4;
template <typename PartT>
__device__ __forceinline__ void reduce_tile(const ReduceJob& J, int chunk, int t) {
  constexpr int EPT = TILE * TILE / (NTHREADS * kReduceChunks);
  constexpr int SB = 8;  // splits per round trip
  constexpr uint32_t es = sizeof(PartT);
  const rsrc_t rp = make_rsrc(J.part);
  const int e0 = chunk * (NTHREADS * EPT) + t;
  double sum[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) sum[i] = 0.0;
  for (int s0 = 0; s0 < J.parts; s0 += SB) {
    PartT v[SB][EPT];
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const bool live = s0 + b < J.parts;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const uint32_t off = (uint32_t)(((int64_t)(s0 + b) * J.stride_part + e0 + NTHREADS * i) * es);
        v[b][i] = bload<PartT>(rp, live ? off : kOob);
      }
    }
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int i = 0; i < EPT; ++i) sum[i] += (double)v[b][i];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = e0 + NTHREADS * i;
    const int r = e & (TILE - 1), c = e / TILE;
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
__global__ __launch_bounds__(NTHREADS) void tile_reduce_kernel(const ReduceJob* __restrict__ jobs) {
  const ReduceJob J = jobs[blockIdx.x];
  if (J.part_f64)
    reduce_tile<double>(J, blockIdx.y, threadIdx.x);
  else
    reduce_tile<float>(J, blockIdx.y, threadIdx.x);
}

template <class S, class D>
__device__ __forceinline__ void copy_chunk(const S* __restrict__ src, D* __restrict__ dst,
                                           int64_t base, int64_t n, int t, const double* norm2,
                                           double mul) {
  constexpr int E = kCopyChunk / 256;
  S v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int64_t e = base + k * 256 + t;
    v[k] = e < n ? src[e] : S(0);
  }
  if (norm2 != nullptr) {
    const double sc = mul * sqrt(*norm2);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int64_t e = base + k * 256 + t;
      if (e < n) dst[e] = (D)((double)v[k] * sc);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int64_t e = base + k * 256 + t;
    if (e < n) dst[e] = (D)v[k];
  }
}

// One workgroup per chunk of kCopyChunk elements; the job holding the chunk
// is found by binary search over the jobs' first chunks.
__global__ __launch_bounds__(256) void copy_kernel(const CopyJob* __restrict__ jobs, int count) {
  const int64_t chunk = blockIdx.x;
  const int lo = find_last_le(count, chunk, [&](int i) { return (int64_t)jobs[i].chunk_begin; });
  const CopyJob& J = jobs[lo];
  const int64_t n = J.rows * J.cols;
  const int64_t base = (chunk - J.chunk_begin) * kCopyChunk;
  const int t = threadIdx.x;
  if (J.src_f64) {
    if (J.dst_f64) copy_chunk((const double*)J.src, (double*)J.dst, base, n, t, J.norm2, J.mul);
    else copy_chunk((const double*)J.src, (float*)J.dst, base, n, t, J.norm2, J.mul);
  } else {
    if (J.dst_f64) copy_chunk((const float*)J.src, (double*)J.dst, base, n, t, J.norm2, J.mul);
    else copy_chunk((const float*)J.src, (float*)J.dst, base, n, t, J.norm2, J.mul);
  }
}

__global__ __launch_bounds__(256) void block_scatter_kernel(const BlockJob* __restrict__ jobs,
                                                            int count) {
  const int64_t chunk = blockIdx.x;
  const int lo = find_last_le(count, chunk, [&](int i) { return (int64_t)jobs[i].chunk_begin; });
  const BlockJob& J = jobs[lo];
  const int64_t base = (chunk - J.chunk_begin) * kCopyChunk;
  for (int k = 0; k < kCopyChunk / 256; ++k) {
    const int64_t e = base + k * 256 + threadIdx.x;
    if (e >= J.count) break;
    int64_t rem = e, off = 0, stride = 1;
    for (int m = 0; m < J.order; ++m) {
      const int64_t i = rem % J.r[m];
      rem /= J.r[m];
      off += (i + J.off[m]) * stride;
      stride *= J.ext[m];
    }
    const double v = J.src_f64 ? ((const double*)J.src)[e] : (double)((const float*)J.src)[e];
    J.dst[off] = J.alpha * v;
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
                         const GemmSeg* segs, hipStream_t stream, bool grouped) {
  const dim3 block(NTHREADS);
  if (grouped) {
    if (role != R_PROJ_TTM) return hipErrorInvalidValue;
    gemm_kernel<P, R_PROJ_TTM, false, true><<<grid, block, 0, stream>>>(descs, ndesc, segs);
    return hipGetLastError();
  }
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
                       int64_t total_tiles, hipStream_t stream, bool a32, bool grouped) {
  if (ndesc <= 0 || total_tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_tiles), block(NTHREADS);
  if (grouped && (a32 || role != R_PROJ_TTM)) return hipErrorInvalidValue;
  if (a32) {
    // FP32 A operands in an FP64 product: the sketch of FP32-stored inputs
    if (prec != P_FP64) return hipErrorInvalidValue;
    if (role == R_FACTOR_SKETCH)
      gemm_kernel<P_FP64, R_FACTOR_SKETCH, true><<<grid, block, 0, stream>>>(descs, ndesc, segs);
    else if (role == R_TERM_EXPAND)
      gemm_kernel<P_FP64, R_TERM_EXPAND, true><<<grid, block, 0, stream>>>(descs, ndesc, segs);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
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
      return launch_gemm_p<P_FP64>(role, grid, descs, ndesc, segs, stream, grouped);
    case P_FP32: return launch_gemm_p<P_FP32>(role, grid, descs, ndesc, segs, stream, grouped);
    case P_BF16X1: return launch_gemm_p<P_BF16X1>(role, grid, descs, ndesc, segs, stream, grouped);
    case P_BF16X3: return launch_gemm_p<P_BF16X3>(role, grid, descs, ndesc, segs, stream, grouped);
    case P_BF16X6: return launch_gemm_p<P_BF16X6>(role, grid, descs, ndesc, segs, stream, grouped);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_krp(int prec, const KrpDesc* descs, int ndesc, int64_t total_tiles,
                      int lds_elems, hipStream_t stream, bool g32) {
  if (ndesc <= 0 || total_tiles <= 0) return hipSuccess;
  if (lds_elems < 0 || lds_elems > kKrpLds) return hipErrorInvalidValue;
  if (g32) {
    // FP32 cores in an FP64 core sketch
    if (prec != P_FP64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)total_tiles), block(NTHREADS);
    const size_t dyn = (size_t)lds_elems * sizeof(double);
    krp_kernel<P_FP64, true><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)total_tiles), block(NTHREADS);
  const size_t dyn = (size_t)lds_elems * (prec == P_FP64 ? sizeof(double) : sizeof(float));
  switch (prec) {
    case P_FP64: krp_kernel<P_FP64><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems); break;
    case P_FP32: krp_kernel<P_FP32><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems); break;
    case P_BF16X1: krp_kernel<P_BF16X1><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems); break;
    case P_BF16X3: krp_kernel<P_BF16X3><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems); break;
    case P_BF16X6: krp_kernel<P_BF16X6><<<grid, block, dyn, stream>>>(descs, ndesc, lds_elems); break;
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
  tile_reduce_kernel<<<dim3((unsigned)count, kReduceChunks), dim3(NTHREADS), 0, stream>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_block_scatter(const BlockJob* jobs, int count, int64_t chunks,
                                hipStream_t stream) {
  if (count <= 0 || chunks <= 0) return hipSuccess;
  block_scatter_kernel<<<dim3((unsigned)chunks), dim3(256), 0, stream>>>(jobs, count);
  return hipGetLastError();
}

hipError_t launch_copy(const CopyJob* jobs, int count, int64_t chunks, hipStream_t stream) {
  if (count <= 0 || chunks <= 0) return hipSuccess;
  copy_kernel<<<dim3((unsigned)chunks), dim3(256), 0, stream>>>(jobs, count);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  fill_i32_kernel<<<dim3(8), dim3(256), 0, stream>>>(p, count, value);
  return hipGetLastError();
}

}  // namespace tsk
