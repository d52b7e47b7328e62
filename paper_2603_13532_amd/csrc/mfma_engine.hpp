// MFMA tile engine for gfx950 (CDNA4): a 256-thread workgroup (four wave64s)
// computes a 64 x 64 output tile; wave w owns the 32 x 32 quadrant
// (w & 1, w >> 1) as 2 x 2 blocks of 16 x 16 MFMA accumulators.
//
// FP64 tiles use v_mfma_f64_16x16x4_f64 and FP32 tiles v_mfma_f32_16x16x4_f32:
// per instruction each lane supplies A[lane % 16][lane / 16] and
// B[lane / 16][lane % 16] of a 16x4 / 4x16 step.  The FP32 result lands as
// D[4 * (lane / 16) + v][lane % 16], v = 0..3; the FP64 result as
// D[lane / 16 + 4 * v][lane % 16] (both measured on gfx950).
// BF16 tiles use v_mfma_f32_16x16x32_bf16: each lane supplies eight
// consecutive k of its row (A) or column (B), k = 8 * (lane / 16) + 0..7.
//
// Operands are staged through LDS one K-tile at a time, k-major for the
// 4-deep instructions ([BK][64 + pad]) and row-major with k contiguous for
// the BF16 planes ([64][BK + pad]) so that each lane reads its eight k with
// one 16-byte LDS load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace tsk {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

constexpr int TILE = 64;     // output tile edge
constexpr int NTHREADS = 256;

// ------------------------------------------------------------ precision traits
template <int P> struct PT;
template <> struct PT<P_FP64> {
  typedef double in_t;
  typedef v4d acc_t;
  static constexpr int BK = 16;
};
template <> struct PT<P_FP32> {
  typedef float in_t;
  typedef v4f acc_t;
  static constexpr int BK = 16;
};
template <int NP> struct PTBf {
  typedef float in_t;
  typedef v4f acc_t;
  static constexpr int BK = 32;
};
template <> struct PT<P_BF16X1> : PTBf<1> { static constexpr int PARTS = 1; };
template <> struct PT<P_BF16X3> : PTBf<3> { static constexpr int PARTS = 2; };
template <> struct PT<P_BF16X6> : PTBf<6> { static constexpr int PARTS = 3; };

__device__ __forceinline__ v4d mma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mma_bf(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

// ------------------------------------------------------------ LDS layouts
// 4-deep instructions: k-major panels.
template <typename T, int BK> struct LdsK {
  T a[BK][TILE + 2];
  T b[BK][TILE + 2];
};
// BF16: row-major, k contiguous, one plane per split part.
template <int BK, int PARTS> struct alignas(16) LdsBf {
  uint16_t a[PARTS][TILE][BK + 8];
  uint16_t b[PARTS][TILE][BK + 8];
};

template <int P> struct Lds;
template <> struct Lds<P_FP64> { typedef LdsK<double, 16> type; };
template <> struct Lds<P_FP32> { typedef LdsK<float, 16> type; };
template <> struct Lds<P_BF16X1> { typedef LdsBf<32, 1> type; };
template <> struct Lds<P_BF16X3> { typedef LdsBf<32, 2> type; };
template <> struct Lds<P_BF16X6> { typedef LdsBf<32, 3> type; };

// Elements each thread stages per operand per K-tile.
template <int P> struct Stage {
  static constexpr int BK = PT<P>::BK;
  static constexpr int PER_THREAD = TILE * BK / NTHREADS;  // 4 (BK 16) or 8 (BK 32)
};

// Store one staged element (row x in [0,64), depth k in [0,BK)) of operand
// `which` (0 = A, 1 = B) into LDS, splitting into BF16 parts if needed.
template <int P>
__device__ __forceinline__ void lds_put(typename Lds<P>::type& s, int which, int x, int k,
                                        typename PT<P>::in_t v) {
  if constexpr (P == P_FP64 || P == P_FP32) {
    if (which == 0) s.a[k][x] = v; else s.b[k][x] = v;
  } else {
    constexpr int PARTS = PT<P>::PARTS;
    float rest = v;
#pragma unroll
    for (int p = 0; p < PARTS; ++p) {
      uint16_t h = bf16_bits(rest);
      if (which == 0) s.a[p][x][k] = h; else s.b[p][x][k] = h;
      rest = rest - bf16_value(h);
    }
  }
}

// ------------------------------------------------------------ compute step
// One K-tile of the wave's 32 x 32 quadrant, straight-line code with no
// test of the tile edge: rows and columns past it multiply the zeros that
// staging put there.  A branch here would split the K-loop iteration into
// basic blocks that the scheduler cannot interleave, and one wave issues in
// order, so the loads, staging and address arithmetic of the next tile could
// not hide behind these MFMAs.
//
// KW waves share one quadrant (FP64/FP32 only): the wave with `phase` p
// takes the 4-deep steps p, p + KW, ... of each K-tile, so a tile whose
// valid region covers fewer than four quadrants still keeps every wave's
// MFMA pipe busy; the partial accumulators are summed in the epilogue.
//
// MB = 1 (FP64/FP32 only): the quadrant's valid rows all lie in its first
// 16-row block, so only that block row is computed (the second one's
// accumulators stay zero); chosen per wave outside the K-loop.
template <int P, int KW = 1, int MB = 2>
__device__ __forceinline__ void mma_tile(const typename Lds<P>::type& s,
                                         typename PT<P>::acc_t (&acc)[2][2], int lane, int wm,
                                         int wn, int phase = 0) {
  const int r = lane & 15, kq = lane >> 4;
  static_assert(MB == 2 || P == P_FP64 || P == P_FP32, "row-block skipping is FP64/FP32 only");
  if constexpr (P == P_FP64 || P == P_FP32) {
    // Fragments of the whole K-tile are read up front; every 16 x 16 block
    // is computed (MFMAs under per-block branches also make the compiler
    // copy the accumulators between register sets after each one).
    constexpr int NS = PT<P>::BK / 4;
    static_assert(NS % KW == 0, "the waves of a quadrant split the K-tile's steps evenly");
    constexpr int NQ = NS / KW;
    typename PT<P>::in_t a[NQ][2], b[NQ][2];
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
      const int q = (KW == 1) ? qq : phase + KW * qq;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i < MB) a[qq][i] = s.a[4 * q + kq][wm * 32 + 16 * i + r];
        b[qq][i] = s.b[4 * q + kq][wn * 32 + 16 * i + r];
      }
    }
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq)
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mma(a[qq][i], b[qq][j], acc[i][j]);
  } else {
    static_assert(KW == 1, "BF16 K-tiles are one MFMA step deep");
    constexpr int PARTS = PT<P>::PARTS;
    v8s a[PARTS][2], b[PARTS][2];
#pragma unroll
    for (int p = 0; p < PARTS; ++p) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[p][i] = *reinterpret_cast<const v8s*>(&s.a[p][wm * 32 + 16 * i + r][8 * kq]);
        b[p][i] = *reinterpret_cast<const v8s*>(&s.b[p][wn * 32 + 16 * i + r][8 * kq]);
      }
    }
    // smallest cross products first so they are not absorbed early
    auto block = [&](int i, int j) {
      if constexpr (PARTS == 3) {
        acc[i][j] = mma_bf(a[0][i], b[2][j], acc[i][j]);
        acc[i][j] = mma_bf(a[2][i], b[0][j], acc[i][j]);
        acc[i][j] = mma_bf(a[1][i], b[1][j], acc[i][j]);
      }
      if constexpr (PARTS >= 2) {
        acc[i][j] = mma_bf(a[0][i], b[1][j], acc[i][j]);
        acc[i][j] = mma_bf(a[1][i], b[0][j], acc[i][j]);
      }
      acc[i][j] = mma_bf(a[0][i], b[0][j], acc[i][j]);
    };
    block(0, 0);
    block(0, 1);
    block(1, 0);
    block(1, 1);
  }
}

template <int P>
__device__ __forceinline__ void acc_zero(typename PT<P>::acc_t (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
}

// Row/column of accumulator element (i, j, v) inside the 64 x 64 tile.
template <int P>
__device__ __forceinline__ int acc_row(int wm, int i, int lane, int v) {
  if constexpr (P == P_FP64) return wm * 32 + i * 16 + (lane >> 4) + 4 * v;
  else return wm * 32 + i * 16 + 4 * (lane >> 4) + v;
}
__device__ __forceinline__ int acc_col(int wn, int j, int lane) {
  return wn * 32 + j * 16 + (lane & 15);
}

// ------------------------------------------------------------ operand staging
// A 64 x BK panel element (x, k) lives at base[x*sx + k*sk]; exactly one of
// sx, sk is 1.  For the 4-deep FP64/FP32 instructions the thread mapping
// follows the contiguous direction so that the global loads coalesce.  For
// the BF16 forms every thread holds eight consecutive k of one row x
// (x = t % 64), so that each split part goes to LDS as one 16-byte store;
// across a wave the 64 rows of one k are still one coalesced load when x is
// the contiguous direction.  Out-of-range elements are staged as zero.
template <int P>
struct PanelMap {
  static constexpr int BK = PT<P>::BK;
  // element j of thread t
  static __device__ __forceinline__ void xk(bool x_contig, int t, int j, int& x, int& k) {
    if constexpr (P == P_FP64 || P == P_FP32) {
      // both candidates, then a select (no branch between the outputs)
      const int xa = t & (TILE - 1), ka = (t >> 6) + (NTHREADS / TILE) * j;
      const int kb = t % BK, xb = t / BK + (NTHREADS / BK) * j;
      x = x_contig ? xa : xb;
      k = x_contig ? ka : kb;
    } else {
      x = t & (TILE - 1);
      k = 8 * (t >> 6) + j;
    }
  }
};

// BF16 forms: split a thread's eight consecutive k of row x into PARTS bf16
// planes and write each plane with one 16-byte LDS store.
template <int P>
__device__ __forceinline__ void stage_bf(uint16_t (*plane)[TILE][PT<P>::BK + 8], int t,
                                         const float (&v)[8], float scale) {
  constexpr int PARTS = PT<P>::PARTS;
  const int x = t & (TILE - 1), k0 = 8 * (t >> 6);
  v8s out[PARTS];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float rest = v[e] * scale;
#pragma unroll
    for (int p = 0; p < PARTS; ++p) {
      const uint16_t h = bf16_bits(rest);
      out[p][e] = (short)h;
      rest = rest - bf16_value(h);
    }
  }
#pragma unroll
  for (int p = 0; p < PARTS; ++p) *reinterpret_cast<v8s*>(&plane[p][x][k0]) = out[p];
}

// ------------------------------------------------------------ global loads
// Operand loads go through buffer resources: a 32-bit byte offset from a
// tile origin, and any offset past the resource's record count reads as
// zero.  Out-of-range elements therefore cost no branch and no select on the
// loaded value, so a load is never waited for before its K-tile is staged
// (the memory counter completes in order: an early wait would drain every
// K-tile in flight behind it).
// Values that are the same in every lane but reach the compiler through a
// vector register (LDS reads, block-wide counts) are moved to scalar
// registers explicitly; a buffer resource must be scalar, and the compiler
// would otherwise loop over the lanes to make it so.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double uni(double v) {
  return __longlong_as_double((long long)uni((int64_t)__double_as_longlong(v)));
}
template <typename T> __device__ __forceinline__ T* uni(T* p) {
  return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRawWord3 = 0x00020000;       // raw 32-bit data format (CDNA buffer descriptor)
constexpr uint32_t kOob = 0x80000000u;      // an offset that reads as zero
__device__ __forceinline__ rsrc_t make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7FFFFFFF,
                                           kRawWord3);
}
template <typename T> __device__ __forceinline__ T bload(rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

}  // namespace tsk
