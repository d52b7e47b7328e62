// Host side of the C ABI in include/tsk.h: argument validation, the size
// planner, workspace layout, and the stream-ordered launch program of
// Stages 2 and 3 of Algorithms 4 (Kronecker) and 5 (Khatri-Rao).
//
// Every call plans the whole launch sequence first: descriptor tables for
// all grouped kernels are packed into one host blob, copied to the device
// workspace with a single asynchronous upload from pinned staging memory,
// and the kernels read their work lists from there.  Nothing is enqueued
// until validation and planning succeed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tsk.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace tsk;

struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
};

struct ProfRecord {
  std::string name;
  hipEvent_t begin, end;
  double flops, bytes;
  int step = -1;  // index of the launch in its program
};

// One autotuned choice: the value of a launch parameter for a class of
// launches, keyed by (kernel role, precision, log2 of the launch's tiles
// before splitting, log2 of its K-tiles); `us` is the time it measured.
struct TuneEntry {
  int value;
  double us;
};

struct tsk_handle_ {
  int device = 0;
  std::string err;
  bool prof = false;                   // record events around every launch
  std::vector<ProfRecord> prof_records;
  std::vector<hipEvent_t> event_pool;  // reusable timing events
  int64_t* d_counter = nullptr;
  std::vector<Staging> ring;
  size_t ring_next = 0;
  std::vector<void*> device_keep;  // descriptor copies owned by captured graphs
  // tucker_sum_recompress_noalloc: the device address of this device's
  // static scratch array, and pinned staging for its descriptor upload,
  // both set up by tsk_create
  char* scratch_dev = nullptr;
  void* fixed_stage = nullptr;
  hipEvent_t fixed_stage_done = nullptr;
  // autotuned launch parameters (split-K targets, KRP quadrant sharing);
  // while tsk_autotune measures, force_* override every class
  std::map<uint32_t, TuneEntry> tune;
  int force_split = 0, force_kw = 0;
  std::string arch;
  // second stream (default priority, non-blocking) and the events that fork
  // work onto it and join it back
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

// Device memory of tucker_sum_recompress_noalloc: one array per device,
// held from library load until the process ends.  Host code never uses the
// array's name as an address; it uses the per-device pointer that
// hipGetSymbolAddress returns (tsk_handle_::scratch_dev).
constexpr size_t kScratchBytes = TSK_NOALLOC_SCRATCH_BYTES;
constexpr size_t kFixedStageBytes = TSK_NOALLOC_DESCRIPTOR_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kGemmBK64 = 16;

tsk_status fail(tsk_handle h, tsk_status st, const char* fmt, ...) {
  if (h != nullptr) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return st;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
bool is_fp64(int prec) { return prec == P_FP64; }

// ------------------------------------------------------------------ problem
struct Problem {
  int d = 0, s = 0;
  std::vector<int64_t> dims;
  std::vector<int32_t> ranks;  // s*d
  std::vector<const void*> cores, factors;
  std::vector<double> coeffs;
  bool in_f64 = true;
  int kind = TSK_SKETCH_KRP;
  std::vector<int64_t> ow;  // columns of Omega_k
  std::vector<int64_t> W;   // columns of Y_n
  std::vector<int64_t> w;   // columns of Q_n
  uint64_t seed = 0;
  std::vector<const void*> omega;  // caller-given or empty
  int ps = P_FP64, pp = P_FP64;
  int qr_policy = 0;
  int r(int i, int k) const { return ranks[(size_t)i * d + k]; }
};

tsk_status validate_sum(tsk_handle h, const tsk_tucker_sum* sum, Problem& P);
tsk_status validate_spec(tsk_handle h, const tsk_sketch_spec* spec, Problem& P);

tsk_status validate(tsk_handle h, const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                    Problem& P) {
  if (sum == nullptr || spec == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "sum or spec is NULL");
  if (spec->kind != TSK_SKETCH_KRP && spec->kind != TSK_SKETCH_KRON)
    return fail(h, TSK_ERR_INVALID_ARG, "bad sketch kind %d", (int)spec->kind);
  if (spec->sizes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "sketch sizes is NULL");
  if (spec->sketch_prec < TSK_PREC_FP64 || spec->sketch_prec > TSK_PREC_BF16X6 ||
      spec->project_prec < TSK_PREC_FP64 || spec->project_prec > TSK_PREC_BF16X6)
    return fail(h, TSK_ERR_INVALID_ARG, "bad precision");
  if (spec->qr_policy < 0 || spec->qr_policy > 2)
    return fail(h, TSK_ERR_INVALID_ARG, "bad qr_policy %d", spec->qr_policy);
  if (tsk_status st = validate_sum(h, sum, P); st != TSK_OK) return st;
  P.kind = spec->kind;
  P.seed = spec->seed;
  P.ps = spec->sketch_prec;
  P.pp = spec->project_prec;
  P.qr_policy = spec->qr_policy;
  return validate_spec(h, spec, P);
}

// The Tucker sum alone: order, terms, sizes and pointers.
tsk_status validate_sum(tsk_handle h, const tsk_tucker_sum* sum, Problem& P) {
  if (sum == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "sum is NULL");
  if (sum->order < 2 || sum->order > kMaxOrder)
    return fail(h, TSK_ERR_INVALID_ARG, "order %d outside [2, %d]", sum->order, kMaxOrder);
  if (sum->num_terms < 1) return fail(h, TSK_ERR_INVALID_ARG, "num_terms %d < 1", sum->num_terms);
  if (sum->dims == nullptr || sum->ranks == nullptr || sum->cores == nullptr ||
      sum->factors == nullptr)
    return fail(h, TSK_ERR_INVALID_ARG, "dims, ranks, cores or factors is NULL");
  if (sum->dtype != TSK_F64 && sum->dtype != TSK_F32)
    return fail(h, TSK_ERR_INVALID_ARG, "bad dtype %d", (int)sum->dtype);
  P.d = sum->order;
  P.s = sum->num_terms;
  P.in_f64 = sum->dtype == TSK_F64;
  for (int k = 0; k < P.d; ++k) {
    if (sum->dims[k] < 1) return fail(h, TSK_ERR_INVALID_ARG, "dims[%d] = %lld < 1", k, (long long)sum->dims[k]);
    if (sum->dims[k] > (1 << 30)) return fail(h, TSK_ERR_UNSUPPORTED, "dims[%d] too large", k);
    P.dims.push_back(sum->dims[k]);
  }
  for (int i = 0; i < P.s; ++i) {
    if (sum->cores[i] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "cores[%d] is NULL", i);
    P.cores.push_back(sum->cores[i]);
    int64_t csize = 1;
    for (int k = 0; k < P.d; ++k) {
      const int32_t r = sum->ranks[(size_t)i * P.d + k];
      if (r < 1) return fail(h, TSK_ERR_INVALID_ARG, "ranks[%d][%d] = %d < 1", i, k, r);
      if (r > (1 << 20)) return fail(h, TSK_ERR_UNSUPPORTED, "ranks[%d][%d] too large", i, k);
      P.ranks.push_back(r);
      csize *= r;
      if (csize > (int64_t(1) << 40)) return fail(h, TSK_ERR_UNSUPPORTED, "core %d too large", i);
      const void* f = sum->factors[(size_t)i * P.d + k];
      if (f == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "factors[%d][%d] is NULL", i, k);
      P.factors.push_back(f);
    }
    P.coeffs.push_back(sum->coeffs ? sum->coeffs[i] : 1.0);
  }
  return TSK_OK;
}

// Sketch sizes and widths of a validated sum.
tsk_status validate_spec(tsk_handle h, const tsk_sketch_spec* spec, Problem& P) {
  if (P.kind == TSK_SKETCH_KRP) {
    if (spec->sizes[0] < 1) return fail(h, TSK_ERR_INVALID_ARG, "KRP width %d < 1", spec->sizes[0]);
    for (int k = 0; k < P.d; ++k) {
      P.ow.push_back(spec->sizes[0]);
      P.W.push_back(spec->sizes[0]);
    }
  } else {
    for (int k = 0; k < P.d; ++k) {
      if (spec->sizes[k] < 1) return fail(h, TSK_ERR_INVALID_ARG, "Kron q[%d] = %d < 1", k, spec->sizes[k]);
      P.ow.push_back(spec->sizes[k]);
    }
    for (int n = 0; n < P.d; ++n) {
      int64_t S = 1;
      for (int k = 0; k < P.d; ++k)
        if (k != n) {
          S *= P.ow[k];
          if (S > (1 << 24)) return fail(h, TSK_ERR_UNSUPPORTED, "Kron sketch width too large");
        }
      P.W.push_back(S);
    }
  }
  if (P.kind == TSK_SKETCH_KRP) {
    // the Khatri-Rao kernels address a whole core through 31-bit byte offsets
    const int64_t es = P.ps == P_FP64 ? 8 : 4;
    for (int i = 0; i < P.s; ++i) {
      int64_t cs = 1;
      for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
      if (cs * es >= (int64_t(1) << 31))
        return fail(h, TSK_ERR_UNSUPPORTED, "core %d exceeds 2^31 bytes in the sketch precision", i);
    }
  }
  for (int n = 0; n < P.d; ++n) {
    P.w.push_back(std::min(P.dims[n], P.W[n]));
    if (P.dims[n] * P.W[n] > (int64_t(1) << 34))
      return fail(h, TSK_ERR_UNSUPPORTED, "sketch of mode %d too large", n);
  }
  if (spec->omega != nullptr) {
    for (int k = 0; k < P.d; ++k) {
      if (spec->omega[k] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "omega[%d] is NULL", k);
      P.omega.push_back(spec->omega[k]);
    }
  }
  return TSK_OK;
}

// ------------------------------------------------------------------ program
// S_FORK makes the handle's second stream wait for the work enqueued so
// far; steps marked `side` then run on that stream, and S_JOIN makes the
// caller's stream wait for them (in a captured graph: two branches).
enum StepKind { S_OMEGA, S_GEMM, S_KRP, S_REDUCE, S_TILE_REDUCE, S_COPY, S_FILL, S_CHOL, S_HOUSE,
                S_KRP_ADJ, S_SYM, S_TRSM, S_EIG, S_SCATTER, S_FORK, S_JOIN };

struct Step {
  StepKind kind;
  int prec = 0;
  int role = R_OTHER;
  double flops = 0, bytes = 0;  // algorithmic work of the launch
  size_t meta = 0, meta2 = 0;  // offsets into the meta blob
  int count = 0;
  int64_t tiles = 0;
  // omega / fill
  uint64_t seed = 0;
  int mode = 0, pass = 0, force = 0;
  int64_t rows = 0, cols = 0;
  void* ptr = nullptr;  // workspace address (resolved)
  bool f64 = true;
  int32_t value = 0;
  double tol = 0;
  int wmax = 0;  // chol: widest Gram of the launch
  int hh_sel = 3;             // householder: modes taken (bit 0 direct, bit 1 broken down)
  int hh_grid[2] = {0, 0};    // householder: workgroups of the register / general kernel
  bool side = false;          // runs on the handle's second stream (between S_FORK and S_JOIN)
  int krp_lds = 0;     // krp: LDS elements for the P slices (largest that fits)
  std::vector<uint32_t> keys;  // autotuning classes whose choices shaped this launch
  bool a32 = false;  // FP64 GEMM / core sketch whose A operands (cores) are stored in FP32
  bool grouped = false;  // GEMM: some descriptors group one-tile batch elements (bpw > 1)
};

// LDS elements a KRP launch needs for its P slices: the largest slice set
// (64 columns of every P_k, k != n) among its descriptors that fits
// kKrpLds; larger ones read P from global memory.
int krp_lds_elems(const KrpDesc* kd, size_t count) {
  int need = 0;
  for (size_t j = 0; j < count; ++j) {
    int tot = 0;
    for (int k = 0; k < kd[j].order; ++k)
      if (k != kd[j].mode) tot += 64 * kd[j].r[k];
    if (tot <= kKrpLds) need = std::max(need, tot);
  }
  return need;
}

// Workspace arena: addresses are planned against a base that may be null
// (size query) and resolved when the caller's workspace is known.
struct Arena {
  char* base = nullptr;
  size_t top = 0;
  // int32 words of per-mode state (QR breakdown flags), one block; each flag
  // is written by the first Cholesky pass before anything reads it
  int32_t* ctr_base = nullptr;
  int64_t ctr_used = 0;
  // Set when a planned launch would address an operand element beyond what
  // the kernels' 31-bit in-tile byte offsets reach; the call then fails with
  // TSK_ERR_UNSUPPORTED before anything is enqueued.
  std::string too_far;
  void* take(size_t bytes) {
    top = align_up(top, 256);
    void* p = base + top;
    top += align_up(bytes, 256);
    return p;
  }
  int32_t* counters(int64_t n) {
    int32_t* p = ctr_base + ctr_used;
    ctr_used += n;
    return p;
  }
};

struct Program {
  std::vector<char> blob;
  std::vector<Step> steps;
  size_t meta_region = 0;  // workspace offset of the blob
  template <typename T>
  size_t put(const std::vector<T>& v) {
    size_t off = align_up(blob.size(), 64);
    blob.resize(off + sizeof(T) * v.size());
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), sizeof(T) * v.size());
    return off;
  }
};

// Collects grouped-GEMM descriptors for one launch.
struct GemmBatch {
  int prec;
  int role;
  std::vector<GemmDesc> descs;
  std::vector<GemmSeg> segs;
  std::vector<ReduceJob> reduces;
  int64_t tiles = 0;
  double flops = 0, bytes = 0;
  std::vector<uint32_t> keys;  // autotuning classes of its split decisions
  bool a32 = false;            // every A operand stored in FP32 (prec FP64)
  GemmBatch(int p, int r, Arena* a) : prec(p), role(r), ar(a) {}
  // Add one descriptor; `splits` > 1 writes partials to `part` and queues a
  // reduction into C.
  Arena* ar = nullptr;
  void add(void* C, bool c_f64, int64_t ldc, int64_t strideC, int M, int N, int batch, int beta,
           const std::vector<GemmSeg>& sg, int splits = 1, void* part_unused = nullptr) {
    (void)part_unused;
    if (M <= 0 || N <= 0 || batch <= 0) return;
    GemmDesc D{};
    D.M = M;
    D.N = N;
    D.batch = batch;
    D.tiles_m = (int)ceil_div(M, 64);
    D.tiles_n = (int)ceil_div(N, 64);
    D.seg_begin = (int)segs.size();
    D.seg_count = (int)sg.size();
    D.c_f64 = c_f64 ? 1 : 0;
    D.splits = splits;
    D.C = C;
    D.ldc = ldc;
    D.strideC = strideC;
    D.bpw = 1;
    D.beta = beta;
    D.part = nullptr;
    if (splits > 1) {
      const int64_t ntiles = (int64_t)D.tiles_m * D.tiles_n * batch;
      const size_t pe = prec == P_FP64 ? 8 : 4;
      D.part = ar->take((size_t)ntiles * splits * 64 * 64 * pe);
      // one reduce job per output tile, in the kernel's tile order
      for (int64_t tl = 0; tl < ntiles; ++tl) {
        const int tm = (int)(tl % D.tiles_m);
        const int tn = (int)((tl / D.tiles_m) % D.tiles_n);
        const int64_t bb = tl / ((int64_t)D.tiles_m * D.tiles_n);
        ReduceJob J{};
        J.out = (char*)C + ((size_t)bb * strideC + (size_t)tm * 64 + (size_t)tn * 64 * ldc) * (c_f64 ? 8 : 4);
        J.part = (char*)D.part + (size_t)tl * splits * 64 * 64 * pe;
        J.rows = std::min<int64_t>(64, M - tm * 64);
        J.cols = std::min<int64_t>(64, N - tn * 64);
        J.ld_out = ldc;
        J.ld_part = 64;
        J.stride_part = 64 * 64;
        J.parts = splits;
        J.beta = beta;
        J.out_f64 = c_f64 ? 1 : 0;
        J.part_f64 = prec == P_FP64 ? 1 : 0;
        reduces.push_back(J);
      }
    }
    D.tile_begin = tiles;
    tiles += (int64_t)D.tiles_m * D.tiles_n * batch * splits;
    const double ein = prec == P_FP64 ? 8.0 : 4.0, ec = c_f64 ? 8.0 : 4.0;
    for (const auto& g : sg) {
      // The K-loop reads a 64 x BK panel through 32-bit byte offsets from the
      // panel origin, and offsets from 2^31 up read as zero: the farthest
      // element, 63 rows and BK - 1 depths away, must stay below that.
      const int64_t es = prec == P_FP64 ? 8 : 4, bk = 32;
      const int64_t farA = (63 * std::abs(g.a_sx) + (bk - 1) * std::abs(g.a_sk)) * es;
      const int64_t farB = (63 * std::abs(g.b_sx) + (bk - 1) * std::abs(g.b_sk)) * es;
      if (std::max(farA, farB) >= (int64_t(1) << 31) && ar->too_far.empty())
        ar->too_far = "an operand stride reaches past 2^31 bytes inside one 64-row tile";
      segs.push_back(g);
      flops += 2.0 * M * N * (double)g.K * batch;
      bytes += ein * (double)M * g.K * (g.strideA != 0 ? batch : 1) +
               ein * (double)g.K * N * (g.strideB != 0 ? batch : 1);
    }
    bytes += ec * (double)M * N * batch * (beta ? 2 : 1);
    descs.push_back(D);
  }
};

GemmSeg seg(const void* A, int64_t a_sx, int64_t a_sk, int64_t sA, const void* B, int64_t b_sx,
            int64_t b_sk, int64_t sB, int64_t K, double alpha = 1.0) {
  GemmSeg g{};
  g.A = A;
  g.B = B;
  g.a_sx = a_sx;
  g.a_sk = a_sk;
  g.strideA = sA;
  g.b_sx = b_sx;
  g.b_sk = b_sk;
  g.strideB = sB;
  g.K = (int32_t)K;
  g.alpha = alpha;
  return g;
}

int64_t tiles_of(const GemmDesc& d) {
  return (int64_t)d.tiles_m * d.tiles_n * ceil_div(d.batch, std::max<int32_t>(d.bpw, 1)) * d.splits;
}
int64_t tiles_of(const KrpDesc& d) { return (int64_t)d.tiles_m * d.tiles_n * d.splits; }

// Workgroups are dispatched in tile order, so a descriptor's place in its
// launch decides when its tiles start.  Descriptors go longest tile first
// (K per split, descending; equal ones keep their order) so that no long
// tile starts last and runs alone at the end of the launch, and tile_begin
// is renumbered.  Each tile's arithmetic does not depend on the order.
template <typename D, typename KofD>
int64_t longest_first(std::vector<D>& ds, KofD k_of) {
  std::vector<size_t> idx(ds.size());
  std::vector<int64_t> key(ds.size());
  for (size_t i = 0; i < ds.size(); ++i) {
    idx[i] = i;
    key[i] = ceil_div(k_of(ds[i]), (int64_t)std::max<int32_t>(ds[i].splits, 1));
  }
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return key[a] > key[b]; });
  std::vector<D> out;
  out.reserve(ds.size());
  int64_t tiles = 0;
  for (size_t i : idx) {
    D d = ds[i];
    d.tile_begin = tiles;
    tiles += tiles_of(d);
    out.push_back(d);
  }
  ds.swap(out);
  return tiles;
}

// Projection TTM launches of many one-tile batch elements (the later modes,
// one element per trailing index; such a launch runs a separate grouped
// kernel, so every other launch keeps the one-tile body) give each
// workgroup bpw consecutive elements, so that a tile's descriptor search and segment load are paid
// once per group; bpw grows with the launch's element count (one per
// kBpwElems elements, at most kMaxBpw), keeping several rounds of workgroups.
constexpr int64_t kBpwElems = 8192;
constexpr int kMaxBpw = 8;
bool groupable(const GemmDesc& d) { return d.tiles_m == 1 && d.tiles_n == 1 && d.splits == 1 && d.batch > 1; }
void group_batches(std::vector<GemmDesc>& ds) {
  int64_t elems = 0;
  for (const GemmDesc& d : ds)
    if (groupable(d)) elems += d.batch;
  const int bpw = (int)std::min<int64_t>(kMaxBpw, std::max<int64_t>(1, elems / kBpwElems));
  if (bpw < 2) return;
  for (GemmDesc& d : ds)
    if (groupable(d)) d.bpw = bpw;
}

void emit_gemm(Program& prog, GemmBatch& gb) {
  if (gb.descs.empty()) return;
  if (gb.role == R_PROJ_TTM) group_batches(gb.descs);  // the only role with a grouped kernel
  gb.tiles = longest_first(gb.descs, [&](const GemmDesc& d) {
    int64_t K = 0;
    for (int j = 0; j < d.seg_count; ++j) K += gb.segs[d.seg_begin + j].K;
    return K * std::min<int64_t>(std::max<int32_t>(d.bpw, 1), d.batch);
  });
  Step st{};
  st.kind = S_GEMM;
  st.prec = gb.prec;
  st.role = gb.role;
  // algorithmic flops: the QR's Gram is symmetric and its basis step a
  // triangular solve, n W^2 each, although the kernel forms the full product
  st.flops = (gb.role == R_QR_GRAM || gb.role == R_QR_BASIS) ? gb.flops / 2 : gb.flops;
  st.bytes = gb.bytes;
  st.meta = prog.put(gb.descs);
  st.meta2 = prog.put(gb.segs);
  st.count = (int)gb.descs.size();
  st.tiles = gb.tiles;
  st.keys = gb.keys;
  st.a32 = gb.a32;
  for (const GemmDesc& d : gb.descs) st.grouped = st.grouped || d.bpw > 1;
  prog.steps.push_back(st);
  if (!gb.reduces.empty()) {
    Step r{};
    r.kind = S_TILE_REDUCE;
    r.keys = gb.keys;  // the split choice also sets the reduction's work
    for (const ReduceJob& J : gb.reduces)
      r.bytes += (double)J.rows * J.cols * (J.parts + 1 + J.beta) * (J.out_f64 ? 8 : 4);
    r.meta = prog.put(gb.reduces);
    r.count = (int)gb.reduces.size();
    prog.steps.push_back(r);
  }
}

void emit_copies(Program& prog, std::vector<CopyJob> jobs) {
  if (jobs.empty()) return;
  Step c{};
  c.kind = S_COPY;
  int64_t chunks = 0;
  for (CopyJob& J : jobs) {
    J.chunk_begin = chunks;
    chunks += (J.rows * J.cols + kCopyChunk - 1) / kCopyChunk;
    c.bytes += (double)(J.rows * J.cols) * ((J.src_f64 ? 8 : 4) + (J.dst_f64 ? 8 : 4));
  }
  c.tiles = chunks;
  c.meta = prog.put(jobs);
  c.count = (int)jobs.size();
  prog.steps.push_back(c);
}

// K-splits so that a launch stays within one round of resident workgroups
// (target = CUs x workgroups per CU): a launch just past that size would run
// a second, nearly empty round and take twice as long.
int choose_splits(int64_t tiles_without_split, int64_t k_tiles, int64_t target = 512) {
  if (tiles_without_split >= target || k_tiles < 4) return 1;
  int64_t s = target / tiles_without_split;
  s = std::min<int64_t>(s, k_tiles / 2);
  s = std::min<int64_t>(s, 32);
  return (int)std::max<int64_t>(s, 1);
}

// Autotuning classes.  A key packs the launch parameter (split-K target of
// a GEMM role or of the KRP core sketch, or the KRP quadrant sharing), the
// precision and two log2 shape buckets: the output tiles the launch has
// before splitting, and the K-tiles of its longest product.
constexpr int kTuneKrpSplit = 16, kTuneKrpKw = 17;
int lg2(int64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    ++l;
  }
  return l;
}
uint32_t tune_key(int cls, int prec, int64_t tiles, int64_t ktiles) {
  return (uint32_t)(cls & 31) << 20 | (uint32_t)(prec & 15) << 16 |
         (uint32_t)std::min(lg2(tiles), 255) << 8 | (uint32_t)std::min(lg2(ktiles), 255);
}

size_t esize(bool f64) { return f64 ? 8 : 4; }

// What the call produces.
struct Outputs {
  bool recompress = false;
  std::vector<double*> Y;  // sketch-only: caller Y buffers
  std::vector<void*> Q;
  void* H = nullptr;
  bool out_f64 = true;
  std::vector<double*> R;
};

// Stages of the launch program, in execution order.  Every sum planned into
// one Builder contributes descriptors to the same stage launches, so a batch
// of independent sums costs the same number of launches as one sum.
enum StageId {
  ST_CONVERT = 0, ST_OMEGA = 1, ST_FACTOR = 2, ST_KRP = 3, ST_KRON = 4,  // ST_KRON + step
  ST_EXPAND = 20, ST_GRAM1 = 21, ST_BASIS1 = 22, ST_GRAM2 = 23, ST_BASIS2 = 24,
  ST_QCOPY = 30, ST_PROJW = 31, ST_TTM = 32,  // ST_TTM + k
  ST_FINAL = 50
};

typedef OmegaJobDev OmegaJob;

struct Builder {
  Arena& ar;
  int nsums = 1;  // sums sharing the launches (scales the split-K decision)
  std::map<int, GemmBatch> gemm;
  std::map<int, std::vector<CopyJob>> copies;
  std::vector<OmegaJob> omega;
  double omega_bytes = 0;
  std::vector<KrpDesc> krp;
  std::vector<ReduceJob> krp_red;
  int krp_prec = 0;
  int64_t krp_tiles = 0;
  double krp_flops = 0, krp_bytes = 0;
  std::vector<QrDesc> qr;
  bool any_chol = false;
  int64_t* d_counter = nullptr;
  const tsk_handle_* th = nullptr;  // its tuning table, if any
  std::vector<uint32_t> krp_keys;
  // FP64 sketch of FP32-stored inputs (every sum of the plan, KRP): the
  // factor sketch, core sketch and term expansion read the FP32 cores and
  // factors directly instead of FP64 copies
  bool direct32 = false;
  explicit Builder(Arena& a) : ar(a) {}
  GemmBatch& g(int stage, int prec, int role) {
    auto it = gemm.find(stage);
    if (it == gemm.end()) it = gemm.emplace(stage, GemmBatch(prec, role, &ar)).first;
    return it->second;
  }
  // The tuned value of class `key`, the forced one while tuning, else dflt.
  int tuned(uint32_t key, int force, int dflt) const {
    if (th == nullptr) return dflt;
    if (force > 0) return force;
    auto it = th->tune.find(key);
    return it == th->tune.end() ? dflt : it->second.value;
  }
  // K-splits of one sum's share of a grouped GEMM launch (the launch holds
  // nsums such shares): the split target comes from the tuning table.
  int splits(GemmBatch& gb, int64_t tiles_without_split, int64_t k_tiles, int64_t target = 512) {
    const int64_t tiles = tiles_without_split * nsums;
    const uint32_t key = tune_key(gb.role, gb.prec, tiles, k_tiles);
    if (std::find(gb.keys.begin(), gb.keys.end(), key) == gb.keys.end()) gb.keys.push_back(key);
    return choose_splits(tiles, k_tiles, tuned(key, th ? th->force_split : 0, (int)target));
  }
  int krp_splits(int prec, int64_t tiles_without_split, int64_t k_tiles) {
    const int64_t tiles = tiles_without_split * nsums;
    const uint32_t key = tune_key(kTuneKrpSplit, prec, tiles, k_tiles);
    if (std::find(krp_keys.begin(), krp_keys.end(), key) == krp_keys.end()) krp_keys.push_back(key);
    return choose_splits(tiles, k_tiles, tuned(key, th ? th->force_split : 0, 1024));
  }
  int krp_kw(int prec, int64_t tiles_without_split, int64_t k_tiles) {
    const uint32_t key = tune_key(kTuneKrpKw, prec, tiles_without_split * nsums, k_tiles);
    if (std::find(krp_keys.begin(), krp_keys.end(), key) == krp_keys.end()) krp_keys.push_back(key);
    return tuned(key, th ? th->force_kw : 0, 4);
  }
  void emit(Program& prog);
};

// Thin QR (FP64, diag R >= 0) of the n_k x W_k matrices Y[k] into Q[k]
// (n_k x min(n_k, W_k)) and, when R is not empty, R[k] (min(n_k, W_k) x
// W_k): Cholesky QR2 where W_k <= 96 <= ... fits (W_k <= min(96, n_k) and
// policy != 1), with a device-side Householder fallback on breakdown, and
// Householder directly otherwise.  `rank_bound` (optional): an upper bound
// on rank(Y[k]); under policy 0 a mode whose bound is below W_k has a
// singular Gram, so it skips the Cholesky attempt that would break down.
void plan_qr(Builder& B, const std::vector<int64_t>& dims, const std::vector<int64_t>& Wd,
             const std::vector<const double*>& Y, const std::vector<double*>& Q,
             const std::vector<double*>& R, int qr_policy,
             const std::vector<int64_t>& rank_bound = {}) {
  Arena& ar = B.ar;
  const int d = (int)dims.size();
  std::vector<QrDesc> qd(d);
  int32_t* flags = ar.counters(d);
  for (int n = 0; n < d; ++n) {
    const int64_t nn = dims[n], W = Wd[n], w = std::min(nn, W);
    QrDesc& q = qd[n];
    q.Y = Y[n];
    q.Q = Q[n];
    q.R = R.empty() ? nullptr : R[n];
    q.n = nn;
    q.W = W;
    q.w = w;
    q.flag = flags + n;
    q.hh = (double*)ar.take((nn * W + W) * 8);  // panel, then the R-diagonal signs
    q.tau = (double*)ar.take(W * 8);
    const bool deficient = qr_policy == 0 && !rank_bound.empty() && rank_bound[n] < W;
    const bool chol = qr_policy != 1 && W <= 96 && W <= nn && !deficient;
    q.hh_direct = chol ? 0 : 1;
    q.report_only = qr_policy == 2 ? 1 : 0;
    if (chol) {
      B.any_chol = true;
      q.gram_splits = (int)std::min<int64_t>(16, std::max<int64_t>(1, nn / 64));
      q.gram_part = (double*)ar.take((size_t)q.gram_splits * W * W * 8);
      q.rinv = (double*)ar.take(W * W * 8);
      q.r1 = (double*)ar.take(W * W * 8);
      q.q1 = (double*)ar.take(nn * W * 8);
    }
  }
  for (int pass = 1; pass <= 2; ++pass) {
    GemmBatch& gram = B.g(pass == 1 ? ST_GRAM1 : ST_GRAM2, P_FP64, R_QR_GRAM);
    GemmBatch& qq = B.g(pass == 1 ? ST_BASIS1 : ST_BASIS2, P_FP64, R_QR_BASIS);
    for (int n = 0; n < d; ++n) {
      const QrDesc& q = qd[n];
      if (q.gram_part == nullptr) continue;
      const double* src = pass == 1 ? q.Y : q.q1;
      // K-split of the Gram over row blocks, partials summed by the Cholesky kernel
      const int64_t rows_per = ceil_div(q.n, q.gram_splits);
      for (int sp = 0; sp < q.gram_splits; ++sp) {
        const int64_t r0 = sp * rows_per, rl = std::max<int64_t>(0, std::min<int64_t>(rows_per, q.n - r0));
        double* C = q.gram_part + (size_t)sp * q.W * q.W;
        // an empty block (K = 0) writes zeros
        gram.add(C, true, q.W, 0, (int)q.W, (int)q.W, 1, 0,
                 {seg(rl > 0 ? src + r0 : src, q.n, 1, 0, rl > 0 ? src + r0 : src, q.n, 1, 0, rl)});
      }
      double* dst = pass == 1 ? q.q1 : q.Q;
      qq.add(dst, true, q.n, 0, (int)q.n, (int)q.W, 1, 0,
             {seg(src, 1, q.n, 0, q.rinv, q.W, 1, 0, q.W)});
    }
  }
  for (auto& q : qd) B.qr.push_back(q);
}

// Stage 3 (Section 3.3): W_k^(i) = Q_k^T U_k^(i), then the multi-TTM
// H = sum_i c_i G^(i) x_1 W_1^(i) ... x_d W_d^(i), modes 0..d-2 per term and
// the last mode K-concatenated over the terms.  Q[n] is n_n x w_n (FP64 when
// q_f64, else FP32); core_s / fac_s are the inputs already held in the
// sketch element type (s64), reused when it is also the projection's.
void build_projection(const Problem& P, const std::vector<const void*>& Q, bool q_f64,
                      const std::vector<const void*>& core_s,
                      const std::vector<const void*>& fac_s, bool s64, void* H, bool out_f64,
                      Builder& B) {
  Arena& ar = B.ar;
  const int d = P.d, s = P.s;
  const bool tp64 = is_fp64(P.pp);
  const size_t ep = esize(tp64);
  const bool ts64 = s64;
  std::vector<const void*> Qp(d);
  std::vector<CopyJob>& cq = B.copies[ST_QCOPY];
  for (int n = 0; n < d; ++n) {
    if (tp64 == q_f64) {
      Qp[n] = Q[n];
    } else {
      void* p = ar.take(P.dims[n] * P.w[n] * ep);
      cq.push_back(CopyJob{p, Q[n], P.dims[n], P.w[n], P.dims[n], P.dims[n], tp64 ? 1 : 0,
                           q_f64 ? 1 : 0});
      Qp[n] = p;
    }
  }
  // inputs in the projection element type
  std::vector<const void*> core_p(s), fac_p((size_t)s * d);
  for (int i = 0; i < s; ++i) {
    int64_t csize = 1;
    for (int k = 0; k < d; ++k) csize *= P.r(i, k);
    if (P.in_f64 == tp64) {
      core_p[i] = P.cores[i];
    } else if (ts64 == tp64) {
      core_p[i] = core_s[i];
    } else {
      void* p = ar.take(csize * ep);
      cq.push_back(CopyJob{p, P.cores[i], csize, 1, csize, csize, tp64, P.in_f64});
      core_p[i] = p;
    }
    for (int k = 0; k < d; ++k) {
      const size_t idx = (size_t)i * d + k;
      if (P.in_f64 == tp64) {
        fac_p[idx] = P.factors[idx];
      } else if (ts64 == tp64) {
        fac_p[idx] = fac_s[idx];
      } else {
        void* p = ar.take(P.dims[k] * P.r(i, k) * ep);
        cq.push_back(CopyJob{p, P.factors[idx], P.dims[k], P.r(i, k), P.dims[k], P.dims[k], tp64,
                             P.in_f64});
        fac_p[idx] = p;
      }
    }
  }
  // The last mode is contracted over all terms at once: its W blocks (each
  // scaled by its term's coefficient) sit side by side in one w x sum_i r
  // matrix, and the last TTM writes every term's result side by side in one
  // L x sum_i r matrix, so that the final product is one dense K range.
  std::vector<int64_t> koff(s + 1, 0);
  for (int i = 0; i < s; ++i) koff[i + 1] = koff[i] + P.r(i, d - 1);
  int64_t Lfin = 1;
  for (int k = 0; k < d - 1; ++k) Lfin *= P.w[k];
  char* Wlast = (char*)ar.take(P.w[d - 1] * koff[s] * ep);
  char* Ucat = (char*)ar.take(Lfin * koff[s] * ep);
  std::vector<void*> Wm((size_t)s * d);
  {
    GemmBatch& gb = B.g(ST_PROJW, P.pp, R_PROJ_W);
    int64_t tiles0 = 0, kt = 0;
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        tiles0 += ceil_div(P.w[k], 64) * ceil_div(P.r(i, k), 64);
        kt = std::max<int64_t>(kt, ceil_div(P.dims[k], tp64 ? 16 : 32));
      }
    const int splits = B.splits(gb, tiles0, kt);
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        const int64_t n = P.dims[k], r = P.r(i, k), w = P.w[k];
        const bool last = k == d - 1;
        void* p = last ? (void*)(Wlast + (size_t)(w * koff[i]) * ep) : ar.take(w * r * ep);
        Wm[(size_t)i * d + k] = p;
        gb.add(p, tp64, w, 0, (int)w, (int)r, 1, 0,
               {seg(Qp[k], n, 1, 0, fac_p[(size_t)i * d + k], n, 1, 0, n,
                    last ? P.coeffs[i] : 1.0)}, splits);
      }
  }
  // multi-TTM, modes 0..d-2 per term, then the last mode K-concatenated over terms
  std::vector<std::vector<int64_t>> shape(s);
  std::vector<const void*> cur(s);
  std::vector<void*> buf0(s), buf1(s);
  for (int i = 0; i < s; ++i) {
    for (int k = 0; k < d; ++k) shape[i].push_back(P.r(i, k));
    // outputs of the TTMs before the last (which writes into Ucat), in two
    // alternating buffers
    int64_t mx = 0;
    std::vector<int64_t> sh = shape[i];
    for (int k = 0; k < d - 2; ++k) {
      sh[k] = P.w[k];
      int64_t sz = 1;
      for (auto x : sh) sz *= x;
      mx = std::max(mx, sz);
    }
    buf0[i] = d > 2 ? ar.take(mx * ep) : nullptr;
    buf1[i] = d > 3 ? ar.take(mx * ep) : nullptr;
    cur[i] = core_p[i];
  }
  for (int k = 0; k < d - 1; ++k) {
    GemmBatch& gb = B.g(ST_TTM + k, P.pp, R_PROJ_TTM);
    for (int i = 0; i < s; ++i) {
      const int64_t rk = shape[i][k], w = P.w[k];
      const void* Wk = Wm[(size_t)i * d + k];  // w x r_k
      void* outp = (k == d - 2) ? (void*)(Ucat + (size_t)(Lfin * koff[i]) * ep)
                                : ((k % 2 == 0) ? buf0[i] : buf1[i]);
      int64_t L = 1, Rr = 1;
      for (int j = 0; j < k; ++j) L *= shape[i][j];
      for (int j = k + 1; j < d; ++j) Rr *= shape[i][j];
      if (k == 0) {
        gb.add(outp, tp64, w, 0, (int)w, (int)Rr, 1, 0, {seg(Wk, 1, w, 0, cur[i], rk, 1, 0, rk)});
      } else {
        gb.add(outp, tp64, L, L * w, (int)L, (int)w, (int)Rr, 0,
               {seg(cur[i], 1, L, L * rk, Wk, 1, w, 0, rk)});
      }
      shape[i][k] = w;
      cur[i] = outp;
    }
  }
  {
    GemmBatch& gb = B.g(ST_FINAL, P.pp, R_PROJ_FINAL);
    const int64_t L = Lfin, w = P.w[d - 1];
    const int64_t kt = ceil_div(koff[s], tp64 ? 16 : 32);
    const int splits = B.splits(gb, ceil_div(L, 64) * ceil_div(w, 64), kt);
    gb.add(H, out_f64, L, 0, (int)L, (int)w, 1, 0, {seg(Ucat, 1, L, 0, Wlast, 1, w, 0, koff[s])},
           splits);
  }
}


// Build the launch program for one Tucker sum.  All workspace addresses come
// from `ar`; the meta blob is placed last by the caller.
void build_sum(const Problem& P, const Outputs& out, Builder& B) {
  Arena& ar = B.ar;
  const int d = P.d, s = P.s;
  const bool ts64 = is_fp64(P.ps);  // sketch-stage element type
  const bool tp64 = is_fp64(P.pp);  // projection-stage element type
  const size_t es = esize(ts64), ep = esize(tp64);

  // ---- inputs in the sketch element type (converted copies if needed)
  std::vector<CopyJob>& conv = B.copies[ST_CONVERT];
  std::vector<const void*> core_s(s), fac_s((size_t)s * d);
  for (int i = 0; i < s; ++i) {
    int64_t csize = 1;
    for (int k = 0; k < d; ++k) csize *= P.r(i, k);
    if (P.in_f64 == ts64 || B.direct32) {
      core_s[i] = P.cores[i];
    } else {
      void* p = ar.take(csize * es);
      conv.push_back(CopyJob{p, P.cores[i], csize, 1, csize, csize, ts64, P.in_f64});
      core_s[i] = p;
    }
    for (int k = 0; k < d; ++k) {
      const int64_t n = P.dims[k], r = P.r(i, k);
      const void* u = P.factors[(size_t)i * d + k];
      if (P.in_f64 == ts64 || B.direct32) {
        fac_s[(size_t)i * d + k] = u;
      } else {
        void* p = ar.take(n * r * es);
        conv.push_back(CopyJob{p, u, n, r, n, n, ts64, P.in_f64});
        fac_s[(size_t)i * d + k] = p;
      }
    }
  }
  // ---- Omega_k (Section 3.1), in the sketch element type
  std::vector<const void*> om(d);
  for (int k = 0; k < d; ++k) {
    if (!P.omega.empty()) {
      if (P.in_f64 == ts64) {
        om[k] = P.omega[k];
      } else {
        void* p = ar.take(P.dims[k] * P.ow[k] * es);
        conv.push_back(CopyJob{p, P.omega[k], P.dims[k], P.ow[k], P.dims[k], P.dims[k], ts64,
                               P.in_f64});
        om[k] = p;
      }
    } else {
      void* p = ar.take(P.dims[k] * P.ow[k] * es);
      B.omega.push_back(OmegaJob{p, P.dims[k] * P.ow[k], P.seed, k, ts64 ? 1 : 0});
      B.omega_bytes += (double)P.dims[k] * P.ow[k] * es;
      om[k] = p;
    }
  }
  // ---- factor sketches P_k^(i) = U_k^(i)^T Omega_k  (r x ow), all terms and modes
  std::vector<void*> Pf((size_t)s * d);
  {
    GemmBatch& gb = B.g(ST_FACTOR, P.ps, R_FACTOR_SKETCH);
    gb.a32 = B.direct32;
    int64_t tiles0 = 0, kt = 0;
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        tiles0 += ceil_div(P.r(i, k), 64) * ceil_div(P.ow[k], 64);
        kt = std::max<int64_t>(kt, ceil_div(P.dims[k], ts64 ? 16 : 32));
      }
    const int splits = B.splits(gb, tiles0, kt);
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        const int64_t n = P.dims[k], r = P.r(i, k), m = P.ow[k];
        void* p = ar.take(r * m * es);
        Pf[(size_t)i * d + k] = p;
        gb.add(p, ts64, r, 0, (int)r, (int)m, 1, 0,
               {seg(fac_s[(size_t)i * d + k], n, 1, 0, om[k], n, 1, 0, n)}, splits);
      }
  }

  // ---- core sketches V^(i)_(n)
  std::vector<void*> V((size_t)s * d);
  if (P.kind == TSK_SKETCH_KRP) {
    const int64_t m = P.ow[0];
    std::vector<KrpDesc>& kd = B.krp;
    std::vector<ReduceJob>& red = B.krp_red;
    int64_t tiles0 = 0, ktmax = 0;
    for (int i = 0; i < s; ++i)
      for (int n = 0; n < d; ++n) {
        int64_t Kc = 1;
        for (int k = 0; k < d; ++k)
          if (k != n) Kc *= P.r(i, k);
        tiles0 += ceil_div(P.r(i, n), 64) * ceil_div(m, 64);
        ktmax = std::max<int64_t>(ktmax, ceil_div(Kc, ts64 ? 16 : 32));
      }
    // the Khatri-Rao expansion makes a KRP K-tile costly, so several rounds
    // of short workgroups beat one round of long ones
    const int splits = B.krp_splits(P.ps, tiles0, ktmax);
    const int kw_max = B.krp_kw(P.ps, tiles0, ktmax);
    int64_t& tiles = B.krp_tiles;
    const size_t kd_first = kd.size();
    for (int i = 0; i < s; ++i)
      for (int n = 0; n < d; ++n) {
        KrpDesc D{};
        D.G = core_s[i];
        int64_t Kc = 1;
        for (int k = 0; k < kMaxOrder; ++k) {
          D.r[k] = k < d ? P.r(i, k) : 1;
          D.P[k] = k < d ? Pf[(size_t)i * d + k] : nullptr;
          if (k < d && k != n) Kc *= P.r(i, k);
        }
        const int64_t rn = P.r(i, n);
        D.order = d;
        D.mode = n;
        D.m = (int)m;
        D.Kc = Kc;
        D.alpha = 1.0;
        D.tiles_m = (int)ceil_div(rn, 64);
        D.tiles_n = (int)ceil_div(m, 64);
        void* v = ar.take(rn * m * es);
        V[(size_t)i * d + n] = v;
        const int sp = (int)std::min<int64_t>(splits, std::max<int64_t>(1, ceil_div(Kc, ts64 ? 16 : 32) / 2));
        D.splits = sp;
        D.V = v;
        D.kw_max = kw_max;
        D.part = nullptr;
            if (sp > 1) {
          const int64_t ntiles = (int64_t)D.tiles_m * D.tiles_n;
          D.part = ar.take((size_t)ntiles * sp * 64 * 64 * es);
          for (int64_t tl = 0; tl < ntiles; ++tl) {
            const int tm = (int)(tl % D.tiles_m), tn = (int)(tl / D.tiles_m);
            ReduceJob J{};
            J.out = (char*)v + ((size_t)tm * 64 + (size_t)tn * 64 * rn) * es;
            J.part = (char*)D.part + (size_t)tl * sp * 64 * 64 * es;
            J.rows = std::min<int64_t>(64, rn - tm * 64);
            J.cols = std::min<int64_t>(64, m - tn * 64);
            J.ld_out = rn;
            J.ld_part = 64;
            J.stride_part = 64 * 64;
            J.parts = sp;
            J.beta = 0;
            J.out_f64 = J.part_f64 = ts64 ? 1 : 0;
            red.push_back(J);
          }
        }
        D.tile_begin = tiles;
        tiles += (int64_t)D.tiles_m * D.tiles_n * sp;
        kd.push_back(D);
      }
    B.krp_prec = P.ps;
    for (size_t j = kd_first; j < kd.size(); ++j) {
      const KrpDesc& D = kd[j];
      int64_t cs = 1;
      double pbytes = 0;
      for (int k = 0; k < d; ++k) {
        cs *= D.r[k];
        if (k != D.mode) pbytes += (double)D.r[k] * D.m * es;
      }
      B.krp_flops += 2.0 * D.r[D.mode] * D.m * (double)D.Kc;
      // algorithmic bytes: each core once per term (not once per mode), the
      // factor sketches it multiplies, and the output
      B.krp_bytes += (D.mode == 0 ? (double)cs * es : 0.0) + pbytes + (double)D.r[D.mode] * D.m * es;
    }
  } else {
    // Kronecker: V = G x_{k != n} (Omega_k^T U_k), TTM chain in ascending mode order
    // (Algorithm 4, inner loop), all (term, mode) chains advanced together.
    struct Chain {
      std::vector<int64_t> shape;
      const void* cur;
      void* buf[2];
      int which;
      int i, n;
    };
    std::vector<Chain> ch;
    for (int i = 0; i < s; ++i)
      for (int n = 0; n < d; ++n) {
        Chain c;
        for (int k = 0; k < d; ++k) c.shape.push_back(P.r(i, k));
        c.cur = core_s[i];
        // largest intermediate along the chain
        int64_t mx = 1;
        std::vector<int64_t> sh = c.shape;
        for (int k = 0; k < d; ++k) {
          if (k == n) continue;
          sh[k] = P.ow[k];
          int64_t sz = 1;
          for (auto x : sh) sz *= x;
          mx = std::max(mx, sz);
        }
        c.buf[0] = ar.take(mx * es);
        c.buf[1] = ar.take(mx * es);
        c.which = 0;
        c.i = i;
        c.n = n;
        ch.push_back(c);
      }
    for (int step = 0; step < d - 1; ++step) {
      GemmBatch& gb = B.g(ST_KRON + step, P.ps, R_KRON_TTM);
      for (auto& c : ch) {
        // the step-th mode other than n
        int k = -1, cnt = 0;
        for (int j = 0; j < d; ++j)
          if (j != c.n) {
            if (cnt == step) k = j;
            ++cnt;
          }
        const int64_t rk = c.shape[k], q = P.ow[k];
        const void* Pk = Pf[(size_t)c.i * d + k];  // r_k x q_k
        void* outp = c.buf[c.which];
        int64_t L = 1, Rr = 1;
        for (int j = 0; j < k; ++j) L *= c.shape[j];
        for (int j = k + 1; j < d; ++j) Rr *= c.shape[j];
        if (k == 0) {
          // out (q x Rr) = P_0^T (q x r_0) . T_(0) (r_0 x Rr)
          gb.add(outp, ts64, q, 0, (int)q, (int)Rr, 1, 0,
                 {seg(Pk, rk, 1, 0, c.cur, rk, 1, 0, rk)});
        } else {
          // per trailing index: out_b (L x q) = T_b (L x r_k) . P_k (r_k x q)
          gb.add(outp, ts64, L, L * q, (int)L, (int)q, (int)Rr, 0,
                 {seg(c.cur, 1, L, L * rk, Pk, rk, 1, 0, rk)});
        }
        c.shape[k] = q;
        c.cur = outp;
        c.which ^= 1;
      }
    }
    for (auto& c : ch) V[(size_t)c.i * d + c.n] = (void*)c.cur;
  }

  // ---- term expansion Y_n = sum_i c_i U_n^(i) V^(i)_(n)  (FP64 output)
  std::vector<double*> Y(d);
  for (int n = 0; n < d; ++n)
    Y[n] = out.recompress ? (double*)ar.take(P.dims[n] * P.W[n] * 8) : out.Y[n];
  {
    GemmBatch& gb = B.g(ST_EXPAND, P.ps, R_TERM_EXPAND);
    gb.a32 = B.direct32;
    // K-split over the term concatenation when the output tiles alone cannot fill the GPU
    int64_t tiles0 = 0, kt = 0;
    const int bk = ts64 ? 16 : 32;
    for (int n = 0; n < d; ++n) {
      int64_t L = 1, T = 1;
      if (P.kind == TSK_SKETCH_KRON) {
        for (int k = 0; k < n; ++k) L *= P.ow[k];
        for (int k = n + 1; k < d; ++k) T *= P.ow[k];
      } else {
        L = P.W[n];
      }
      tiles0 += ceil_div(P.dims[n], 64) * ceil_div(L, 64) * T;
      int64_t ktn = 0;
      for (int i = 0; i < s; ++i) ktn += ceil_div(P.r(i, n), bk);
      kt = std::max(kt, ktn);
    }
    const int splits = B.splits(gb, tiles0, kt);
    for (int n = 0; n < d; ++n) {
      const int64_t nn = P.dims[n];
      std::vector<GemmSeg> sg;
      if (P.kind == TSK_SKETCH_KRP) {
        for (int i = 0; i < s; ++i) {
          const int64_t r = P.r(i, n);
          sg.push_back(seg(fac_s[(size_t)i * d + n], 1, nn, 0, V[(size_t)i * d + n], r, 1, 0, r,
                           P.coeffs[i]));
        }
        gb.add(Y[n], true, nn, 0, (int)nn, (int)P.W[n], 1, 0, sg, splits);
      } else {
        int64_t L = 1, T = 1;
        for (int k = 0; k < n; ++k) L *= P.ow[k];
        for (int k = n + 1; k < d; ++k) T *= P.ow[k];
        for (int i = 0; i < s; ++i) {
          const int64_t r = P.r(i, n);
          sg.push_back(seg(fac_s[(size_t)i * d + n], 1, nn, 0, V[(size_t)i * d + n], 1, L, L * r,
                           r, P.coeffs[i]));
        }
        gb.add(Y[n], true, nn, nn * L, (int)nn, (int)L, (int)T, 0, sg, splits);
      }
    }
  }
  if (!out.recompress) return;

  // ---- thin QR of every Y_n in FP64
  std::vector<double*> Qd(d);
  for (int n = 0; n < d; ++n)
    Qd[n] = out.out_f64 ? (double*)out.Q[n] : (double*)ar.take(P.dims[n] * P.w[n] * 8);
  // Y_n = X_(n) S_n lies in the span of the terms' mode-n factors, so its
  // rank is at most the sum's total mode-n rank
  std::vector<int64_t> total_rank(d, 0);
  for (int n = 0; n < d; ++n)
    for (int i = 0; i < s; ++i) total_rank[n] += P.r(i, n);
  plan_qr(B, P.dims, P.W, std::vector<const double*>(Y.begin(), Y.end()), Qd, out.R, P.qr_policy,
          total_rank);

  // ---- core projection (Section 3.3)
  std::vector<CopyJob>& cq = B.copies[ST_QCOPY];
  if (!out.out_f64)
    for (int n = 0; n < d; ++n)
      cq.push_back(CopyJob{out.Q[n], Qd[n], P.dims[n], P.w[n], P.dims[n], P.dims[n], 0, 1});
  // an FP32-class projection reads the FP32 output bases (written by the
  // same copy launch, before it) instead of converting Q a second time
  const bool q_out32 = !out.out_f64 && !is_fp64(P.pp);
  std::vector<const void*> Qc = q_out32 ? std::vector<const void*>(out.Q.begin(), out.Q.end())
                                        : std::vector<const void*>(Qd.begin(), Qd.end());
  build_projection(P, Qc, !q_out32, core_s, fac_s, ts64 && !B.direct32, out.H, out.out_f64, B);
}

void Builder::emit(Program& prog) {
  auto emit_copy_stage = [&](int stage) {
    auto it = copies.find(stage);
    if (it != copies.end()) emit_copies(prog, it->second);
  };
  auto emit_gemm_stage = [&](int stage) {
    auto it = gemm.find(stage);
    if (it != gemm.end()) emit_gemm(prog, it->second);
  };
  emit_copy_stage(ST_CONVERT);
  if (!omega.empty()) {
    Step st{};
    st.kind = S_OMEGA;
    st.meta = prog.put(omega);
    st.count = (int)omega.size();
    st.bytes = omega_bytes;
    for (const OmegaJob& j : omega) st.rows = std::max<int64_t>(st.rows, j.count);
    prog.steps.push_back(st);
  }
  emit_gemm_stage(ST_FACTOR);
  if (!krp.empty()) {
    Step st{};
    st.kind = S_KRP;
    st.prec = krp_prec;
    st.flops = krp_flops;
    st.bytes = krp_bytes;
    longest_first(krp, [](const KrpDesc& d) { return d.Kc; });
    st.meta = prog.put(krp);
    st.count = (int)krp.size();
    st.tiles = krp_tiles;
    st.krp_lds = krp_lds_elems(krp.data(), krp.size());
    st.keys = krp_keys;
    st.a32 = direct32;
    prog.steps.push_back(st);
    if (!krp_red.empty()) {
      Step r{};
      r.kind = S_TILE_REDUCE;
      r.keys = krp_keys;
      for (const ReduceJob& J : krp_red)
        r.bytes += (double)J.rows * J.cols * (J.parts + 1) * (J.out_f64 ? 8 : 4);
      r.meta = prog.put(krp_red);
      r.count = (int)krp_red.size();
      prog.steps.push_back(r);
    }
  }
  for (int st = ST_KRON; st < ST_EXPAND; ++st) emit_gemm_stage(st);
  emit_gemm_stage(ST_EXPAND);
  if (!qr.empty()) {
    const size_t qmeta = prog.put(qr);
    // modes planned for Householder directly and modes that try Cholesky QR
    // first, per kernel kind (register kernel, general kernel)
    int direct[2] = {0, 0}, tried[2] = {0, 0};
    int64_t general_elems = 0;
    for (const QrDesc& q : qr) {
      const int k = hh_wide_panel(q.n, q.W) ? 0 : 1;
      (q.hh_direct ? direct : tried)[k] += 1;
      if (k == 1) general_elems = std::max<int64_t>(general_elems, (q.n + 1) * q.W + 2 * q.W);
    }
    auto house = [&](int sel, int grid_reg, int grid_gen, bool side) {
      Step hh{};
      hh.kind = S_HOUSE;
      hh.meta = qmeta;
      hh.count = (int)qr.size();
      hh.ptr = d_counter;
      hh.hh_sel = sel;
      hh.hh_grid[0] = grid_reg;
      hh.hh_grid[1] = grid_gen;
      hh.rows = general_elems;
      hh.side = side;
      prog.steps.push_back(hh);
    };
    // the direct modes need nothing from the Cholesky passes: they run on the
    // second stream, beside the passes of the other modes
    const bool fork = any_chol && direct[0] + direct[1] > 0;
    if (fork) {
      Step f{};
      f.kind = S_FORK;
      prog.steps.push_back(f);
      house(1, direct[0], direct[1], true);
    }
    if (any_chol) {
      for (int pass = 1; pass <= 2; ++pass) {
        emit_gemm_stage(pass == 1 ? ST_GRAM1 : ST_GRAM2);
        Step c{};
        c.kind = S_CHOL;
        c.meta = qmeta;
        c.count = (int)qr.size();
        c.pass = pass;
        c.tol = pass == 1 ? 1e-11 : 1e-2;
        for (const QrDesc& q : qr)
          if (q.gram_part != nullptr) {
            c.wmax = std::max(c.wmax, (int)q.W);
            const double W = (double)q.W;
            c.flops += W * W * W / 3.0;  // the Cholesky factorization
            c.bytes += 8.0 * W * W * (q.gram_splits + 2);
          }
        prog.steps.push_back(c);
        emit_gemm_stage(pass == 1 ? ST_BASIS1 : ST_BASIS2);
      }
    }
    if (fork)
      house(2, tried[0], tried[1], false);
    else
      house(3, direct[0] + tried[0], direct[1] + tried[1], false);
    if (fork) {
      Step j{};
      j.kind = S_JOIN;
      prog.steps.push_back(j);
    }
  }
  emit_copy_stage(ST_QCOPY);
  emit_gemm_stage(ST_PROJW);
  for (int st = ST_TTM; st < ST_FINAL; ++st) emit_gemm_stage(st);
  emit_gemm_stage(ST_FINAL);
}

// ------------------------------------------------------------------ backward
// Buffers of one backward call (see tucker_sum_recompress_backward).
struct BackwardIO {
  std::vector<const void*> Q;       // forward Q_n (out dtype)
  std::vector<const double*> R;     // forward R_n (FP64, w x w)
  const void* Hbar = nullptr;       // out dtype
  std::vector<const void*> Qbar;    // out dtype, or empty
  bool out_f64 = true;              // dtype of Q, Hbar, Qbar
  std::vector<void*> core_bar;      // sum dtype
  std::vector<void*> factor_bar;    // sum dtype, [s*d]
  unsigned long long* singular = nullptr;  // counter of singular R_n (or null)
};

// Reverse mode of the KRP recompression, in the order of the oracle's
// derivation: recompute P, V, W; project H_bar back (G_bar, W_bar, Q_bar);
// thin-QR adjoint in FP64; term expansion, core sketch and factor sketch
// adjoints; sum the contributions.
void build_backward(const Problem& P, const BackwardIO& io, Arena& ar, Program& prog) {
  const int d = P.d, s = P.s;
  const int pc = P.ps;                 // one arithmetic for every contraction
  const bool tc64 = is_fp64(pc);
  const size_t ec = esize(tc64);
  std::vector<CopyJob> conv;
  auto as_tc = [&](const void* src, bool src_f64, int64_t rows, int64_t cols) -> const void* {
    if (src_f64 == tc64) return src;
    void* p = ar.take(rows * cols * ec);
    conv.push_back(CopyJob{p, src, rows, cols, rows, rows, tc64, src_f64});
    return p;
  };
  std::vector<const void*> core(s), fac((size_t)s * d);
  std::vector<int64_t> csize(s, 1);
  for (int i = 0; i < s; ++i) {
    for (int k = 0; k < d; ++k) csize[i] *= P.r(i, k);
    core[i] = as_tc(P.cores[i], P.in_f64, csize[i], 1);
    for (int k = 0; k < d; ++k)
      fac[(size_t)i * d + k] = as_tc(P.factors[(size_t)i * d + k], P.in_f64, P.dims[k], P.r(i, k));
  }
  std::vector<const void*> Qc(d);
  std::vector<const double*> Q64(d);
  int64_t hsize = 1;
  for (int n = 0; n < d; ++n) {
    Qc[n] = as_tc(io.Q[n], io.out_f64, P.dims[n], P.w[n]);
    Q64[n] = (const double*)(io.out_f64 ? io.Q[n] : as_tc(io.Q[n], false, P.dims[n], P.w[n]));
    hsize *= P.w[n];
  }
  if (!io.out_f64 && !tc64) {
    // as_tc above returned the float Q for Q64: make a real FP64 copy
    for (int n = 0; n < d; ++n) {
      void* p = ar.take(P.dims[n] * P.w[n] * 8);
      conv.push_back(CopyJob{p, io.Q[n], P.dims[n], P.w[n], P.dims[n], P.dims[n], 1, 0});
      Q64[n] = (const double*)p;
    }
  }
  const void* Hb = as_tc(io.Hbar, io.out_f64, hsize, 1);
  // Q_bar accumulators (FP64), seeded with the caller's Q_bar
  std::vector<double*> Qb(d);
  for (int n = 0; n < d; ++n) {
    Qb[n] = (double*)ar.take(P.dims[n] * P.w[n] * 8);
    if (!io.Qbar.empty())
      conv.push_back(CopyJob{Qb[n], io.Qbar[n], P.dims[n], P.w[n], P.dims[n], P.dims[n], 1,
                             io.out_f64 ? 1 : 0});
  }
  // Omega
  std::vector<OmegaJob> om_jobs;
  std::vector<const void*> om(d);
  for (int k = 0; k < d; ++k) {
    if (!P.omega.empty()) {
      om[k] = as_tc(P.omega[k], P.in_f64, P.dims[k], P.ow[k]);
    } else {
      void* p = ar.take(P.dims[k] * P.ow[k] * ec);
      om_jobs.push_back(OmegaJob{p, P.dims[k] * P.ow[k], P.seed, k, tc64 ? 1 : 0});
      om[k] = p;
    }
  }
  emit_copies(prog, conv);
  if (!om_jobs.empty()) {
    Step st{};
    st.kind = S_OMEGA;
    st.meta = prog.put(om_jobs);
    st.count = (int)om_jobs.size();
    for (const OmegaJob& j : om_jobs) st.rows = std::max<int64_t>(st.rows, j.count);
    prog.steps.push_back(st);
  }
  const int64_t m = P.ow[0];
  const int bk = tc64 ? 16 : 32;
  // ---- recompute P_k = U_k^T Omega_k and W_k = Q_k^T U_k
  std::vector<void*> Pf((size_t)s * d), Wm((size_t)s * d);
  {
    GemmBatch gb(pc, R_FACTOR_SKETCH, &ar);
    GemmBatch gw(pc, R_PROJ_W, &ar);
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        const int64_t n = P.dims[k], r = P.r(i, k), w = P.w[k];
        Pf[(size_t)i * d + k] = ar.take(r * m * ec);
        gb.add(Pf[(size_t)i * d + k], tc64, r, 0, (int)r, (int)m, 1, 0,
               {seg(fac[(size_t)i * d + k], n, 1, 0, om[k], n, 1, 0, n)},
               choose_splits((int64_t)s * d * ceil_div(r, 64) * ceil_div(m, 64), ceil_div(n, bk)));
        Wm[(size_t)i * d + k] = ar.take(w * r * ec);
        gw.add(Wm[(size_t)i * d + k], tc64, w, 0, (int)w, (int)r, 1, 0,
               {seg(Qc[k], n, 1, 0, fac[(size_t)i * d + k], n, 1, 0, n)},
               choose_splits((int64_t)s * d * ceil_div(w, 64) * ceil_div(r, 64), ceil_div(n, bk)));
      }
    emit_gemm(prog, gb);
    emit_gemm(prog, gw);
  }
  // ---- recompute V_n = G_(n) KR_n (KRP kernel, no split)
  std::vector<void*> V((size_t)s * d);
  auto krp_step = [&](std::vector<KrpDesc>& kd, int64_t tiles) {
    if (kd.empty()) return;
    Step st{};
    st.kind = S_KRP;
    st.prec = pc;
    st.meta = prog.put(kd);
    st.count = (int)kd.size();
    st.tiles = tiles;
    st.krp_lds = krp_lds_elems(kd.data(), kd.size());
    prog.steps.push_back(st);
  };
  auto krp_desc = [&](int i, int mode, const std::vector<const void*>& fs, void* out,
                      int64_t& tiles) {
    KrpDesc D{};
    D.G = core[i];
    int64_t Kc = 1;
    for (int k = 0; k < kMaxOrder; ++k) {
      D.r[k] = k < d ? P.r(i, k) : 1;
      D.P[k] = k < d ? fs[k] : nullptr;
      if (k < d && k != mode) Kc *= P.r(i, k);
    }
    D.order = d;
    D.mode = mode;
    D.m = (int)m;
    D.Kc = Kc;
    D.alpha = 1.0;
    D.tiles_m = (int)ceil_div(P.r(i, mode), 64);
    D.tiles_n = (int)ceil_div(m, 64);
    D.splits = 1;
    D.kw_max = 4;
    D.V = out;
    D.tile_begin = tiles;
    tiles += (int64_t)D.tiles_m * D.tiles_n;
    return D;
  };
  {
    std::vector<KrpDesc> kd;
    int64_t tiles = 0;
    for (int i = 0; i < s; ++i) {
      std::vector<const void*> fs(d);
      for (int k = 0; k < d; ++k) fs[k] = Pf[(size_t)i * d + k];
      for (int n = 0; n < d; ++n) {
        V[(size_t)i * d + n] = ar.take(P.r(i, n) * m * ec);
        kd.push_back(krp_desc(i, n, fs, V[(size_t)i * d + n], tiles));
      }
    }
    krp_step(kd, tiles);
  }
  // ---- projection adjoint: Z_k = H_bar x_{j != k} W_j^T (chains), W_bar, G_bar
  std::vector<void*> Zk((size_t)s * d);
  {
    struct Chain {
      std::vector<int64_t> shape;
      const void* cur;
      void* buf[2];
      int which, i, k;
    };
    std::vector<Chain> ch;
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        Chain c;
        for (int j = 0; j < d; ++j) c.shape.push_back(P.w[j]);
        c.cur = Hb;
        int64_t mx = 1;
        std::vector<int64_t> sh = c.shape;
        for (int j = 0; j < d; ++j) {
          if (j == k) continue;
          sh[j] = P.r(i, j);
          int64_t sz = 1;
          for (auto x : sh) sz *= x;
          mx = std::max(mx, sz);
        }
        c.buf[0] = ar.take(mx * ec);
        c.buf[1] = ar.take(mx * ec);
        c.which = 0;
        c.i = i;
        c.k = k;
        ch.push_back(c);
      }
    for (int step = 0; step < d - 1; ++step) {
      GemmBatch gb(pc, R_PROJ_TTM, &ar);
      for (auto& c : ch) {
        int j = -1, cnt = 0;
        for (int q = 0; q < d; ++q)
          if (q != c.k) {
            if (cnt == step) j = q;
            ++cnt;
          }
        const int64_t wj = c.shape[j], rj = P.r(c.i, j);
        const void* Wj = Wm[(size_t)c.i * d + j];  // w_j x r_j
        void* outp = c.buf[c.which];
        int64_t L = 1, Rr = 1;
        for (int q = 0; q < j; ++q) L *= c.shape[q];
        for (int q = j + 1; q < d; ++q) Rr *= c.shape[q];
        if (j == 0) {
          // out (r_0 x Rr) = W_0^T (r_0 x w_0) . T_(0) (w_0 x Rr)
          gb.add(outp, tc64, rj, 0, (int)rj, (int)Rr, 1, 0, {seg(Wj, wj, 1, 0, c.cur, wj, 1, 0, wj)});
        } else {
          // out_b (L x r_j) = T_b (L x w_j) . W_j (w_j x r_j)
          gb.add(outp, tc64, L, L * rj, (int)L, (int)rj, (int)Rr, 0,
                 {seg(c.cur, 1, L, L * wj, Wj, wj, 1, 0, wj)});
        }
        c.shape[j] = rj;
        c.cur = outp;
        c.which ^= 1;
      }
      emit_gemm(prog, gb);
    }
    for (auto& c : ch) Zk[(size_t)c.i * d + c.k] = (void*)c.cur;
  }
  // W_bar_k = c_i Z_k,(k) G_(k)^T (w_k x r_k); G_bar_proj = c_i Z_{d-1} x_{d-1} W_{d-1}^T
  std::vector<void*> Wb((size_t)s * d), gparts(s);
  {
    GemmBatch gb(pc, R_OTHER, &ar);
    GemmBatch gg(pc, R_PROJ_FINAL, &ar);
    for (int i = 0; i < s; ++i) {
      gparts[i] = ar.take((size_t)(d + 1) * csize[i] * ec);  // slot 0: projection, 1..d: sketch
      for (int k = 0; k < d; ++k) {
        const int64_t w = P.w[k], r = P.r(i, k);
        Wb[(size_t)i * d + k] = ar.take(w * r * ec);
        const void* Z = Zk[(size_t)i * d + k];
        int64_t L = 1, T = 1;
        for (int q = 0; q < k; ++q) L *= P.r(i, q);
        for (int q = k + 1; q < d; ++q) T *= P.r(i, q);
        std::vector<GemmSeg> sg;
        int64_t ktiles = 0;
        if (k == 0) {
          sg.push_back(seg(Z, 1, w, 0, core[i], 1, r, 0, csize[i] / r, P.coeffs[i]));
          ktiles = ceil_div(csize[i] / r, bk);
        } else {
          for (int64_t t = 0; t < T; ++t) {
            sg.push_back(seg((const char*)Z + (size_t)t * L * w * ec, L, 1, 0,
                             (const char*)core[i] + (size_t)t * L * r * ec, L, 1, 0, L, P.coeffs[i]));
            ktiles += ceil_div(L, bk);
          }
        }
        gb.add(Wb[(size_t)i * d + k], tc64, w, 0, (int)w, (int)r, 1, 0, sg,
               choose_splits((int64_t)s * d * ceil_div(w, 64) * ceil_div(r, 64), ktiles));
      }
      // slot 0 of G_bar: c_i Z_{d-1} (L x w) . W_{d-1} (w x r)
      const int k = d - 1;
      const int64_t w = P.w[k], r = P.r(i, k);
      const int64_t L = csize[i] / r;
      gg.add(gparts[i], tc64, L, 0, (int)L, (int)r, 1, 0,
             {seg(Zk[(size_t)i * d + k], 1, L, 0, Wm[(size_t)i * d + k], w, 1, 0, w, P.coeffs[i])});
    }
    emit_gemm(prog, gb);
    emit_gemm(prog, gg);
  }
  // ---- Q_bar_k += sum_i U_k^(i) W_bar_k^(i)T (FP64 accumulator)
  {
    GemmBatch gb(pc, R_OTHER, &ar);
    for (int k = 0; k < d; ++k) {
      const int64_t n = P.dims[k], w = P.w[k];
      std::vector<GemmSeg> sg;
      for (int i = 0; i < s; ++i)
        sg.push_back(seg(fac[(size_t)i * d + k], 1, n, 0, Wb[(size_t)i * d + k], 1, w, 0, P.r(i, k)));
      gb.add(Qb[k], true, n, 0, (int)n, (int)w, 1, io.Qbar.empty() ? 0 : 1, sg);
    }
    emit_gemm(prog, gb);
  }
  // ---- thin-QR adjoint (FP64): M = -Q_bar^T Q, S = copyltu(M), Z = Q_bar + Q S, Y_bar = Z R^-T
  std::vector<double*> Mm(d), Sm(d);
  {
    GemmBatch gm(P_FP64, R_OTHER, &ar);
    for (int k = 0; k < d; ++k) {
      const int64_t n = P.dims[k], w = P.w[k];
      Mm[k] = (double*)ar.take(w * w * 8);
      Sm[k] = (double*)ar.take(w * w * 8);
      gm.add(Mm[k], true, w, 0, (int)w, (int)w, 1, 0, {seg(Qb[k], n, 1, 0, Q64[k], n, 1, 0, n, -1.0)},
             choose_splits(d * ceil_div(w, 64) * ceil_div(w, 64), ceil_div(n, 16)));
    }
    emit_gemm(prog, gm);
    std::vector<SymJob> sj;
    for (int k = 0; k < d; ++k) sj.push_back(SymJob{Mm[k], Sm[k], P.w[k]});
    Step st{};
    st.kind = S_SYM;
    st.meta = prog.put(sj);
    st.count = d;
    prog.steps.push_back(st);
    GemmBatch gz(P_FP64, R_OTHER, &ar);
    for (int k = 0; k < d; ++k) {
      const int64_t n = P.dims[k], w = P.w[k];
      gz.add(Qb[k], true, n, 0, (int)n, (int)w, 1, 1, {seg(Q64[k], 1, n, 0, Sm[k], w, 1, 0, w)});
    }
    emit_gemm(prog, gz);
    std::vector<TrsmJob> tj;
    for (int k = 0; k < d; ++k)
      for (int64_t r0 = 0; r0 < P.dims[k]; r0 += 64)
        tj.push_back(TrsmJob{Qb[k], io.R[k], Qb[k], P.dims[k], P.w[k], r0,
                             (int32_t)std::min<int64_t>(64, P.dims[k] - r0), 0, io.singular});
    Step tr{};
    tr.kind = S_TRSM;
    tr.meta = prog.put(tj);
    tr.count = (int)tj.size();
    prog.steps.push_back(tr);
  }
  // Y_bar in the contraction type
  std::vector<const void*> Yb(d);
  {
    std::vector<CopyJob> cj;
    for (int k = 0; k < d; ++k) {
      if (tc64) {
        Yb[k] = Qb[k];
      } else {
        void* p = ar.take(P.dims[k] * P.w[k] * 4);
        cj.push_back(CopyJob{p, Qb[k], P.dims[k], P.w[k], P.dims[k], P.dims[k], 0, 1});
        Yb[k] = p;
      }
    }
    emit_copies(prog, cj);
  }
  // ---- V_bar_n^(i) = c_i U_n^(i)T Y_bar_n
  std::vector<void*> Vb((size_t)s * d);
  {
    GemmBatch gb(pc, R_OTHER, &ar);
    for (int i = 0; i < s; ++i)
      for (int n = 0; n < d; ++n) {
        const int64_t nn = P.dims[n], r = P.r(i, n);
        Vb[(size_t)i * d + n] = ar.take(r * m * ec);
        gb.add(Vb[(size_t)i * d + n], tc64, r, 0, (int)r, (int)m, 1, 0,
               {seg(fac[(size_t)i * d + n], nn, 1, 0, Yb[n], nn, 1, 0, nn, P.coeffs[i])},
               choose_splits((int64_t)s * d * ceil_div(r, 64) * ceil_div(m, 64), ceil_div(nn, bk)));
      }
    emit_gemm(prog, gb);
  }
  // ---- P_bar_k = sum_{n != k} G_(k) KR(P_j, j != k with V_bar_n at n): d-1 slots, then a sum
  std::vector<void*> Pb((size_t)s * d), Pslots((size_t)s * d);
  {
    std::vector<KrpDesc> kd;
    int64_t tiles = 0;
    std::vector<ReduceJob> red;
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        const int64_t r = P.r(i, k);
        Pslots[(size_t)i * d + k] = ar.take((size_t)(d - 1) * r * m * ec);
        Pb[(size_t)i * d + k] = ar.take(r * m * ec);
        int slot = 0;
        for (int n = 0; n < d; ++n) {
          if (n == k) continue;
          std::vector<const void*> fs(d);
          for (int j = 0; j < d; ++j) fs[j] = (j == n) ? Vb[(size_t)i * d + n] : Pf[(size_t)i * d + j];
          kd.push_back(krp_desc(i, k, fs, (char*)Pslots[(size_t)i * d + k] + (size_t)slot * r * m * ec,
                                tiles));
          ++slot;
        }
        red.push_back(ReduceJob{Pb[(size_t)i * d + k], Pslots[(size_t)i * d + k], r, m, r, r, r * m,
                                d - 1, 0, tc64 ? 1 : 0, tc64 ? 1 : 0});
      }
    krp_step(kd, tiles);
    Step st{};
    st.kind = S_REDUCE;
    st.meta = prog.put(red);
    st.count = (int)red.size();
    prog.steps.push_back(st);
  }
  // ---- G_bar slots 1..d: V_bar_n KR_n^T through the mode-n unfolding
  {
    std::vector<KrpAdjDesc> ad;
    int64_t tiles = 0;
    for (int i = 0; i < s; ++i)
      for (int n = 0; n < d; ++n) {
        KrpAdjDesc D{};
        D.Vbar = Vb[(size_t)i * d + n];
        int64_t Nc = 1;
        for (int k = 0; k < kMaxOrder; ++k) {
          D.r[k] = k < d ? P.r(i, k) : 1;
          D.P[k] = k < d ? Pf[(size_t)i * d + k] : nullptr;
          if (k < d && k != n) Nc *= P.r(i, k);
        }
        D.Gout = (char*)gparts[i] + (size_t)(1 + n) * csize[i] * ec;
        D.order = d;
        D.mode = n;
        D.m = (int)m;
        D.Nc = Nc;
        D.alpha = 1.0;
        D.tiles_m = (int)ceil_div(P.r(i, n), 64);
        D.tiles_n = (int)ceil_div(Nc, 64);
        D.tile_begin = tiles;
        tiles += (int64_t)D.tiles_m * D.tiles_n;
        ad.push_back(D);
      }
    Step st{};
    st.kind = S_KRP_ADJ;
    st.prec = pc;
    st.meta = prog.put(ad);
    st.count = (int)ad.size();
    st.tiles = tiles;
    prog.steps.push_back(st);
  }
  // ---- core_bar = sum of the d + 1 slots
  {
    std::vector<ReduceJob> red;
    for (int i = 0; i < s; ++i)
      red.push_back(ReduceJob{io.core_bar[i], gparts[i], P.r(i, 0), csize[i] / P.r(i, 0), P.r(i, 0),
                              P.r(i, 0), csize[i], d + 1, 0, P.in_f64 ? 1 : 0, tc64 ? 1 : 0});
    Step st{};
    st.kind = S_REDUCE;
    st.meta = prog.put(red);
    st.count = (int)red.size();
    prog.steps.push_back(st);
  }
  // ---- factor_bar = Q_k W_bar_k + c_i Y_bar_k V_k^T + Omega_k P_bar_k^T
  {
    GemmBatch gb(pc, R_OTHER, &ar);
    for (int i = 0; i < s; ++i)
      for (int k = 0; k < d; ++k) {
        const int64_t n = P.dims[k], r = P.r(i, k), w = P.w[k];
        const size_t ik = (size_t)i * d + k;
        gb.add(io.factor_bar[ik], P.in_f64, n, 0, (int)n, (int)r, 1, 0,
               {seg(Qc[k], 1, n, 0, Wb[ik], w, 1, 0, w),
                seg(Yb[k], 1, n, 0, V[ik], 1, r, 0, m, P.coeffs[i]),
                seg(om[k], 1, n, 0, Pb[ik], 1, r, 0, m)});
      }
    emit_gemm(prog, gb);
  }
}

// ------------------------------------------------------------------ execution
const char* role_name(int role) {
  switch (role) {
    case R_FACTOR_SKETCH: return "factor_sketch";
    case R_KRON_TTM: return "kron_core_ttm";
    case R_TERM_EXPAND: return "term_expand";
    case R_QR_GRAM: return "qr_gram";
    case R_QR_BASIS: return "qr_basis";
    case R_PROJ_W: return "proj_w";
    case R_PROJ_TTM: return "proj_ttm";
    case R_PROJ_FINAL: return "proj_final";
  }
  return "other";
}

// Name of the kernel symbol a step launches (template arguments as a kernel
// trace prints them, defaulted ones left out), followed by the step's role.
std::string step_name(const Step& st) {
  char buf[96];
  switch (st.kind) {
    case S_OMEGA: return "omega_kernel";
    case S_GEMM: {
      int role = st.role;
      if (role > R_OTHER || role < 0) role = R_OTHER;
      if ((role == R_QR_GRAM || role == R_QR_BASIS) && st.prec != P_FP64) role = R_OTHER;
      // the FP32-source and grouped variants carry their template flags, as a
      // trace prints them
      snprintf(buf, sizeof buf, "gemm_kernel<%d, %d%s> %s", st.prec, role,
               st.grouped ? ", false, true" : (st.a32 ? ", true" : ""), role_name(role));
      return buf;
    }
    case S_KRP:
      snprintf(buf, sizeof buf, "krp_kernel<%d%s> core_sketch", st.prec, st.a32 ? ", true" : "");
      return buf;
    case S_REDUCE: return "reduce_kernel";
    case S_TILE_REDUCE: return "tile_reduce_kernel";
    case S_COPY: return "copy_kernel";
    case S_FILL: return "fill_i32_kernel";
    case S_CHOL: return "chol_kernel";
    case S_HOUSE: return "householder_kernel";
    case S_KRP_ADJ: {
      snprintf(buf, sizeof buf, "krp_adj_kernel<%d> core_sketch_adjoint", st.prec);
      return buf;
    }
    case S_SYM: return "sym_kernel";
    case S_TRSM: return "trsm_rt_kernel";
    case S_EIG: return st.pass == 1 ? "tridiag_eig_kernel" : "jacobi_eig_kernel";
    case S_SCATTER: return "block_scatter_kernel";
    case S_FORK: return "fork";
    case S_JOIN: return "join";
  }
  return "unknown";
}

tsk_status acquire_staging(tsk_handle h, size_t bytes, void** host, hipEvent_t* ev) {
  if (h->ring.empty()) h->ring.resize(8);
  Staging& sl = h->ring[h->ring_next];
  h->ring_next = (h->ring_next + 1) % h->ring.size();
  if (sl.done == nullptr) {
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
      return fail(h, TSK_ERR_DEVICE, "hipEventCreate failed");
  } else if (hipEventSynchronize(sl.done) != hipSuccess) {
    return fail(h, TSK_ERR_DEVICE, "waiting for a staging slot failed");
  }
  if (sl.cap < bytes) {
    if (sl.host) hipHostFree(sl.host);
    sl.host = nullptr;
    const size_t cap = std::max<size_t>(align_up(bytes, 65536), 65536);
    if (hipHostMalloc(&sl.host, cap, hipHostMallocDefault) != hipSuccess) {
      sl.cap = 0;
      return fail(h, TSK_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
    }
    sl.cap = cap;
  }
  *host = sl.host;
  *ev = sl.done;
  return TSK_OK;
}

// `fixed_stage`: upload the descriptors from the handle's preallocated
// pinned buffer (waiting for its previous upload) and record no profiling
// events, so that the call allocates nothing.
tsk_status run_program(tsk_handle h, Program& prog, char* ws, hipStream_t stream,
                       bool fixed_stage = false) {
  char* meta = ws + prog.meta_region;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "hipStreamIsCapturing failed");
  const bool capturing = cs == hipStreamCaptureStatusActive;
  const bool prof = h->prof && !capturing && !fixed_stage;
  if (!prog.blob.empty()) {
    void* host = nullptr;
    hipEvent_t ev = nullptr;
    if (fixed_stage) {
      if (prog.blob.size() > kFixedStageBytes)
        return fail(h, TSK_ERR_UNSUPPORTED, "launch descriptors %zu bytes > %zu", prog.blob.size(),
                    kFixedStageBytes);
      if (hipEventSynchronize(h->fixed_stage_done) != hipSuccess)
        return fail(h, TSK_ERR_DEVICE, "waiting for the previous descriptor upload failed");
      host = h->fixed_stage;
      ev = h->fixed_stage_done;
    } else if (capturing) {
      // A captured call keeps its descriptors in device memory of the
      // handle's (until tsk_destroy), filled once here through the handle's
      // idle second stream; the graph copies them into the workspace on the
      // device, so a replay neither reads host memory over the bus nor relies
      // on the workspace keeping them between replays.
      void* dev = nullptr;
      if (hipMalloc(&dev, prog.blob.size()) != hipSuccess)
        return fail(h, TSK_ERR_OUT_OF_MEMORY, "descriptor copy allocation failed");
      h->device_keep.push_back(dev);
      if (hipMemcpyAsync(dev, prog.blob.data(), prog.blob.size(), hipMemcpyHostToDevice,
                         h->side) != hipSuccess ||
          hipStreamSynchronize(h->side) != hipSuccess)
        return fail(h, TSK_ERR_DEVICE, "descriptor copy failed");
      if (hipMemcpyAsync(meta, dev, prog.blob.size(), hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return fail(h, TSK_ERR_DEVICE, "descriptor upload failed");
    } else {
      tsk_status st = acquire_staging(h, prog.blob.size(), &host, &ev);
      if (st != TSK_OK) return st;
    }
    if (host != nullptr) {
      std::memcpy(host, prog.blob.data(), prog.blob.size());
      if (hipMemcpyAsync(meta, host, prog.blob.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(h, TSK_ERR_DEVICE, "descriptor upload failed");
    }
    if (ev != nullptr && hipEventRecord(ev, stream) != hipSuccess)
      return fail(h, TSK_ERR_DEVICE, "hipEventRecord failed");
  }
  for (const Step& st : prog.steps) {
    hipError_t e = hipSuccess;
    if (st.kind == S_FORK || st.kind == S_JOIN) {
      hipEvent_t ev = st.kind == S_FORK ? h->fork_ev : h->join_ev;
      hipStream_t from = st.kind == S_FORK ? stream : h->side;
      hipStream_t to = st.kind == S_FORK ? h->side : stream;
      if (hipEventRecord(ev, from) != hipSuccess || hipStreamWaitEvent(to, ev, 0) != hipSuccess)
        return fail(h, TSK_ERR_DEVICE, "stream %s failed", st.kind == S_FORK ? "fork" : "join");
      continue;
    }
    const hipStream_t caller = stream;
    hipStream_t stream = st.side ? h->side : caller;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof) {
      for (hipEvent_t* ev : {&ev0, &ev1}) {
        if (!h->event_pool.empty()) {
          *ev = h->event_pool.back();
          h->event_pool.pop_back();
        } else if (hipEventCreate(ev) != hipSuccess) {
          return fail(h, TSK_ERR_DEVICE, "hipEventCreate failed");
        }
      }
      if (hipEventRecord(ev0, stream) != hipSuccess) return fail(h, TSK_ERR_DEVICE, "hipEventRecord failed");
    }
    switch (st.kind) {
      case S_OMEGA: e = launch_omega_jobs((const OmegaJobDev*)(meta + st.meta), st.count, st.rows, stream); break;
      case S_GEMM:
        e = launch_gemm(st.prec, st.role, (const GemmDesc*)(meta + st.meta), st.count,
                        (const GemmSeg*)(meta + st.meta2), st.tiles, stream, st.a32, st.grouped);
        break;
      case S_KRP:
        e = launch_krp(st.prec, (const KrpDesc*)(meta + st.meta), st.count, st.tiles, st.krp_lds,
                       stream, st.a32);
        break;
      case S_REDUCE: e = launch_reduce((const ReduceJob*)(meta + st.meta), st.count, stream); break;
      case S_TILE_REDUCE: e = launch_tile_reduce((const ReduceJob*)(meta + st.meta), st.count, stream); break;
      case S_COPY: e = launch_copy((const CopyJob*)(meta + st.meta), st.count, st.tiles, stream); break;
      case S_FILL: e = launch_fill_i32((int32_t*)st.ptr, st.rows, st.value, stream); break;
      case S_CHOL:
        e = launch_chol((const QrDesc*)(meta + st.meta), st.count, st.pass, st.tol, st.wmax, stream);
        break;
      case S_KRP_ADJ:
        e = launch_krp_adj(st.prec, (const KrpAdjDesc*)(meta + st.meta), st.count, st.tiles, stream);
        break;
      case S_SYM: e = launch_sym((const SymJob*)(meta + st.meta), st.count, stream); break;
      case S_TRSM: e = launch_trsm_rt((const TrsmJob*)(meta + st.meta), st.count, stream); break;
      case S_SCATTER:
        e = launch_block_scatter((const BlockJob*)(meta + st.meta), st.count, st.tiles, stream);
        break;
      case S_EIG:
        e = st.pass == 1 ? launch_tridiag_eig((const EigJob*)(meta + st.meta), st.count, st.wmax, stream)
                         : launch_jacobi_eig((const EigJob*)(meta + st.meta), st.count, st.wmax, stream);
        break;
      case S_FORK:
      case S_JOIN: break;  // handled above
      case S_HOUSE:
        e = launch_householder((const QrDesc*)(meta + st.meta), st.count, st.force, (int64_t*)st.ptr,
                               st.rows, st.hh_sel, st.hh_grid, stream);
        break;
    }
    if (e != hipSuccess) return fail(h, TSK_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    if (ev1 != nullptr) {
      if (hipEventRecord(ev1, stream) != hipSuccess) return fail(h, TSK_ERR_DEVICE, "hipEventRecord failed");
      h->prof_records.push_back(
          ProfRecord{step_name(st), ev0, ev1, st.flops, st.bytes, (int)(&st - prog.steps.data())});
    }
  }
  return TSK_OK;
}

// Plan into a null-based arena to size the workspace, then rebase.
tsk_status plan_many(tsk_handle h, const std::vector<Problem>& Ps, const std::vector<Outputs>& outs,
                     char* ws, Program& prog, size_t* bytes) {
  // the per-mode QR flag words come first: one per mode of every sum whose
  // QR is planned
  int64_t nctr = 0;
  for (size_t j = 0; j < Ps.size(); ++j)
    if (outs[j].recompress) nctr += Ps[j].d;
  Arena ar;
  ar.base = ws;
  ar.ctr_base = (int32_t*)ar.take(sizeof(int32_t) * std::max<int64_t>(nctr, 1));
  Builder B(ar);
  B.nsums = (int)Ps.size();
  B.d_counter = h ? h->d_counter : nullptr;
  B.th = h;
  B.direct32 = !Ps.empty();
  for (const Problem& P : Ps)
    if (P.kind != TSK_SKETCH_KRP || P.in_f64 || !is_fp64(P.ps)) B.direct32 = false;
  for (size_t j = 0; j < Ps.size(); ++j) build_sum(Ps[j], outs[j], B);
  if (!ar.too_far.empty()) return fail(h, TSK_ERR_UNSUPPORTED, "%s", ar.too_far.c_str());
  if (ar.ctr_used != nctr) return fail(h, TSK_ERR_DEVICE, "QR flag words planned %lld, placed %lld",
                                      (long long)ar.ctr_used, (long long)nctr);
  B.emit(prog);
  prog.meta_region = align_up(ar.top, 256);
  *bytes = prog.meta_region + align_up(prog.blob.size(), 256) + 256;
  return TSK_OK;
}

tsk_status plan(tsk_handle h, const Problem& P, const Outputs& out, char* ws, Program& prog,
                size_t* bytes) {
  return plan_many(h, std::vector<Problem>{P}, std::vector<Outputs>{out}, ws, prog, bytes);
}

// Stage 3 alone: bases Q (FP64 when q_f64) of widths P.w.
tsk_status plan_project(tsk_handle h, const Problem& P, const std::vector<const void*>& Q,
                        bool q_f64, void* H, bool out_f64, char* ws, Program& prog,
                        size_t* bytes) {
  Arena ar;
  ar.base = ws;
  ar.ctr_base = (int32_t*)ar.take(256);
  Builder B(ar);
  B.d_counter = h ? h->d_counter : nullptr;
  B.th = h;
  build_projection(P, Q, q_f64, P.cores, P.factors, P.in_f64, H, out_f64, B);
  if (!ar.too_far.empty()) return fail(h, TSK_ERR_UNSUPPORTED, "%s", ar.too_far.c_str());
  B.emit(prog);
  prog.meta_region = align_up(ar.top, 256);
  *bytes = prog.meta_region + align_up(prog.blob.size(), 256) + 256;
  return TSK_OK;
}

// Problem of a Stage-3-only call: the sum, the bases' widths and the
// projection arithmetic.
tsk_status validate_project(tsk_handle h, const tsk_tucker_sum* sum, const int64_t* widths,
                            int32_t project_prec, Problem& P) {
  if (tsk_status st = validate_sum(h, sum, P); st != TSK_OK) return st;
  if (widths == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "widths is NULL");
  if (project_prec < TSK_PREC_FP64 || project_prec > TSK_PREC_BF16X6)
    return fail(h, TSK_ERR_INVALID_ARG, "bad precision");
  P.pp = project_prec;
  P.ps = project_prec;
  int64_t hsize = 1;
  for (int n = 0; n < P.d; ++n) {
    if (widths[n] < 1) return fail(h, TSK_ERR_INVALID_ARG, "widths[%d] < 1", n);
    if (P.dims[n] * widths[n] > (int64_t(1) << 34))
      return fail(h, TSK_ERR_UNSUPPORTED, "basis of mode %d too large", n);
    hsize *= widths[n];
    if (hsize > (int64_t(1) << 34)) return fail(h, TSK_ERR_UNSUPPORTED, "projected core too large");
    P.w.push_back(widths[n]);
    P.W.push_back(widths[n]);
  }
  return TSK_OK;
}

tsk_status set_device(tsk_handle h) {
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, TSK_ERR_DEVICE, "hipSetDevice failed");
  return TSK_OK;
}


// ------------------------------------------------------------------ Stage 4
// ST-HOSVD of the projected core H with relative tolerance eps (Algorithms
// 4/5, Stage 4; rank rule of Algorithm 2, phase 2): for n = 1..d in order,
// the Gram G_(n) G_(n)^T of the current core, its eigendecomposition, the
// rank r_n (smallest r with discarded eigenvalues summing to at most
// theta = eps^2 ||H||^2 / d), and G <- G x_n V_n^T with the r_n leading
// eigenvectors V_n; finally U_n = Q_n V_n.  The ranks decide the shapes of
// the next mode's launches, so each mode ends with a host read of r_n.
struct TruncIO {
  int d = 0;
  std::vector<int64_t> dims, w;  // mode sizes n_k and core widths w_k
  std::vector<const double*> Q;  // n_k x w_k
  const double* H = nullptr;     // w_1 x ... x w_d
  double eps = 0;
  std::vector<double*> U;        // n_k x w_k capacity
  double* G = nullptr;           // prod w_k capacity
};

// Fixed workspace of a batch of truncations: the ranks and theta of every
// job in one block each (so that one copy reads every rank of a phase);
// then per job the Gram, the eigenvectors and eigenvalues of every mode, two
// core buffers and, for widths above the LDS limit, the eigensolver's
// workspace.  One phase region (Gram split-K partials) and the descriptor
// blob follow.
struct TruncJobMem {
  double* C = nullptr;
  std::vector<double*> V, lam;
  double* buf[2] = {nullptr, nullptr};
  double* work = nullptr;
};

struct TruncLayout {
  int32_t* ranks = nullptr;  // [jobs * kMaxOrder]
  double* theta = nullptr;   // [jobs]
  std::vector<TruncJobMem> job;
  size_t phase_base = 0;
};

static void trunc_layout(const std::vector<TruncIO>& ios, Arena& ar, TruncLayout& L) {
  const size_t J = ios.size();
  L.ranks = (int32_t*)ar.take(sizeof(int32_t) * kMaxOrder * J);
  L.theta = (double*)ar.take(sizeof(double) * J);
  L.job.assign(J, TruncJobMem{});
  for (size_t j = 0; j < J; ++j) {
    const TruncIO& io = ios[j];
    TruncJobMem& M = L.job[j];
    int64_t wmax = 1, hs = 1;
    for (int n = 0; n < io.d; ++n) {
      wmax = std::max(wmax, io.w[n]);
      hs *= io.w[n];
    }
    M.C = (double*)ar.take(wmax * wmax * 8);
    M.V.resize(io.d);
    M.lam.resize(io.d);
    for (int n = 0; n < io.d; ++n) {
      M.V[n] = (double*)ar.take(io.w[n] * io.w[n] * 8);
      M.lam[n] = (double*)ar.take(io.w[n] * 8);
    }
    M.buf[0] = (double*)ar.take(hs * 8);
    M.buf[1] = (double*)ar.take(hs * 8);
    if (wmax > kEigMaxW) {
      const int64_t Wp = wmax + (wmax & 1);
      M.work = (double*)ar.take(2 * Wp * Wp * 8);
    }
  }
  L.phase_base = align_up(ar.top, 256);
}

// Where a job stands between phases: the core's current shape, the ranks
// chosen so far, the core the next phase reads and where its TTM writes.
struct TruncState {
  std::vector<int64_t> shape;
  std::vector<int32_t> ranks;
  const double* cur = nullptr;
  double* dst = nullptr;
};

// Launches of phase n of every job: the TTMs that truncate mode n - 1 (if
// n > 0, with rank ranks[n - 1]), then the Grams and eigendecompositions of
// mode n (if n < d); at n == d also U_k = Q_k V_k for every mode of the job.
// Jobs of lower order than n take no part.  Each kind of launch is one
// grouped launch over the jobs.
static void trunc_phase(const std::vector<TruncIO>& ios, const TruncLayout& L, int n,
                        const std::vector<TruncState>& S, Arena& ar, Program& prog) {
  GemmBatch ttm(P_FP64, R_OTHER, &ar), gram(P_FP64, R_OTHER, &ar), fin(P_FP64, R_OTHER, &ar);
  std::vector<EigJob> small, large;
  int wsmall = 0, wlarge = 0;
  int64_t gram_tiles = 0;
  for (size_t j = 0; j < ios.size(); ++j) {
    const TruncIO& io = ios[j];
    if (n < io.d) gram_tiles += ceil_div(S[j].shape[n], 64) * ceil_div(S[j].shape[n], 64);
  }
  for (size_t j = 0; j < ios.size(); ++j) {
    const TruncIO& io = ios[j];
    const TruncJobMem& M = L.job[j];
    const int d = io.d;
    if (n > d) continue;
    std::vector<int64_t> shape = S[j].shape;
    const double* cur = S[j].cur;
    if (n > 0) {
      const int k = n - 1;
      const int64_t Wk = shape[k], rk = S[j].ranks[k];
      int64_t Lo = 1, Ro = 1;
      for (int i = 0; i < k; ++i) Lo *= shape[i];
      for (int i = k + 1; i < d; ++i) Ro *= shape[i];
      if (k == 0) {
        // out (r_0 x R) = V_0^T (r_0 x W_0) . G_(0) (W_0 x R)
        ttm.add(S[j].dst, true, rk, 0, (int)rk, (int)Ro, 1, 0,
                {seg(M.V[k], Wk, 1, 0, cur, Wk, 1, 0, Wk)});
      } else {
        // per trailing index b: out_b (L x r_k) = G_b (L x W_k) . V_k (W_k x r_k)
        ttm.add(S[j].dst, true, Lo, Lo * rk, (int)Lo, (int)rk, (int)Ro, 0,
                {seg(cur, 1, Lo, Lo * Wk, M.V[k], Wk, 1, 0, Wk)});
      }
      shape[k] = rk;
      cur = S[j].dst;
    }
    if (n < d) {
      const int64_t Wn = shape[n];
      int64_t Lo = 1, Ro = 1;
      for (int i = 0; i < n; ++i) Lo *= shape[i];
      for (int i = n + 1; i < d; ++i) Ro *= shape[i];
      std::vector<GemmSeg> sg;
      if (n == 0) {
        sg.push_back(seg(cur, 1, Wn, 0, cur, 1, Wn, 0, Ro));
      } else {
        for (int64_t c = 0; c < Ro; ++c) {
          const double* base = cur + c * Lo * Wn;
          sg.push_back(seg(base, Lo, 1, 0, base, Lo, 1, 0, Lo));
        }
      }
      const int splits = choose_splits(gram_tiles, ceil_div(Lo * Ro, 16));
      gram.add(M.C, true, Wn, 0, (int)Wn, (int)Wn, 1, 0, sg, splits);
      EigJob J{};
      J.C = M.C;
      J.V = M.V[n];
      J.lam = M.lam[n];
      J.theta = L.theta + j;
      J.rank = L.ranks + j * kMaxOrder + n;
      J.ldc = Wn;
      J.ldv = Wn;
      J.tol = 1e-15;
      J.theta_scale = io.eps * io.eps / d;
      J.W = (int32_t)Wn;
      J.set_theta = n == 0 ? 1 : 0;
      J.clip = 1;
      J.work = M.work;
      if (Wn <= kEigMaxW) {
        small.push_back(J);
        wsmall = std::max<int>(wsmall, (int)Wn);
      } else {
        large.push_back(J);
        wlarge = std::max<int>(wlarge, (int)Wn);
      }
    } else {
      for (int k = 0; k < d; ++k) {
        const int64_t nk = io.dims[k], Wk = io.w[k];
        fin.add(io.U[k], true, nk, 0, (int)nk, (int)S[j].ranks[k], 1, 0,
                {seg(io.Q[k], 1, nk, 0, M.V[k], Wk, 1, 0, Wk)});
      }
    }
  }
  emit_gemm(prog, ttm);
  emit_gemm(prog, gram);
  emit_gemm(prog, fin);
  // The LDS Jacobi and its global-memory form are separate launches: the
  // global form reads every job's eigensolver workspace.
  for (int which = 0; which < 2; ++which) {
    const std::vector<EigJob>& js = which == 0 ? small : large;
    if (js.empty()) continue;
    Step st{};
    st.kind = S_EIG;
    st.meta = prog.put(js);
    st.count = (int)js.size();
    st.wmax = which == 0 ? wsmall : wlarge;
    prog.steps.push_back(st);
  }
}

// Workspace of a batch of truncations: the fixed part, then the largest
// phase with every rank at its maximum.  A phase's Gram tiles do not depend
// on the ranks, and smaller ranks only shorten K, which never raises the
// split count, so this bounds the partials and descriptors of any ranks.
static size_t trunc_workspace(const std::vector<TruncIO>& ios, bool* too_far) {
  Arena a0;
  TruncLayout L;
  trunc_layout(ios, a0, L);
  size_t phase = 0, blob = 0;
  std::vector<TruncState> S(ios.size());
  int dmax = 0;
  for (size_t j = 0; j < ios.size(); ++j) {
    S[j].shape = ios[j].w;
    S[j].ranks.assign(ios[j].w.begin(), ios[j].w.end());
    dmax = std::max(dmax, ios[j].d);
  }
  for (int n = 0; n <= dmax; ++n) {
    Arena ar;
    ar.base = nullptr;
    ar.top = L.phase_base;
    Program prog;
    trunc_phase(ios, L, n, S, ar, prog);
    if (!ar.too_far.empty()) *too_far = true;
    phase = std::max(phase, ar.top);
    blob = std::max(blob, prog.blob.size());
  }
  return align_up(phase, 256) + align_up(blob, 256) + 256;
}

static size_t trunc_workspace(const TruncIO& io, bool* too_far) {
  return trunc_workspace(std::vector<TruncIO>{io}, too_far);
}

static tsk_status validate_trunc(tsk_handle h, int32_t order, const int64_t* dims,
                                 const int64_t* widths, double eps, TruncIO& io) {
  if (order < 2 || order > kMaxOrder) return fail(h, TSK_ERR_INVALID_ARG, "order %d outside [2, %d]", order, kMaxOrder);
  if (dims == nullptr || widths == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "dims or widths is NULL");
  if (!(eps >= 0.0) || eps > 1.0) return fail(h, TSK_ERR_INVALID_ARG, "eps must be in [0, 1]");
  io.d = order;
  io.eps = eps;
  int64_t hs = 1;
  for (int k = 0; k < order; ++k) {
    if (dims[k] < 1 || widths[k] < 1) return fail(h, TSK_ERR_INVALID_ARG, "mode %d: size < 1", k);
    if (widths[k] > dims[k]) return fail(h, TSK_ERR_INVALID_ARG, "mode %d: width above the mode size", k);
    if (widths[k] > kEigMaxWGlobal)
      return fail(h, TSK_ERR_UNSUPPORTED, "mode %d: width %lld above %d", k, (long long)widths[k],
                  kEigMaxWGlobal);
    if (dims[k] > (1 << 30)) return fail(h, TSK_ERR_UNSUPPORTED, "dims[%d] too large", k);
    hs *= widths[k];
    io.dims.push_back(dims[k]);
    io.w.push_back(widths[k]);
  }
  if (hs > (int64_t(1) << 31)) return fail(h, TSK_ERR_UNSUPPORTED, "core too large");
  return TSK_OK;
}

// Drives the phases of a batch of truncations in `ws` (of `need` bytes, as
// trunc_workspace computed).  `run(prog)` launches (or checks) a phase's
// program; `rank_of(j, n)` returns the rank job j chose for mode n after
// the phase that decided it (read from the device, or given by a
// self-check), 0 on failure.  The last TTM of a job writes the caller's
// core; the others ping-pong between the job's two buffers.
template <typename Run, typename RankOf>
static tsk_status trunc_drive(tsk_handle h, const std::vector<TruncIO>& ios, const TruncLayout& L,
                              char* ws, size_t need, Run run, RankOf rank_of,
                              std::vector<std::vector<int32_t>>& ranks) {
  const size_t J = ios.size();
  std::vector<TruncState> S(J);
  std::vector<int> which(J, 0);
  int dmax = 0;
  for (size_t j = 0; j < J; ++j) {
    S[j].shape = ios[j].w;
    S[j].ranks.assign(ios[j].d, 0);
    S[j].cur = ios[j].H;
    dmax = std::max(dmax, ios[j].d);
  }
  for (int n = 0; n <= dmax; ++n) {
    for (size_t j = 0; j < J; ++j)
      S[j].dst = (n == ios[j].d) ? ios[j].G : L.job[j].buf[which[j]];
    Arena ar;
    ar.base = ws;
    ar.top = L.phase_base;
    Program prog;
    trunc_phase(ios, L, n, S, ar, prog);
    prog.meta_region = align_up(ar.top, 256);
    if (prog.meta_region + align_up(prog.blob.size(), 256) + 256 > need)
      return fail(h, TSK_ERR_DEVICE, "truncation phase exceeds its planned workspace");
    if (tsk_status st = run(prog); st != TSK_OK) return st;
    for (size_t j = 0; j < J; ++j) {
      if (n > 0 && n <= ios[j].d) {
        S[j].shape[n - 1] = S[j].ranks[n - 1];
        S[j].cur = S[j].dst;
        which[j] ^= 1;
      }
      if (n < ios[j].d) {
        const int32_t r = rank_of(j, n);
        if (r < 1 || r > S[j].shape[n])
          return fail(h, TSK_ERR_DEVICE, "rank %d of mode %d of job %zu out of range", r, n, j);
        S[j].ranks[n] = r;
      }
    }
  }
  ranks.resize(J);
  for (size_t j = 0; j < J; ++j) ranks[j] = S[j].ranks;
  return TSK_OK;
}

// The launches of a batch of truncations; ranks_out[j]: host [d_j].  One
// stream synchronisation per mode reads every job's rank of that mode.
static tsk_status truncate_run(tsk_handle h, const std::vector<TruncIO>& ios, char* ws,
                               size_t need, hipStream_t s, int32_t* const* ranks_out) {
  Arena fixed;
  fixed.base = ws;
  TruncLayout L;
  trunc_layout(ios, fixed, L);
  std::vector<int32_t> host(kMaxOrder * ios.size(), 0);
  int last_read = -1;
  auto run = [&](Program& prog) { return run_program(h, prog, ws, s); };
  auto rank_of = [&](size_t j, int n) -> int32_t {
    if (last_read != n) {
      if (hipStreamSynchronize(s) != hipSuccess ||
          hipMemcpy(host.data(), L.ranks, sizeof(int32_t) * host.size(), hipMemcpyDeviceToHost) !=
              hipSuccess)
        return 0;
      last_read = n;
    }
    return host[j * kMaxOrder + n];
  };
  std::vector<std::vector<int32_t>> ranks;
  if (tsk_status st = trunc_drive(h, ios, L, ws, need, run, rank_of, ranks); st != TSK_OK)
    return st;
  for (size_t j = 0; j < ios.size(); ++j)
    for (int k = 0; k < ios[j].d; ++k) ranks_out[j][k] = ranks[j][k];
  return TSK_OK;
}

static tsk_status truncate_run(tsk_handle h, const TruncIO& io, char* ws, size_t need,
                               hipStream_t s, int32_t* ranks_out) {
  int32_t* const outs[1] = {ranks_out};
  return truncate_run(h, std::vector<TruncIO>{io}, ws, need, s, outs);
}

// ------------------------------------------------------------------ deterministic baseline
// The paper's baseline for the sum: Algorithm 1 (TuckerAxby) over all
// terms, W_n = [U_n^(1), ..., U_n^(s)] (n_n x R_n, R_n = sum_i r_n^(i)) and
// the dense R_1 x ... x R_d core with c_i G^(i) in disjoint blocks along the
// super-diagonal; then Algorithm 2 (TuckerRounding): W_n = Q_n R_n (thin
// QR), C <- C x_n R_n for every n, and the ST-HOSVD of C with tolerance tau
// and theta = tau^2 ||C||^2 / d (the Stage 4 machinery on Q_n and C).
// Phase 1 (one launch sequence): the concatenated factors, their QR, the
// dense core and its TTM chain.
struct DetPlan {
  std::vector<int64_t> R, w;      // concatenated widths and min(n, R)
  std::vector<double*> Wf, Q, Rm;  // n x R factors, n x w bases, w x R triangles
  double* C = nullptr;             // R_1 x ... x R_d super-diagonal core
  double* core = nullptr;          // w_1 x ... x w_d after the TTM chain
};

static void plan_det_phase1(const Problem& P, Arena& ar, Program& prog, DetPlan& D) {
  const int d = P.d, s = P.s;
  ar.ctr_base = (int32_t*)ar.take(sizeof(int32_t) * 64);
  D.R.assign(d, 0);
  for (int n = 0; n < d; ++n)
    for (int i = 0; i < s; ++i) D.R[n] += P.r(i, n);
  std::vector<CopyJob> cat;
  int64_t csz = 1;
  for (int n = 0; n < d; ++n) {
    D.w.push_back(std::min(P.dims[n], D.R[n]));
    D.Wf.push_back((double*)ar.take(P.dims[n] * D.R[n] * 8));
    D.Q.push_back((double*)ar.take(P.dims[n] * D.w[n] * 8));
    D.Rm.push_back((double*)ar.take(D.w[n] * D.R[n] * 8));
    int64_t col = 0;
    for (int i = 0; i < s; ++i) {
      cat.push_back(CopyJob{D.Wf[n] + P.dims[n] * col, P.factors[(size_t)i * d + n], P.dims[n],
                            P.r(i, n), P.dims[n], P.dims[n], 1, P.in_f64 ? 1 : 0});
      col += P.r(i, n);
    }
    csz *= D.R[n];
  }
  D.C = (double*)ar.take(csz * 8);
  Builder B(ar);
  B.copies[ST_CONVERT] = cat;
  plan_qr(B, P.dims, D.R, std::vector<const double*>(D.Wf.begin(), D.Wf.end()), D.Q, D.Rm, 0);
  B.emit(prog);
  // the dense super-diagonal core: zeros, then the scaled cores in their blocks
  Step fill{};
  fill.kind = S_FILL;
  fill.ptr = D.C;
  fill.rows = 2 * csz;
  fill.value = 0;
  prog.steps.push_back(fill);
  std::vector<BlockJob> blocks;
  std::vector<int64_t> off(d, 0);
  int64_t chunks = 0;
  for (int i = 0; i < s; ++i) {
    BlockJob J{};
    J.dst = D.C;
    J.src = P.cores[i];
    J.order = d;
    J.src_f64 = P.in_f64 ? 1 : 0;
    J.alpha = P.coeffs[i];
    J.count = 1;
    for (int k = 0; k < kMaxOrder; ++k) {
      J.r[k] = k < d ? P.r(i, k) : 1;
      J.off[k] = k < d ? off[k] : 0;
      J.ext[k] = k < d ? D.R[k] : 1;
      if (k < d) J.count *= P.r(i, k);
    }
    J.chunk_begin = chunks;
    chunks += ceil_div(J.count, kCopyChunk);
    blocks.push_back(J);
    for (int k = 0; k < d; ++k) off[k] += P.r(i, k);
  }
  Step sc{};
  sc.kind = S_SCATTER;
  sc.meta = prog.put(blocks);
  sc.count = (int)blocks.size();
  sc.tiles = chunks;
  prog.steps.push_back(sc);
  // C <- C x_k R_k, k = 1..d, through two ping-pong buffers; the last into core
  std::vector<int64_t> shape = D.R;
  int64_t mx = 1;
  {
    std::vector<int64_t> sh = D.R;
    for (int k = 0; k < d; ++k) {
      sh[k] = D.w[k];
      int64_t sz = 1;
      for (auto x : sh) sz *= x;
      mx = std::max(mx, sz);
    }
  }
  double* buf[2] = {(double*)ar.take(mx * 8), (double*)ar.take(mx * 8)};
  const double* cur = D.C;
  for (int k = 0; k < d; ++k) {
    double* out = k == d - 1 ? (D.core = (double*)ar.take(mx * 8)) : buf[k & 1];
    const int64_t Rk = shape[k], wk = D.w[k];
    int64_t Lo = 1, Ro = 1;
    for (int j = 0; j < k; ++j) Lo *= shape[j];
    for (int j = k + 1; j < d; ++j) Ro *= shape[j];
    GemmBatch gb(P_FP64, R_OTHER, &ar);
    if (k == 0) {
      // out (w_0 x Ro) = R_0 (w_0 x R_0) . C_(0) (R_0 x Ro)
      const int splits = choose_splits(ceil_div(wk, 64) * ceil_div(Ro, 64), ceil_div(Rk, 16));
      gb.add(out, true, wk, 0, (int)wk, (int)Ro, 1, 0,
             {seg(D.Rm[k], 1, wk, 0, cur, Rk, 1, 0, Rk)}, splits);
    } else {
      // per trailing index b: out_b (Lo x w_k) = C_b (Lo x R_k) . R_k^T (R_k x w_k)
      gb.add(out, true, Lo, Lo * wk, (int)Lo, (int)wk, (int)Ro, 0,
             {seg(cur, 1, Lo, Lo * Rk, D.Rm[k], 1, wk, 0, Rk)});
    }
    emit_gemm(prog, gb);
    shape[k] = wk;
    cur = out;
  }
}

static tsk_status validate_det(tsk_handle h, const tsk_tucker_sum* sum, double tau, Problem& P,
                               TruncIO& io) {
  if (tsk_status st = validate_sum(h, sum, P); st != TSK_OK) return st;
  if (!(tau >= 0.0) || tau > 1.0) return fail(h, TSK_ERR_INVALID_ARG, "tau must be in [0, 1]");
  int64_t csz = 1;
  std::vector<int64_t> w(P.d);
  for (int n = 0; n < P.d; ++n) {
    int64_t R = 0;
    for (int i = 0; i < P.s; ++i) R += P.r(i, n);
    csz *= R;
    if (csz > (int64_t(1) << 32)) return fail(h, TSK_ERR_UNSUPPORTED, "dense core of the formal sum too large");
    w[n] = std::min(P.dims[n], R);
  }
  return validate_trunc(h, P.d, P.dims.data(), w.data(), tau, io);
}

static tsk_status plan_det_sized(tsk_handle h, const Problem& P, char* ws, Program& prog,
                                 DetPlan& D, size_t* phase1_bytes) {
  Arena ar;
  ar.base = ws;
  plan_det_phase1(P, ar, prog, D);
  if (!ar.too_far.empty()) return fail(h, TSK_ERR_UNSUPPORTED, "%s", ar.too_far.c_str());
  prog.meta_region = align_up(ar.top, 256);
  *phase1_bytes = align_up(prog.meta_region + align_up(prog.blob.size(), 256) + 256, 256);
  return TSK_OK;
}

// ------------------------------------------------------------------ Stage 1
// Phase 1 of Algorithm 3 for every mode: V_n = [w_1 U_n^(1), ..., w_s U_n^(s)]
// with w_i = |c_i| ||G^(i)||_F (the summands are c_i X^(i)), the eigenvalues
// of V_n^T V_n clipped at zero in decreasing order, and the smallest rank
// r_n >= 1 whose discarded eigenvalues sum to at most eps^2/d of their
// total.  Launches: FP64 copies of FP32 inputs; the squared core norms (one
// 1 x 1 GEMM per term); V_n assembled by copies scaled on the device;
// V_n^T V_n (one GEMM per mode); the eigenvalues (Jacobi in LDS for
// sum_i r_n^(i) <= 96, tridiagonal reduction and bisection above).
// A batch of sums runs each of these launches once for all of its sums.
struct SubrankOut {
  int32_t* ranks = nullptr;  // device [sums * kMaxOrder]
};

static void plan_subranks(const std::vector<Problem>& Ps, double eps, Arena& ar, Program& prog,
                          SubrankOut& out) {
  const size_t J = Ps.size();
  out.ranks = (int32_t*)ar.take(sizeof(int32_t) * kMaxOrder * J);
  double* theta = (double*)ar.take(sizeof(double) * kMaxOrder * J);
  // inputs in FP64
  std::vector<CopyJob> conv;
  std::vector<std::vector<const double*>> G(J), U(J);
  for (size_t j = 0; j < J; ++j) {
    const Problem& P = Ps[j];
    const int d = P.d, s = P.s;
    G[j].resize(s);
    U[j].resize((size_t)s * d);
    for (int i = 0; i < s; ++i) {
      int64_t cs = 1;
      for (int k = 0; k < d; ++k) cs *= P.r(i, k);
      if (P.in_f64) {
        G[j][i] = (const double*)P.cores[i];
      } else {
        double* p = (double*)ar.take(cs * 8);
        conv.push_back(CopyJob{p, P.cores[i], cs, 1, cs, cs, 1, 0});
        G[j][i] = p;
      }
      for (int k = 0; k < d; ++k) {
        const size_t idx = (size_t)i * d + k;
        if (P.in_f64) {
          U[j][idx] = (const double*)P.factors[idx];
        } else {
          double* p = (double*)ar.take(P.dims[k] * P.r(i, k) * 8);
          conv.push_back(
              CopyJob{p, P.factors[idx], P.dims[k], P.r(i, k), P.dims[k], P.dims[k], 1, 0});
          U[j][idx] = p;
        }
      }
    }
  }
  emit_copies(prog, conv);
  // squared Frobenius norms of the cores (one 1 x 1 product per term)
  std::vector<double*> norm2(J);
  {
    GemmBatch gb(P_FP64, R_OTHER, &ar);
    int64_t kt = 0, terms = 0;
    for (size_t j = 0; j < J; ++j) {
      const Problem& P = Ps[j];
      terms += P.s;
      for (int i = 0; i < P.s; ++i) {
        int64_t cs = 1;
        for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
        kt = std::max<int64_t>(kt, ceil_div(cs, 16));
      }
    }
    const int splits = choose_splits(terms, kt);
    for (size_t j = 0; j < J; ++j) {
      const Problem& P = Ps[j];
      norm2[j] = (double*)ar.take(sizeof(double) * P.s);
      for (int i = 0; i < P.s; ++i) {
        int64_t cs = 1;
        for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
        gb.add(norm2[j] + i, true, 1, 0, 1, 1, 1, 0,
               {seg(G[j][i], 1, 1, 0, G[j][i], 1, 1, 0, cs)},
               (int)std::min<int64_t>(splits, std::max<int64_t>(1, ceil_div(cs, 16) / 2)));
      }
    }
    emit_gemm(prog, gb);
  }
  // V_n, then V_n^T V_n, per sum and mode
  std::vector<CopyJob> scaled;
  struct ModeMem {
    double *V, *B, *lam, *scratch;
    int64_t W, n;
  };
  std::vector<std::vector<ModeMem>> mm(J);
  int64_t gram_tiles = 0;
  for (size_t j = 0; j < J; ++j) {
    const Problem& P = Ps[j];
    mm[j].resize(P.d);
    for (int n = 0; n < P.d; ++n) {
      int64_t W = 0;
      for (int i = 0; i < P.s; ++i) W += P.r(i, n);
      ModeMem& M = mm[j][n];
      M.W = W;
      M.n = P.dims[n];
      M.V = (double*)ar.take(P.dims[n] * W * 8);
      M.B = (double*)ar.take(W * W * 8);
      M.lam = (double*)ar.take(W * 8);
      M.scratch = (double*)ar.take(W * W * 8);
      gram_tiles += ceil_div(W, 64) * ceil_div(W, 64);
      int64_t col = 0;
      for (int i = 0; i < P.s; ++i) {
        CopyJob C{M.V + P.dims[n] * col, U[j][(size_t)i * P.d + n], P.dims[n], P.r(i, n), P.dims[n],
                  P.dims[n], 1, 1};
        C.norm2 = norm2[j] + i;
        C.mul = std::fabs(P.coeffs[i]);
        scaled.push_back(C);
        col += P.r(i, n);
      }
    }
  }
  emit_copies(prog, scaled);
  {
    GemmBatch gb(P_FP64, R_OTHER, &ar);
    for (size_t j = 0; j < J; ++j)
      for (const ModeMem& M : mm[j]) {
        const int splits = choose_splits(gram_tiles, ceil_div(M.n, 16));
        gb.add(M.B, true, M.W, 0, (int)M.W, (int)M.W, 1, 0,
               {seg(M.V, M.n, 1, 0, M.V, M.n, 1, 0, M.n)}, splits);
      }
    emit_gemm(prog, gb);
  }
  std::vector<EigJob> small, large;
  int wsmall = 0, wlarge = 0;
  for (size_t j = 0; j < J; ++j) {
    const Problem& P = Ps[j];
    for (int n = 0; n < P.d; ++n) {
      const ModeMem& M = mm[j][n];
      EigJob E{};
      E.C = M.B;
      E.V = M.scratch;
      E.lam = M.lam;
      E.theta = theta + j * kMaxOrder + n;
      E.rank = out.ranks + j * kMaxOrder + n;
      E.ldc = M.W;
      E.ldv = M.W;
      E.tol = 1e-15;
      E.theta_scale = eps * eps / P.d;
      E.W = (int32_t)M.W;
      E.set_theta = 1;
      E.clip = 1;
      E.values_only = 1;  // Stage 1 needs the eigenvalues only
      if (M.W <= kEigMaxW) {
        small.push_back(E);
        wsmall = std::max<int>(wsmall, (int)M.W);
      } else {
        large.push_back(E);
        wlarge = std::max<int>(wlarge, (int)M.W);
      }
    }
  }
  for (int which = 0; which < 2; ++which) {
    const std::vector<EigJob>& js = which == 0 ? small : large;
    if (js.empty()) continue;
    Step st{};
    st.kind = S_EIG;
    st.pass = which;  // 0: Jacobi in LDS, 1: tridiagonal reduction
    st.meta = prog.put(js);
    st.count = (int)js.size();
    st.wmax = which == 0 ? wsmall : wlarge;
    prog.steps.push_back(st);
  }
}

static tsk_status validate_subranks(tsk_handle h, const tsk_tucker_sum* sum, double eps,
                                    Problem& P) {
  if (tsk_status st = validate_sum(h, sum, P); st != TSK_OK) return st;
  if (!(eps >= 0.0) || eps > 1.0) return fail(h, TSK_ERR_INVALID_ARG, "eps must be in [0, 1]");
  for (int n = 0; n < P.d; ++n) {
    int64_t W = 0;
    for (int i = 0; i < P.s; ++i) W += P.r(i, n);
    if (W > kTriMaxW)
      return fail(h, TSK_ERR_UNSUPPORTED, "mode %d: sum of ranks %lld above %d", n, (long long)W,
                  kTriMaxW);
  }
  return TSK_OK;
}

static tsk_status validate_subranks_batch(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                                          double eps, std::vector<Problem>& Ps) {
  if (batch < 1 || sums == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "batch < 1 or sums is NULL");
  Ps.assign(batch, Problem{});
  for (int j = 0; j < batch; ++j)
    if (tsk_status st = validate_subranks(h, sums + j, eps, Ps[j]); st != TSK_OK) {
      h->err = "sum " + std::to_string(j) + ": " + h->err;
      return st;
    }
  return TSK_OK;
}

static tsk_status plan_subranks_sized(tsk_handle h, const std::vector<Problem>& Ps, double eps,
                                      char* ws, Program& prog, SubrankOut& out, size_t* bytes) {
  Arena ar;
  ar.base = ws;
  plan_subranks(Ps, eps, ar, prog, out);
  if (!ar.too_far.empty()) return fail(h, TSK_ERR_UNSUPPORTED, "%s", ar.too_far.c_str());
  prog.meta_region = align_up(ar.top, 256);
  *bytes = prog.meta_region + align_up(prog.blob.size(), 256) + 256;
  return TSK_OK;
}

static tsk_status plan_subranks_sized(tsk_handle h, const Problem& P, double eps, char* ws,
                                      Program& prog, SubrankOut& out, size_t* bytes) {
  return plan_subranks_sized(h, std::vector<Problem>{P}, eps, ws, prog, out, bytes);
}

// ------------------------------------------------------------------ plan self-check
// Host-only verification that every address a planned launch sequence can
// touch lies inside a buffer it is allowed to touch: the workspace or one of
// the caller's buffers, each given a synthetic, widely separated address.
// Used by the CPU test suite so that descriptor mistakes surface before any
// kernel runs.
struct Region {
  uintptr_t lo, hi;  // [lo, hi)
  const char* name;
};

struct Checker {
  std::vector<Region> regions;
  std::string err;
  bool ok = true;
  void add(const void* p, size_t bytes, const char* name) {
    regions.push_back(Region{(uintptr_t)p, (uintptr_t)p + bytes, name});
  }
  void span(const void* base, int64_t first, int64_t last, size_t es, const char* what) {
    if (!ok) return;
    if (first > last) return;  // empty access
    const uintptr_t lo = (uintptr_t)base + (uintptr_t)(first * (int64_t)es);
    const uintptr_t hi = (uintptr_t)base + (uintptr_t)((last + 1) * (int64_t)es);
    for (const Region& r : regions)
      if (lo >= r.lo && hi <= r.hi) return;
    ok = false;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: [%#zx, %#zx) outside every buffer", what, (size_t)lo, (size_t)hi);
    err = buf;
  }
};

// Largest value of sum_i idx_i * stride_i for 0 <= idx_i < ext_i.
int64_t max_off(std::initializer_list<std::pair<int64_t, int64_t>> terms) {
  int64_t o = 0;
  for (auto& t : terms) o += (t.first - 1) * t.second;
  return o;
}

void check_program(const Program& prog, Checker& ck) {
  const char* blob = prog.blob.data();
  bool forked = false;  // between S_FORK and S_JOIN
  for (const Step& st : prog.steps) {
    if (st.side && !forked) { ck.ok = false; ck.err = "second-stream launch outside a fork"; return; }
    switch (st.kind) {
      case S_FORK:
        if (forked) { ck.ok = false; ck.err = "fork inside a fork"; return; }
        forked = true;
        break;
      case S_JOIN:
        if (!forked) { ck.ok = false; ck.err = "join without a fork"; return; }
        forked = false;
        break;
      case S_OMEGA: {
        const OmegaJob* js = (const OmegaJob*)(blob + st.meta);
        for (int i = 0; i < st.count; ++i) ck.span(js[i].out, 0, js[i].count - 1, js[i].f64 ? 8 : 4, "omega");
        break;
      }
      case S_FILL: ck.span(st.ptr, 0, st.rows - 1, 4, "fill"); break;
      case S_GEMM: {
        const GemmDesc* ds = (const GemmDesc*)(blob + st.meta);
        const GemmSeg* sg = (const GemmSeg*)(blob + st.meta2);
        const size_t ein = st.prec == P_FP64 ? 8 : 4;
        int64_t tiles = 0;
        for (int i = 0; i < st.count; ++i) {
          const GemmDesc& D = ds[i];
          if (D.tile_begin != tiles) { ck.ok = false; ck.err = "gemm tile prefix mismatch"; return; }
          if (D.bpw > 1 && (D.splits != 1 || D.tiles_m != 1 || D.tiles_n != 1 ||
                            st.role != R_PROJ_TTM)) {
            ck.ok = false;
            ck.err = "batch elements grouped on a tile that is split or not alone";
            return;
          }
          tiles += tiles_of(D);
          if (D.tiles_m * 64 < D.M || D.tiles_n * 64 < D.N) { ck.ok = false; ck.err = "gemm tiles too few"; return; }
          for (int j = 0; j < D.seg_count; ++j) {
            const GemmSeg& S = sg[D.seg_begin + j];
            if (S.a_sx != 1 && S.a_sk != 1) { ck.ok = false; ck.err = "gemm A has no unit stride"; return; }
            if (S.b_sx != 1 && S.b_sk != 1) { ck.ok = false; ck.err = "gemm B has no unit stride"; return; }
            if (S.K == 0) continue;
            ck.span(S.A, 0, (D.batch - 1) * S.strideA + max_off({{D.M, S.a_sx}, {S.K, S.a_sk}}),
                    st.a32 ? 4 : ein, "gemm A");
            ck.span(S.B, 0, (D.batch - 1) * S.strideB + max_off({{D.N, S.b_sx}, {S.K, S.b_sk}}), ein, "gemm B");
          }
          ck.span(D.C, 0, (D.batch - 1) * D.strideC + max_off({{D.M, 1}, {D.N, D.ldc}}),
                  D.c_f64 ? 8 : 4, "gemm C");
          if (D.splits > 1) {
            const int64_t nt = (int64_t)D.tiles_m * D.tiles_n * D.batch;
            ck.span(D.part, 0, nt * D.splits * 4096 - 1, ein, "gemm partials");
          }
        }
        if (tiles != st.tiles) { ck.ok = false; ck.err = "gemm total tiles mismatch"; }
        break;
      }
      case S_KRP: {
        const KrpDesc* ds = (const KrpDesc*)(blob + st.meta);
        const size_t e = st.prec == P_FP64 ? 8 : 4;
        int64_t tiles = 0;
        for (int i = 0; i < st.count; ++i) {
          const KrpDesc& D = ds[i];
          if (D.tile_begin != tiles) { ck.ok = false; ck.err = "krp tile prefix mismatch"; return; }
          tiles += (int64_t)D.tiles_m * D.tiles_n * D.splits;
          int64_t cs = 1, Kc = 1;
          for (int k = 0; k < D.order; ++k) {
            cs *= D.r[k];
            if (k != D.mode) {
              Kc *= D.r[k];
              ck.span(D.P[k], 0, (int64_t)D.r[k] * D.m - 1, e, "krp P");
            }
          }
          if (Kc != D.Kc) { ck.ok = false; ck.err = "krp Kc mismatch"; return; }
          if (st.krp_lds < 0 || st.krp_lds > kKrpLds) { ck.ok = false; ck.err = "krp LDS size"; return; }
          ck.span(D.G, 0, cs - 1, st.a32 ? 4 : e, "krp G");
          ck.span(D.V, 0, (int64_t)D.r[D.mode] * D.m - 1, e, "krp V");
          if (D.splits > 1) {
            const int64_t nt = (int64_t)D.tiles_m * D.tiles_n;
            ck.span(D.part, 0, nt * D.splits * 4096 - 1, e, "krp partials");
          }
        }
        if (tiles != st.tiles) { ck.ok = false; ck.err = "krp total tiles mismatch"; }
        break;
      }
      case S_TILE_REDUCE:
      case S_REDUCE: {
        const ReduceJob* js = (const ReduceJob*)(blob + st.meta);
        for (int i = 0; i < st.count; ++i) {
          const ReduceJob& J = js[i];
          ck.span(J.out, 0, max_off({{J.rows, 1}, {J.cols, J.ld_out}}), J.out_f64 ? 8 : 4, "reduce out");
          ck.span(J.part, 0, (J.parts - 1) * J.stride_part + max_off({{J.rows, 1}, {J.cols, J.ld_part}}),
                  J.part_f64 ? 8 : 4, "reduce part");
        }
        break;
      }
      case S_COPY: {
        const CopyJob* js = (const CopyJob*)(blob + st.meta);
        int64_t chunks = 0;
        for (int i = 0; i < st.count; ++i) {
          const CopyJob& J = js[i];
          if (J.ld_dst != J.rows || J.ld_src != J.rows) { ck.ok = false; ck.err = "copy job not contiguous"; return; }
          if (J.chunk_begin != chunks) { ck.ok = false; ck.err = "copy chunk prefix mismatch"; return; }
          chunks += (J.rows * J.cols + kCopyChunk - 1) / kCopyChunk;
          ck.span(J.dst, 0, max_off({{J.rows, 1}, {J.cols, J.ld_dst}}), J.dst_f64 ? 8 : 4, "copy dst");
          ck.span(J.src, 0, max_off({{J.rows, 1}, {J.cols, J.ld_src}}), J.src_f64 ? 8 : 4, "copy src");
          if (J.norm2) ck.span(J.norm2, 0, 0, 8, "copy scale");
        }
        if (chunks != st.tiles) { ck.ok = false; ck.err = "copy chunk count mismatch"; return; }
        break;
      }
      case S_KRP_ADJ: {
        const KrpAdjDesc* ds = (const KrpAdjDesc*)(blob + st.meta);
        const size_t e = st.prec == P_FP64 ? 8 : 4;
        int64_t tiles = 0;
        for (int i = 0; i < st.count; ++i) {
          const KrpAdjDesc& D = ds[i];
          if (D.tile_begin != tiles) { ck.ok = false; ck.err = "krp_adj tile prefix mismatch"; return; }
          tiles += (int64_t)D.tiles_m * D.tiles_n;
          int64_t cs = 1;
          for (int k = 0; k < D.order; ++k) {
            cs *= D.r[k];
            if (k != D.mode) ck.span(D.P[k], 0, (int64_t)D.r[k] * D.m - 1, e, "krp_adj P");
          }
          ck.span(D.Vbar, 0, (int64_t)D.r[D.mode] * D.m - 1, e, "krp_adj Vbar");
          ck.span(D.Gout, 0, cs - 1, e, "krp_adj out");
        }
        if (tiles != st.tiles) { ck.ok = false; ck.err = "krp_adj total tiles mismatch"; }
        break;
      }
      case S_SYM: {
        const SymJob* js = (const SymJob*)(blob + st.meta);
        for (int i = 0; i < st.count; ++i) {
          ck.span(js[i].M, 0, js[i].w * js[i].w - 1, 8, "sym M");
          ck.span(js[i].S, 0, js[i].w * js[i].w - 1, 8, "sym S");
        }
        break;
      }
      case S_TRSM: {
        const TrsmJob* js = (const TrsmJob*)(blob + st.meta);
        for (int i = 0; i < st.count; ++i) {
          const TrsmJob& J = js[i];
          if (J.w > 96 || J.rows > 64) { ck.ok = false; ck.err = "trsm job too large"; return; }
          ck.span(J.R, 0, J.w * J.w - 1, 8, "trsm R");
          ck.span(J.Z, 0, J.n * J.w - 1, 8, "trsm Z");
          ck.span(J.X, 0, J.n * J.w - 1, 8, "trsm X");
          if (J.singular) ck.span(J.singular, 0, 0, 8, "trsm flag");
        }
        break;
      }
      case S_SCATTER: {
        const BlockJob* js = (const BlockJob*)(blob + st.meta);
        int64_t chunks = 0;
        for (int i = 0; i < st.count; ++i) {
          const BlockJob& J = js[i];
          if (J.chunk_begin != chunks) { ck.ok = false; ck.err = "scatter chunk prefix mismatch"; return; }
          chunks += (J.count + kCopyChunk - 1) / kCopyChunk;
          int64_t cnt = 1, last = 0, stride = 1, total = 1;
          for (int m = 0; m < J.order; ++m) {
            if (J.off[m] + J.r[m] > J.ext[m]) { ck.ok = false; ck.err = "scatter block outside"; return; }
            cnt *= J.r[m];
            last += (J.off[m] + J.r[m] - 1) * stride;
            stride *= J.ext[m];
            total *= J.ext[m];
          }
          if (cnt != J.count) { ck.ok = false; ck.err = "scatter count mismatch"; return; }
          ck.span(J.src, 0, J.count - 1, J.src_f64 ? 8 : 4, "scatter src");
          ck.span(J.dst, 0, last, 8, "scatter dst");
        }
        if (chunks != st.tiles) { ck.ok = false; ck.err = "scatter chunk count mismatch"; return; }
        break;
      }
      case S_EIG: {
        const EigJob* js = (const EigJob*)(blob + st.meta);
        for (int i = 0; i < st.count; ++i) {
          const EigJob& J = js[i];
          const int wcap = st.pass == 1 ? kTriMaxW : kEigMaxWGlobal;
          if (J.W < 1 || J.W > wcap || J.W > st.wmax || J.ldc < J.W || J.ldv < J.W) {
            ck.ok = false;
            ck.err = "eigen job outside the kernel's sizes";
            return;
          }
          ck.span(J.C, 0, (J.W - 1) * J.ldc + J.W - 1, 8, "eig C");
          ck.span(J.V, 0, (J.W - 1) * J.ldv + J.W - 1, 8, "eig V");
          ck.span(J.lam, 0, J.W - 1, 8, "eig lam");
          if (st.pass == 0 && st.wmax > kEigMaxW) {
            // the global-memory form runs for every job of such a launch
            const int64_t Wp = J.W + (J.W & 1);
            ck.span(J.work, 0, 2 * Wp * Wp - 1, 8, "eig work");
          }
          if (J.rank) {
            ck.span(J.rank, 0, 0, 4, "eig rank");
            ck.span(J.theta, 0, 0, 8, "eig theta");
          }
        }
        break;
      }
      case S_CHOL:
      case S_HOUSE: {
        const QrDesc* qs = (const QrDesc*)(blob + st.meta);
        int hh_take[2] = {0, 0};
        for (int i = 0; i < st.count; ++i) {
          const QrDesc& q = qs[i];
          ck.span(q.Y, 0, q.n * q.W - 1, 8, "qr Y");
          ck.span(q.Q, 0, q.n * q.w - 1, 8, "qr Q");
          ck.span(q.hh, 0, q.n * q.W + q.W - 1, 8, "qr hh");
          ck.span(q.tau, 0, q.W - 1, 8, "qr tau");
          ck.span(q.flag, 0, 0, 4, "qr flag");
          if (q.R) ck.span(q.R, 0, q.w * q.W - 1, 8, "qr R");
          if (st.kind == S_HOUSE) {
            // every mode the launch may take has a workgroup of its kernel
            const bool takes = (q.hh_direct || st.force) ? (st.hh_sel & 1) : (st.hh_sel & 2);
            if (takes) ++hh_take[hh_wide_panel(q.n, q.W) ? 0 : 1];
          }
          if (st.kind == S_CHOL && q.gram_part && q.W <= 96 && q.W <= q.n) {
            if (q.W > st.wmax) { ck.ok = false; ck.err = "chol LDS sized below a Gram width"; return; }
            ck.span(q.gram_part, 0, (int64_t)q.gram_splits * q.W * q.W - 1, 8, "qr gram");
            ck.span(q.rinv, 0, q.W * q.W - 1, 8, "qr rinv");
            ck.span(q.r1, 0, q.W * q.W - 1, 8, "qr r1");
            ck.span(q.q1, 0, q.n * q.W - 1, 8, "qr q1");
          }
        }
        if (st.kind == S_HOUSE && (hh_take[0] > st.hh_grid[0] || hh_take[1] > st.hh_grid[1])) {
          ck.ok = false;
          ck.err = "householder launch with fewer workgroups than modes";
        }
        break;
      }
    }
    if (!ck.ok) return;
  }
  if (forked) { ck.ok = false; ck.err = "fork without a join"; }
}

// One line per launch of a checked plan: kernel, descriptors, workgroups,
// largest K-split and segment count (a planning aid for the tests and for
// tuning; not part of the ABI header).
static std::string describe_program(const Program& prog) {
  std::string out;
  const char* blob = prog.blob.data();
  char line[256];
  for (const Step& st : prog.steps) {
    int max_split = 1, max_seg = 0;
    int64_t blocks = st.tiles;
    if (st.kind == S_GEMM) {
      const GemmDesc* ds = (const GemmDesc*)(blob + st.meta);
      for (int i = 0; i < st.count; ++i) {
        max_split = std::max(max_split, (int)ds[i].splits);
        max_seg = std::max(max_seg, (int)ds[i].seg_count);
      }
    } else if (st.kind == S_KRP) {
      const KrpDesc* ds = (const KrpDesc*)(blob + st.meta);
      for (int i = 0; i < st.count; ++i) max_split = std::max(max_split, (int)ds[i].splits);
    } else if (st.kind == S_CHOL) {
      blocks = st.count;
    } else if (st.kind == S_HOUSE) {
      blocks = st.hh_grid[0] + st.hh_grid[1];
    }
    snprintf(line, sizeof line, "%-40s descs=%d blocks=%lld max_split=%d max_seg=%d flops=%.3g\n",
             step_name(st).c_str(), st.count, (long long)blocks, max_split, max_seg, st.flops);
    out += line;
  }
  return out;
}

static int selfcheck_impl(int32_t batch, const tsk_tucker_sum* sums, const tsk_sketch_spec* specs,
                          int out_dtype, int sketch_only, int with_r, char* msg, size_t msglen,
                          bool describe = false) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  tsk_handle_ scratch_handle;
  std::vector<Problem> Ps(batch);
  for (int b = 0; b < batch; ++b) {
    tsk_status st = validate(&scratch_handle, &sums[b], &specs[b], Ps[b]);
    if (st != TSK_OK) {
      say(scratch_handle.err);
      return st;
    }
  }
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* p = (void*)next;
    ck.add(p, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return p;
  };
  std::vector<Outputs> outs(batch);
  for (int b = 0; b < batch; ++b) {
    Problem& P = Ps[b];
    const size_t ein = P.in_f64 ? 8 : 4;
    for (int i = 0; i < P.s; ++i) {
      int64_t cs = 1;
      for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
      P.cores[i] = fake(cs * ein, "core");
      for (int k = 0; k < P.d; ++k)
        P.factors[(size_t)i * P.d + k] = fake(P.dims[k] * P.r(i, k) * ein, "factor");
    }
    for (size_t k = 0; k < P.omega.size(); ++k) P.omega[k] = fake(P.dims[k] * P.ow[k] * ein, "omega");
    Outputs& out = outs[b];
    out.recompress = !sketch_only;
    out.out_f64 = out_dtype == TSK_F64;
    const size_t eo = out.out_f64 ? 8 : 4;
    int64_t hsize = 1;
    for (int n = 0; n < P.d; ++n) {
      if (sketch_only) out.Y.push_back((double*)fake(P.dims[n] * P.W[n] * 8, "Y"));
      out.Q.push_back(fake(P.dims[n] * P.w[n] * eo, "Q"));
      if (with_r) out.R.push_back((double*)fake(P.w[n] * P.W[n] * 8, "R"));
      hsize *= P.w[n];
    }
    out.H = fake(hsize * eo, "H");
  }
  tsk_handle_ fake_handle;
  fake_handle.d_counter = (int64_t*)fake(256, "counter");
  Program p0;
  size_t need = 0;
  if (tsk_status st = plan_many(&fake_handle, Ps, outs, nullptr, p0, &need); st != TSK_OK) {
    say(fake_handle.err);
    return st;
  }
  char* ws = (char*)fake(need, "workspace");
  Program prog;
  size_t need2 = 0;
  plan_many(&fake_handle, Ps, outs, ws, prog, &need2);
  if (need2 != need) {
    say("workspace size differs between the size query and the call");
    return 99;
  }
  check_program(prog, ck);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  if (describe) {
    char tail[128];
    snprintf(tail, sizeof tail, "workspace %zu bytes, descriptors %zu bytes\n", need,
             prog.blob.size());
    say(describe_program(prog) + tail);
  } else {
    say("ok");
  }
  return 0;
}

}  // namespace

static tsk_status plan_backward(const Problem& P, const BackwardIO& io, char* ws, Program& prog,
                                size_t* bytes) {
  Arena ar;
  ar.base = ws;
  ar.ctr_base = (int32_t*)ar.take(256);
  build_backward(P, io, ar, prog);
  if (!ar.too_far.empty()) return TSK_ERR_UNSUPPORTED;
  prog.meta_region = align_up(ar.top, 256);
  *bytes = prog.meta_region + align_up(prog.blob.size(), 256) + 256;
  return TSK_OK;
}

static tsk_status validate_backward(tsk_handle h, const Problem& P) {
  if (P.kind != TSK_SKETCH_KRP)
    return fail(h, TSK_ERR_UNSUPPORTED, "backward is implemented for the Khatri-Rao sketch");
  for (int n = 0; n < P.d; ++n) {
    if (P.W[n] > P.dims[n])
      return fail(h, TSK_ERR_UNSUPPORTED, "backward needs sketch width <= n_k (mode %d)", n);
    if (P.w[n] > 96) return fail(h, TSK_ERR_UNSUPPORTED, "backward needs sketch width <= 96");
  }
  return TSK_OK;
}


// Host-only bounds self-check of a backward plan (tests; not part of the ABI header).
extern "C" int tsk_plan_selfcheck_backward(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                                           int out_dtype, int with_qbar, char* msg, size_t msglen) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  tsk_handle_ hh;
  Problem P;
  tsk_status st = validate(&hh, sum, spec, P);
  if (st == TSK_OK) st = validate_backward(&hh, P);
  if (st != TSK_OK) {
    say(hh.err);
    return st;
  }
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* p = (void*)next;
    ck.add(p, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return p;
  };
  const size_t ein = P.in_f64 ? 8 : 4, eo = out_dtype == TSK_F64 ? 8 : 4;
  BackwardIO io;
  io.out_f64 = out_dtype == TSK_F64;
  int64_t hsize = 1;
  for (int i = 0; i < P.s; ++i) {
    int64_t cs = 1;
    for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
    P.cores[i] = fake(cs * ein, "core");
    io.core_bar.push_back(fake(cs * ein, "core_bar"));
    for (int k = 0; k < P.d; ++k) {
      P.factors[(size_t)i * P.d + k] = fake(P.dims[k] * P.r(i, k) * ein, "factor");
      io.factor_bar.push_back(fake(P.dims[k] * P.r(i, k) * ein, "factor_bar"));
    }
  }
  for (int n = 0; n < P.d; ++n) {
    io.Q.push_back(fake(P.dims[n] * P.w[n] * eo, "Q"));
    io.R.push_back((const double*)fake(P.w[n] * P.w[n] * 8, "R"));
    if (with_qbar) io.Qbar.push_back(fake(P.dims[n] * P.w[n] * eo, "Qbar"));
    hsize *= P.w[n];
  }
  io.Hbar = fake(hsize * eo, "Hbar");
  io.singular = (unsigned long long*)fake(256, "counter");
  Program p0;
  size_t need = 0;
  if (plan_backward(P, io, nullptr, p0, &need) != TSK_OK) {
    say("an operand stride reaches past 2^31 bytes inside one tile");
    return TSK_ERR_UNSUPPORTED;
  }
  char* ws = (char*)fake(need, "workspace");
  Program prog;
  size_t need2 = 0;
  plan_backward(P, io, ws, prog, &need2);
  if (need != need2) {
    say("workspace size differs between the size query and the call");
    return 99;
  }
  check_program(prog, ck);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  say("ok");
  return 0;
}


extern "C" int tsk_plan_selfcheck_project(const tsk_tucker_sum* sum, const int64_t* widths,
                                          int basis_dtype, int project_prec, int out_dtype,
                                          char* msg, size_t msglen) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  tsk_handle_ scratch_handle;
  Problem P;
  if (tsk_status st = validate_project(&scratch_handle, sum, widths, project_prec, P); st != TSK_OK) {
    say(scratch_handle.err);
    return st;
  }
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* p = (void*)next;
    ck.add(p, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return p;
  };
  const size_t ein = P.in_f64 ? 8 : 4, eb = basis_dtype == TSK_F64 ? 8 : 4,
               eo = out_dtype == TSK_F64 ? 8 : 4;
  for (int i = 0; i < P.s; ++i) {
    int64_t cs = 1;
    for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
    P.cores[i] = fake(cs * ein, "core");
    for (int k = 0; k < P.d; ++k)
      P.factors[(size_t)i * P.d + k] = fake(P.dims[k] * P.r(i, k) * ein, "factor");
  }
  std::vector<const void*> Q;
  int64_t hsize = 1;
  for (int n = 0; n < P.d; ++n) {
    Q.push_back(fake(P.dims[n] * P.w[n] * eb, "basis"));
    hsize *= P.w[n];
  }
  void* H = fake(hsize * eo, "H");
  tsk_handle_ fake_handle;
  Program p0;
  size_t need = 0;
  if (tsk_status st = plan_project(&fake_handle, P, Q, basis_dtype == TSK_F64, H,
                                   out_dtype == TSK_F64, nullptr, p0, &need);
      st != TSK_OK) {
    say(fake_handle.err);
    return st;
  }
  char* ws = (char*)fake(need, "workspace");
  Program prog;
  size_t need2 = 0;
  plan_project(&fake_handle, P, Q, basis_dtype == TSK_F64, H, out_dtype == TSK_F64, ws, prog,
               &need2);
  if (need2 != need) {
    say("workspace size differs between the size query and the call");
    return 99;
  }
  check_program(prog, ck);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  say("ok");
  return 0;
}

// Every phase of a truncation planned with the given ranks (as the device
// would report them), each launch checked against the workspace and the
// caller's buffers.
// Host-only bounds check of a batch of truncations of one order: job j has
// dims[j*order..], widths[j*order..] and takes the ranks ranks[j*order..]
// (as if the device had chosen them).
extern "C" int tsk_plan_selfcheck_truncate_batched(int32_t batch, int32_t order,
                                                   const int64_t* dims, const int64_t* widths,
                                                   const int32_t* ranks, char* msg,
                                                   size_t msglen) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  if (batch < 1 || dims == nullptr || widths == nullptr || ranks == nullptr) {
    say("bad batch or NULL arrays");
    return TSK_ERR_INVALID_ARG;
  }
  tsk_handle_ scratch_handle;
  std::vector<TruncIO> ios(batch);
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* p = (void*)next;
    ck.add(p, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return p;
  };
  for (int j = 0; j < batch; ++j) {
    const int64_t* dj = dims + (size_t)j * order;
    const int64_t* wj = widths + (size_t)j * order;
    if (tsk_status st = validate_trunc(&scratch_handle, order, dj, wj, 0.5, ios[j]); st != TSK_OK) {
      say(scratch_handle.err);
      return st;
    }
    int64_t hs = 1;
    for (int k = 0; k < order; ++k) {
      const int32_t r = ranks[(size_t)j * order + k];
      if (r < 1 || r > wj[k]) {
        say("rank outside [1, width]");
        return TSK_ERR_INVALID_ARG;
      }
      ios[j].Q.push_back((const double*)fake(dj[k] * wj[k] * 8, "Q"));
      ios[j].U.push_back((double*)fake(dj[k] * wj[k] * 8, "U"));
      hs *= wj[k];
    }
    ios[j].H = (const double*)fake(hs * 8, "H");
    ios[j].G = (double*)fake(hs * 8, "G");
  }
  bool far = false;
  const size_t need = trunc_workspace(ios, &far);
  if (far) {
    say("stride beyond 31-bit offsets");
    return TSK_ERR_UNSUPPORTED;
  }
  char* ws = (char*)fake(need, "workspace");
  Arena fixed;
  fixed.base = ws;
  TruncLayout L;
  trunc_layout(ios, fixed, L);
  auto run = [&](Program& prog) -> tsk_status {
    check_program(prog, ck);
    return ck.ok ? TSK_OK : TSK_ERR_DEVICE;
  };
  auto rank_of = [&](size_t j, int n) -> int32_t { return ranks[j * order + n]; };
  std::vector<std::vector<int32_t>> out;
  const tsk_status st = trunc_drive(&scratch_handle, ios, L, ws, need, run, rank_of, out);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  if (st != TSK_OK) {
    say(scratch_handle.err);
    return 99;
  }
  say("ok");
  return 0;
}

extern "C" int tsk_plan_selfcheck_truncate(int32_t order, const int64_t* dims,
                                           const int64_t* widths, const int32_t* ranks,
                                           char* msg, size_t msglen) {
  return tsk_plan_selfcheck_truncate_batched(1, order, dims, widths, ranks, msg, msglen);
}

extern "C" int tsk_plan_selfcheck_subranks_batched(int32_t batch, const tsk_tucker_sum* sums,
                                                   char* msg, size_t msglen) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  tsk_handle_ scratch_handle;
  std::vector<Problem> Ps;
  if (tsk_status st = validate_subranks_batch(&scratch_handle, batch, sums, 0.5, Ps); st != TSK_OK) {
    say(scratch_handle.err);
    return st;
  }
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* q = (void*)next;
    ck.add(q, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return q;
  };
  for (Problem& P : Ps) {
    const size_t ein = P.in_f64 ? 8 : 4;
    for (int i = 0; i < P.s; ++i) {
      int64_t cs = 1;
      for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
      P.cores[i] = fake(cs * ein, "core");
      for (int k = 0; k < P.d; ++k)
        P.factors[(size_t)i * P.d + k] = fake(P.dims[k] * P.r(i, k) * ein, "factor");
    }
  }
  tsk_handle_ fake_handle;
  Program p0;
  SubrankOut o0;
  size_t need = 0;
  if (tsk_status st = plan_subranks_sized(&fake_handle, Ps, 0.5, nullptr, p0, o0, &need); st != TSK_OK) {
    say(fake_handle.err);
    return st;
  }
  char* ws = (char*)fake(need, "workspace");
  Program prog;
  SubrankOut o1;
  size_t need2 = 0;
  plan_subranks_sized(&fake_handle, Ps, 0.5, ws, prog, o1, &need2);
  if (need2 != need) {
    say("workspace size differs between the size query and the call");
    return 99;
  }
  check_program(prog, ck);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  say("ok");
  return 0;
}

extern "C" int tsk_plan_selfcheck_subranks(const tsk_tucker_sum* sum, char* msg, size_t msglen) {
  return tsk_plan_selfcheck_subranks_batched(1, sum, msg, msglen);
}

extern "C" int tsk_plan_selfcheck_deterministic(const tsk_tucker_sum* sum, char* msg,
                                                size_t msglen) {
  auto say = [&](const std::string& s) {
    if (msg && msglen) {
      std::strncpy(msg, s.c_str(), msglen - 1);
      msg[msglen - 1] = 0;
    }
  };
  tsk_handle_ scratch_handle;
  Problem P;
  TruncIO io;
  if (tsk_status st = validate_det(&scratch_handle, sum, 0.1, P, io); st != TSK_OK) {
    say(scratch_handle.err);
    return st;
  }
  Checker ck;
  uintptr_t next = (uintptr_t)1 << 44;
  auto fake = [&](size_t bytes, const char* name) {
    void* q = (void*)next;
    ck.add(q, bytes, name);
    next += align_up(bytes, (size_t)1 << 20) + ((size_t)1 << 30);
    return q;
  };
  const size_t ein = P.in_f64 ? 8 : 4;
  for (int i = 0; i < P.s; ++i) {
    int64_t cs = 1;
    for (int k = 0; k < P.d; ++k) cs *= P.r(i, k);
    P.cores[i] = fake(cs * ein, "core");
    for (int k = 0; k < P.d; ++k)
      P.factors[(size_t)i * P.d + k] = fake(P.dims[k] * P.r(i, k) * ein, "factor");
  }
  tsk_handle_ fake_handle;
  Program p0;
  DetPlan d0;
  size_t need = 0;
  if (tsk_status st = plan_det_sized(&fake_handle, P, nullptr, p0, d0, &need); st != TSK_OK) {
    say(fake_handle.err);
    return st;
  }
  char* ws = (char*)fake(need, "workspace");
  Program prog;
  DetPlan d1;
  size_t need2 = 0;
  plan_det_sized(&fake_handle, P, ws, prog, d1, &need2);
  if (need2 != need) {
    say("workspace size differs between the size query and the call");
    return 99;
  }
  check_program(prog, ck);
  if (!ck.ok) {
    say(ck.err);
    return 98;
  }
  say("ok");
  return 0;
}

// Host-only bounds self-check of a planned call (tests; not part of the ABI header).
extern "C" int tsk_plan_describe(int32_t batch, const tsk_tucker_sum* sums,
                                 const tsk_sketch_spec* specs, int out_dtype, char* msg,
                                 size_t msglen) {
  return selfcheck_impl(batch, sums, specs, out_dtype, 0, 0, msg, msglen, true);
}

extern "C" int tsk_plan_selfcheck(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                                  int out_dtype, int sketch_only, int with_r, char* msg,
                                  size_t msglen) {
  return selfcheck_impl(1, sum, spec, out_dtype, sketch_only, with_r, msg, msglen);
}

extern "C" int tsk_plan_selfcheck_batched(int32_t batch, const tsk_tucker_sum* sums,
                                          const tsk_sketch_spec* specs, int out_dtype, char* msg,
                                          size_t msglen) {
  return selfcheck_impl(batch, sums, specs, out_dtype, 0, 0, msg, msglen);
}

// ====================================================================== C ABI
extern "C" {

tsk_status tsk_create(tsk_handle* handle, int device) {
  if (handle == nullptr) return TSK_ERR_INVALID_ARG;
  *handle = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return TSK_ERR_INVALID_ARG;
  tsk_handle h = new (std::nothrow) tsk_handle_();
  if (h == nullptr) return TSK_ERR_OUT_OF_MEMORY;
  h->device = device;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      h->arch = prop.gcnArchName;
      h->arch = h->arch.substr(0, h->arch.find(':'));
    }
  }
  if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&h->d_counter, 256) != hipSuccess) {
    delete h;
    return TSK_ERR_DEVICE;
  }
  if (hipMemset(h->d_counter, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    hipFree(h->d_counter);
    delete h;
    return TSK_ERR_DEVICE;
  }
  {
    // each device holds its own copy of `scratch`: look its address up once
    // per device, with that device current
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        hipFree(h->d_counter);
        delete h;
        return TSK_ERR_DEVICE;
      }
      it = addr.emplace(device, (char*)p).first;
    }
    h->scratch_dev = it->second;
  }
  if (hipHostMalloc(&h->fixed_stage, kFixedStageBytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&h->fixed_stage_done, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(h->fixed_stage_done, nullptr) != hipSuccess ||
      hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess) {
    if (h->fixed_stage) hipHostFree(h->fixed_stage);
    if (h->fixed_stage_done) hipEventDestroy(h->fixed_stage_done);
    if (h->side) hipStreamDestroy(h->side);
    if (h->fork_ev) hipEventDestroy(h->fork_ev);
    hipFree(h->d_counter);
    delete h;
    return TSK_ERR_OUT_OF_MEMORY;
  }
  *handle = h;
  return TSK_OK;
}

tsk_status tsk_destroy(tsk_handle h) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  hipSetDevice(h->device);
  hipDeviceSynchronize();
  for (auto& sl : h->ring) {
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.host) hipHostFree(sl.host);
  }
  for (void* p : h->device_keep) hipFree(p);
  if (h->fixed_stage_done) hipEventDestroy(h->fixed_stage_done);
  if (h->fixed_stage) hipHostFree(h->fixed_stage);
  if (h->fork_ev) hipEventDestroy(h->fork_ev);
  if (h->join_ev) hipEventDestroy(h->join_ev);
  if (h->side) hipStreamDestroy(h->side);
  for (auto& r : h->prof_records) {
    hipEventDestroy(r.begin);
    hipEventDestroy(r.end);
  }
  for (hipEvent_t e : h->event_pool) hipEventDestroy(e);
  if (h->d_counter) hipFree(h->d_counter);
  delete h;
  return TSK_OK;
}

const char* tsk_status_string(tsk_status st) {
  switch (st) {
    case TSK_OK: return "TSK_OK";
    case TSK_ERR_INVALID_ARG: return "TSK_ERR_INVALID_ARG";
    case TSK_ERR_UNSUPPORTED: return "TSK_ERR_UNSUPPORTED";
    case TSK_ERR_OUT_OF_MEMORY: return "TSK_ERR_OUT_OF_MEMORY";
    case TSK_ERR_WORKSPACE_TOO_SMALL: return "TSK_ERR_WORKSPACE_TOO_SMALL";
    case TSK_ERR_DEVICE: return "TSK_ERR_DEVICE";
    case TSK_ERR_RANK_DEFICIENT: return "TSK_ERR_RANK_DEFICIENT";
  }
  return "unknown tsk_status";
}

const char* tsk_last_error_detail(tsk_handle h) { return h ? h->err.c_str() : ""; }

tsk_status tsk_krp_width(int32_t order, const int32_t* ell, int32_t* m_out) {
  if (order < 1 || ell == nullptr || m_out == nullptr) return TSK_ERR_INVALID_ARG;
  int32_t m = 0;
  for (int k = 0; k < order; ++k) {
    if (ell[k] < 1) return TSK_ERR_INVALID_ARG;
    m = std::max(m, ell[k]);
  }
  *m_out = m;
  return TSK_OK;
}

tsk_status tsk_kron_sizes(int32_t order, const int32_t* ell, int32_t* q_out) {
  if (order < 2 || order > kMaxOrder || ell == nullptr || q_out == nullptr) return TSK_ERR_INVALID_ARG;
  // prod_j ell_j as an exact integer (unsigned __int128 holds up to 8 factors < 2^16)
  unsigned __int128 prod = 1;
  for (int k = 0; k < order; ++k) {
    if (ell[k] < 1 || ell[k] > 65535) return TSK_ERR_INVALID_ARG;
    prod *= (unsigned)ell[k];
  }
  for (int k = 0; k < order; ++k) {
    for (int64_t q = 1;; ++q) {
      unsigned __int128 p = 1;
      bool big = false;
      for (int e = 0; e < order - 1; ++e) {
        p *= (unsigned __int128)(q * ell[k]);
        if (p >= prod) { big = true; break; }
      }
      if (big || p >= prod) {
        q_out[k] = (int32_t)q;
        break;
      }
    }
  }
  return TSK_OK;
}

tsk_status tsk_sketch_widths(const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                             int64_t* sketch_width, int64_t* basis_width) {
  Problem P;
  tsk_status st = validate(nullptr, sum, spec, P);
  if (st != TSK_OK) return st;
  for (int n = 0; n < P.d; ++n) {
    if (sketch_width) sketch_width[n] = P.W[n];
    if (basis_width) basis_width[n] = P.w[n];
  }
  return TSK_OK;
}

tsk_status tsk_sketch_omega(tsk_handle h, uint64_t seed, int32_t mode, int64_t rows,
                            int64_t cols, void* out, tsk_dtype out_dtype, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  if (out == nullptr || rows < 1 || cols < 1 || mode < 0)
    return fail(h, TSK_ERR_INVALID_ARG, "bad omega arguments");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad dtype");
  tsk_status st = set_device(h);
  if (st != TSK_OK) return st;
  if (launch_omega(seed, mode, rows, cols, out, out_dtype == TSK_F64, (hipStream_t)stream) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "omega launch failed");
  return TSK_OK;
}

tsk_status tucker_sum_workspace_size(tsk_handle h, const tsk_tucker_sum* sum,
                                     const tsk_sketch_spec* spec, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st != TSK_OK) return st;
  // the recompress plan needs at least what the sketch-only plan needs
  // the recompress plan needs at least what the sketch-only plan needs; the
  // FP32- and FP64-output plans differ (Q staging vs. partial sizes): take both
  size_t best = 0;
  for (int o = 0; o < 2; ++o) {
    Outputs out;
    out.recompress = true;
    out.out_f64 = o == 1;
    out.Q.assign(P.d, nullptr);
    out.R.assign(P.d, nullptr);
    Program prog;
    size_t b = 0;
    if (tsk_status pst = plan(h, P, out, nullptr, prog, &b); pst != TSK_OK) return pst;
    best = std::max(best, b);
  }
  *bytes = best;
  return TSK_OK;
}

tsk_status tucker_sum_sketch(tsk_handle h, const tsk_tucker_sum* sum, const tsk_sketch_spec* spec,
                             double* const* Y_out, void* ws, size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st != TSK_OK) return st;
  if (Y_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Y_out is NULL");
  Outputs out;
  out.recompress = false;
  for (int n = 0; n < P.d; ++n) {
    if (Y_out[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Y_out[%d] is NULL", n);
    out.Y.push_back(Y_out[n]);
  }
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  size_t need = 0;
  if (tsk_status pst = plan(h, P, out, (char*)ws, prog, &need); pst != TSK_OK) return pst;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}

tsk_status tucker_sum_recompress(tsk_handle h, const tsk_tucker_sum* sum,
                                 const tsk_sketch_spec* spec, void* const* Q_out, void* H_out,
                                 tsk_dtype out_dtype, double* const* R_out, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st != TSK_OK) return st;
  if (Q_out == nullptr || H_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out or H_out is NULL");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  Outputs out;
  out.recompress = true;
  out.out_f64 = out_dtype == TSK_F64;
  out.H = H_out;
  for (int n = 0; n < P.d; ++n) {
    if (Q_out[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d] is NULL", n);
    out.Q.push_back(Q_out[n]);
    if (R_out != nullptr) {
      if (R_out[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "R_out[%d] is NULL", n);
      out.R.push_back(R_out[n]);
    }
  }
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  size_t need = 0;
  if (tsk_status pst = plan(h, P, out, (char*)ws, prog, &need); pst != TSK_OK) return pst;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}

tsk_status tucker_sum_recompress_noalloc(tsk_handle h, const tsk_tucker_sum* sum,
                                         const tsk_sketch_spec* spec, void* const* Q_out,
                                         void* H_out, tsk_dtype out_dtype, double* const* R_out,
                                         void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st != TSK_OK) return st;
  if (Q_out == nullptr || H_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out or H_out is NULL");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  Outputs out;
  out.recompress = true;
  out.out_f64 = out_dtype == TSK_F64;
  out.H = H_out;
  for (int n = 0; n < P.d; ++n) {
    if (Q_out[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d] is NULL", n);
    out.Q.push_back(Q_out[n]);
    if (R_out != nullptr) {
      if (R_out[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "R_out[%d] is NULL", n);
      out.R.push_back(R_out[n]);
    }
  }
  if (h->scratch_dev == nullptr) return fail(h, TSK_ERR_DEVICE, "no scratch address for the device");
  Program prog;
  size_t need = 0;
  if (tsk_status pst = plan(h, P, out, h->scratch_dev, prog, &need); pst != TSK_OK) return pst;
  if (need > kScratchBytes)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL,
                "problem needs %zu bytes of device scratch; the no-allocation call holds %zu", need,
                kScratchBytes);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, h->scratch_dev, (hipStream_t)stream, true);
}

tsk_status tucker_sum_project_workspace_size(tsk_handle h, const tsk_tucker_sum* sum,
                                             const int64_t* widths, tsk_dtype basis_dtype,
                                             tsk_precision project_prec, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  Problem P;
  tsk_status st = validate_project(h, sum, widths, project_prec, P);
  if (st != TSK_OK) return st;
  if (basis_dtype != TSK_F64 && basis_dtype != TSK_F32)
    return fail(h, TSK_ERR_INVALID_ARG, "bad basis dtype");
  std::vector<const void*> Q(P.d, nullptr);
  size_t best = 0;
  for (int o = 0; o < 2; ++o) {
    Program prog;
    size_t b = 0;
    if ((st = plan_project(h, P, Q, basis_dtype == TSK_F64, nullptr, o == 1, nullptr, prog, &b)) !=
        TSK_OK)
      return st;
    best = std::max(best, b);
  }
  *bytes = best;
  return TSK_OK;
}

tsk_status tucker_sum_project(tsk_handle h, const tsk_tucker_sum* sum, const void* const* bases,
                              const int64_t* widths, tsk_dtype basis_dtype,
                              tsk_precision project_prec, void* H_out, tsk_dtype out_dtype,
                              void* ws, size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate_project(h, sum, widths, project_prec, P);
  if (st != TSK_OK) return st;
  if (basis_dtype != TSK_F64 && basis_dtype != TSK_F32)
    return fail(h, TSK_ERR_INVALID_ARG, "bad basis dtype");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  if (bases == nullptr || H_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "bases or H_out is NULL");
  std::vector<const void*> Q;
  for (int n = 0; n < P.d; ++n) {
    if (bases[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "bases[%d] is NULL", n);
    Q.push_back(bases[n]);
  }
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  size_t need = 0;
  if ((st = plan_project(h, P, Q, basis_dtype == TSK_F64, H_out, out_dtype == TSK_F64, (char*)ws,
                         prog, &need)) != TSK_OK)
    return st;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}

tsk_status tucker_truncate_workspace_size(tsk_handle h, int32_t order, const int64_t* dims,
                                         const int64_t* widths, double eps, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  TruncIO io;
  tsk_status st = validate_trunc(h, order, dims, widths, eps, io);
  if (st != TSK_OK) return st;
  io.Q.assign(order, nullptr);
  io.U.assign(order, nullptr);
  bool far = false;
  *bytes = trunc_workspace(io, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  return TSK_OK;
}

tsk_status tucker_truncate(tsk_handle h, int32_t order, const int64_t* dims,
                           const int64_t* widths, const double* const* Q, const double* H,
                           double eps, double* const* U_out, double* G_out, int32_t* ranks_out,
                           void* ws, size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  TruncIO io;
  tsk_status st = validate_trunc(h, order, dims, widths, eps, io);
  if (st != TSK_OK) return st;
  if (Q == nullptr || H == nullptr || U_out == nullptr || G_out == nullptr || ranks_out == nullptr)
    return fail(h, TSK_ERR_INVALID_ARG, "NULL Q, H, U_out, G_out or ranks_out");
  for (int k = 0; k < order; ++k) {
    if (Q[k] == nullptr || U_out[k] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q[%d] or U_out[%d] is NULL", k, k);
    io.Q.push_back(Q[k]);
    io.U.push_back(U_out[k]);
  }
  io.H = H;
  io.G = G_out;
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  bool far = false;
  const size_t need = trunc_workspace(io, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return truncate_run(h, io, (char*)ws, need, (hipStream_t)stream, ranks_out);
}

tsk_status tucker_sum_subranks_workspace_size(tsk_handle h, const tsk_tucker_sum* sum,
                                              size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  Problem P;
  tsk_status st = validate_subranks(h, sum, 0.5, P);
  if (st != TSK_OK) return st;
  Program prog;
  SubrankOut out;
  return plan_subranks_sized(h, P, 0.5, nullptr, prog, out, bytes);
}

tsk_status tucker_sum_subranks(tsk_handle h, const tsk_tucker_sum* sum, double eps,
                               const int32_t* p, int32_t* ell_out, void* ws, size_t ws_bytes,
                               void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate_subranks(h, sum, eps, P);
  if (st != TSK_OK) return st;
  if (p == nullptr || ell_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "p or ell_out is NULL");
  for (int n = 0; n < P.d; ++n)
    if (p[n] < 0) return fail(h, TSK_ERR_INVALID_ARG, "p[%d] < 0", n);
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  SubrankOut out;
  size_t need = 0;
  if ((st = plan_subranks_sized(h, P, eps, (char*)ws, prog, out, &need)) != TSK_OK) return st;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = run_program(h, prog, (char*)ws, s)) != TSK_OK) return st;
  int32_t r[kMaxOrder];
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(r, out.ranks, sizeof(int32_t) * P.d, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "reading the effective subranks failed");
  for (int n = 0; n < P.d; ++n) ell_out[n] = r[n] + p[n];
  return TSK_OK;
}

tsk_status tucker_sum_subranks_batched_workspace_size(tsk_handle h, int32_t batch,
                                                      const tsk_tucker_sum* sums, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  std::vector<Problem> Ps;
  tsk_status st = validate_subranks_batch(h, batch, sums, 0.5, Ps);
  if (st != TSK_OK) return st;
  Program prog;
  SubrankOut out;
  return plan_subranks_sized(h, Ps, 0.5, nullptr, prog, out, bytes);
}

tsk_status tucker_sum_subranks_batched(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                                       double eps, const int32_t* p, int32_t* ell_out, void* ws,
                                       size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  std::vector<Problem> Ps;
  tsk_status st = validate_subranks_batch(h, batch, sums, eps, Ps);
  if (st != TSK_OK) return st;
  if (p == nullptr || ell_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "p or ell_out is NULL");
  size_t total = 0;
  for (const Problem& P : Ps) total += P.d;
  for (size_t i = 0; i < total; ++i)
    if (p[i] < 0) return fail(h, TSK_ERR_INVALID_ARG, "p[%zu] < 0", i);
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  SubrankOut out;
  size_t need = 0;
  if ((st = plan_subranks_sized(h, Ps, eps, (char*)ws, prog, out, &need)) != TSK_OK) return st;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = run_program(h, prog, (char*)ws, s)) != TSK_OK) return st;
  std::vector<int32_t> r((size_t)kMaxOrder * batch);
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(r.data(), out.ranks, sizeof(int32_t) * r.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "reading the effective subranks failed");
  size_t at = 0;
  for (int j = 0; j < batch; ++j)
    for (int n = 0; n < Ps[j].d; ++n, ++at) ell_out[at] = r[(size_t)j * kMaxOrder + n] + p[at];
  return TSK_OK;
}

static tsk_status validate_trunc_batch(tsk_handle h, int32_t batch, const tsk_truncation* jobs,
                                       bool need_ptrs, std::vector<TruncIO>& ios) {
  if (batch < 1 || jobs == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "batch < 1 or jobs is NULL");
  ios.assign(batch, TruncIO{});
  for (int j = 0; j < batch; ++j) {
    const tsk_truncation& T = jobs[j];
    if (tsk_status st = validate_trunc(h, T.order, T.dims, T.widths, T.eps, ios[j]); st != TSK_OK) {
      h->err = "job " + std::to_string(j) + ": " + h->err;
      return st;
    }
    if (!need_ptrs) {
      ios[j].Q.assign(T.order, nullptr);
      ios[j].U.assign(T.order, nullptr);
      continue;
    }
    if (T.Q == nullptr || T.H == nullptr || T.U_out == nullptr || T.G_out == nullptr ||
        T.ranks_out == nullptr)
      return fail(h, TSK_ERR_INVALID_ARG, "job %d: NULL Q, H, U_out, G_out or ranks_out", j);
    for (int k = 0; k < T.order; ++k) {
      if (T.Q[k] == nullptr || T.U_out[k] == nullptr)
        return fail(h, TSK_ERR_INVALID_ARG, "job %d: Q[%d] or U_out[%d] is NULL", j, k, k);
      ios[j].Q.push_back(T.Q[k]);
      ios[j].U.push_back(T.U_out[k]);
    }
    ios[j].H = T.H;
    ios[j].G = T.G_out;
  }
  return TSK_OK;
}

tsk_status tucker_truncate_batched_workspace_size(tsk_handle h, int32_t batch,
                                                  const tsk_truncation* jobs, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  std::vector<TruncIO> ios;
  tsk_status st = validate_trunc_batch(h, batch, jobs, false, ios);
  if (st != TSK_OK) return st;
  bool far = false;
  *bytes = trunc_workspace(ios, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  return TSK_OK;
}

tsk_status tucker_truncate_batched(tsk_handle h, int32_t batch, const tsk_truncation* jobs,
                                   void* ws, size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  std::vector<TruncIO> ios;
  tsk_status st = validate_trunc_batch(h, batch, jobs, true, ios);
  if (st != TSK_OK) return st;
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  bool far = false;
  const size_t need = trunc_workspace(ios, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  std::vector<int32_t*> outs(batch);
  for (int j = 0; j < batch; ++j) outs[j] = jobs[j].ranks_out;
  return truncate_run(h, ios, (char*)ws, need, (hipStream_t)stream, outs.data());
}

tsk_status tucker_sum_round_deterministic_workspace_size(tsk_handle h,
                                                        const tsk_tucker_sum* sum, double tau,
                                                        size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  Problem P;
  TruncIO io;
  tsk_status st = validate_det(h, sum, tau, P, io);
  if (st != TSK_OK) return st;
  Program prog;
  DetPlan D;
  size_t p1 = 0;
  if ((st = plan_det_sized(h, P, nullptr, prog, D, &p1)) != TSK_OK) return st;
  io.Q.assign(P.d, nullptr);
  io.U.assign(P.d, nullptr);
  bool far = false;
  *bytes = p1 + trunc_workspace(io, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  return TSK_OK;
}

tsk_status tucker_sum_round_deterministic(tsk_handle h, const tsk_tucker_sum* sum, double tau,
                                          double* const* U_out, double* G_out,
                                          int32_t* ranks_out, void* ws, size_t ws_bytes,
                                          void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  TruncIO io;
  tsk_status st = validate_det(h, sum, tau, P, io);
  if (st != TSK_OK) return st;
  if (U_out == nullptr || G_out == nullptr || ranks_out == nullptr)
    return fail(h, TSK_ERR_INVALID_ARG, "NULL U_out, G_out or ranks_out");
  for (int k = 0; k < P.d; ++k)
    if (U_out[k] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "U_out[%d] is NULL", k);
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  DetPlan D;
  size_t p1 = 0;
  if ((st = plan_det_sized(h, P, (char*)ws, prog, D, &p1)) != TSK_OK) return st;
  for (int k = 0; k < P.d; ++k) {
    io.Q.push_back(D.Q[k]);
    io.U.push_back(U_out[k]);
  }
  io.H = D.core;
  io.G = G_out;
  bool far = false;
  const size_t tneed = trunc_workspace(io, &far);
  if (far) return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  if (ws_bytes < p1 + tneed)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, p1 + tneed);
  if ((st = set_device(h)) != TSK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = run_program(h, prog, (char*)ws, s)) != TSK_OK) return st;
  return truncate_run(h, io, (char*)ws + p1, tneed, s, ranks_out);
}

tsk_status tsk_profile_enable(tsk_handle h, int32_t on) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->prof = on != 0;
  return TSK_OK;
}

tsk_status tsk_profile_report(tsk_handle h, char* buf, size_t buf_len, size_t* needed) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  struct Agg {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::vector<std::pair<std::string, Agg>> agg;
  for (auto& r : h->prof_records) {
    if (hipEventSynchronize(r.end) != hipSuccess) return fail(h, TSK_ERR_DEVICE, "event wait failed");
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.begin, r.end) != hipSuccess)
      return fail(h, TSK_ERR_DEVICE, "hipEventElapsedTime failed");
    size_t j = 0;
    while (j < agg.size() && agg[j].first != r.name) ++j;
    if (j == agg.size()) agg.push_back({r.name, Agg{}});
    agg[j].second.launches += 1;
    agg[j].second.ms += ms;
    agg[j].second.flops += r.flops;
    agg[j].second.bytes += r.bytes;
  }
  std::string js = "{";
  for (size_t j = 0; j < agg.size(); ++j) {
    char line[384];
    snprintf(line, sizeof line, "%s\"%s\": {\"launches\": %lld, \"ms\": %.9g, \"flops\": %.17g, \"bytes\": %.17g}",
             j ? ", " : "", agg[j].first.c_str(), (long long)agg[j].second.launches, agg[j].second.ms,
             agg[j].second.flops, agg[j].second.bytes);
    js += line;
  }
  js += "}";
  if (needed) *needed = js.size() + 1;
  if (buf == nullptr || buf_len < js.size() + 1)
    return buf == nullptr ? TSK_OK : fail(h, TSK_ERR_INVALID_ARG, "report buffer too small");
  std::memcpy(buf, js.c_str(), js.size() + 1);
  for (auto& r : h->prof_records) {
    h->event_pool.push_back(r.begin);
    h->event_pool.push_back(r.end);
  }
  h->prof_records.clear();
  return TSK_OK;
}

// ---- batched form: many independent sums in one launch sequence
static tsk_status validate_batch(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                                 const tsk_sketch_spec* specs, std::vector<Problem>& Ps) {
  if (batch < 1 || sums == nullptr || specs == nullptr)
    return fail(h, TSK_ERR_INVALID_ARG, "batch < 1 or NULL sums/specs");
  Ps.resize(batch);
  for (int b = 0; b < batch; ++b) {
    tsk_status st = validate(h, &sums[b], &specs[b], Ps[b]);
    if (st != TSK_OK) {
      if (h) h->err = "sum " + std::to_string(b) + ": " + h->err;
      return st;
    }
    if (Ps[b].d != Ps[0].d || Ps[b].kind != Ps[0].kind || Ps[b].ps != Ps[0].ps ||
        Ps[b].pp != Ps[0].pp)
      return fail(h, TSK_ERR_INVALID_ARG,
                  "sum %d: order, sketch kind and precisions must match across the batch", b);
  }
  return TSK_OK;
}

tsk_status tucker_sum_batched_workspace_size(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                                             const tsk_sketch_spec* specs, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  std::vector<Problem> Ps;
  tsk_status st = validate_batch(h, batch, sums, specs, Ps);
  if (st != TSK_OK) return st;
  size_t best = 0;
  for (int o = 0; o < 2; ++o) {
    std::vector<Outputs> outs(batch);
    for (int b = 0; b < batch; ++b) {
      outs[b].recompress = true;
      outs[b].out_f64 = o == 1;
      outs[b].Q.assign(Ps[b].d, nullptr);
    }
    Program prog;
    size_t nb = 0;
    if (tsk_status pst = plan_many(h, Ps, outs, nullptr, prog, &nb); pst != TSK_OK) return pst;
    best = std::max(best, nb);
  }
  *bytes = best;
  return TSK_OK;
}

tsk_status tucker_sum_recompress_batched(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                                         const tsk_sketch_spec* specs, void* const* const* Q_out,
                                         void* const* H_out, tsk_dtype out_dtype, void* ws,
                                         size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  std::vector<Problem> Ps;
  tsk_status st = validate_batch(h, batch, sums, specs, Ps);
  if (st != TSK_OK) return st;
  if (Q_out == nullptr || H_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out or H_out is NULL");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  std::vector<Outputs> outs(batch);
  for (int b = 0; b < batch; ++b) {
    outs[b].recompress = true;
    outs[b].out_f64 = out_dtype == TSK_F64;
    if (Q_out[b] == nullptr || H_out[b] == nullptr)
      return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d] or H_out[%d] is NULL", b, b);
    outs[b].H = H_out[b];
    for (int n = 0; n < Ps[b].d; ++n) {
      if (Q_out[b][n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d][%d] is NULL", b, n);
      outs[b].Q.push_back(Q_out[b][n]);
    }
  }
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  size_t need = 0;
  if (tsk_status pst = plan_many(h, Ps, outs, (char*)ws, prog, &need); pst != TSK_OK) return pst;
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}

// ---- autotuning: measured choices of the planner's launch parameters
static const char* prec_name(int p) {
  switch (p) {
    case P_FP64: return "fp64";
    case P_FP32: return "fp32";
    case P_BF16X1: return "bf16x1";
    case P_BF16X3: return "bf16x3";
    case P_BF16X6: return "bf16x6";
  }
  return "?";
}

static const char* tune_kernel_name(int cls) {
  return (cls == kTuneKrpSplit || cls == kTuneKrpKw) ? "krp_core_sketch" : role_name(cls);
}

static const char* tune_param_name(int cls) {
  return cls == kTuneKrpKw ? "waves_per_quadrant" : "split_target";
}

static std::string tune_dump(const std::map<uint32_t, TuneEntry>& t, const std::string& arch) {
  std::string js = "{\n  \"arch\": \"" + arch + "\",\n  \"entries\": [";
  bool first = true;
  for (const auto& kv : t) {
    const uint32_t k = kv.first;
    const int cls = (k >> 20) & 31, prec = (k >> 16) & 15, tl = (k >> 8) & 255, kl = k & 255;
    char line[512];
    snprintf(line, sizeof line,
             "%s\n    {\"kernel\": \"%s\", \"param\": \"%s\", \"prec\": \"%s\", \"tiles_log2\": %d, "
             "\"ktiles_log2\": %d, \"value\": %d, \"us\": %.3f}",
             first ? "" : ",", tune_kernel_name(cls), tune_param_name(cls), prec_name(prec), tl, kl,
             kv.second.value, kv.second.us);
    js += line;
    first = false;
  }
  js += "\n  ]\n}\n";
  return js;
}

// Reads the text tune_dump writes (keys in any order, any whitespace).
// Fails, leaving `out` untouched, on malformed input, an unknown kernel,
// parameter or precision, a value outside its range, or another arch.
static bool tune_parse(const std::string& text, const std::string& arch,
                std::map<uint32_t, TuneEntry>& out, std::string& err) {
  size_t i = 0;
  const size_t n = text.size();
  auto ws = [&]() {
    while (i < n && (text[i] == ' ' || text[i] == '\n' || text[i] == '\t' || text[i] == '\r')) ++i;
  };
  auto expect = [&](char c) {
    ws();
    if (i < n && text[i] == c) {
      ++i;
      return true;
    }
    err = std::string("expected '") + c + "' at offset " + std::to_string(i);
    return false;
  };
  auto str = [&](std::string& v) {
    if (!expect('"')) return false;
    const size_t b = i;
    while (i < n && text[i] != '"') ++i;
    if (i >= n) {
      err = "unterminated string";
      return false;
    }
    v = text.substr(b, i - b);
    ++i;
    return true;
  };
  auto num = [&](double& v) {
    ws();
    const char* b = text.c_str() + i;
    char* e = nullptr;
    v = std::strtod(b, &e);
    if (e == b) {
      err = "expected a number at offset " + std::to_string(i);
      return false;
    }
    i += (size_t)(e - b);
    return true;
  };
  std::map<uint32_t, TuneEntry> table;
  std::string file_arch;
  bool have_entries = false;
  if (!expect('{')) return false;
  for (;;) {
    std::string key;
    if (!str(key) || !expect(':')) return false;
    if (key == "arch") {
      if (!str(file_arch)) return false;
    } else if (key == "entries") {
      have_entries = true;
      if (!expect('[')) return false;
      ws();
      if (i < n && text[i] == ']') {
        ++i;
      } else {
        for (;;) {
          if (!expect('{')) return false;
          std::string kernel, param, prec;
          double tl = -1, kl = -1, value = -1, us = 0;
          for (;;) {
            std::string f;
            if (!str(f) || !expect(':')) return false;
            bool ok = true;
            if (f == "kernel") ok = str(kernel);
            else if (f == "param") ok = str(param);
            else if (f == "prec") ok = str(prec);
            else if (f == "tiles_log2") ok = num(tl);
            else if (f == "ktiles_log2") ok = num(kl);
            else if (f == "value") ok = num(value);
            else if (f == "us") ok = num(us);
            else {
              err = "unknown field " + f;
              return false;
            }
            if (!ok) return false;
            ws();
            if (i < n && text[i] == ',') {
              ++i;
              continue;
            }
            if (!expect('}')) return false;
            break;
          }
          int cls = -1;
          if (kernel == "krp_core_sketch")
            cls = param == "split_target" ? kTuneKrpSplit
                  : param == "waves_per_quadrant" ? kTuneKrpKw : -1;
          else if (param == "split_target")
            for (int r = 0; r < R_OTHER; ++r)
              if (kernel == role_name(r)) cls = r;
          int pc = -1;
          for (int q = 0; q <= P_BF16X6; ++q)
            if (prec == prec_name(q)) pc = q;
          if (cls < 0 || pc < 0) {
            err = "unknown kernel, parameter or precision: " + kernel + " " + param + " " + prec;
            return false;
          }
          const bool kw = cls == kTuneKrpKw;
          if (tl < 0 || tl > 62 || kl < 0 || kl > 62 || tl != (int)tl || kl != (int)kl ||
              (kw ? !(value == 1 || value == 2 || value == 4) : !(value >= 1 && value <= 65536)) ||
              value != (int)value) {
            err = "entry for " + kernel + " out of range";
            return false;
          }
          const uint32_t k = (uint32_t)cls << 20 | (uint32_t)pc << 16 | (uint32_t)tl << 8 | (uint32_t)kl;
          table[k] = TuneEntry{(int)value, us};
          ws();
          if (i < n && text[i] == ',') {
            ++i;
            continue;
          }
          if (!expect(']')) return false;
          break;
        }
      }
    } else {
      err = "unknown key " + key;
      return false;
    }
    ws();
    if (i < n && text[i] == ',') {
      ++i;
      continue;
    }
    if (!expect('}')) return false;
    break;
  }
  if (!have_entries) {
    err = "no entries";
    return false;
  }
  if (file_arch != arch) {
    err = "cache is for '" + file_arch + "', the device is '" + arch + "'";
    return false;
  }
  out = table;
  return true;
}

// Median time (ms) of every launch of `prog` over `reps` runs after one
// warm-up run.
static tsk_status time_steps(tsk_handle h, Program& prog, char* ws, hipStream_t s, int reps,
                             std::vector<double>& med) {
  const bool was = h->prof;
  std::vector<std::vector<double>> samples(prog.steps.size());
  auto recycle = [&]() {
    for (auto& r : h->prof_records) {
      h->event_pool.push_back(r.begin);
      h->event_pool.push_back(r.end);
    }
    h->prof_records.clear();
  };
  recycle();
  h->prof = true;
  tsk_status st = TSK_OK;
  for (int r = 0; r <= reps && st == TSK_OK; ++r) {
    st = run_program(h, prog, ws, s);
    if (st == TSK_OK && hipStreamSynchronize(s) != hipSuccess)
      st = fail(h, TSK_ERR_DEVICE, "stream synchronisation failed");
    if (st == TSK_OK && r > 0)
      for (auto& rec : h->prof_records) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, rec.begin, rec.end) != hipSuccess) {
          st = fail(h, TSK_ERR_DEVICE, "hipEventElapsedTime failed");
          break;
        }
        if (rec.step >= 0 && rec.step < (int)samples.size()) samples[rec.step].push_back(ms);
      }
    recycle();
  }
  h->prof = was;
  if (st != TSK_OK) return st;
  med.assign(prog.steps.size(), 0.0);
  for (size_t j = 0; j < samples.size(); ++j) {
    auto& v = samples[j];
    if (v.empty()) continue;
    std::sort(v.begin(), v.end());
    med[j] = v[v.size() / 2];
  }
  return TSK_OK;
}

// One tuning pass: every candidate value forced on every class of the pass
// at once (the launches of different classes do not share their choices),
// each class then keeping the value under which its launches were fastest.
static tsk_status tune_pass(tsk_handle h, const std::vector<Problem>& Ps,
                            const std::vector<Outputs>& outs, hipStream_t s, int reps, bool kw_pass,
                            char*& ws, size_t& cap, std::map<uint32_t, TuneEntry>& best) {
  static const int kSplitTargets[] = {128, 256, 512, 1024, 2048, 4096};
  static const int kKw[] = {1, 4};
  const int* cand = kw_pass ? kKw : kSplitTargets;
  const int ncand = kw_pass ? 2 : 6;
  tsk_status st = TSK_OK;
  for (int c = 0; c < ncand && st == TSK_OK; ++c) {
    h->force_split = kw_pass ? 0 : cand[c];
    h->force_kw = kw_pass ? cand[c] : 0;
    Program p0, prog;
    size_t need = 0;
    if ((st = plan_many(h, Ps, outs, nullptr, p0, &need)) != TSK_OK) break;
    if (need > cap) {
      if (ws != nullptr && hipFree(ws) != hipSuccess) {
        st = fail(h, TSK_ERR_DEVICE, "hipFree failed");
        break;
      }
      ws = nullptr;
      cap = 0;
      if (hipMalloc((void**)&ws, need) != hipSuccess) {
        st = fail(h, TSK_ERR_OUT_OF_MEMORY, "tuning workspace of %zu bytes", need);
        break;
      }
      cap = need;
    }
    if ((st = plan_many(h, Ps, outs, ws, prog, &need)) != TSK_OK) break;
    std::vector<double> med;
    if ((st = time_steps(h, prog, ws, s, reps, med)) != TSK_OK) break;
    std::map<uint32_t, double> cost;
    for (size_t j = 0; j < prog.steps.size(); ++j)
      for (uint32_t k : prog.steps[j].keys)
        if ((((k >> 20) & 31) == kTuneKrpKw) == kw_pass) cost[k] += med[j];
    for (const auto& kv : cost) {
      auto it = best.find(kv.first);
      const double us = kv.second * 1e3;
      if (it == best.end() || us < it->second.us) best[kv.first] = TuneEntry{cand[c], us};
    }
  }
  h->force_split = 0;
  h->force_kw = 0;
  return st;
}

tsk_status tsk_autotune(tsk_handle h, int32_t batch, const tsk_tucker_sum* sums,
                        const tsk_sketch_spec* specs, void* const* const* Q_out,
                        void* const* H_out, tsk_dtype out_dtype, int32_t reps, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  if (reps < 1 || reps > 100) return fail(h, TSK_ERR_INVALID_ARG, "reps must be in [1, 100]");
  std::vector<Problem> Ps;
  tsk_status st = validate_batch(h, batch, sums, specs, Ps);
  if (st != TSK_OK) return st;
  if (Q_out == nullptr || H_out == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out or H_out is NULL");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  std::vector<Outputs> outs(batch);
  for (int b = 0; b < batch; ++b) {
    outs[b].recompress = true;
    outs[b].out_f64 = out_dtype == TSK_F64;
    if (Q_out[b] == nullptr || H_out[b] == nullptr)
      return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d] or H_out[%d] is NULL", b, b);
    outs[b].H = H_out[b];
    for (int n = 0; n < Ps[b].d; ++n) {
      if (Q_out[b][n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_out[%d][%d] is NULL", b, n);
      outs[b].Q.push_back(Q_out[b][n]);
    }
  }
  if ((st = set_device(h)) != TSK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = nullptr;
  size_t cap = 0;
  std::map<uint32_t, TuneEntry> split_best, kw_best;
  // the measured classes start from the planner's defaults, so that the
  // split pass sees the default quadrant sharing and vice versa
  std::map<uint32_t, TuneEntry> saved = h->tune;
  st = tune_pass(h, Ps, outs, s, reps, false, ws, cap, split_best);
  if (st == TSK_OK) {
    for (const auto& kv : split_best) h->tune[kv.first] = kv.second;
    st = tune_pass(h, Ps, outs, s, reps, true, ws, cap, kw_best);
  }
  if (st == TSK_OK)
    for (const auto& kv : kw_best) h->tune[kv.first] = kv.second;
  else
    h->tune = saved;
  if (hipStreamSynchronize(s) != hipSuccess && st == TSK_OK)
    st = fail(h, TSK_ERR_DEVICE, "stream synchronisation failed");
  if (ws != nullptr && hipFree(ws) != hipSuccess && st == TSK_OK)
    st = fail(h, TSK_ERR_DEVICE, "hipFree failed");
  return st;
}

// Host-only check of the tuning cache format (tests; not part of the ABI
// header): parse `json` for `arch` and write the table back as text.
int tsk_tune_json_check(const char* json, const char* arch, char* out, size_t outlen) {
  if (json == nullptr || arch == nullptr || out == nullptr || outlen == 0) return TSK_ERR_INVALID_ARG;
  std::map<uint32_t, TuneEntry> table;
  std::string err;
  const bool ok = tune_parse(json, arch, table, err);
  const std::string text = ok ? tune_dump(table, arch) : err;
  std::strncpy(out, text.c_str(), outlen - 1);
  out[outlen - 1] = 0;
  return ok ? TSK_OK : TSK_ERR_INVALID_ARG;
}

tsk_status tsk_autotune_clear(tsk_handle h) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->tune.clear();
  return TSK_OK;
}

tsk_status tsk_autotune_save(tsk_handle h, const char* path) {
  if (h == nullptr || path == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or path");
  h->err.clear();
  const std::string js = tune_dump(h->tune, h->arch);
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "cannot open %s for writing", path);
  const bool ok = std::fwrite(js.data(), 1, js.size(), f) == js.size();
  if (std::fclose(f) != 0 || !ok) return fail(h, TSK_ERR_INVALID_ARG, "writing %s failed", path);
  return TSK_OK;
}

tsk_status tsk_autotune_load(tsk_handle h, const char* path) {
  if (h == nullptr || path == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or path");
  h->err.clear();
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "cannot open %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  std::map<uint32_t, TuneEntry> table;
  std::string err;
  if (!tune_parse(text, h->arch, table, err)) return fail(h, TSK_ERR_INVALID_ARG, "%s: %s", path, err.c_str());
  h->tune = table;
  return TSK_OK;
}

static tsk_status backward_io(tsk_handle h, const Problem& P, const void* const* Q,
                              const double* const* R, const void* H_bar, const void* const* Q_bar,
                              tsk_dtype out_dtype, void* const* core_bar, void* const* factor_bar,
                              BackwardIO& io) {
  if (Q == nullptr || R == nullptr || H_bar == nullptr || core_bar == nullptr || factor_bar == nullptr)
    return fail(h, TSK_ERR_INVALID_ARG, "NULL Q, R, H_bar, core_bar or factor_bar");
  if (out_dtype != TSK_F64 && out_dtype != TSK_F32) return fail(h, TSK_ERR_INVALID_ARG, "bad out_dtype");
  io.out_f64 = out_dtype == TSK_F64;
  io.Hbar = H_bar;
  for (int n = 0; n < P.d; ++n) {
    if (Q[n] == nullptr || R[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q[%d] or R[%d] is NULL", n, n);
    io.Q.push_back(Q[n]);
    io.R.push_back(R[n]);
    if (Q_bar != nullptr) {
      if (Q_bar[n] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "Q_bar[%d] is NULL", n);
      io.Qbar.push_back(Q_bar[n]);
    }
  }
  for (int i = 0; i < P.s; ++i) {
    if (core_bar[i] == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "core_bar[%d] is NULL", i);
    io.core_bar.push_back(core_bar[i]);
    for (int k = 0; k < P.d; ++k) {
      void* f = factor_bar[(size_t)i * P.d + k];
      if (f == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "factor_bar[%d][%d] is NULL", i, k);
      io.factor_bar.push_back(f);
    }
  }
  return TSK_OK;
}

tsk_status tucker_sum_backward_workspace_size(tsk_handle h, const tsk_tucker_sum* sum,
                                              const tsk_sketch_spec* spec, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL handle or bytes");
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st == TSK_OK) st = validate_backward(h, P);
  if (st != TSK_OK) return st;
  size_t best = 0;
  for (int o = 0; o < 2; ++o)
    for (int qb = 0; qb < 2; ++qb) {
      BackwardIO io;
      io.out_f64 = o == 1;
      io.Q.assign(P.d, nullptr);
      io.R.assign(P.d, nullptr);
      if (qb) io.Qbar.assign(P.d, nullptr);
      io.core_bar.assign(P.s, nullptr);
      io.factor_bar.assign((size_t)P.s * P.d, nullptr);
      Program prog;
      size_t nb = 0;
      if (plan_backward(P, io, nullptr, prog, &nb) != TSK_OK)
        return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
      best = std::max(best, nb);
    }
  *bytes = best;
  return TSK_OK;
}

tsk_status tucker_sum_recompress_backward(tsk_handle h, const tsk_tucker_sum* sum,
                                          const tsk_sketch_spec* spec, const void* const* Q,
                                          const double* const* R, const void* H_bar,
                                          const void* const* Q_bar, tsk_dtype out_dtype,
                                          void* const* core_bar, void* const* factor_bar, void* ws,
                                          size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  h->err.clear();
  Problem P;
  tsk_status st = validate(h, sum, spec, P);
  if (st == TSK_OK) st = validate_backward(h, P);
  if (st != TSK_OK) return st;
  BackwardIO io;
  if ((st = backward_io(h, P, Q, R, H_bar, Q_bar, out_dtype, core_bar, factor_bar, io)) != TSK_OK)
    return st;
  io.singular = (unsigned long long*)(h->d_counter + 2);
  if (ws == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(h, TSK_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Program prog;
  size_t need = 0;
  if (plan_backward(P, io, (char*)ws, prog, &need) != TSK_OK)
    return fail(h, TSK_ERR_UNSUPPORTED, "an operand stride reaches past 2^31 bytes inside one tile");
  if (ws_bytes < need)
    return fail(h, TSK_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if ((st = set_device(h)) != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}

tsk_status tsk_qr_fallback_count(tsk_handle h, void* stream, int64_t* count) {
  if (h == nullptr || count == nullptr) return fail(h, TSK_ERR_INVALID_ARG, "NULL argument");
  tsk_status st = set_device(h);
  if (st != TSK_OK) return st;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "stream synchronisation failed");
  int64_t c[3] = {0, 0, 0};
  if (hipMemcpy(c, h->d_counter, sizeof c, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, TSK_ERR_DEVICE, "counter read failed");
  *count = c[0];
  if (c[2] != 0) {
    // singular R_n met by a backward call: reported once, then cleared
    if (hipMemset(h->d_counter + 2, 0, sizeof(int64_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
      return fail(h, TSK_ERR_DEVICE, "counter reset failed");
    return fail(h, TSK_ERR_RANK_DEFICIENT,
                "%lld mode(s) of a backward call had a numerically singular R_n",
                (long long)c[2]);
  }
  if (c[1] != 0) {
    // breakdowns under qr_policy 2 are reported once, then cleared
    if (hipMemset(h->d_counter + 1, 0, sizeof(int64_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
      return fail(h, TSK_ERR_DEVICE, "counter reset failed");
    return fail(h, TSK_ERR_RANK_DEFICIENT, "%lld Cholesky QR breakdown(s) under qr_policy 2",
                (long long)c[1]);
  }
  return TSK_OK;
}

}  // extern "C"

// Single GEMM through the grouped kernel, for kernel-level tests (not part of
// the ABI header): C (M x N, ldc) = op(A) op(B) with op(A)[m][k] =
// A[m*a_sx + k*a_sk] and op(B)[k][n] = B[n*b_sx + k*b_sk], `splits` K-splits.
extern "C" int tsk_debug_gemm(tsk_handle h, int prec, int M, int N, int K, const void* A,
                              int64_t a_sx, int64_t a_sk, const void* B, int64_t b_sx,
                              int64_t b_sk, void* C, int64_t ldc, int c_f64, int splits, void* ws,
                              size_t ws_bytes, void* stream) {
  if (h == nullptr) return TSK_ERR_INVALID_ARG;
  Program prog;
  Arena ar;
  ar.base = (char*)ws;
  ar.ctr_base = (int32_t*)ar.take(sizeof(int32_t) * 65536);
  GemmBatch gb(prec, R_OTHER, &ar);
  gb.add(C, c_f64 != 0, ldc, 0, M, N, 1, 0, {seg(A, a_sx, a_sk, 0, B, b_sx, b_sk, 0, K)}, splits);
  emit_gemm(prog, gb);
  if (ar.ctr_used > 65536) return TSK_ERR_UNSUPPORTED;
  Step f{};
  f.kind = S_FILL;
  f.ptr = ar.ctr_base;
  f.rows = std::max<int64_t>(ar.ctr_used, 1);
  prog.steps.insert(prog.steps.begin(), f);
  prog.meta_region = align_up(ar.top, 256);
  if (prog.meta_region + prog.blob.size() > ws_bytes) return TSK_ERR_WORKSPACE_TOO_SMALL;
  tsk_status st = set_device(h);
  if (st != TSK_OK) return st;
  return run_program(h, prog, (char*)ws, (hipStream_t)stream);
}
