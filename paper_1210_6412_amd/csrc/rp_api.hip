// rp_api.hip -- C ABI of librp: context and system management, and the host
// drivers of the solvers (iteration loops, FP64 iterative refinement, the
// error certificate and the adjoint).  Every arithmetic step runs in the HIP
// kernels of rp_kernels.hip; this file only sequences them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/rp.h"
#include "rp_internal.h"

using namespace rpk;

namespace {

// ---------------------------------------------------------------------------
// small RAII helpers

// Device blocks released by the buffers of a context, kept for reuse by
// exact size (rounded to 256 bytes): hipFree costs ~170 us and hipMalloc ~30 us
// here (a stream-ordered pool measured the same), and a system built and
// freed per batch holds dozens of buffers.  All use is on the context's one
// stream, so a block handed out again is only touched by work enqueued after
// its previous user's.  Everything is freed with the context.
struct BlockCache {
  std::multimap<size_t, void*> blocks;
  size_t cached = 0;
  static constexpr size_t kCap = size_t(32) << 30;  // beyond this, released blocks are freed
  static size_t round(size_t bytes) { return (bytes + 255) / 256 * 256; }
  void* take(size_t bytes) {
    auto it = blocks.find(bytes);
    if (it == blocks.end()) return nullptr;
    void* p = it->second;
    blocks.erase(it);
    cached -= bytes;
    return p;
  }
  void give(void* p, size_t bytes) {
    if (cached + bytes > kCap) {
      (void)hipFree(p);
      return;
    }
    blocks.emplace(bytes, p);
    cached += bytes;
  }
  ~BlockCache() {
    for (auto& kv : blocks) (void)hipFree(kv.second);
  }
};

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  BlockCache* cache = nullptr;  // where the block goes back (null: hipFree)
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) {
      if (cache) cache->give(p, BlockCache::round(n * sizeof(T)));
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
  }
  hipError_t alloc(size_t count, BlockCache* c) {
    release();
    if (count == 0) count = 1;
    cache = c;
    const size_t bytes = BlockCache::round(count * sizeof(T));
    void* q = c ? c->take(bytes) : nullptr;
    if (!q) {
      hipError_t e = hipMalloc(&q, bytes);
      if (e != hipSuccess) {
        p = nullptr;
        return e;
      }
    }
    p = static_cast<T*>(q);
    n = count;
    return hipSuccess;
  }

};

struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  ~HostPinned() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t reserve(size_t b) {
    if (b <= bytes) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e == hipSuccess) bytes = b;
    return e;
  }
};

struct Fail {  // thrown inside the library only; converted to a status code at the ABI
  int code;
};

}  // namespace

// Per-kernel timing with HIP events (measurement hook, off by default).
struct ProfStat {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

struct rp_context {
  int device = 0;
  int cus = 256;
  hipStream_t stream = nullptr;
  BlockCache blocks;              // device memory of the systems, kept for reuse
  // lanes per row chosen by timing, per (padded rows, entries, instances,
  // value width, transposed)
  std::map<std::array<int64_t, 5>, int> lane_choice;
  int32_t* flag_h = nullptr;      // host-mapped {value, sequence} for status reads
  int32_t* flag_d = nullptr;      // the same memory as the device sees it
  unsigned char* scratch = nullptr;  // device address of this GPU's no-allocation working memory
  int32_t flag_seq = 0;
  hipStream_t cap_stream = nullptr;  // private stream that graphs are captured on (never run)
  std::string err;
  HostPinned pin;
  bool prof = false;
  ProfStat stat[RP_PROF_NKERNELS];
  struct Pend {
    int k;
    hipEvent_t a, b;
    int64_t count;  // iterations covered by the event pair
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pend> pend;
  ~rp_context() {
    for (auto& p : pend) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(stream);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (flag_h) (void)hipHostFree(flag_h);
  }
};

// Working memory of rp_classify_noalloc: a fixed device array (each GPU the
// library runs on holds its own copy until the process ends), so that the
// call allocates nothing.  Layout: bytes [0, 8) the validation key, [8, 12)
// the search's change flag, [16, 16 + 8(K+1)) the instance offsets (needed
// by the validation only, so they may run into the marks), from byte
// kScratchHead the goal-search marks (n uint32) and then the second search's
// marks (n uint32).  Host code never uses the array's name as an address:
// rp_context_create takes the address of this GPU's copy with
// hipGetSymbolAddress once per device (scratch_address).
constexpr int64_t kNoAllocMaxStates = (int64_t)1 << 23;  // RP_NOALLOC_MAX_STATES
constexpr size_t kScratchHead = 256;
static __device__ __align__(256) unsigned char scratch[kScratchHead + 8 * (size_t)kNoAllocMaxStates];

namespace {

// Device address of the current device's copy of `scratch`, looked up once
// per device (the caller has made `device` current); null if the lookup fails.
unsigned char* scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, unsigned char*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  addr[device] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

// Workspace of the inner iteration in precision T.
template <typename T>
struct VecSet {
  DBuf<T> xa, xb, r, q, p, v, s, t, rhs;
  bool ready = false;
  hipError_t ensure(size_t n, BlockCache* cache) {
    if (ready) return hipSuccess;
    DBuf<T>* all[] = {&xa, &xb, &r, &q, &p, &v, &s, &t, &rhs};
    for (DBuf<T>* b : all) {
      hipError_t e = b->alloc(n, cache);
      if (e != hipSuccess) return e;
    }
    ready = true;
    return hipSuccess;
  }
};

// Sliced rows of one (tile set, matrix) pair, built on first use.
template <typename T>
struct SlicedSet {
  bool built = false, ok = false;
  DBuf<int32_t> t_s0, off, width, row, c32;
  DBuf<T> d, val;
  DBuf<uint16_t> c16;
  // column panels
  DBuf<int32_t> npan, hoff, pent, pend;
  DBuf<uint8_t> cnt;
  int32_t npaneled = 0;          // paneled tiles
  std::vector<int32_t> npan_h;   // panels per tile (empty: none paneled)
  Sliced<T> v{};
};

struct Mat {
  DBuf<int32_t> rp, col;
  DBuf<uint16_t> c16;
  DBuf<double> v64;
  DBuf<float> v32;
};

}  // namespace

struct rp_system {
  int32_t K = 0;
  int64_t n = 0, nnz = 0, npad = 0, z = 0, nq_total = 0;
  int L = 1;
  int R = 64;
  std::vector<int64_t> inst_off_h, roff_h, nq_h, z_h;
  std::vector<int32_t> chunk_inst_h, chunk_c0_h;
  // device
  DBuf<int64_t> inst_off, roff, nq;
  DBuf<uint8_t> cls;
  DBuf<int32_t> map, row_state, prp, pcol;
  DBuf<double> d64, b64;
  DBuf<float> d32;
  Mat fwd, tr;
  bool have_tr = false;
  DBuf<int32_t> c_row0, c_nrows, c_inst, c_inst0;
  Chunks ch{};
  // LDS-staged tiles (every instance block fits one workgroup's LDS), one set
  // per value width: FP64 windows use a whole LDS, FP32 windows half of it
  struct TileSet {
    bool ok = false;
    DBuf<int32_t> row0, nrows, inst, inst0, w0, nw, kind, order;
    std::vector<uint8_t> whole_h;  // per instance: window kind WIN_WHOLE (16-bit columns)
    std::vector<int32_t> nrows_h;  // rows per tile
    std::vector<int32_t> kind_h;   // window kind per tile
    std::vector<int32_t> inst_h;   // instance per tile
    std::vector<int32_t> inst0_h;  // tiles of instance k: [inst0_h[k], inst0_h[k+1])
    Tiles tl{};
  } t64, t32;
  // sliced rows of t64 / t32 for the forward [0] and transposed [1] matrix
  SlicedSet<double> sl64[2];
  SlicedSet<float> sl32[2];
  bool sliced = false;  // per call: tiled sweeps use the sliced rows
  int jvariant = 0;     // per call, Jacobi: 1 in-place update, 2 segmented-scan row sums (row chunks)
  DBuf<int32_t> erow[2];  // row of every stored entry, forward [0] / transposed [1] (segmented scan)
  // strongly connected components of S_? (forward graph), per reduced row:
  // component id (a row of it), level; per component id: smallest row, size
  DBuf<int32_t> scc_comp, scc_lvl, scc_minrow, scc_size;
  bool have_scc = false;
  rp_scc_info scc_counts{};
  // one tile per instance for the resident Jacobi kernel (small instances
  // only: both iterates fit the LDS and a sweep moves little data)
  TileSet res64, res32;
  // the last running instances of a tiled Jacobi solve, resident (build_tail);
  // on sliced rows with the slices of each: [tail_slo[c], tail_shi[c])
  TileSet tail;
  DBuf<int32_t> tail_slo, tail_shi;
  bool tail_sliced = false;
  int32_t ntile_max = 0;
  bool tiles_on = true;  // per call: opts.tiling
  DBuf<double> tp, tpa, tps, tpb, tpc, rho2;
  // certificate factors ||(I-A)^{-1} 1|| and ||(I-A)^{-T} 1|| per instance
  DBuf<double> tb_fwd, tb_tr;
  bool have_tb_fwd = false, have_tb_tr = false;
  std::vector<double> tb_fwd_h, tb_tr_h;
  // workspaces
  VecSet<double> w64;
  VecSet<float> w32;
  DBuf<double> x64, r64, b_one, lam64;
  DBuf<double> pa, pb, pc, ps;
  DBuf<int32_t> status_in, status_out, counters;
  DBuf<int64_t> iters_in, outer_it;
  DBuf<double> meas_in, thr_in, rho, alpha, omega, beta, rn, scale, tmp_k, rbest, last_meas;
  DBuf<int32_t> stall;
  DBuf<int64_t> tot_it;
  // stagnation watch of the paper's stopping rule: best measure, and the
  // iteration count when it was last halved
  DBuf<double> sbest;
  DBuf<int64_t> sbest_it;
  bool work_ready = false;
  // a general system A x = b (rp_matrix_system) rather than a chain's
  bool general = false;
  bool dominant = true;  // general: every row strictly diagonally dominant
};

namespace {

// ---------------------------------------------------------------------------
// error plumbing

void set_err(rp_context* ctx, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      set_err(ctx, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,    \
              __LINE__);                                                               \
      throw Fail{e_ == hipErrorOutOfMemory ? RP_ERR_OOM : RP_ERR_HIP};                 \
    }                                                                                  \
  } while (0)

template <typename T>
void dalloc(rp_context* ctx, DBuf<T>& b, size_t n) {
  hipError_t e = b.alloc(n, &ctx->blocks);
  if (e != hipSuccess) {
    set_err(ctx, "device allocation of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
    throw Fail{e == hipErrorOutOfMemory ? RP_ERR_OOM : RP_ERR_HIP};
  }
}

void* pinned(rp_context* ctx, size_t bytes) {
  HIPCHK(ctx, ctx->pin.reserve(bytes));
  return ctx->pin.p;
}

// Fold completed event pairs into the per-kernel totals (after a sync).
void prof_resolve(rp_context* ctx) {
  for (auto& p : ctx->pend) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->stat[p.k].ms += ms;
      ctx->stat[p.k].launches += p.count;
    }
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  ctx->pend.clear();
}

hipEvent_t prof_event(rp_context* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  HIPCHK(ctx, hipEventCreate(&e));
  return e;
}

// Brackets one kernel launch with an event pair when profiling is on.
struct ProfScope {
  rp_context* c;
  int k;
  hipEvent_t a = nullptr;
  ProfScope(rp_context* ctx, int kernel) : c(ctx), k(kernel) {
    if (c->prof) {
      a = prof_event(c);
      HIPCHK(c, hipEventRecord(a, c->stream));
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!c->pool.empty()) {
      b = c->pool.back();
      c->pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      c->pool.push_back(a);
      return;
    }
    if (hipEventRecord(b, c->stream) == hipSuccess) {
      c->pend.push_back({k, a, b, 1});
    } else {
      c->pool.push_back(a);
      c->pool.push_back(b);
    }
  }
};
#define PROF(ctx, kernel, expr)       \
  do {                                \
    ProfScope ps_(ctx, kernel);       \
    HIPCHK(ctx, expr);                \
  } while (0)

// One event pair around a batch of iteration launches (no-op when off).
struct ProfSpan {
  rp_context* c;
  hipEvent_t a = nullptr;
  explicit ProfSpan(rp_context* ctx) : c(ctx) {
    if (c->prof) {
      a = prof_event(c);
      HIPCHK(c, hipEventRecord(a, c->stream));
    }
  }
  void end(int k, int64_t count) {
    if (!a) return;
    if (count == 0) {  // nothing launched: drop the span
      c->pool.push_back(a);
      a = nullptr;
      return;
    }
    hipEvent_t b = prof_event(c);
    HIPCHK(c, hipEventRecord(b, c->stream));
    c->pend.push_back({k, a, b, count});
    a = nullptr;
  }
  // start a new span (after end)
  void restart() {
    if (c->prof && !a) {
      a = prof_event(c);
      HIPCHK(c, hipEventRecord(a, c->stream));
    }
  }
  ~ProfSpan() {
    if (a) c->pool.push_back(a);
  }
};

template <typename T>
void to_host(rp_context* ctx, T* host, const T* dev, size_t count) {
  if (count == 0) return;
  void* p = pinned(ctx, count * sizeof(T));
  HIPCHK(ctx, hipMemcpyAsync(p, dev, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::memcpy(host, p, count * sizeof(T));
  if (ctx->prof) prof_resolve(ctx);
}

template <typename T>
void to_dev(rp_context* ctx, T* dev, const T* host, size_t count) {
  if (count == 0) return;
  void* p = pinned(ctx, count * sizeof(T));
  std::memcpy(p, host, count * sizeof(T));
  HIPCHK(ctx, hipMemcpyAsync(dev, p, count * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
}

// One device int32 read back without a copy command or a stream
// synchronisation: a one-thread kernel stores it, with a sequence number, into
// host-mapped pinned memory, and the host spins on the sequence number.  The
// wait is bounded; past the bound (or without the mapped buffer) the stream is
// synchronised, which also reports a failed launch.
// Asynchronous form: publish_i32 enqueues the store and returns its sequence
// number (0 without the mapped buffer: the value is then read by
// wait_i32 with a copy); wait_i32 returns the value of that publication or of
// a later one on the same stream (later values of the counters read this
// way are never smaller).
int32_t publish_i32(rp_context* ctx, const int32_t* dev) {
  if (!ctx->flag_h) return 0;
  const int32_t seq = ++ctx->flag_seq;
  HIPCHK(ctx, launch_publish(ctx->stream, dev, ctx->flag_d, seq));
  return seq;
}

int32_t wait_i32(rp_context* ctx, const int32_t* dev, int32_t seq) {
  if (!ctx->flag_h) {
    int32_t v = 0;
    to_host(ctx, &v, dev, 1);
    return v;
  }
  volatile int32_t* f = ctx->flag_h;
  const auto t0 = std::chrono::steady_clock::now();
  int spins = 0;
  while ((int32_t)(f[1] - seq) < 0) {
    if (++spins % 4096 == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  const int32_t v = f[0];
  if (ctx->prof) prof_resolve(ctx);
  return v;
}

int32_t read_i32(rp_context* ctx, const int32_t* dev) { return wait_i32(ctx, dev, publish_i32(ctx, dev)); }

const char* reason_text(unsigned r) {
  switch (r) {
    case 1: return "row pointers not monotone or out of range";
    case 2: return "column index out of range";
    case 3: return "columns not strictly ascending (or duplicated) within the row";
    case 4: return "transition probability not finite or outside [0, 1]";
    case 5: return "row does not sum to 1 within rowsum_tol";
    case 6: return "transition leaves the row's own instance";
    case 7: return "matrix entry not finite";
    case 8: return "no nonzero diagonal entry stored";
    default: return "invalid";
  }
}

// Lanes per row for the sparse products: about half the mean row length
// (measured best on gfx950 for short rows: 4 lanes at ~8 entries per row).
int auto_lanes(double mean_row) {
  int L = 1;
  while (L < 64 && 4.0 * L <= mean_row + 1e-9) L *= 2;
  return L;
}

// ---------------------------------------------------------------------------
// workspace

void ensure_work(rp_context* ctx, rp_system* s) {
  if (s->work_ready) return;
  const size_t np = (size_t)s->npad, nc = (size_t)s->ch.nchunk, K = (size_t)s->K;
  dalloc(ctx, s->x64, np);
  dalloc(ctx, s->r64, np);
  dalloc(ctx, s->b_one, np);
  dalloc(ctx, s->lam64, np);
  HIPCHK(ctx, launch_fill_f64(ctx->stream, s->b_one.p, (int64_t)np, 1.0));
  dalloc(ctx, s->pa, nc * 2);
  dalloc(ctx, s->pb, nc * 2);
  dalloc(ctx, s->pc, nc * 2);
  dalloc(ctx, s->ps, nc * 2);
  if (s->ntile_max > 0) {
    const size_t nt = (size_t)s->ntile_max;
    dalloc(ctx, s->tp, 2 * nt);
    dalloc(ctx, s->tpa, nt);
    dalloc(ctx, s->tps, nt);
    dalloc(ctx, s->tpb, 2 * nt);
    dalloc(ctx, s->tpc, 2 * nt);
    dalloc(ctx, s->rho2, 2 * K);
  }
  dalloc(ctx, s->status_in, K);
  dalloc(ctx, s->status_out, K);
  dalloc(ctx, s->counters, 4);
  dalloc(ctx, s->iters_in, K);
  dalloc(ctx, s->outer_it, K);
  dalloc(ctx, s->stall, K);
  dalloc(ctx, s->tot_it, K);
  dalloc(ctx, s->sbest, K);
  dalloc(ctx, s->sbest_it, K);
  DBuf<double>* ks[] = {&s->meas_in, &s->thr_in, &s->rho, &s->alpha, &s->omega, &s->beta, &s->rn, &s->scale,
                        &s->tmp_k, &s->rbest, &s->last_meas};
  for (auto* b : ks) dalloc(ctx, *b, K);
  s->work_ready = true;
}

template <typename T>
VecSet<T>& vecs(rp_system* s);
template <>
VecSet<double>& vecs<double>(rp_system* s) { return s->w64; }
template <>
VecSet<float>& vecs<float>(rp_system* s) { return s->w32; }

template <typename T>
MatView<T> view(rp_system* s, bool transposed);
template <>
MatView<double> view<double>(rp_system* s, bool tr) {
  Mat& m = tr ? s->tr : s->fwd;
  return MatView<double>{m.rp.p, m.col.p, m.v64.p, s->d64.p, m.c16.p};
}
template <>
MatView<float> view<float>(rp_system* s, bool tr) {
  Mat& m = tr ? s->tr : s->fwd;
  return MatView<float>{m.rp.p, m.col.p, m.v32.p, s->d32.p, m.c16.p};
}

void ensure_transpose(rp_context* ctx, rp_system* s) {
  if (s->have_tr) return;
  const int64_t np = s->npad;
  const size_t z1 = (size_t)std::max<int64_t>(s->z, 1);
  DBuf<int32_t> erow, idx, key, perm;
  DBuf<uint8_t> temp;
  dalloc(ctx, erow, z1);
  dalloc(ctx, idx, z1);
  dalloc(ctx, key, z1);
  dalloc(ctx, perm, z1);
  size_t tb = 0;
  HIPCHK(ctx, transpose_temp_bytes(np, s->z, &tb));
  dalloc(ctx, temp, tb);
  dalloc(ctx, s->tr.rp, (size_t)np + 1);
  dalloc(ctx, s->tr.col, (size_t)s->z);
  dalloc(ctx, s->tr.v64, (size_t)s->z);
  dalloc(ctx, s->tr.v32, (size_t)s->z);
  HIPCHK(ctx, launch_transpose(ctx->stream, np, s->z, s->fwd.rp.p, s->fwd.col.p, s->fwd.v64.p, s->tr.rp.p,
                               s->tr.col.p, s->tr.v64.p, s->tr.v32.p, erow.p, idx.p, key.p, perm.p, temp.p, tb));
  dalloc(ctx, s->tr.c16, (size_t)s->z);
  HIPCHK(ctx, launch_col16(ctx->stream, s->ch, s->roff.p, s->tr.rp.p, s->tr.col.p, s->tr.c16.p));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  s->have_tr = true;
}


// Tiles of the LDS-staged kernels for values of `width` bytes.  Each instance
// is cut into row ranges, about `per_cu` tiles per compute unit over the whole
// system, and each tile gets an x window in LDS:
//  - the instance's whole padded row block when it fits, with few enough
//    tiles per instance that copying the window into LDS stays below half of
//    the sweep's own traffic;
//  - otherwise a band [row0 - B, row0 + nr + B) around the tile's rows, B
//    chosen from `hist` (per instance: 32 bins of log2(|col - row| + 1));
//  - otherwise (no band covers half of the entries) no window, nw = 0.
// Reads outside a tile's window go to global memory in every case.
constexpr double kGatherBytes = 32.0;  // cost of one x read from L2/HBM instead of LDS
// Most rows of a tile whose columns are staged panel by panel (see Sliced),
// for values of type T.
template <typename T>
constexpr int64_t panel_rows() { return (int64_t)PanelShape<T>::MAXS * 1024; }
// Column panels are used while the copies of the instance's iterate into LDS
// (one per tile and sweep, served by L2 to the tiles of one instance) stay
// below this multiple of the sweep's own bytes.
constexpr double kPanelCopyShare = 1.5;
// Most rows of a tile of an instance without a window.  Measured on the
// 256-chain batch (uniform targets), 200 fixed sweeps, FP64 with two lanes
// per row: 331 us with the panel-driven tile counts (up to 16,384 rows),
// 294 (8,192), 276 (4,096), 284 (2,048), 319 (1,024); FP32 one lane per row
// 243 -> 201 at 4,096.
constexpr int64_t kNoWindowTileRows = 4096;

// Tiles of instance k (no window) for column panels of values `width` bytes
// wide, given its share of the GPU; 0 when panels are not viable (a tile's
// rows would not fit the registers within the copy budget).
int64_t panel_tiles(const rp_system* s, int k, size_t width, int64_t share) {
  const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
  if (rows <= 0) return 0;
  const double w = (double)width;
  const double sweep = (4.0 + w) * (double)s->z_h[k] + (4.0 + 4.0 * w) * (double)s->nq_h[k];
  const int64_t cap = (int64_t)std::floor(kPanelCopyShare * sweep / (w * (double)rows));
  const int64_t prow = width == 4 ? panel_rows<float>() : panel_rows<double>();
  const int64_t need = (rows + prow - 1) / prow;
  if (need > cap) return 0;
  return std::max(need, std::min(share, cap));
}

// Block-to-tile order of a launch of one block per tile.  Block b runs on
// XCD b mod 8 (workgroups are handed to the XCDs in turn), so each XCD gets a
// fixed number of blocks.  Instances, largest first, go whole to the XCD with
// the least work among those with room for all their tiles (split over the
// least loaded XCDs when none has), so the tiles of one instance share an L2;
// each XCD then takes its tiles largest first (an instance's tiles are equal
// and stay together), which keeps a large tile from starting last.
std::vector<int32_t> balanced_order(const std::vector<int32_t>& tc0, const std::vector<double>& cost) {
  constexpr int X = 8;
  const int K = (int)tc0.size() - 1;
  const int nt = (int)cost.size();
  std::array<int, X> room{};
  std::array<double, X> load{};
  std::array<std::vector<int32_t>, X> list;
  for (int x = 0; x < X; x++) room[x] = (nt - x + X - 1) / X;
  std::vector<double> icost(K, 0.0);
  std::vector<int> idx;
  for (int k = 0; k < K; k++) {
    for (int t = tc0[k]; t < tc0[k + 1]; t++) icost[k] += cost[t];
    if (tc0[k + 1] > tc0[k]) idx.push_back(k);
  }
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return icost[a] > icost[b]; });
  for (int k : idx) {
    int t = tc0[k];
    while (t < tc0[k + 1]) {
      const int m = tc0[k + 1] - t;
      int best = -1;
      for (int x = 0; x < X; x++)
        if (room[x] >= m && (best < 0 || load[x] < load[best])) best = x;
      if (best < 0)  // no XCD has room for all: fill the least loaded one with room
        for (int x = 0; x < X; x++)
          if (room[x] > 0 && (best < 0 || load[x] < load[best])) best = x;
      const int take = std::min(m, room[best]);
      for (int i = 0; i < take; i++, t++) {
        list[best].push_back(t);
        load[best] += cost[t];
      }
      room[best] -= take;
    }
  }
  std::vector<int32_t> order((size_t)nt, 0);
  for (int x = 0; x < X; x++) {
    std::stable_sort(list[x].begin(), list[x].end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    for (size_t i = 0; i < list[x].size(); i++) order[(size_t)x + X * i] = list[x][i];
  }
  return order;
}

void build_tiles(rp_context* ctx, rp_system* s, rp_system::TileSet& ts, size_t width, int per_cu,
                 const std::vector<int32_t>& hist) {
  const int K = s->K;
  const int64_t np = s->npad;
  const int64_t wmax = (int64_t)(TILE_LDS_BYTES / width) / PAD * PAD;
  ts.ok = np > 0;
  if (!ts.ok) return;
  std::vector<int32_t> trow0, tnr, tinst, tw0, tnw, tkind, tc0(K + 1, 0);
  std::vector<double> tcost;
  ts.whole_h.assign(K, 0);
  const double target = (double)ctx->cus * per_cu;
  const double w = (double)width;
  int64_t maxw = 0;
  auto ceil_pad = [](int64_t v) { return (v + PAD - 1) / PAD * PAD; };
  // first pass: tiles per instance and window kind
  std::vector<int64_t> ntiles(K, 0), bands(K, -1), shares(K, 0);
  int64_t total = 0;
  for (int k = 0; k < K; k++) {
    const int64_t lo = s->roff_h[k], hi = s->roff_h[k + 1];
    const int64_t rows = hi - lo;
    if (rows == 0) continue;
    const double share = std::max(1.0, std::round(target * (double)rows / (double)np));
    int64_t ntk, band = -1;  // band -1: whole block; -2: no window; >= 0: band half-width
    if (rows <= wmax) {
      const double sweep_bytes = (4.0 + w) * (double)s->z_h[k] + (4.0 + 4.0 * w) * (double)s->nq_h[k];
      const double cap = std::max(1.0, std::floor(0.5 * sweep_bytes / (w * (double)rows)));
      ntk = (int64_t)std::min(share, cap);
    } else {
      // Band half-width B from the instance's distance histogram: bin i holds
      // |col - row| in [2^i - 1, 2^(i+1) - 2].  Pick the B that minimises the
      // extra bytes copied into LDS (2B rows per tile) plus kGatherBytes per
      // entry left outside the band; no window when no band covers half of
      // the entries.
      band = -2;
      auto tiles_at = [&](int64_t B) {
        const int64_t cap = wmax - 2 * B - 2 * PAD;  // rows of one tile
        return std::max<int64_t>((int64_t)share, (rows + cap - 1) / cap);
      };
      if (!hist.empty()) {
        const int32_t* h = hist.data() + (size_t)k * 32;
        int64_t tot = 0, cov = 0;
        for (int i = 0; i < 32; i++) tot += h[i];
        double best = 0.0;
        for (int i = 0; i < 31 && tot > 0; i++) {
          const int64_t B = ((int64_t)2 << i) - 2;
          if (4 * (B + PAD) > wmax) break;  // keep at least half of the window for the tile's rows
          cov += h[i];
          if (2 * cov < tot) continue;
          const double cost = w * 2.0 * (double)B * (double)tiles_at(B) + kGatherBytes * (double)(tot - cov);
          if (band == -2 || cost < best) {
            band = B;
            best = cost;
          }
        }
      }
      if (band >= 0) {
        ntk = tiles_at(band);
      } else {
        // No window: the sliced rows can stage the columns panel by panel,
        // each tile copying the instance's whole iterate once per sweep.
        // When that is viable (panel_tiles) such an instance takes one tile
        // per compute unit's share (also in FP32), at least as many as keep
        // a tile's rows in a wavefront's registers and at most as many as
        // keep the copies within kPanelCopyShare of the sweep's bytes.
        const double share1 = std::max(1.0, std::round((double)ctx->cus * (double)rows / (double)np));
        // (FP64 only: FP32 tiles keep the CU share, which measured faster --
        // 256-chain batch without sinks 50 -> 31 us per FP32 sweep, with sinks
        // unchanged -- and then rarely fit the panel budget)
        const int64_t pt = width == sizeof(double) ? panel_tiles(s, k, width, (int64_t)share1) : 0;
        ntk = pt > 0 ? pt : (int64_t)share;
        // Tiles of at most kNoWindowTileRows rows: the gathers of such an
        // instance come from L2 (or panels staged from it), and with the
        // balanced order an instance's tiles run side by side on one XCD, so
        // more, shorter tiles put fewer instances' iterates in one L2 at a
        // time (and even out the blocks).  Panels remain where their copies
        // still fit the budget (instances up to ~70,000 rows).
        ntk = std::max<int64_t>(ntk, (rows + kNoWindowTileRows - 1) / kNoWindowTileRows);
      }
    }
    ntk = std::max<int64_t>(1, std::min<int64_t>(ntk, rows / PAD));
    ntiles[k] = ntk;
    bands[k] = band;
    shares[k] = (int64_t)share;
    total += ntk;
  }
  // The window-copy cap only matters while the tiles fill the GPU; with fewer
  // tiles than that (one chain, or a few), whole-window instances take their
  // full share of blocks: a sweep is then latency-bound and more blocks each
  // with fewer rows finish sooner (the copies come from L2).
  if (total < (int64_t)target)
    for (int k = 0; k < K; k++) {
      const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
      if (rows > 0 && bands[k] == -1) ntiles[k] = std::max(ntiles[k], std::min(shares[k], rows / PAD));
    }
  // second pass: emit the tiles
  for (int k = 0; k < K; k++) {
    tc0[k] = (int32_t)trow0.size();
    const int64_t lo = s->roff_h[k], hi = s->roff_h[k + 1];
    const int64_t rows = hi - lo;
    if (rows == 0) continue;
    const int64_t ntk = ntiles[k], band = bands[k];
    const int64_t per = ceil_pad((rows + ntk - 1) / ntk);
    for (int64_t r = lo; r < hi; r += per) {
      const int64_t nr = std::min<int64_t>(per, hi - r);
      int64_t w0 = lo, nw = rows;
      int32_t kind = WIN_WHOLE;
      if (band == -2) {
        nw = 0;
        kind = WIN_NONE;
      } else if (band >= 0) {
        w0 = std::max(lo, (r - band) / PAD * PAD);
        nw = std::min(hi, ceil_pad(r + nr + band)) - w0;
        kind = (w0 == lo && nw == rows) ? WIN_WHOLE : WIN_BAND;
      }
      trow0.push_back((int32_t)r);
      tnr.push_back((int32_t)nr);
      tinst.push_back(k);
      tw0.push_back((int32_t)w0);
      tnw.push_back((int32_t)nw);
      tkind.push_back(kind);
      ts.whole_h[k] = kind == WIN_WHOLE;
      maxw = std::max(maxw, nw);
      // bytes the tile moves per sweep: its share of the instance's entries
      // and rows, plus what it copies into LDS (its window, or the whole
      // block panel by panel)
      const double zt = (double)s->z_h[k] * (double)nr / (double)rows;
      const double copy = kind == WIN_NONE ? (double)rows * w : (double)nw * w;
      tcost.push_back(zt * (w + 2.0) + (double)nr * (4.0 * w + 8.0) + copy);
    }
  }
  if (maxw > wmax) {
    set_err(ctx, "internal error: tile window of %lld rows exceeds LDS", (long long)maxw);
    throw Fail{RP_ERR_HIP};
  }
  tc0[K] = (int32_t)trow0.size();
  const int32_t nt = (int32_t)trow0.size();
  dalloc(ctx, ts.row0, (size_t)nt);
  dalloc(ctx, ts.nrows, (size_t)nt);
  dalloc(ctx, ts.inst, (size_t)nt);
  dalloc(ctx, ts.inst0, (size_t)K + 1);
  dalloc(ctx, ts.w0, (size_t)nt);
  dalloc(ctx, ts.nw, (size_t)nt);
  dalloc(ctx, ts.kind, (size_t)nt);
  to_dev(ctx, ts.row0.p, trow0.data(), (size_t)nt);
  to_dev(ctx, ts.nrows.p, tnr.data(), (size_t)nt);
  to_dev(ctx, ts.inst.p, tinst.data(), (size_t)nt);
  to_dev(ctx, ts.inst0.p, tc0.data(), (size_t)K + 1);
  to_dev(ctx, ts.w0.p, tw0.data(), (size_t)nt);
  to_dev(ctx, ts.nw.p, tnw.data(), (size_t)nt);
  to_dev(ctx, ts.kind.p, tkind.data(), (size_t)nt);
  ts.nrows_h = tnr;
  ts.kind_h = tkind;
  ts.inst_h = tinst;
  ts.inst0_h = tc0;
  ts.tl = Tiles{ts.row0.p, ts.nrows.p, ts.inst.p, ts.inst0.p, ts.w0.p, ts.nw.p, ts.kind.p, nt, K, (int32_t)maxw};
  const std::vector<int32_t> order = balanced_order(tc0, tcost);
  dalloc(ctx, ts.order, (size_t)nt);
  to_dev(ctx, ts.order.p, order.data(), (size_t)nt);
  ts.tl.order = ts.order.p;
}

// Resident Jacobi (one block per instance, many sweeps per launch) pays off
// where a sweep is too small to spread over several CUs: every non-empty
// instance's two iterates fit the LDS and its sweep moves at most
// kResidentBytes.
constexpr double kResidentBytes = 512.0 * 1024.0;

void build_resident(rp_context* ctx, rp_system* s, rp_system::TileSet& ts, size_t width) {
  const int K = s->K;
  ts.ok = false;
  if (s->npad <= 0) return;
  const double w = (double)width;
  int64_t maxw = 0;
  for (int k = 0; k < K; k++) {
    const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
    const double sweep_bytes = (2.0 + w) * (double)s->z_h[k] + (4.0 + 4.0 * w) * (double)s->nq_h[k];
    if (rows > 65536 || 2.0 * w * (double)rows > (double)TILE_LDS_BYTES || sweep_bytes > kResidentBytes) return;
    maxw = std::max(maxw, rows);
  }
  std::vector<int32_t> trow0, tnr, tinst, tw0, tnw, tkind, tc0(K + 1, 0);
  ts.whole_h.assign(K, 1);
  for (int k = 0; k < K; k++) {
    tc0[k] = (int32_t)trow0.size();
    const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
    if (rows == 0) continue;
    trow0.push_back((int32_t)s->roff_h[k]);
    tnr.push_back((int32_t)rows);
    tinst.push_back(k);
    tw0.push_back((int32_t)s->roff_h[k]);
    tnw.push_back((int32_t)rows);
    tkind.push_back(WIN_WHOLE);
  }
  tc0[K] = (int32_t)trow0.size();
  const int32_t nt = (int32_t)trow0.size();
  dalloc(ctx, ts.row0, (size_t)nt);
  dalloc(ctx, ts.nrows, (size_t)nt);
  dalloc(ctx, ts.inst, (size_t)nt);
  dalloc(ctx, ts.inst0, (size_t)K + 1);
  dalloc(ctx, ts.w0, (size_t)nt);
  dalloc(ctx, ts.nw, (size_t)nt);
  dalloc(ctx, ts.kind, (size_t)nt);
  to_dev(ctx, ts.row0.p, trow0.data(), (size_t)nt);
  to_dev(ctx, ts.nrows.p, tnr.data(), (size_t)nt);
  to_dev(ctx, ts.inst.p, tinst.data(), (size_t)nt);
  to_dev(ctx, ts.inst0.p, tc0.data(), (size_t)K + 1);
  to_dev(ctx, ts.w0.p, tw0.data(), (size_t)nt);
  to_dev(ctx, ts.nw.p, tnw.data(), (size_t)nt);
  to_dev(ctx, ts.kind.p, tkind.data(), (size_t)nt);
  ts.tl = Tiles{ts.row0.p, ts.nrows.p, ts.inst.p, ts.inst0.p, ts.w0.p, ts.nw.p, ts.kind.p, nt, K, (int32_t)maxw};
  ts.ok = true;
}

// The tail of a tiled Jacobi solve: instances converge at different sweep
// counts, and the last few of a batch (often small chains that mix slowly)
// can need as many sweeps again as the rest, each a launch over every tile
// for one or two instances' rows.  Once at most kTailInstances still run and
// each fits the resident kernel (the limits of build_resident), s->tail gets
// one tile per running instance and the remaining sweeps run resident, many
// per launch.  False (s->tail untouched) when none runs or one does not fit.
// With the slice starts of the tiled sweeps' sliced rows (t_s0_h, per tile of
// `main`), and every tile of the running instances a whole-block window, the
// tail keeps the sliced rows (s->tail_sliced, slices in s->tail_slo/shi).
constexpr int kTailInstances = 16;

bool build_tail(rp_context* ctx, rp_system* s, size_t width, const std::vector<int32_t>& status_h,
                const rp_system::TileSet& main, const std::vector<int32_t>* t_s0_h) {
  const int K = s->K;
  const double w = (double)width;
  std::vector<int32_t> trow0, tnr, tinst, tkind, tc0(K + 1, 0);
  int64_t maxw = 0;
  for (int k = 0; k < K; k++) {
    tc0[k] = (int32_t)trow0.size();
    const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
    if (status_h[k] != ST_RUN || rows == 0) continue;
    const double sweep_bytes = (2.0 + w) * (double)s->z_h[k] + (4.0 + 4.0 * w) * (double)s->nq_h[k];
    if (rows > 65536 || 2.0 * w * (double)rows > (double)TILE_LDS_BYTES || sweep_bytes > kResidentBytes) return false;
    maxw = std::max(maxw, rows);
    trow0.push_back((int32_t)s->roff_h[k]);
    tnr.push_back((int32_t)rows);
    tinst.push_back(k);
    tkind.push_back(WIN_WHOLE);
  }
  tc0[K] = (int32_t)trow0.size();
  const int32_t nt = tc0[K];
  if (nt == 0) return false;
  std::vector<int32_t> slo, shi;
  bool sliced = t_s0_h != nullptr;
  for (int32_t c = 0; c < nt && sliced; c++) {
    const int k = tinst[c];
    for (int32_t t = main.inst0_h[k]; t < main.inst0_h[k + 1]; t++) sliced = sliced && main.kind_h[t] == WIN_WHOLE;
    slo.push_back((*t_s0_h)[main.inst0_h[k]]);
    shi.push_back((*t_s0_h)[main.inst0_h[k + 1]]);
  }
  if (sliced) {
    dalloc(ctx, s->tail_slo, (size_t)nt);
    dalloc(ctx, s->tail_shi, (size_t)nt);
    to_dev(ctx, s->tail_slo.p, slo.data(), (size_t)nt);
    to_dev(ctx, s->tail_shi.p, shi.data(), (size_t)nt);
  }
  s->tail_sliced = sliced;
  rp_system::TileSet& ts = s->tail;
  dalloc(ctx, ts.row0, (size_t)nt);
  dalloc(ctx, ts.nrows, (size_t)nt);
  dalloc(ctx, ts.inst, (size_t)nt);
  dalloc(ctx, ts.inst0, (size_t)K + 1);
  dalloc(ctx, ts.kind, (size_t)nt);
  to_dev(ctx, ts.row0.p, trow0.data(), (size_t)nt);
  to_dev(ctx, ts.nrows.p, tnr.data(), (size_t)nt);
  to_dev(ctx, ts.inst.p, tinst.data(), (size_t)nt);
  to_dev(ctx, ts.inst0.p, tc0.data(), (size_t)K + 1);
  to_dev(ctx, ts.kind.p, tkind.data(), (size_t)nt);
  // the window of a resident tile is its instance block: w0 = row0, nw = nrows
  ts.tl = Tiles{ts.row0.p, ts.nrows.p, ts.inst.p, ts.inst0.p, ts.row0.p, ts.nrows.p, ts.kind.p, nt, K, (int32_t)maxw};
  ts.ok = true;
  return true;
}

// Chunk view of a tile set (same per-instance partial layout), for the
// per-instance finishing kernels.
Chunks tile_chunks(const Tiles& tl) { return Chunks{tl.row0, tl.nrows, tl.inst, tl.inst_t0, tl.ntile, tl.K}; }

template <typename T>
rp_system::TileSet& tiles_for(rp_system* s) {
  return sizeof(T) == 4 ? s->t32 : s->t64;
}

// Whether this call runs the LDS-staged tile kernels for values of type T.
template <typename T>
bool tiled(rp_system* s) {
  return s->tiles_on && tiles_for<T>(s).ok;
}

template <typename T>
rp_system::TileSet& resident_for(rp_system* s) {
  return sizeof(T) == 4 ? s->res32 : s->res64;
}

template <typename T>
SlicedSet<T>& sliced_for(rp_system* s, bool tr);
template <>
SlicedSet<double>& sliced_for<double>(rp_system* s, bool tr) { return s->sl64[tr ? 1 : 0]; }
template <>
SlicedSet<float>& sliced_for<float>(rp_system* s, bool tr) { return s->sl32[tr ? 1 : 0]; }

// Slice bytes above which a sweep streams them past the caches (the MI355X
// last-level cache holds 256 MB; the vectors need room beside the matrix).
constexpr double kStreamBytes = 192.0 * 1024.0 * 1024.0;

// Rows per sort window of the sliced layout (see k_slice_order).  Wider
// windows pad less, narrower ones keep the x' lines more local.  Measured:
// rows of 1-4 entries (program graphs of 2 M and 2^25 states) sweep 4-5%
// faster with 512-row windows than with 2,048; rows of 0-15 entries (the
// 64-chain batch, 7.3 per row) sweep 2% slower with 1,024 than with 2,048.
int32_t sort_window(const rp_system* s) {
  const double mean = s->npad > 0 ? (double)s->z / (double)s->npad : 0.0;
  return mean < 5.0 ? 512 : 2048;
}

// Sliced rows of the tile set for T and the forward or transposed matrix,
// built once: a block per tile orders its rows and measures its slices, the
// host lays the slices out (64-bit offsets, checked against int32), and a
// wavefront per slice copies the entries.  Returns false (the lane-group
// tiles are used) when the tile set is absent or the slices would not fit
// 32-bit offsets.
template <typename T>
bool ensure_sliced(rp_context* ctx, rp_system* s, bool tr) {
  SlicedSet<T>& ss = sliced_for<T>(s, tr);
  if (ss.built) return ss.ok;
  rp_system::TileSet& ts = tiles_for<T>(s);
  if (!ts.ok) {
    ss.built = true;
    return false;
  }
  if (tr) ensure_transpose(ctx, s);
  hipStream_t st = ctx->stream;
  const Tiles& tl = ts.tl;
  const int32_t nt = tl.ntile;
  std::vector<int32_t> t_s0(nt + 1, 0), stile;
  for (int32_t t = 0; t < nt; t++) {
    const int32_t ns = (ts.nrows_h[t] + SLICE - 1) / SLICE;
    t_s0[t + 1] = t_s0[t] + ns;
    stile.insert(stile.end(), ns, t);
  }
  const int32_t nslice = t_s0[nt];
  dalloc(ctx, ss.t_s0, (size_t)nt + 1);
  dalloc(ctx, ss.row, (size_t)nslice * SLICE);
  dalloc(ctx, ss.width, (size_t)nslice);
  to_dev(ctx, ss.t_s0.p, t_s0.data(), (size_t)nt + 1);
  MatView<T> m = view<T>(s, tr);
  HIPCHK(ctx, launch_slice_order(st, m.rp, tl, ss.t_s0.p, sort_window(s), ss.row.p, ss.width.p));
  std::vector<int32_t> width(nslice);
  to_host(ctx, width.data(), ss.width.p, (size_t)nslice);
  // Column panels for the tiles of instances without a window (no band, too
  // large for the LDS), when the copies of the instance's iterate (once per
  // tile and sweep) stay below kPanelCopyShare of the sweep's bytes, the
  // tile's rows fit the wavefronts' registers and no row has more than 255
  // entries (count bytes).  Their slices get no regular slots (width 0).
  const int64_t pw = (int64_t)(TILE_LDS_BYTES / sizeof(T)) / PAD * PAD;
  const double w = (double)sizeof(T);
  std::vector<int32_t> npan(nt, 0), pend(nt, 0), hoff(nt, 0);
  std::vector<int32_t> pslice, ptile;
  int64_t ncnt = 0;
  int32_t npaneled = 0;
  for (int32_t t = 0; t < nt; t++) {
    if (ts.kind_h[t] != WIN_NONE || ts.nrows_h[t] > panel_rows<T>()) continue;
    const int k = ts.inst_h[t];
    const int64_t rows = s->roff_h[k + 1] - s->roff_h[k];
    const double copy = (double)(ts.inst0_h[k + 1] - ts.inst0_h[k]) * (double)rows * w;
    const double sweep = (4.0 + w) * (double)s->z_h[k] + (4.0 + 4.0 * w) * (double)s->nq_h[k];
    if (copy > kPanelCopyShare * sweep * (1.0 + 1e-9)) continue;
    int32_t longest = 0;
    for (int32_t q = t_s0[t]; q < t_s0[t + 1]; q++) longest = std::max(longest, width[q]);
    if (longest > 255) continue;
    npan[t] = (int32_t)((rows + pw - 1) / pw);
    pend[t] = (int32_t)s->roff_h[k + 1];
    hoff[t] = (int32_t)std::min<int64_t>(ncnt, INT32_MAX);
    ncnt += (int64_t)(t_s0[t + 1] - t_s0[t]) * npan[t] * SLICE;
    for (int32_t q = t_s0[t]; q < t_s0[t + 1]; q++) {
      width[q] = 0;
      pslice.push_back(q);
      ptile.push_back(t);
    }
    npaneled++;
  }
  std::vector<int32_t> off(nslice);
  int64_t total = 0;
  for (int32_t i = 0; i < nslice; i++) {
    off[i] = (int32_t)std::min<int64_t>(total, INT32_MAX);
    total += (int64_t)width[i] * SLICE;
  }
  ss.built = true;
  if (total > INT32_MAX || ncnt >= INT32_MAX) return false;
  bool any_whole = false, any_other = false;
  for (int32_t t = 0; t < nt; t++)
    if (npan[t] == 0) (ts.kind_h[t] == WIN_WHOLE ? any_whole : any_other) = true;
  // paneled slices: count bytes and entries per slice, then the entries laid
  // out after the regular slots
  const int32_t nps = (int32_t)pslice.size();
  DBuf<int32_t> ps_d, pt_d;
  int64_t pent = 0;
  if (npaneled > 0) {
    dalloc(ctx, ss.npan, (size_t)nt);
    dalloc(ctx, ss.hoff, (size_t)nt);
    dalloc(ctx, ss.pend, (size_t)nt);
    dalloc(ctx, ss.cnt, (size_t)ncnt);
    to_dev(ctx, ss.npan.p, npan.data(), (size_t)nt);
    to_dev(ctx, ss.hoff.p, hoff.data(), (size_t)nt);
    to_dev(ctx, ss.pend.p, pend.data(), (size_t)nt);
    DBuf<int32_t> ent_d;
    dalloc(ctx, ps_d, (size_t)nps);
    dalloc(ctx, pt_d, (size_t)nps);
    dalloc(ctx, ent_d, (size_t)nps);
    to_dev(ctx, ps_d.p, pslice.data(), (size_t)nps);
    to_dev(ctx, pt_d.p, ptile.data(), (size_t)nps);
    Sliced<T> pv{};
    pv.t_s0 = ss.t_s0.p;
    pv.row = ss.row.p;
    pv.npan = ss.npan.p;
    pv.hoff = ss.hoff.p;
    pv.pend = ss.pend.p;
    pv.pw = (int32_t)pw;
    HIPCHK(ctx, launch_panel_count<T>(st, m, tl, pv, ps_d.p, pt_d.p, nps, ss.cnt.p, ent_d.p));
    std::vector<int32_t> ent((size_t)nps);
    to_host(ctx, ent.data(), ent_d.p, (size_t)nps);
    std::vector<int32_t> pstart((size_t)nslice, 0);
    for (int32_t i = 0; i < nps; i++) {
      pstart[pslice[i]] = (int32_t)std::min<int64_t>(total + pent, INT32_MAX);
      pent += ent[i];
    }
    if (total + pent > INT32_MAX) return false;
    dalloc(ctx, ss.pent, (size_t)nslice);
    to_dev(ctx, ss.pent.p, pstart.data(), (size_t)nslice);
    to_dev(ctx, ss.width.p, width.data(), (size_t)nslice);  // paneled slices: no regular slots
  }
  const int64_t nent = total + pent + (npaneled > 0 ? PANEL_SLACK : 0);
  DBuf<int32_t> stile_d;
  dalloc(ctx, stile_d, (size_t)nslice);
  dalloc(ctx, ss.off, (size_t)nslice);
  dalloc(ctx, ss.d, (size_t)nslice * SLICE);
  dalloc(ctx, ss.val, (size_t)std::max<int64_t>(nent, 1));
  if (any_whole || npaneled > 0) dalloc(ctx, ss.c16, (size_t)std::max<int64_t>(nent, 1));
  if (any_other) dalloc(ctx, ss.c32, (size_t)std::max<int64_t>(total, 1));
  to_dev(ctx, stile_d.p, stile.data(), (size_t)nslice);
  to_dev(ctx, ss.off.p, off.data(), (size_t)nslice);
  HIPCHK(ctx, launch_slice_fill<T>(st, m, tl, stile_d.p, nslice, ss.off.p, ss.width.p, ss.row.p, ss.d.p, ss.val.p,
                                   ss.c16.p, ss.c32.p));
  // Slices larger than the last-level cache are read with nontemporal loads:
  // they cannot stay cached from one sweep to the next anyway, and streaming
  // them keeps the vectors' lines (x', the right-hand side) cached.
  const double slice_bytes = (double)total * (double)(sizeof(T) + (any_other ? 4 : 2)) +
                             (double)pent * (double)(sizeof(T) + 2) + (double)ncnt;
  const int32_t stream = slice_bytes > kStreamBytes ? 1 : 0;
  ss.v = Sliced<T>{ss.t_s0.p, ss.off.p, ss.width.p, ss.row.p, ss.d.p, ss.val.p, ss.c16.p, ss.c32.p, stream};
  if (npaneled > 0) {
    HIPCHK(ctx, hipMemsetAsync(ss.val.p + (total + pent), 0, sizeof(T) * PANEL_SLACK, st));
    HIPCHK(ctx, hipMemsetAsync(ss.c16.p + (total + pent), 0, sizeof(uint16_t) * PANEL_SLACK, st));
    ss.v.npan = ss.npan.p;
    ss.v.hoff = ss.hoff.p;
    ss.v.cnt = ss.cnt.p;
    ss.v.pent = ss.pent.p;
    ss.v.pend = ss.pend.p;
    ss.v.pw = (int32_t)pw;
    ss.v.paneled = 1;
    HIPCHK(ctx, launch_panel_fill<T>(st, m, tl, ss.v, ps_d.p, pt_d.p, nps, ss.val.p, ss.c16.p));
  }
  HIPCHK(ctx, hipStreamSynchronize(st));
  ss.npaneled = npaneled;
  if (npaneled > 0) ss.npan_h = npan;
  ss.ok = true;
  return true;
}

// Iterations of the next batch queued before the host waits for the done
// count of the previous one.
constexpr int64_t kLookahead = 4;

// Most tiled BiCGStab steps between two checks.  With the look-ahead a check
// no longer idles the GPU, while every step launched after the last instance
// stopped still costs five short launches (measured: ~0.3 ms per solve of
// such steps with batches of up to 32 on the bench workload).
constexpr int kBicgBatch = 8;

// Sweeps per launch of the resident Jacobi kernel (it stops early once its
// instance has decided).
constexpr int kResidentSweeps = 256;

// Algorithmic bytes of batched launches, from each instance's final count:
// batch [j0, j0+n) did min(n, max(0, m_k - j0)) iterations of instance k.
// Several device -> host reads with one stream synchronisation: add() the
// reads, then run() copies them all into the pinned staging buffer and waits
// once (each read alone costs a copy command and a synchronisation).
struct HostReads {
  struct Item {
    void* host;
    const void* dev;
    size_t off, bytes;
  };
  rp_context* ctx;
  std::vector<Item> items;
  size_t total = 0;
  explicit HostReads(rp_context* c) : ctx(c) {}
  template <typename T>
  HostReads& add(T* host, const T* dev, size_t count) {
    if (count == 0) return *this;
    items.push_back({host, dev, total, count * sizeof(T)});
    total += (count * sizeof(T) + 15) / 16 * 16;
    return *this;
  }
  void run() {
    if (total == 0) return;
    unsigned char* p = static_cast<unsigned char*>(pinned(ctx, total));
    for (const Item& it : items)
      HIPCHK(ctx, hipMemcpyAsync(p + it.off, it.dev, it.bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (const Item& it : items) std::memcpy(it.host, p + it.off, it.bytes);
    if (ctx->prof) prof_resolve(ctx);
  }
};

void prof_batches(rp_context* ctx, rp_system* s, int kernel, const std::vector<std::pair<int64_t, int64_t>>& batches,
                  double zcoef, double ncoef) {
  if (!ctx->prof || batches.empty()) return;
  const int K = s->K;
  std::vector<int64_t> m(K);
  std::vector<int32_t> st(K);
  HostReads(ctx).add(m.data(), s->iters_in.p, K).add(st.data(), s->status_in.p, K).run();
  for (int k = 0; k < K; k++) {
    if (st[k] == ST_SKIP) continue;
    const double per = zcoef * (double)s->z_h[k] + ncoef * (double)s->nq_h[k];
    for (const auto& b : batches) {
      const int64_t d = std::min<int64_t>(b.second, std::max<int64_t>(0, m[k] - b.first));
      ctx->stat[kernel].bytes += per * (double)d;
    }
  }
}

// ---------------------------------------------------------------------------
// inner iterations (run on every instance whose status_in is ST_RUN)

struct InnerCfg {
  int method;        // 0 Jacobi, 1 BiCGStab
  int measmode;      // MEAS_*
  int strict;        // Jacobi: stop on m < thr instead of m <= thr
  int64_t max_iter;  // per instance
  int chunk;         // iterations between host checks
  bool x_zero;       // start from x = 0 (else from the contents of xa)
  bool stall = false;  // stop instances whose measure stagnates (paper's rule)
  bool graph = false;  // tiled Jacobi: replay full batches as one captured graph
};

// Fewest iterations without a halving of the best stopping measure before
// the paper's rule gives up on an instance (see k_stall): far above the
// halving interval of any chain that converges in a useful time (spectral
// radius 0.99999 halves in ~69,000 sweeps), while a tolerance below the
// rounding floor now ends after ~2^16 iterations instead of max_iter.
constexpr int64_t kStallWindow = 65536;

// Iterations launched before the first host check of an inner solve; the
// batch doubles after every check up to cfg.chunk.  Short solves (a
// BiCGStab correction takes ~10 steps) then launch few idle iterations and
// long ones few checks.
int first_batch(const InnerCfg& cfg) { return std::min(4, cfg.chunk); }

// Returns the number of iterations launched (an upper bound on every
// instance's count).  On return the solution of instance k is in xa, or in
// xb when the Jacobi count iters_in[k] is odd.
// Tiled Jacobi batches as replays of one captured HIP graph: cfg.chunk
// sweeps (an even count), the check of the last one, the publication of the
// done count and the advance of the sweep base.  The sweep and check kernels
// take their sweep numbers relative to a device word (Tiles::sbase), so the
// same graph serves every batch; the sequence number of the publication is
// kept on the device too.  The graph is captured on the context's private
// stream and replayed on its own stream, one replay ahead of the host's wait
// (a replay after every instance stopped costs its launches only).  Returns
// true when every instance finished; otherwise the caller continues from
// `launched` with ordinary launches (fewer than cfg.chunk sweeps left before
// max_iter, or the sweep count not even).
template <typename T>
bool jacobi_graph_batches(rp_context* ctx, rp_system* s, bool tr, const T* rhs, const InnerCfg& cfg, bool sl_on,
                          int64_t& launched, std::vector<std::pair<int64_t, int64_t>>& batches) {
  const int64_t B = cfg.chunk;
  if (!ctx->flag_h || B < 2 || B % 2 != 0 || launched % 2 != 0 || launched + B > cfg.max_iter) return false;
  hipStream_t st = ctx->stream;
  if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = ctx->cap_stream;
  const int K = s->K;
  VecSet<T>& w = vecs<T>(s);
  MatView<T> m = view<T>(s, tr);
  const Sliced<T> slv = sl_on ? sliced_for<T>(s, tr).v : Sliced<T>{};
  DBuf<int64_t> base;
  DBuf<int32_t> gseq;
  dalloc(ctx, base, 1);
  dalloc(ctx, gseq, 1);
  HIPCHK(ctx, launch_set_i64(st, base.p, launched));
  HIPCHK(ctx, launch_set_i32(st, gseq.p, ctx->flag_seq));
  Tiles tl = tiles_for<T>(s).tl;
  tl.sbase = base.p;
  double* P0 = s->tp.p;
  double* P1 = s->tp.p + tl.ntile;
  int32_t* ndone = s->counters.p;
  const int wd = cfg.measmode == MEAS_WDELTA;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIPCHK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  for (int64_t i = 0; i < B && e == hipSuccess; i++) {
    const T* x = (i & 1) ? w.xb.p : w.xa.p;
    T* xn = (i & 1) ? w.xa.p : w.xb.p;
    double* pcur = (i & 1) ? P1 : P0;
    const double* pprev = (i & 1) ? P0 : P1;
    e = sl_on ? launch_jacobi_sliced<T>(cs, slv, rhs, x, xn, tl, i, pprev, pcur, s->status_in.p, s->iters_in.p,
                                        s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter, ndone, wd)
              : launch_jacobi_tile<T>(cs, s->L, m, rhs, x, xn, tl, i, pprev, pcur, s->status_in.p, s->iters_in.p,
                                      s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter, ndone, wd);
  }
  if (e == hipSuccess)
    e = launch_jacobi_check(cs, tl, B, P1, s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, cfg.strict,
                            cfg.max_iter, ndone);
  if (e == hipSuccess) e = launch_publish_next(cs, ndone, ctx->flag_d, gseq.p);
  if (e == hipSuccess) e = launch_advance(cs, base.p, B);
  const hipError_t ee = hipStreamEndCapture(cs, &graph);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_err(ctx, "graph capture of the Jacobi batches failed: %s", hipGetErrorString(e));
    throw Fail{RP_ERR_HIP};
  }
  struct Cleanup {
    hipGraph_t g;
    hipGraphExec_t x;
    ~Cleanup() {
      (void)hipGraphExecDestroy(x);
      (void)hipGraphDestroy(g);
    }
  } cleanup{graph, exec};
  const int kJ = std::is_same<T, float>::value ? RP_PROF_JACOBI_FP32 : RP_PROF_JACOBI_FP64;
  std::deque<int32_t> pending;
  bool done = false;
  while (true) {
    while (pending.size() < 2 && launched + B <= cfg.max_iter) {
      ProfSpan span(ctx);
      HIPCHK(ctx, hipGraphLaunch(exec, st));
      span.end(kJ, B);
      batches.push_back({launched, B});
      launched += B;
      pending.push_back(++ctx->flag_seq);
    }
    if (pending.empty()) break;
    const int32_t sq = pending.front();
    pending.pop_front();
    if (wait_i32(ctx, ndone, sq) >= K) {
      done = true;
      break;
    }
  }
  // replays still queued end before the graph and its words are released
  HIPCHK(ctx, hipStreamSynchronize(st));
  return done;
}

template <typename T>
int64_t run_inner(rp_context* ctx, rp_system* s, bool tr, const T* rhs, const InnerCfg& cfg) {
  VecSet<T>& w = vecs<T>(s);
  MatView<T> m = view<T>(s, tr);
  hipStream_t st = ctx->stream;
  const Chunks& ch = s->ch;
  int32_t* ndone = s->counters.p;
  const int32_t K = s->K;
  int64_t launched = 0;
  const double tb_ = (double)sizeof(T);
  // stagnation watch after a batch (paper's rule only); queued before the
  // done count is published so that the look-ahead iterations see it
  auto watch = [&]() {
    if (cfg.stall)
      HIPCHK(ctx, launch_stall(st, K, launched, s->status_in.p, s->iters_in.p, s->meas_in.p, s->sbest.p,
                               s->sbest_it.p, kStallWindow, ndone));
  };
  // tiled sweeps on sliced rows when this call chose them
  const bool sl_on = s->sliced && tiled<T>(s) && ensure_sliced<T>(ctx, s, tr);
  const Sliced<T> slv = sl_on ? sliced_for<T>(s, tr).v : Sliced<T>{};
  const int kJ = std::is_same<T, float>::value ? RP_PROF_JACOBI_FP32 : RP_PROF_JACOBI_FP64;
  const int kT = std::is_same<T, float>::value ? RP_PROF_JACOBI_TAIL_FP32 : RP_PROF_JACOBI_TAIL_FP64;
  const int kS = std::is_same<T, float>::value ? RP_PROF_SPMV_FP32 : RP_PROF_SPMV_FP64;
  const int kV = std::is_same<T, float>::value ? RP_PROF_VECTOR_FP32 : RP_PROF_VECTOR_FP64;
  // algorithmic bytes of the iterations done since the last call
  std::vector<int64_t> seen(K, 0);
  auto account = [&]() {
    if (!ctx->prof) return;
    std::vector<int64_t> it(K);
    to_host(ctx, it.data(), s->iters_in.p, K);
    for (int k = 0; k < K; k++) {
      const double d = (double)(it[k] - seen[k]);
      seen[k] = it[k];
      const double z = (double)s->z_h[k], n = (double)s->nq_h[k];
      if (cfg.method == 0) {
        ctx->stat[kJ].bytes += d * ((4 + tb_) * z + (4 + 4 * tb_) * n);
      } else {
        ctx->stat[kS].bytes += d * (2 * (4 + tb_) * z + (8 + 7 * tb_) * n);
        ctx->stat[kV].bytes += d * (14 * tb_ * n);
      }
    }
  };
  if (cfg.x_zero) HIPCHK(ctx, hipMemsetAsync(w.xa.p, 0, sizeof(T) * (size_t)s->npad, st));
  if (cfg.method == 0) {
    // Jacobi; xb must hold a copy of xa wherever an instance is skipped
    // (padding rows included) so that either buffer is a valid iterate.
    HIPCHK(ctx, hipMemcpyAsync(w.xb.p, w.xa.p, sizeof(T) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    const int jv = s->jvariant;
    if (jv == 0 && s->tiles_on && resident_for<T>(s).ok) {
      // small instances: one block per instance, many sweeps per launch
      const Tiles& tl = resident_for<T>(s).tl;
      std::vector<std::pair<int64_t, int64_t>> batches;
      while (launched < cfg.max_iter) {
        ProfSpan span(ctx);
        const int64_t j0 = launched;
        const int n = (int)std::min<int64_t>(kResidentSweeps, cfg.max_iter - launched);
        HIPCHK(ctx, launch_jacobi_resident<T>(st, s->L, m, rhs, w.xa.p, w.xb.p, tl, launched, n, s->status_in.p,
                                              s->iters_in.p, s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter,
                                              ndone, cfg.measmode == MEAS_WDELTA));
        launched += n;
        span.end(kJ, n);
        batches.push_back({j0, n});
        watch();
        if (read_i32(ctx, ndone) >= K) break;
      }
      prof_batches(ctx, s, kJ, batches, 4 + tb_, 4 + 4 * tb_);
      return launched;
    }
    if (jv == 0 && tiled<T>(s)) {
      // LDS-staged sweeps; the decision on sweep j is taken inside sweep j+1
      // (or by the check kernel after the last sweep of a batch)
      const Tiles& tl = tiles_for<T>(s).tl;
      double* P0 = s->tp.p;
      double* P1 = s->tp.p + tl.ntile;
      std::vector<std::pair<int64_t, int64_t>> batches;
      auto sweep = [&](int64_t j) {
        const T* x = (j & 1) ? w.xb.p : w.xa.p;
        T* xn = (j & 1) ? w.xa.p : w.xb.p;
        double* pcur = (j & 1) ? P1 : P0;
        const double* pprev = (j & 1) ? P0 : P1;
        if (sl_on)
          HIPCHK(ctx, launch_jacobi_sliced<T>(st, slv, rhs, x, xn, tl, j, pprev, pcur, s->status_in.p, s->iters_in.p,
                                              s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter, ndone,
                                              cfg.measmode == MEAS_WDELTA));
        else
          HIPCHK(ctx, launch_jacobi_tile<T>(st, s->L, m, rhs, x, xn, tl, j, pprev, pcur, s->status_in.p,
                                            s->iters_in.p, s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter,
                                            ndone, cfg.measmode == MEAS_WDELTA));
      };
      // After each batch the check kernel publishes how many instances are
      // done; the first sweeps of the next batch are queued before the host
      // waits for that count, so the GPU does not idle during the round trip
      // (sweeps of finished instances return at once).  One timing span per
      // batch: its look-ahead sweeps and the rest.
      int batch = first_batch(cfg);
      int64_t ahead = 0;  // sweeps of the current batch launched ahead
      if (cfg.graph && !cfg.stall) {
        if (jacobi_graph_batches<T>(ctx, s, tr, rhs, cfg, sl_on, launched, batches)) {
          prof_batches(ctx, s, kJ, batches, 4 + tb_, 4 + 4 * tb_);
          return launched;
        }
        batch = cfg.chunk;
      }
      ProfSpan span(ctx);
      int64_t j0 = launched;
      int32_t tail_tried = -1;  // done count at the last look at the tail
      bool tail = false;
      // (ahead > 0 at max_iter: one more pass runs the check of those sweeps)
      while (launched < cfg.max_iter || ahead > 0) {
        const int64_t end = std::min<int64_t>(cfg.max_iter, j0 + batch);
        for (; launched < end; launched++) sweep(launched);
        span.end(kJ, launched - j0);
        if (launched > j0) batches.push_back({j0, launched - j0});
        const double* plast = ((launched - 1) & 1) ? P1 : P0;
        HIPCHK(ctx, launch_jacobi_check(st, tl, launched, plast, s->status_in.p, s->iters_in.p, s->meas_in.p,
                                        s->thr_in.p, cfg.strict, cfg.max_iter, ndone));
        watch();
        const int32_t seq = publish_i32(ctx, ndone);
        batch = std::min(2 * batch, cfg.chunk);
        ahead = std::min<int64_t>({kLookahead, batch, cfg.max_iter - launched});
        span.restart();
        j0 = launched;
        for (int64_t i = 0; i < ahead; i++, launched++) sweep(launched);
        const int32_t nd = wait_i32(ctx, ndone, seq);
        if (nd >= K) {
          span.end(kJ, launched - j0);
          if (launched > j0) batches.push_back({j0, launched - j0});
          break;
        }
        if (K - nd <= kTailInstances && nd != tail_tried && launched < cfg.max_iter) {
          // few instances left: close the look-ahead sweeps (their span and
          // the decision on the last of them) and go resident if they fit
          tail_tried = nd;
          span.end(kJ, launched - j0);
          if (launched > j0) batches.push_back({j0, launched - j0});
          const double* pl = ((launched - 1) & 1) ? P1 : P0;
          HIPCHK(ctx, launch_jacobi_check(st, tl, launched, pl, s->status_in.p, s->iters_in.p, s->meas_in.p,
                                          s->thr_in.p, cfg.strict, cfg.max_iter, ndone));
          std::vector<int32_t> st_h((size_t)K), ts0_h;
          to_host(ctx, st_h.data(), s->status_in.p, (size_t)K);
          if (std::none_of(st_h.begin(), st_h.end(), [](int32_t v) { return v == ST_RUN; })) break;
          if (sl_on) {
            ts0_h.resize((size_t)tl.ntile + 1);
            to_host(ctx, ts0_h.data(), slv.t_s0, (size_t)tl.ntile + 1);
          }
          if (build_tail(ctx, s, sizeof(T), st_h, tiles_for<T>(s), sl_on ? &ts0_h : nullptr)) {
            tail = true;
            break;
          }
          span.restart();
          j0 = launched;
        }
      }
      if (tail) {
        // resident sweeps from sweep `launched` on, with the row sums of the
        // tiled layout in use (the sliced rows themselves, or one lane per row
        // in CSR order, which sums alike), so the iterates are those the tiled
        // sweeps would have produced
        const Tiles& tt = s->tail.tl;
        const int lanes = sl_on ? 1 : s->L;
        std::vector<std::pair<int64_t, int64_t>> tb;
        while (launched < cfg.max_iter) {
          ProfSpan sp(ctx);
          const int64_t j1 = launched;
          const int n = (int)std::min<int64_t>(kResidentSweeps, cfg.max_iter - launched);
          if (s->tail_sliced)
            HIPCHK(ctx, launch_jacobi_resident_sliced<T>(st, slv, rhs, w.xa.p, w.xb.p, tt, s->tail_slo.p,
                                                         s->tail_shi.p, launched, n, s->status_in.p, s->iters_in.p,
                                                         s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter, ndone,
                                                         cfg.measmode == MEAS_WDELTA));
          else
            HIPCHK(ctx, launch_jacobi_resident<T>(st, lanes, m, rhs, w.xa.p, w.xb.p, tt, launched, n, s->status_in.p,
                                                  s->iters_in.p, s->meas_in.p, s->thr_in.p, cfg.strict, cfg.max_iter,
                                                  ndone, cfg.measmode == MEAS_WDELTA));
          launched += n;
          sp.end(kT, n);
          tb.push_back({j1, n});
          watch();
          if (read_i32(ctx, ndone) >= K) break;
        }
        prof_batches(ctx, s, kT, tb, 4 + tb_, 4 + 4 * tb_);
      }
      // (after the tail: the byte counts read the final iteration counts)
      prof_batches(ctx, s, kJ, batches, 4 + tb_, 4 + 4 * tb_);
      return launched;
    }
    while (launched < cfg.max_iter) {
      for (int i = 0; i < cfg.chunk && launched < cfg.max_iter; i++, launched++) {
        const T* x = (launched & 1) ? w.xb.p : w.xa.p;
        T* xn = (launched & 1) ? w.xa.p : w.xb.p;
        const int wd = cfg.measmode == MEAS_WDELTA;
        if (jv == 1)  // one vector, xa, overwritten in place
          PROF(ctx, kJ, launch_jacobi_inplace<T>(st, s->L, m, rhs, w.xa.p, ch, s->status_in.p, s->pa.p, wd));
        else if (jv == 2)
          PROF(ctx, kJ, launch_jacobi_segscan<T>(st, m, s->erow[tr ? 1 : 0].p, rhs, x, xn, ch, s->status_in.p,
                                                 s->pa.p, wd));
        else
          PROF(ctx, kJ, launch_jacobi<T>(st, s->L, m, rhs, x, xn, ch, s->status_in.p, s->pa.p, wd));
        HIPCHK(ctx, launch_fin_jacobi(st, ch, s->pa.p, s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p,
                                      cfg.strict, cfg.max_iter, ndone));
      }
      watch();
      const bool done = read_i32(ctx, ndone) >= K;
      account();
      if (done) break;
    }
    // in place: both buffers hold the iterate, whichever the sweep count
    // selects
    if (jv == 1)
      HIPCHK(ctx, hipMemcpyAsync(w.xb.p, w.xa.p, sizeof(T) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
  } else if (s->tiles_on && resident_for<T>(s).ok && resident_for<T>(s).tl.maxw <= bicg_resident_rows(s->L)) {
    // small instances: one block per instance, many steps per launch
    const Tiles& tl = resident_for<T>(s).tl;
    const int kB = std::is_same<T, float>::value ? RP_PROF_BICGSTAB_FP32 : RP_PROF_BICGSTAB_FP64;
    BicgState b{s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, s->rho2.p, s->alpha.p, s->omega.p,
                ndone, cfg.measmode, cfg.max_iter};
    std::vector<std::pair<int64_t, int64_t>> batches;
    while (true) {
      ProfSpan span(ctx);
      const int64_t j0 = launched;
      const int n = (int)std::min<int64_t>(kResidentSweeps, cfg.max_iter - launched);
      HIPCHK(ctx, launch_bicg_resident<T>(st, s->L, m, rhs, w.xa.p, w.r.p, w.q.p, w.p.p, w.v.p, tl, launched, n,
                                          cfg.x_zero ? 1 : 0, s->tpc.p, s->tps.p, b));
      launched += n;
      span.end(kB, n);
      batches.push_back({j0, n});
      watch();
      if (read_i32(ctx, ndone) >= K || launched >= cfg.max_iter) break;
    }
    prof_batches(ctx, s, kB, batches, 2 * (4 + tb_), 8 + 21 * tb_);
  } else if (tiled<T>(s)) {
    // tiled BiCGStab: five launches per step, scalars reduced in-kernel
    const Tiles& tl = tiles_for<T>(s).tl;
    const int kB = std::is_same<T, float>::value ? RP_PROF_BICGSTAB_FP32 : RP_PROF_BICGSTAB_FP64;
    BicgState b{s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, s->rho2.p, s->alpha.p, s->omega.p,
                ndone, cfg.measmode, cfg.max_iter};
    HIPCHK(ctx, launch_bicg_tile_init<T>(st, s->L, m, rhs, w.xa.p, cfg.x_zero ? 1 : 0, w.r.p, w.q.p, w.p.p, w.v.p, tl,
                                         s->status_in.p, s->tpc.p));
    std::vector<std::pair<int64_t, int64_t>> batches;
    auto bstep = [&](int64_t j) {
      HIPCHK(ctx, launch_bicg_p_tile<T>(st, w.r.p, w.p.p, w.v.p, tl, j, s->tpc.p, s->tps.p, b));
      if (sl_on) HIPCHK(ctx, launch_spmv_sliced<T>(st, 0, slv, w.p.p, w.v.p, w.q.p, tl, s->status_in.p, s->tpa.p));
      else HIPCHK(ctx, launch_spmv_tile<T>(st, s->L, 0, m, w.p.p, w.v.p, w.q.p, tl, s->status_in.p, s->tpa.p));
      HIPCHK(ctx, launch_bicg_s_tile<T>(st, w.r.p, w.v.p, w.s.p, tl, j, s->tpa.p, s->tps.p, b));
      if (sl_on) HIPCHK(ctx, launch_spmv_sliced<T>(st, 1, slv, w.s.p, w.t.p, w.q.p, tl, s->status_in.p, s->tpb.p));
      else HIPCHK(ctx, launch_spmv_tile<T>(st, s->L, 1, m, w.s.p, w.t.p, w.q.p, tl, s->status_in.p, s->tpb.p));
      HIPCHK(ctx, launch_bicg_xr_tile<T>(st, w.xa.p, w.p.p, w.s.p, w.r.p, w.t.p, w.q.p, tl, j, s->tpb.p, s->tpc.p,
                                         b));
    };
    // as for the tiled Jacobi sweeps: the first steps of the next batch are
    // queued before the host waits for the done count of this one
    int batch = first_batch(cfg);
    int64_t ahead = 0;
    ProfSpan span(ctx);
    int64_t j0 = launched;
    while (launched < cfg.max_iter || ahead > 0) {
      const int64_t end = std::min<int64_t>(cfg.max_iter, j0 + batch);
      for (; launched < end; launched++) bstep(launched);
      span.end(kB, launched - j0);
      if (launched > j0) batches.push_back({j0, launched - j0});
      HIPCHK(ctx, launch_bicg_check(st, tl, launched, s->tpc.p, s->tps.p, b));
      watch();
      const int32_t seq = publish_i32(ctx, ndone);
      batch = std::min({2 * batch, cfg.chunk, kBicgBatch});
      ahead = std::min<int64_t>({kLookahead / 2, batch, cfg.max_iter - launched});
      span.restart();
      j0 = launched;
      for (int64_t i = 0; i < ahead; i++, launched++) bstep(launched);
      if (wait_i32(ctx, ndone, seq) >= K) {
        span.end(kB, launched - j0);
        if (launched > j0) batches.push_back({j0, launched - j0});
        break;
      }
    }
    prof_batches(ctx, s, kB, batches, 2 * (4 + tb_), 8 + 21 * tb_);
  } else {
    HIPCHK(ctx, launch_bicg_init<T>(st, s->L, m, rhs, w.xa.p, cfg.x_zero ? 1 : 0, w.r.p, w.q.p, w.p.p, w.v.p, ch,
                                    s->status_in.p, s->pa.p));
    HIPCHK(ctx, launch_fin_bicg_init(st, ch, s->pa.p, s->status_in.p, s->rho.p, s->alpha.p, s->omega.p, s->beta.p,
                                     s->meas_in.p, s->thr_in.p, cfg.measmode, ndone));
    if (read_i32(ctx, ndone) < K) {
      while (launched < cfg.max_iter) {
        for (int i = 0; i < cfg.chunk && launched < cfg.max_iter; i++, launched++) {
          PROF(ctx, kV, launch_bicg_p<T>(st, w.r.p, w.p.p, w.v.p, s->beta.p, s->omega.p, ch, s->status_in.p));
          PROF(ctx, kS, launch_spmv_dot<T>(st, s->L, 0, m, w.p.p, w.v.p, w.q.p, ch, s->status_in.p, s->pa.p));
          HIPCHK(ctx, launch_fin_alpha(st, ch, s->pa.p, s->status_in.p, s->rho.p, s->alpha.p, ndone));
          PROF(ctx, kV, launch_bicg_s<T>(st, w.r.p, w.v.p, w.s.p, s->alpha.p, ch, s->status_in.p, s->ps.p));
          PROF(ctx, kS, launch_spmv_dot<T>(st, s->L, 1, m, w.s.p, w.t.p, w.q.p, ch, s->status_in.p, s->pb.p));
          HIPCHK(ctx, launch_fin_omega(st, ch, s->pb.p, s->status_in.p, s->omega.p, ndone));
          PROF(ctx, kV, launch_bicg_xr<T>(st, w.xa.p, w.p.p, w.s.p, w.r.p, w.t.p, w.q.p, s->alpha.p, s->omega.p, ch,
                                          s->status_in.p, s->pc.p));
          HIPCHK(ctx, launch_fin_rho(st, ch, s->pc.p, s->ps.p, s->status_in.p, s->rho.p, s->alpha.p, s->omega.p,
                                     s->beta.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, cfg.measmode,
                                     cfg.max_iter, ndone));
        }
        watch();
        const bool done = read_i32(ctx, ndone) >= K;
        account();
        if (done) break;
      }
    }
  }
  return launched;
}

// ---------------------------------------------------------------------------
// per-instance host bookkeeping of a solve

struct SolveLog {
  std::vector<int64_t> iters, refinements;
  std::vector<double> delta, resid, bound;
  std::vector<int32_t> status;  // device status codes (ST_*)
  int32_t lanes = 0;             // lanes per row of the sparse products
  std::vector<int32_t> panels;   // per instance: column panels of its sliced rows (0: none)
  explicit SolveLog(int K)
      : iters(K, 0), refinements(K, 0), delta(K, 0.0), resid(K, 0.0), bound(K, -1.0), status(K, ST_RUN) {}
};

void accumulate_inner(rp_context* ctx, rp_system* s, SolveLog& log, const std::vector<int32_t>& active) {
  const int K = s->K;
  std::vector<int64_t> it(K);
  std::vector<double> me(K);
  std::vector<int32_t> stin(K);
  HostReads(ctx).add(it.data(), s->iters_in.p, K).add(me.data(), s->meas_in.p, K)
      .add(stin.data(), s->status_in.p, K).run();
  for (int k = 0; k < K; k++) {
    if (!active[k]) continue;
    log.iters[k] += it[k];
    log.delta[k] = me[k];
  }
  (void)stin;
}

constexpr int64_t kInnerCap = 200000;

// FP64 iterative refinement on (I - A) x = b (or the transposed system):
// r = b - M x in FP64; stop per instance when certified (tb * ||r|| <= tol)
// or when ||r|| <= tol; otherwise solve M d = r / ||r|| in precision T with
// the inner method and add ||r|| d to x.  x64 holds the starting point.
template <typename T>
void refine(rp_context* ctx, rp_system* s, bool tr, int method, const double* b64, bool certified, double tol,
            const double* tb, const rp_opts& o, SolveLog& log) {
  hipStream_t st = ctx->stream;
  const int K = s->K;
  VecSet<T>& w = vecs<T>(s);
  HIPCHK(ctx, w.ensure((size_t)s->npad, &ctx->blocks));
  MatView<double> m64 = view<double>(s, tr);
  int32_t* ndone_out = s->counters.p + 1;
  // outer status: skip empty instances
  HIPCHK(ctx, launch_inner_init(st, K, nullptr, s->nq.p, s->status_out.p, s->outer_it.p, ndone_out));
  // Rounding floor of the inner stopping measure, relative to the scaled
  // right-hand side: the inner solution is as large as ||(I-A)^{-1}||, so its
  // last-bit noise is about unit roundoff times that (tb when known).
  const double floor_rel = std::is_same<T, float>::value ? 8.0 * 5.9604644775390625e-08 : 8.0 * 1.1102230246251565e-16;
  // Share of what the final tolerance still needs that an inner solve must
  // reach.  Jacobi's weighted measure after m sweeps, max d_i |x_m - x_{m-1}|,
  // is the residual of x_{m-1} (up to rounding), and that iterate is the
  // correction handed on (k_correct with prev set), so in FP64 the corrected
  // x misses the target only by rounding and 0.9 is enough; the stopping test
  // is always on the FP64 residual of the corrected x.  BiCGStab's recurrence
  // residual can drift from the true one and FP32 measures carry FP32
  // rounding, so those keep 0.5.
  const double margin = (std::is_same<T, double>::value && method == 0 && s->jvariant != 1) ? 0.9 : 0.5;
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 10000000;
  // per-instance inner-iteration totals and last stopping measure, on device
  HIPCHK(ctx, hipMemsetAsync(s->tot_it.p, 0, sizeof(int64_t) * (size_t)K, st));
  HIPCHK(ctx, hipMemsetAsync(s->last_meas.p, 0, sizeof(double) * (size_t)K, st));
  // upper bound on every instance's total (sum of the inner launches)
  int64_t launched_total = 0;
  std::vector<int32_t> sto(K);
  while (true) {
    const bool t64 = tiled<double>(s);
    if (ctx->prof) to_host(ctx, sto.data(), s->status_out.p, K);
    // sliced rows when this call uses them and the FP64 slices exist
    const SlicedSet<double>& sl64 = sliced_for<double>(s, tr);
    if (t64 && s->sliced && sl64.ok)
      PROF(ctx, RP_PROF_RESIDUAL_FP64,
           launch_spmv_sliced<double>(st, 2, sl64.v, s->x64.p, s->r64.p, b64, s->t64.tl, s->status_out.p, s->tpa.p));
    else if (t64)
      PROF(ctx, RP_PROF_RESIDUAL_FP64,
           launch_residual_tile(st, s->L, m64, b64, s->x64.p, s->r64.p, s->t64.tl, s->status_out.p, s->tpa.p));
    else
      PROF(ctx, RP_PROF_RESIDUAL_FP64,
           launch_residual64(st, s->L, m64, b64, s->x64.p, s->r64.p, s->ch, s->status_out.p, s->pa.p));
    if (ctx->prof)
      for (int k = 0; k < K; k++)
        if (sto[k] == ST_RUN)
          ctx->stat[RP_PROF_RESIDUAL_FP64].bytes += 12.0 * (double)s->z_h[k] + 36.0 * (double)s->nq_h[k];
    HIPCHK(ctx, launch_fin_outer(st, t64 ? tile_chunks(s->t64.tl) : s->ch, t64 ? s->tpa.p : s->pa.p,
                                 s->status_out.p, s->outer_it.p, s->rn.p, s->scale.p, tb, tol,
                                 certified ? 1 : 0, o.max_refine, s->thr_in.p, o.inner_tol, floor_rel, margin, s->rbest.p,
                                 s->stall.p, s->tot_it.p, max_iter, ndone_out));
    if (read_i32(ctx, ndone_out) >= K) break;
    HIPCHK(ctx, launch_inner_init(st, K, s->status_out.p, s->nq.p, s->status_in.p, s->iters_in.p, s->counters.p));
    HIPCHK(ctx, launch_scale_rhs<T>(st, s->r64.p, s->scale.p, w.rhs.p, s->ch, s->status_out.p));
    InnerCfg cfg;
    cfg.method = method;
    cfg.measmode = method == 0 ? MEAS_WDELTA : MEAS_R;
    cfg.strict = 0;
    // cap one inner solve; an inner solve cut short still yields a useful
    // correction and the outer loop continues from the improved x
    int64_t room = kInnerCap;
    if (launched_total + kInnerCap > max_iter) {
      // near the budget: the exact per-instance totals bound this inner solve
      std::vector<int64_t> tot(K);
      HostReads(ctx).add(tot.data(), s->tot_it.p, K).add(sto.data(), s->status_out.p, K).run();
      int64_t worst = 0;
      for (int k = 0; k < K; k++)
        if (sto[k] == ST_RUN) worst = std::max(worst, tot[k]);
      room = std::min<int64_t>(kInnerCap, max_iter - worst);
    }
    cfg.max_iter = std::max<int64_t>(1, room);
    cfg.chunk = o.chunk > 0 ? o.chunk : 32;
    cfg.x_zero = true;
    cfg.graph = o.graph != 0;
    launched_total += run_inner<T>(ctx, s, tr, w.rhs.p, cfg);
    HIPCHK(ctx, launch_correct<T>(st, s->x64.p, w.xa.p, w.xb.p, method == 0 ? s->iters_in.p : nullptr,
                                  cfg.measmode == MEAS_WDELTA ? 1 : 0, s->status_in.p, s->scale.p, s->ch,
                                  s->status_out.p));
    HIPCHK(ctx, launch_accum_inner(st, K, s->status_out.p, s->iters_in.p, s->meas_in.p, s->tot_it.p,
                                   s->last_meas.p));
  }
  std::vector<int64_t> tot(K);
  std::vector<double> lastm(K);
  std::vector<int64_t> oit(K);
  std::vector<double> rn(K), tbh(K, -1.0);
  {
    HostReads hr(ctx);
    hr.add(tot.data(), s->tot_it.p, K).add(lastm.data(), s->last_meas.p, K).add(sto.data(), s->status_out.p, K);
    hr.add(oit.data(), s->outer_it.p, K).add(rn.data(), s->rn.p, K);
    if (tb) hr.add(tbh.data(), tb, K);
    hr.run();
  }
  for (int k = 0; k < K; k++) {
    log.iters[k] += tot[k];
    if (tot[k] > 0) log.delta[k] = lastm[k];
  }
  for (int k = 0; k < K; k++) {
    if (s->nq_h[k] == 0) {
      log.status[k] = ST_CONVERGED;
      log.resid[k] = 0.0;
      log.bound[k] = 0.0;
      continue;
    }
    log.status[k] = sto[k];
    log.refinements[k] = oit[k];
    log.resid[k] = rn[k];
    log.bound[k] = tb ? tbh[k] * rn[k] : -1.0;
  }
}

// Bound on ||(I-A)^{-1} 1||_inf per instance (or of the transpose): solve
// M T = 1 in FP64 refinement until ||1 - M T||_inf <= 1e-3, then
// ||T||_inf <= ||T^||_inf / (1 - ||1 - M T^||_inf).
void ensure_tbound(rp_context* ctx, rp_system* s, bool tr, int method) {
  bool& have = tr ? s->have_tb_tr : s->have_tb_fwd;
  if (have) return;
  DBuf<double>& tbd = tr ? s->tb_tr : s->tb_fwd;
  std::vector<double>& tbh = tr ? s->tb_tr_h : s->tb_fwd_h;
  const int K = s->K;
  dalloc(ctx, tbd, (size_t)K);
  rp_opts o;
  rp_opts_default(&o);
  o.inner_tol = 1e-2;
  o.max_refine = 200;
  std::vector<double> bound(K, std::numeric_limits<double>::infinity());
  // BiCGStab first (few iterations, whichever method the solve itself uses:
  // the bound is a property of the matrix); any instance it fails on is
  // redone by Jacobi, which converges on every M-matrix.  Small instances
  // that the resident Jacobi kernel serves go to Jacobi directly: its sweeps
  // cost about a microsecond, while BiCGStab's five launches per step cost
  // several and it can stall on ill-conditioned chains.
  // The first pass runs its inner iterations in FP32 (the bound only needs
  // T^ and its residual, and both are FP64: the residual is recomputed in
  // FP64 and T^ is the FP64 refinement iterate); the fallback passes are
  // FP64, for chains too ill-conditioned for FP32 inner solves.
  (void)method;
  const bool jacobi_first = s->tiles_on && s->res64.ok;
  const int m0 = jacobi_first ? 0 : 1, m1 = 1 - m0;
  const int methods[3] = {m0, m1, m0};
  const bool fp32[3] = {true, false, false};
  for (int pass = 0; pass < 3; pass++) {
    SolveLog log(K);
    HIPCHK(ctx, hipMemsetAsync(s->x64.p, 0, sizeof(double) * (size_t)s->npad, ctx->stream));
    if (fp32[pass]) refine<float>(ctx, s, tr, methods[pass], s->b_one.p, false, 1e-3, nullptr, o, log);
    else refine<double>(ctx, s, tr, methods[pass], s->b_one.p, false, 1e-3, nullptr, o, log);
    HIPCHK(ctx, launch_absmax(ctx->stream, s->x64.p, s->ch, s->pa.p));
    HIPCHK(ctx, launch_fin_absmax(ctx->stream, s->ch, s->pa.p, s->tmp_k.p));
    std::vector<double> tmax(K);
    to_host(ctx, tmax.data(), s->tmp_k.p, K);
    bool all = true;
    for (int k = 0; k < K; k++) {
      if (std::isfinite(bound[k])) continue;
      if (s->nq_h[k] == 0) {
        bound[k] = 0.0;
        continue;
      }
      if (log.status[k] == ST_CONVERGED && log.resid[k] < 1.0 && std::isfinite(tmax[k])) {
        bound[k] = tmax[k] / (1.0 - log.resid[k]);
      } else {
        all = false;
      }
    }
    if (all) break;
  }
  tbh = bound;
  to_dev(ctx, tbd.p, bound.data(), K);
  have = true;
}

int status_to_rp(int32_t st) {
  switch (st) {
    case ST_CONVERGED: return RP_OK;
    case ST_MAXITER: return RP_ERR_NOT_CONVERGED;
    case ST_STALLED: return RP_ERR_NOT_CONVERGED;
    case ST_BREAKDOWN: return RP_ERR_BREAKDOWN;
    case ST_NONFINITE: return RP_ERR_NONFINITE;
    case ST_RUN: return RP_ERR_NOT_CONVERGED;
    default: return RP_OK;
  }
}
int severity(int code) {
  switch (code) {
    case RP_OK: return 0;
    case RP_ERR_NOT_CONVERGED: return 1;
    case RP_ERR_BREAKDOWN: return 2;
    case RP_ERR_NONFINITE: return 3;
    default: return 4;
  }
}

void check_opts(rp_context* ctx, const rp_opts* o) {
  if (!o) return;
  if (!(o->tol >= 0.0)) { set_err(ctx, "opts.tol must be >= 0"); throw Fail{RP_ERR_INVALID_ARG}; }
  if (o->stop < RP_STOP_DELTA || o->stop > RP_STOP_RESIDUAL) {
    set_err(ctx, "opts.stop must be RP_STOP_DELTA, RP_STOP_CERTIFIED or RP_STOP_RESIDUAL");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->precision != RP_FP64 && o->precision != RP_FP32_REFINED) {
    set_err(ctx, "opts.precision must be RP_FP64 or RP_FP32_REFINED");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->stop == RP_STOP_DELTA && o->precision != RP_FP64) {
    set_err(ctx, "RP_STOP_DELTA (the paper's rule) needs RP_FP64");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->schedule != RP_SCHEDULE_SEGSCAN && o->schedule != -1 && o->schedule != 0 && o->schedule != 1 &&
      o->schedule != 2 && o->schedule != 4 && o->schedule != 8 && o->schedule != 16 && o->schedule != 32 &&
      o->schedule != 64) {
    set_err(ctx, "opts.schedule must be RP_SCHEDULE_SEGSCAN, -1, 0 or a power of two in 1..64");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->update != RP_UPDATE_TWO_BUFFER && o->update != RP_UPDATE_IN_PLACE) {
    set_err(ctx, "opts.update must be RP_UPDATE_TWO_BUFFER or RP_UPDATE_IN_PLACE");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->graph != 0 && o->graph != 1) {
    set_err(ctx, "opts.graph must be 0 or 1");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->update == RP_UPDATE_IN_PLACE && o->schedule == RP_SCHEDULE_SEGSCAN) {
    set_err(ctx, "RP_UPDATE_IN_PLACE and RP_SCHEDULE_SEGSCAN do not combine");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (o->tiling != RP_TILING_AUTO && o->tiling != RP_TILING_OFF) {
    set_err(ctx, "opts.tiling must be RP_TILING_AUTO or RP_TILING_OFF");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (!(o->inner_tol > 0.0 && o->inner_tol < 1.0)) {
    set_err(ctx, "opts.inner_tol must be in (0, 1)");
    throw Fail{RP_ERR_INVALID_ARG};
  }
}

// Row layout of the tiled kernels, chosen by timing: the sliced rows (one
// lane per row), and lane groups of the mean-row-length choice L and of its
// neighbours L/2 and 2L, each run a few Jacobi sweeps (on the workspace,
// never converging); a lane-group layout replaces the sliced rows only when
// clearly faster.  The choice (0 = sliced rows, else L) is kept for every
// later system of the same shape on this context.  Systems served by the
// resident kernels keep the mean-row-length lane groups.
template <typename T>
int tuned_layout(rp_context* ctx, rp_system* s, bool tr) {
  if (!tiled<T>(s) || resident_for<T>(s).ok) return s->L;
  const std::array<int64_t, 5> key{s->npad, s->z, (int64_t)s->K, (int64_t)sizeof(T), tr ? 1 : 0};
  auto it = ctx->lane_choice.find(key);
  if (it != ctx->lane_choice.end()) return it->second;
  const bool have_sliced = ensure_sliced<T>(ctx, s, tr);
  hipStream_t st = ctx->stream;
  VecSet<T>& w = vecs<T>(s);
  HIPCHK(ctx, w.ensure((size_t)s->npad, &ctx->blocks));
  MatView<T> m = view<T>(s, tr);
  const Tiles& tl = tiles_for<T>(s).tl;
  const Sliced<T> slv = have_sliced ? sliced_for<T>(s, tr).v : Sliced<T>{};
  HIPCHK(ctx, hipMemsetAsync(w.xa.p, 0, sizeof(T) * (size_t)s->npad, st));
  HIPCHK(ctx, hipMemsetAsync(w.rhs.p, 0, sizeof(T) * (size_t)s->npad, st));
  HIPCHK(ctx, launch_inner_init(st, s->K, nullptr, s->nq.p, s->status_in.p, s->iters_in.p, s->counters.p));
  HIPCHK(ctx, launch_fill_f64(st, s->thr_in.p, s->K, -1.0));  // never met: every sweep runs
  hipEvent_t e0 = prof_event(ctx), e1 = prof_event(ctx);
  const int base = s->L;
  int best = -1;
  float best_ms = 0.f;
  constexpr int kWarm = 2, kTimed = 4;
  std::vector<int> cands;
  if (have_sliced) cands.push_back(0);
  for (int L : {base, base / 2, base * 2})
    if (L >= 1 && L <= 64) cands.push_back(L);
  for (int L : cands) {
    double* P0 = s->tp.p;
    double* P1 = s->tp.p + tl.ntile;
    for (int i = 0; i < kWarm + kTimed; i++) {
      if (i == kWarm) HIPCHK(ctx, hipEventRecord(e0, st));
      const T* x = (i & 1) ? w.xb.p : w.xa.p;
      T* xn = (i & 1) ? w.xa.p : w.xb.p;
      if (L == 0)
        HIPCHK(ctx, launch_jacobi_sliced<T>(st, slv, w.rhs.p, x, xn, tl, i, (i & 1) ? P0 : P1, (i & 1) ? P1 : P0,
                                            s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, 0,
                                            int64_t(1) << 40, s->counters.p, 0));
      else
        HIPCHK(ctx, launch_jacobi_tile<T>(st, L, m, w.rhs.p, x, xn, tl, i, (i & 1) ? P0 : P1, (i & 1) ? P1 : P0,
                                          s->status_in.p, s->iters_in.p, s->meas_in.p, s->thr_in.p, 0,
                                          int64_t(1) << 40, s->counters.p, 0));
    }
    HIPCHK(ctx, hipEventRecord(e1, st));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
    // a later candidate must be clearly faster: within 5% the earlier one
    // (sliced rows first) stays, so close timings do not flip the choice
    // from one run to the next
    if (best < 0 || ms < 0.95f * best_ms) {
      best = L;
      best_ms = ms;
    }
  }
  ctx->pool.push_back(e0);
  ctx->pool.push_back(e1);
  ctx->lane_choice[key] = best;
  return best;
}

// Core of rp_jacobi / rp_bicgstab and of the adjoint solve.  Solves the
// forward (tr = false) or transposed system with right-hand side b64 (padded
// reduced layout) and leaves the FP64 solution in s->x64.  x0_red, when not
// null, is a padded reduced starting point.
// Row of every stored entry of the forward or transposed reduced matrix,
// built the first time a segmented-scan sweep needs it.
void ensure_erow(rp_context* ctx, rp_system* s, bool tr) {
  DBuf<int32_t>& e = s->erow[tr ? 1 : 0];
  if (e.p) return;
  dalloc(ctx, e, (size_t)std::max<int64_t>(s->z, 1));
  HIPCHK(ctx, launch_fill_erow(ctx->stream, s->npad, view<double>(s, tr).rp, e.p));
}

void solve_core(rp_context* ctx, rp_system* s, bool tr, int method, const double* b64, const rp_opts& o,
                const double* x0_full, SolveLog& log) {
  hipStream_t st = ctx->stream;
  const int K = s->K;
  ensure_work(ctx, s);
  if (s->nq_total == 0) {
    // nothing undecided: every state is in S_{=0} or S_{=1}
    for (int k = 0; k < K; k++) {
      log.status[k] = ST_CONVERGED;
      log.resid[k] = 0.0;
      log.bound[k] = 0.0;
    }
    return;
  }
  if (s->general && o.stop == RP_STOP_CERTIFIED && !s->dominant) {
    set_err(ctx, "a certified stop needs every row strictly diagonally dominant (Varah's bound); use "
                 "RP_STOP_RESIDUAL or RP_STOP_DELTA");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (s->general && tr) {
    set_err(ctx, "the adjoint is defined for Markov chains only");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  if (method != 0 && (o.update != RP_UPDATE_TWO_BUFFER || o.schedule == RP_SCHEDULE_SEGSCAN)) {
    set_err(ctx, "RP_UPDATE_IN_PLACE and RP_SCHEDULE_SEGSCAN are Jacobi variants");
    throw Fail{RP_ERR_INVALID_ARG};
  }
  const int saved_L = s->L;
  s->tiles_on = o.tiling != RP_TILING_OFF;
  // Jacobi variants run on row chunks read from device memory
  s->jvariant = o.update == RP_UPDATE_IN_PLACE ? 1 : o.schedule == RP_SCHEDULE_SEGSCAN ? 2 : 0;
  if (s->jvariant == 2) ensure_erow(ctx, s, tr);
  // row layout of the tiled kernels: 0 = sliced rows, L > 0 = L lanes per row
  const bool f32 = o.precision == RP_FP32_REFINED;
  int layout = s->jvariant ? s->L : o.schedule;
  if (layout < 0) layout = f32 ? tuned_layout<float>(ctx, s, tr) : tuned_layout<double>(ctx, s, tr);
  // sliced rows need the tile kernels and slices that fit 32-bit offsets
  if (layout == 0 && !(s->tiles_on && (f32 ? (tiled<float>(s) && ensure_sliced<float>(ctx, s, tr))
                                           : (tiled<double>(s) && ensure_sliced<double>(ctx, s, tr)))))
    layout = s->L;
  s->sliced = layout == 0;
  if (layout > 0) s->L = layout;
  log.lanes = s->sliced ? 0 : s->L;
  log.panels.assign(K, 0);
  if (s->sliced) {
    const std::vector<int32_t>& np = f32 ? sliced_for<float>(s, tr).npan_h : sliced_for<double>(s, tr).npan_h;
    const rp_system::TileSet& ts = f32 ? s->t32 : s->t64;
    if (!np.empty())
      for (int k = 0; k < K; k++)
        if (ts.inst0_h[k] < ts.inst0_h[k + 1]) log.panels[k] = np[ts.inst0_h[k]];
  }
  struct Restore {
    rp_system* s;
    int L;
    ~Restore() {
      s->L = L;
      s->tiles_on = true;
      s->sliced = false;
      s->jvariant = 0;
    }
  } restore{s, saved_L};

  if (x0_full) HIPCHK(ctx, launch_gather_full<double>(st, s->npad, s->row_state.p, x0_full, s->x64.p));
  else HIPCHK(ctx, hipMemsetAsync(s->x64.p, 0, sizeof(double) * (size_t)s->npad, st));

  if (o.stop == RP_STOP_DELTA) {
    // The paper's algorithms verbatim in FP64: Jacobi stops on max|dx| < tol,
    // BiCGStab once every |s_i| <= tol.
    VecSet<double>& w = s->w64;
    HIPCHK(ctx, w.ensure((size_t)s->npad, &ctx->blocks));
    HIPCHK(ctx, hipMemcpyAsync(w.xa.p, s->x64.p, sizeof(double) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, launch_inner_init(st, K, nullptr, s->nq.p, s->status_in.p, s->iters_in.p, s->counters.p));
    HIPCHK(ctx, launch_fill_f64(st, s->thr_in.p, K, o.tol));
    InnerCfg cfg;
    cfg.method = method;
    cfg.measmode = method == 0 ? MEAS_DELTA : MEAS_S;
    cfg.strict = 1;
    cfg.max_iter = o.max_iter > 0 ? o.max_iter : 10000000;
    cfg.chunk = o.chunk > 0 ? o.chunk : 32;
    cfg.x_zero = false;
    cfg.stall = true;
    HIPCHK(ctx, launch_fill_f64(st, s->sbest.p, K, HUGE_VAL));
    HIPCHK(ctx, hipMemsetAsync(s->sbest_it.p, 0, sizeof(int64_t) * (size_t)K, st));
    run_inner<double>(ctx, s, tr, b64, cfg);
    if (method == 0) HIPCHK(ctx, launch_copy_sel(st, s->ch, w.xa.p, w.xb.p, s->iters_in.p, s->x64.p));
    else HIPCHK(ctx, hipMemcpyAsync(s->x64.p, w.xa.p, sizeof(double) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    std::vector<int32_t> all(K, 1);
    accumulate_inner(ctx, s, log, all);
    std::vector<int32_t> stin(K);
    to_host(ctx, stin.data(), s->status_in.p, K);
    // FP64 residual of the returned iterate, for the report
    HIPCHK(ctx, launch_inner_init(st, K, nullptr, s->nq.p, s->status_out.p, s->outer_it.p, s->counters.p + 1));
    HIPCHK(ctx, launch_residual64(st, s->L, view<double>(s, tr), b64, s->x64.p, s->r64.p, s->ch, s->status_out.p,
                                  s->pa.p));
    HIPCHK(ctx, launch_fin_absmax(st, s->ch, s->pa.p, s->tmp_k.p));
    std::vector<double> rn(K);
    to_host(ctx, rn.data(), s->tmp_k.p, K);
    const std::vector<double>& tbh = tr ? s->tb_tr_h : s->tb_fwd_h;
    const bool have_tb = tr ? s->have_tb_tr : s->have_tb_fwd;
    for (int k = 0; k < K; k++) {
      log.status[k] = (s->nq_h[k] == 0) ? ST_CONVERGED : stin[k];
      log.resid[k] = s->nq_h[k] == 0 ? 0.0 : rn[k];
      log.bound[k] = have_tb ? tbh[k] * log.resid[k] : -1.0;
    }
    return;
  }

  const bool certified = o.stop == RP_STOP_CERTIFIED;
  const double* tb = nullptr;
  if (certified) {
    // keep x64 (starting point) safe while the certificate solve runs
    DBuf<double> keep;
    if (x0_full) {
      dalloc(ctx, keep, (size_t)s->npad);
      HIPCHK(ctx, hipMemcpyAsync(keep.p, s->x64.p, sizeof(double) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    }
    ensure_tbound(ctx, s, tr, method);
    if (x0_full) HIPCHK(ctx, hipMemcpyAsync(s->x64.p, keep.p, sizeof(double) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    else HIPCHK(ctx, hipMemsetAsync(s->x64.p, 0, sizeof(double) * (size_t)s->npad, st));
    tb = tr ? s->tb_tr.p : s->tb_fwd.p;
  }
  if (o.precision == RP_FP32_REFINED) refine<float>(ctx, s, tr, method, b64, certified, o.tol, tb, o, log);
  else refine<double>(ctx, s, tr, method, b64, certified, o.tol, tb, o, log);
}

// Pull-step batches of a search before its states of equal reachability are
// merged (a search that has not settled by then is a deep one).
constexpr int kPlainBatches = 4;

// The two backward searches of Section 2.2 (the second never passes a goal
// state), into reach_goal and, unless prob0_only, reach_s0 (n marks each);
// changed is one device word (the number of the last pull step that marked a
// state).  Chains of at most REACH_RESIDENT_MAX states run the whole search
// in one workgroup, larger ones in pull steps, batches of 8 launches per host
// check (the steps after the fixed point return at once).  With parent and cmark (n words each, or
// null), a search still running after kPlainBatches batches merges the
// states of equal reachability (launch_reach_contract) and continues on the
// classes.  Allocates nothing.
void partition_searches(rp_context* ctx, const rp_chain* chain, const uint8_t* goal_mask, bool prob0_only,
                        uint32_t* reach_goal, uint32_t* reach_s0, int32_t* changed, int32_t* parent,
                        uint32_t* cmark) {
  hipStream_t st = ctx->stream;
  const int64_t n = chain->n;
  auto search = [&](uint32_t* mark, const uint8_t* blocked) {
    if (n <= REACH_RESIDENT_MAX) {
      HIPCHK(ctx, launch_reach_resident(st, n, chain->row_ptr, chain->col, chain->val, blocked, mark));
      return;
    }
    // pull steps in batches; a step that marks nothing has reached the fixed
    // point, which the batch's last step shows when it is not the last step
    // that marked
    const int batch = 8;
    bool merged = false;
    int32_t step = 0;
    HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(changed), 1, 0u));
    for (int b = 0;; b++) {
      if (!merged && parent && cmark && b == kPlainBatches) {
        HIPCHK(ctx, launch_reach_contract(st, n, chain->row_ptr, chain->col, chain->val, blocked, mark, parent,
                                          cmark));
        merged = true;
      }
      for (int i = 0; i < batch; i++) {
        step++;
        if (merged)
          HIPCHK(ctx, launch_reach_step_classes(st, n, chain->row_ptr, chain->col, chain->val, blocked, parent,
                                                cmark, changed, step));
        else
          HIPCHK(ctx, launch_reach_step(st, n, chain->row_ptr, chain->col, chain->val, blocked, mark, changed,
                                        step));
      }
      if (read_i32(ctx, changed) < step) break;
    }
    if (merged) HIPCHK(ctx, launch_classes_expand(st, n, blocked, parent, cmark, mark));
  };
  HIPCHK(ctx, launch_seed_goal(st, n, goal_mask, reach_goal));
  search(reach_goal, nullptr);
  if (!prob0_only) {
    HIPCHK(ctx, launch_seed_complement(st, n, reach_goal, reach_s0));
    search(reach_s0, goal_mask);
  }
}

// Reduced system of a classified chain (s->cls set, flags_sq[i] = 1 for the
// states of S_?): numbering with instance blocks padded to PAD rows, the
// off-diagonal CSR with d = 1 - P(s,s) and b = P(s, S_{=1}) (Section 2.3),
// the chunk and tile layouts.  Shared by rp_precompute and rp_matrix_system.
void assemble_system(rp_context* ctx, rp_system* s, const rp_chain* chain, int32_t* flags_sq_p) {
  hipStream_t st = ctx->stream;
  const int64_t n = chain->n, nnz = chain->nnz;
  const int32_t K = chain->num_instances;
  DBuf<int32_t> rank, scan_tmp;
  // -- reduced numbering with instance blocks padded to PAD rows
  dalloc(ctx, rank, (size_t)n + 1);
  dalloc(ctx, scan_tmp, scan_scratch_elems(n));
  HIPCHK(ctx, launch_scan(st, flags_sq_p, rank.p, n, scan_tmp.p));
  DBuf<int32_t> counts;
  dalloc(ctx, counts, (size_t)K);
  HIPCHK(ctx, launch_inst_counts(st, K, s->inst_off.p, rank.p, counts.p));
  std::vector<int32_t> cnt_h(K);
  to_host(ctx, cnt_h.data(), counts.p, K);
  s->nq_h.resize(K);
  s->roff_h.assign(K + 1, 0);
  for (int k = 0; k < K; k++) {
    s->nq_h[k] = cnt_h[k];
    s->nq_total += cnt_h[k];
    s->roff_h[k + 1] = s->roff_h[k] + ((cnt_h[k] + PAD - 1) / PAD) * PAD;
  }
  s->npad = s->roff_h[K];
  dalloc(ctx, s->roff, (size_t)K + 1);
  to_dev(ctx, s->roff.p, s->roff_h.data(), (size_t)K + 1);
  dalloc(ctx, s->nq, (size_t)K);
  to_dev(ctx, s->nq.p, s->nq_h.data(), (size_t)K);

  const int64_t np = s->npad;
  dalloc(ctx, s->map, (size_t)n);
  dalloc(ctx, s->row_state, (size_t)np);
  if (np > 0) HIPCHK(ctx, hipMemsetAsync(s->row_state.p, 0xFF, sizeof(int32_t) * (size_t)np, st));
  HIPCHK(ctx, launch_map(st, n, s->cls.p, rank.p, s->inst_off.p, K, s->roff.p, s->map.p, s->row_state.p, nullptr));

  // -- reduced system (Section 2.3): d = 1 - P(s,s), b = P(s, S=1), A_off
  DBuf<int32_t> rcnt;
  dalloc(ctx, rcnt, (size_t)np);
  dalloc(ctx, s->d64, (size_t)np);
  dalloc(ctx, s->d32, (size_t)np);
  dalloc(ctx, s->b64, (size_t)np);
  HIPCHK(ctx, launch_row_count(st, np, s->row_state.p, chain->row_ptr, chain->col, chain->val, s->cls.p, rcnt.p,
                               s->d64.p, s->d32.p, s->b64.p, s->general ? 1 : 0));
  dalloc(ctx, s->fwd.rp, (size_t)np + 1);
  DBuf<int32_t> scratch2;
  dalloc(ctx, scratch2, scan_scratch_elems(np));
  HIPCHK(ctx, launch_scan(st, rcnt.p, s->fwd.rp.p, np, scratch2.p));
  int32_t z = 0;
  to_host(ctx, &z, s->fwd.rp.p + np, 1);
  s->z = z;
  {
    // off-diagonal entries per instance (row pointers at the block starts)
    DBuf<int32_t> at;
    dalloc(ctx, at, (size_t)K + 1);
    HIPCHK(ctx, launch_gather_at(st, s->fwd.rp.p, s->roff.p, K + 1, at.p));
    std::vector<int32_t> ath(K + 1);
    to_host(ctx, ath.data(), at.p, (size_t)K + 1);
    s->z_h.resize(K);
    for (int k = 0; k < K; k++) s->z_h[k] = ath[k + 1] - ath[k];
  }
  dalloc(ctx, s->fwd.col, (size_t)z);
  dalloc(ctx, s->fwd.v64, (size_t)z);
  dalloc(ctx, s->fwd.v32, (size_t)z);
  HIPCHK(ctx, launch_fill_rows(st, np, s->row_state.p, chain->row_ptr, chain->col, chain->val, s->cls.p, s->map.p,
                               s->fwd.rp.p, s->fwd.col.p, s->fwd.v64.p, s->fwd.v32.p, s->general ? 1 : 0));

  // keep P's structure for the gradient
  dalloc(ctx, s->prp, (size_t)n + 1);
  dalloc(ctx, s->pcol, (size_t)nnz);
  HIPCHK(ctx, hipMemcpyAsync(s->prp.p, chain->row_ptr, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, st));
  if (nnz > 0)
    HIPCHK(ctx, hipMemcpyAsync(s->pcol.p, chain->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, st));

  // -- work decomposition: chunks of R rows inside each instance block
  const double mean_row = s->nq_total > 0 ? (double)z / (double)s->nq_total : 1.0;
  s->L = auto_lanes(mean_row);
  int64_t R = PAD;
  while (R < 1024 && np / (2 * R) >= 2048) R *= 2;
  s->R = (int)R;
  std::vector<int32_t> row0, nrows, cinst;
  std::vector<int32_t> c0(K + 1, 0);
  for (int k = 0; k < K; k++) {
    c0[k] = (int32_t)row0.size();
    for (int64_t r = s->roff_h[k]; r < s->roff_h[k + 1]; r += R) {
      row0.push_back((int32_t)r);
      nrows.push_back((int32_t)std::min<int64_t>(R, s->roff_h[k + 1] - r));
      cinst.push_back(k);
    }
  }
  c0[K] = (int32_t)row0.size();
  const int32_t nchunk = (int32_t)row0.size();
  dalloc(ctx, s->c_row0, (size_t)nchunk);
  dalloc(ctx, s->c_nrows, (size_t)nchunk);
  dalloc(ctx, s->c_inst, (size_t)nchunk);
  dalloc(ctx, s->c_inst0, (size_t)K + 1);
  to_dev(ctx, s->c_row0.p, row0.data(), (size_t)nchunk);
  to_dev(ctx, s->c_nrows.p, nrows.data(), (size_t)nchunk);
  to_dev(ctx, s->c_inst.p, cinst.data(), (size_t)nchunk);
  to_dev(ctx, s->c_inst0.p, c0.data(), (size_t)K + 1);
  s->chunk_inst_h = cinst;
  s->chunk_c0_h = c0;
  s->ch = Chunks{s->c_row0.p, s->c_nrows.p, s->c_inst.p, s->c_inst0.p, nchunk, K};
  dalloc(ctx, s->fwd.c16, (size_t)z);
  HIPCHK(ctx, launch_col16(st, s->ch, s->roff.p, s->fwd.rp.p, s->fwd.col.p, s->fwd.c16.p));

  // -- LDS tiles for FP64 and FP32 windows; instances too large for a
  // whole-block window get a band sized from their |col - row| histogram
  std::vector<int32_t> hist;
  int64_t maxrows = 0;
  for (int k = 0; k < K; k++) maxrows = std::max<int64_t>(maxrows, s->roff_h[k + 1] - s->roff_h[k]);
  if (maxrows > (int64_t)(TILE_LDS_BYTES / sizeof(double)) / PAD * PAD && z > 0) {
    DBuf<int32_t> dh;
    dalloc(ctx, dh, (size_t)K * 32);
    HIPCHK(ctx, hipMemsetAsync(dh.p, 0, sizeof(int32_t) * (size_t)K * 32, st));
    HIPCHK(ctx, launch_band_hist(st, s->ch, s->fwd.rp.p, s->fwd.col.p, dh.p));
    hist.resize((size_t)K * 32);
    to_host(ctx, hist.data(), dh.p, (size_t)K * 32);
  }
  build_tiles(ctx, s, s->t64, sizeof(double), 1, hist);
  build_tiles(ctx, s, s->t32, sizeof(float), 2, hist);
  build_resident(ctx, s, s->res64, sizeof(double));
  build_resident(ctx, s, s->res32, sizeof(float));
  s->ntile_max = std::max(s->t64.ok ? s->t64.tl.ntile : 0, s->t32.ok ? s->t32.tl.ntile : 0);
  HIPCHK(ctx, hipStreamSynchronize(st));
}

int finish(rp_context* ctx, rp_system* s, const SolveLog& log, rp_solve_info* info) {
  int worst = RP_OK;
  for (int k = 0; k < s->K; k++) {
    const int code = status_to_rp(log.status[k]);
    if (severity(code) > severity(worst)) worst = code;
    if (info) {
      info[k].iterations = log.iters[k];
      info[k].refinements = log.refinements[k];
      info[k].final_delta = log.delta[k];
      info[k].residual_inf = log.resid[k];
      info[k].error_bound = log.bound[k];
      info[k].status = code;
      info[k].lanes = log.lanes;
      info[k].panels = log.panels.empty() ? 0 : log.panels[k];
      info[k].reserved = 0;
    }
  }
  if (worst != RP_OK) {
    int bad = 0;
    for (int k = 0; k < s->K; k++)
      if (status_to_rp(log.status[k]) == worst) { bad = k; break; }
    set_err(ctx, "instance %d: %s", bad,
            log.status[bad] == ST_STALLED
                ? "the stopping measure stopped falling above the tolerance (no halving of its best value in "
                  "65,536 iterations or in as many as it took to reach it): the tolerance is below what the "
                  "arithmetic reaches"
            : worst == RP_ERR_NOT_CONVERGED ? "iteration cap reached before the stopping rule held"
            : worst == RP_ERR_BREAKDOWN   ? "BiCGStab breakdown"
                                          : "non-finite value during the iteration");
  }
  return worst;
}

// Strongly connected components of the forward reduced graph (coloring
// algorithm, see the kernels).  Each "until stable" loop runs pairs of
// ascending and descending passes and stops at a host check after which
// none of its passes changed anything.  Every round assigns at least the component of the
// largest unassigned row (its color is its own index), so the rounds end.
void scc_decompose(rp_context* ctx, rp_system* s) {
  if (s->have_scc) return;
  hipStream_t st = ctx->stream;
  const int64_t n = s->npad;
  const MatView<double> m = view<double>(s, false);
  dalloc(ctx, s->scc_comp, (size_t)std::max<int64_t>(n, 1));
  dalloc(ctx, s->scc_lvl, (size_t)std::max<int64_t>(n, 1));
  dalloc(ctx, s->scc_minrow, (size_t)std::max<int64_t>(n, 1));
  dalloc(ctx, s->scc_size, (size_t)std::max<int64_t>(n, 1));
  DBuf<int32_t> color, mark, flag;
  dalloc(ctx, color, (size_t)std::max<int64_t>(n, 1));
  dalloc(ctx, mark, (size_t)std::max<int64_t>(n, 1));
  dalloc(ctx, flag, 4);
  // Between two host reads of the change flag, 1, 2, 4, ... up to 16 pairs
  // of passes while the loop keeps changing (a long chain of dependencies
  // then costs few round trips); the loop ends at a read after which none of
  // the passes since the previous read changed anything.
  auto until_stable = [&](auto&& pass) {
    int pairs = 1;
    while (true) {
      HIPCHK(ctx, hipMemsetAsync(flag.p, 0, sizeof(int32_t), st));
      for (int i = 0; i < pairs; i++) {
        HIPCHK(ctx, pass(0));
        HIPCHK(ctx, pass(1));
      }
      if (read_i32(ctx, flag.p) == 0) break;
      pairs = std::min(2 * pairs, 16);
    }
  };
  HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(s->scc_comp.p), n, 0xFFFFFFFFu));
  int rounds = 0;
  while (n > 0) {
    until_stable([&](int dir) { return launch_scc_trim(st, n, m.rp, m.col, m.val, s->scc_comp.p, dir, flag.p); });
    HIPCHK(ctx, launch_scc_color_init(st, n, s->scc_comp.p, color.p, mark.p));
    until_stable([&](int dir) {
      return launch_scc_color(st, n, m.rp, m.col, m.val, s->scc_comp.p, color.p, dir, flag.p);
    });
    HIPCHK(ctx, launch_scc_root(st, n, s->scc_comp.p, color.p, mark.p));
    until_stable([&](int dir) {
      return launch_scc_mark(st, n, m.rp, m.col, m.val, s->scc_comp.p, color.p, mark.p, dir, flag.p);
    });
    HIPCHK(ctx, hipMemsetAsync(flag.p + 1, 0, sizeof(int32_t), st));
    HIPCHK(ctx, launch_scc_assign(st, n, s->scc_comp.p, color.p, mark.p, flag.p + 1));
    rounds++;
    if (read_i32(ctx, flag.p + 1) == 0) break;
  }
  HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(s->scc_minrow.p), n, 0x7FFFFFFFu));
  HIPCHK(ctx, hipMemsetAsync(s->scc_size.p, 0, sizeof(int32_t) * (size_t)n, st));
  HIPCHK(ctx, hipMemsetAsync(s->scc_lvl.p, 0, sizeof(int32_t) * (size_t)n, st));
  HIPCHK(ctx, hipMemsetAsync(flag.p, 0, sizeof(int32_t) * 4, st));
  HIPCHK(ctx, launch_scc_stats(st, n, s->scc_comp.p, s->row_state.p, s->scc_minrow.p, s->scc_size.p, flag.p));
  int32_t cnt[3];
  to_host(ctx, cnt, flag.p, 3);
  until_stable([&](int dir) {
    return launch_scc_level(st, n, m.rp, m.col, m.val, s->scc_comp.p, s->scc_lvl.p, dir, flag.p);
  });
  rp_scc_info& c = s->scc_counts;
  c = rp_scc_info{};
  c.components = cnt[0];
  c.cyclic_components = cnt[1];
  c.largest = cnt[2];
  c.rounds = rounds;
  s->have_scc = true;
}

// Reduced rows sorted by level and, inside a level, one-state components
// first (stable: ascending rows inside each part); count[2 l] rows of
// one-state components of level l, count[2 l + 1] rows of larger ones.
struct SccLevels {
  DBuf<int32_t> rows;
  std::vector<int32_t> count;
};

void scc_levels(rp_context* ctx, rp_system* s, SccLevels& L) {
  hipStream_t st = ctx->stream;
  const int64_t n = s->npad;
  DBuf<int32_t> key, rowid, key2, misc;
  dalloc(ctx, key, (size_t)n);
  dalloc(ctx, rowid, (size_t)n);
  dalloc(ctx, key2, (size_t)n);
  dalloc(ctx, L.rows, (size_t)n);
  dalloc(ctx, misc, 2);
  HIPCHK(ctx, hipMemsetAsync(misc.p, 0, sizeof(int32_t) * 2, st));
  HIPCHK(ctx, launch_scc_rowlevel(st, n, s->scc_comp.p, s->scc_lvl.p, s->scc_size.p, key.p, rowid.p, misc.p,
                                  misc.p + 1));
  int32_t mx[2];
  to_host(ctx, mx, misc.p, 2);
  const int32_t nl = mx[0] + 1;
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) <= 2 * (int64_t)mx[0] + 1) bits++;
  size_t tb = 0;
  HIPCHK(ctx, launch_sort_by_key(st, key.p, rowid.p, key2.p, L.rows.p, n, bits, nullptr, &tb));
  DBuf<uint8_t> temp;
  dalloc(ctx, temp, std::max<size_t>(tb, 1));
  HIPCHK(ctx, launch_sort_by_key(st, key.p, rowid.p, key2.p, L.rows.p, n, bits, temp.p, &tb));
  DBuf<int32_t> cnt;
  dalloc(ctx, cnt, 2 * (size_t)nl);
  HIPCHK(ctx, hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * 2 * (size_t)nl, st));
  HIPCHK(ctx, launch_scc_levelcount(st, n, key.p, cnt.p));
  L.count.resize(2 * (size_t)nl);
  to_host(ctx, L.count.data(), cnt.p, 2 * (size_t)nl);
  s->scc_counts.levels = nl;
}

// Level-by-level solve into s->x64 (see rp_scc_solve).
void scc_solve_levels(rp_context* ctx, rp_system* s, const rp_opts& o, rp_scc_info& out) {
  hipStream_t st = ctx->stream;
  SccLevels L;
  scc_levels(ctx, s, L);
  const MatView<double> m = view<double>(s, false);
  DBuf<unsigned long long> dmax;
  dalloc(ctx, dmax, 1);
  if (o.x0) HIPCHK(ctx, launch_gather_full<double>(st, s->npad, s->row_state.p, o.x0, s->x64.p));
  else HIPCHK(ctx, hipMemsetAsync(s->x64.p, 0, sizeof(double) * (size_t)s->npad, st));
  const double tol_in = o.tol / 100.0;
  const int64_t cap = o.max_iter > 0 ? o.max_iter : 10000000;
  constexpr int kBatch = 16;  // sweeps between two reads of the largest change
  int64_t off = 0;
  out = s->scc_counts;
  for (size_t l = 0; l < L.count.size(); l++) {
    const int32_t nr = L.count[l];
    const int32_t* rows = L.rows.p + off;
    off += nr;
    if (nr == 0) continue;
    if (l % 2 == 0) {
      // one-state components: every dependency lies in a solved level, so
      // one substitution pass
      HIPCHK(ctx, launch_scc_rows(st, rows, nr, m, s->b64.p, s->x64.p, dmax.p));
      out.substitution_levels++;
      out.substitution_rows += nr;
      continue;
    }
    out.jacobi_levels++;
    out.jacobi_rows += nr;
    int64_t sweeps = 0;
    while (sweeps < cap) {
      const int64_t nb = std::min<int64_t>(kBatch, cap - sweeps);
      for (int64_t i = 0; i < nb; i++) {
        if (i == nb - 1) HIPCHK(ctx, hipMemsetAsync(dmax.p, 0, sizeof(unsigned long long), st));
        HIPCHK(ctx, launch_scc_rows(st, rows, nr, m, s->b64.p, s->x64.p, dmax.p));
      }
      sweeps += nb;
      unsigned long long bits = 0;
      to_host(ctx, &bits, dmax.p, 1);
      double d;
      std::memcpy(&d, &bits, sizeof d);
      if (!(d > tol_in)) break;
    }
    out.jacobi_sweeps += sweeps;
  }
}

int solve_entry(rp_context* ctx, rp_system* s, const rp_opts* opts, double* x_out, rp_solve_info* info,
                int method) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s || !x_out) {
    set_err(ctx, "null system or x_out");
    return RP_ERR_INVALID_ARG;
  }
  try {
    rp_opts o;
    if (opts) o = *opts; else rp_opts_default(&o);
    check_opts(ctx, &o);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    SolveLog log(s->K);
    solve_core(ctx, s, false, method, s->b64.p, o, o.x0, log);
    HIPCHK(ctx, launch_scatter_full(ctx->stream, s->n, s->cls.p, s->map.p, s->inst_off.p, s->K, s->x64.p,
                                    s->x64.p, nullptr, 1.0, x_out));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return finish(ctx, s, log, info);
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int rp_scc(rp_context* ctx, rp_system* s, int32_t* label_out, int32_t* level_out, rp_scc_info* info) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s) {
    set_err(ctx, "null system");
    return RP_ERR_INVALID_ARG;
  }
  if (s->general) {
    set_err(ctx, "components are defined here for Markov-chain systems (edges A > 0)");
    return RP_ERR_INVALID_ARG;
  }
  try {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    scc_decompose(ctx, s);
    SccLevels L;  // (for the level count)
    scc_levels(ctx, s, L);
    if (label_out || level_out)
      HIPCHK(ctx, launch_scc_out(ctx->stream, s->n, s->map.p, s->scc_comp.p, s->scc_minrow.p, s->scc_lvl.p,
                                 s->row_state.p, label_out, level_out));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (info) *info = s->scc_counts;
    return RP_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

int rp_scc_solve(rp_context* ctx, rp_system* s, const rp_opts* opts, double* x_out, rp_solve_info* info,
                 rp_scc_info* scc_info) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s || !x_out) {
    set_err(ctx, "null system or x_out");
    return RP_ERR_INVALID_ARG;
  }
  if (s->general) {
    set_err(ctx, "components are defined here for Markov-chain systems (edges A > 0)");
    return RP_ERR_INVALID_ARG;
  }
  try {
    rp_opts o;
    if (opts) o = *opts; else rp_opts_default(&o);
    check_opts(ctx, &o);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ensure_work(ctx, s);
    scc_decompose(ctx, s);
    rp_scc_info si{};
    scc_solve_levels(ctx, s, o, si);
    // the level solution, as a full vector, starts the ordinary refinement
    DBuf<double> xf;
    dalloc(ctx, xf, (size_t)std::max<int64_t>(s->n, 1));
    HIPCHK(ctx, launch_scatter_full(st, s->n, s->cls.p, s->map.p, s->inst_off.p, s->K, s->x64.p, s->x64.p, nullptr,
                                    1.0, xf.p));
    o.update = RP_UPDATE_TWO_BUFFER;
    if (o.schedule == RP_SCHEDULE_SEGSCAN) o.schedule = -1;
    SolveLog log(s->K);
    solve_core(ctx, s, false, 0, s->b64.p, o, xf.p, log);
    HIPCHK(ctx, launch_scatter_full(st, s->n, s->cls.p, s->map.p, s->inst_off.p, s->K, s->x64.p, s->x64.p, nullptr,
                                    1.0, x_out));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (scc_info) *scc_info = si;
    return finish(ctx, s, log, info);
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

void rp_opts_default(rp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-10;
  o->stop = RP_STOP_CERTIFIED;
  o->precision = RP_FP64;
  o->max_iter = 10000000;
  o->inner_tol = 1e-2;
  o->max_refine = 60;
  o->chunk = 32;
  o->schedule = -1;
  o->x0 = nullptr;
}

int rp_context_create(rp_context** out, int device, void* stream) {
  if (!out) return RP_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return RP_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return RP_ERR_HIP;
  rp_context* c = new (std::nothrow) rp_context();
  if (!c) return RP_ERR_OOM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->scratch = scratch_address(device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->cus = prop.multiProcessorCount;
  void* fh = nullptr;
  if (hipHostMalloc(&fh, 2 * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
    void* fd = nullptr;
    if (hipHostGetDevicePointer(&fd, fh, 0) == hipSuccess) {
      c->flag_h = static_cast<int32_t*>(fh);
      c->flag_d = static_cast<int32_t*>(fd);
      c->flag_h[0] = 0;
      c->flag_h[1] = 0;
    } else {
      (void)hipHostFree(fh);
    }
  }
  (void)hipGetLastError();
  *out = c;
  return RP_OK;
}

int rp_context_destroy(rp_context* ctx) {
  delete ctx;
  return RP_OK;
}

const char* rp_last_error(const rp_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int rp_precompute(rp_context* ctx, const rp_chain* chain, const uint8_t* goal_mask, uint32_t flags,
                  double rowsum_tol, uint8_t* class_out, rp_system** sys_out) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!chain || !goal_mask || !sys_out || !chain->inst_state_offset || !chain->row_ptr ||
      (chain->nnz > 0 && (!chain->col || !chain->val))) {
    set_err(ctx, "null argument");
    return RP_ERR_INVALID_ARG;
  }
  *sys_out = nullptr;
  if ((flags & ~RP_PROB0_ONLY) != 0) {
    set_err(ctx, "unknown flags 0x%x", flags);
    return RP_ERR_INVALID_ARG;
  }
  const int64_t n = chain->n, nnz = chain->nnz;
  const int32_t K = chain->num_instances;
  if (n < 1 || nnz < 0 || K < 1 || K > n) {
    set_err(ctx, "bad sizes (n=%lld, nnz=%lld, K=%d)", (long long)n, (long long)nnz, K);
    return RP_ERR_INVALID_ARG;
  }
  if (n >= (int64_t)INT32_MAX - 2 * PAD * (int64_t)K || nnz >= (int64_t)INT32_MAX) {
    set_err(ctx, "chain too large for 32-bit indices (n=%lld, nnz=%lld)", (long long)n, (long long)nnz);
    return RP_ERR_TOO_LARGE;
  }
  const int64_t* off = chain->inst_state_offset;
  if (off[0] != 0 || off[K] != n) {
    set_err(ctx, "inst_state_offset must start at 0 and end at n");
    return RP_ERR_INVALID_ARG;
  }
  for (int k = 0; k < K; k++)
    if (off[k + 1] <= off[k]) {
      set_err(ctx, "inst_state_offset must be strictly increasing (instance %d)", k);
      return RP_ERR_INVALID_ARG;
    }
  const double tol = rowsum_tol > 0 ? rowsum_tol : 1e-12;
  rp_system* s = new (std::nothrow) rp_system();
  if (!s) return RP_ERR_OOM;
  try {
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    s->K = K;
    s->n = n;
    s->nnz = nnz;
    s->inst_off_h.assign(off, off + K + 1);
    dalloc(ctx, s->inst_off, (size_t)K + 1);
    to_dev(ctx, s->inst_off.p, off, (size_t)K + 1);

    // -- validation (Section 2: a row-stochastic transition function)
    int32_t ends[2];
    to_host(ctx, &ends[0], chain->row_ptr, 1);
    to_host(ctx, &ends[1], chain->row_ptr + n, 1);
    if (ends[0] != 0 || ends[1] != nnz) {
      set_err(ctx, "row %lld: %s (row_ptr[0] = %d, row_ptr[n] = %d, nnz = %lld)", (long long)n, reason_text(1),
              ends[0], ends[1], (long long)nnz);
      throw Fail{RP_ERR_BAD_CHAIN};
    }
    {
      DBuf<unsigned long long> bad;
      dalloc(ctx, bad, 1);
      HIPCHK(ctx, hipMemsetAsync(bad.p, 0xFF, sizeof(unsigned long long), st));
      HIPCHK(ctx, launch_validate(st, n, nnz, chain->row_ptr, chain->col, chain->val, s->inst_off.p, K, tol, 0, bad.p));
      unsigned long long key = 0;
      to_host(ctx, &key, bad.p, 1);
      if (key != ~0ull) {
        set_err(ctx, "row %lld: %s", (long long)(key >> 8), reason_text((unsigned)(key & 0xFF)));
        throw Fail{RP_ERR_BAD_CHAIN};
      }
    }

    // -- partition (Section 2.2)
    DBuf<uint32_t> reach_goal, reach_s0;
    DBuf<int32_t> changed;
    dalloc(ctx, reach_goal, (size_t)n);
    dalloc(ctx, changed, 1);
    const bool prob0_only = (flags & RP_PROB0_ONLY) != 0;
    if (!prob0_only) dalloc(ctx, reach_s0, (size_t)n);
    DBuf<int32_t> uf_parent;
    DBuf<uint32_t> uf_cmark;
    if (n > REACH_RESIDENT_MAX) {
      dalloc(ctx, uf_parent, (size_t)n);
      dalloc(ctx, uf_cmark, (size_t)n);
    }
    partition_searches(ctx, chain, goal_mask, prob0_only, reach_goal.p, reach_s0.p, changed.p, uf_parent.p,
                       uf_cmark.p);
    DBuf<int32_t> flags_sq;
    dalloc(ctx, s->cls, (size_t)n);
    dalloc(ctx, flags_sq, (size_t)n);
    HIPCHK(ctx, launch_classes(st, n, reach_goal.p, prob0_only ? nullptr : reach_s0.p, goal_mask, prob0_only ? 1 : 0,
                               s->cls.p, class_out, flags_sq.p));
    reach_goal.release();
    reach_s0.release();

    assemble_system(ctx, s, chain, flags_sq.p);
    *sys_out = s;
    return RP_OK;
  } catch (const Fail& f) {
    delete s;
    return f.code;
  } catch (...) {
    delete s;
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

int rp_matrix_system(rp_context* ctx, int32_t num_instances, const int64_t* inst_row_offset, int64_t n, int64_t nnz,
                     const int32_t* row_ptr, const int32_t* col, const double* val, const double* rhs,
                     rp_system** sys_out) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!sys_out || !inst_row_offset || !row_ptr || !rhs || (nnz > 0 && (!col || !val))) {
    set_err(ctx, "null argument");
    return RP_ERR_INVALID_ARG;
  }
  *sys_out = nullptr;
  const int32_t K = num_instances;
  if (n < 1 || nnz < 0 || K < 1 || K > n) {
    set_err(ctx, "bad sizes (n=%lld, nnz=%lld, K=%d)", (long long)n, (long long)nnz, K);
    return RP_ERR_INVALID_ARG;
  }
  if (n >= (int64_t)INT32_MAX - 2 * PAD * (int64_t)K || nnz >= (int64_t)INT32_MAX) {
    set_err(ctx, "matrix too large for 32-bit indices (n=%lld, nnz=%lld)", (long long)n, (long long)nnz);
    return RP_ERR_TOO_LARGE;
  }
  const int64_t* off = inst_row_offset;
  if (off[0] != 0 || off[K] != n) {
    set_err(ctx, "inst_row_offset must start at 0 and end at n");
    return RP_ERR_INVALID_ARG;
  }
  for (int k = 0; k < K; k++)
    if (off[k + 1] <= off[k]) {
      set_err(ctx, "inst_row_offset must be strictly increasing (instance %d)", k);
      return RP_ERR_INVALID_ARG;
    }
  rp_system* s = new (std::nothrow) rp_system();
  if (!s) return RP_ERR_OOM;
  try {
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    s->K = K;
    s->n = n;
    s->nnz = nnz;
    s->general = true;
    s->inst_off_h.assign(off, off + K + 1);
    dalloc(ctx, s->inst_off, (size_t)K + 1);
    to_dev(ctx, s->inst_off.p, off, (size_t)K + 1);
    int32_t ends[2];
    to_host(ctx, &ends[0], row_ptr, 1);
    to_host(ctx, &ends[1], row_ptr + n, 1);
    if (ends[0] != 0 || ends[1] != nnz) {
      set_err(ctx, "row %lld: %s (row_ptr[0] = %d, row_ptr[n] = %d, nnz = %lld)", (long long)n, reason_text(1),
              ends[0], ends[1], (long long)nnz);
      throw Fail{RP_ERR_BAD_CHAIN};
    }
    {
      DBuf<unsigned long long> bad;
      dalloc(ctx, bad, 1);
      HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(bad.p), 2, 0xFFFFFFFFu));
      HIPCHK(ctx, launch_validate(st, n, nnz, row_ptr, col, val, s->inst_off.p, K, 0.0, 1, bad.p));
      unsigned long long key = 0;
      to_host(ctx, &key, bad.p, 1);
      if (key != ~0ull) {
        set_err(ctx, "row %lld: %s", (long long)(key >> 8), reason_text((unsigned)(key & 0xFF)));
        throw Fail{RP_ERR_BAD_CHAIN};
      }
    }
    // the solvers' form: P' = I - A on the same structure, every row undecided
    DBuf<double> pval;
    dalloc(ctx, pval, (size_t)std::max<int64_t>(nnz, 1));
    HIPCHK(ctx, launch_identity_minus(st, n, row_ptr, col, val, pval.p));
    dalloc(ctx, s->cls, (size_t)n);
    HIPCHK(ctx, hipMemsetAsync(s->cls.p, RP_SQ, (size_t)n, st));
    DBuf<int32_t> flags_sq;
    dalloc(ctx, flags_sq, (size_t)n);
    HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(flags_sq.p), n, 1u));
    const rp_chain pc{K, off, n, nnz, row_ptr, col, pval.p};
    assemble_system(ctx, s, &pc, flags_sq.p);
    // right-hand side (no S_{=1} columns: b was assembled as 0)
    HIPCHK(ctx, launch_gather_full<double>(st, s->npad, s->row_state.p, rhs, s->b64.p));
    // certificate factor: Varah's bound per instance (dominant rows only)
    ensure_work(ctx, s);
    HIPCHK(ctx, launch_inv_gap(st, s->npad, s->row_state.p, s->fwd.rp.p, s->fwd.v64.p, s->d64.p, s->r64.p));
    HIPCHK(ctx, launch_absmax(st, s->r64.p, s->ch, s->pa.p));
    dalloc(ctx, s->tb_fwd, (size_t)K);
    HIPCHK(ctx, launch_fin_absmax(st, s->ch, s->pa.p, s->tb_fwd.p));
    s->tb_fwd_h.resize(K);
    to_host(ctx, s->tb_fwd_h.data(), s->tb_fwd.p, K);
    for (int k = 0; k < K; k++)
      if (!std::isfinite(s->tb_fwd_h[k])) s->dominant = false;
    s->have_tb_fwd = s->dominant;
    HIPCHK(ctx, hipStreamSynchronize(st));
    *sys_out = s;
    return RP_OK;
  } catch (const Fail& f) {
    delete s;
    return f.code;
  } catch (...) {
    delete s;
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

int rp_classify_noalloc(rp_context* ctx, const rp_chain* chain, const uint8_t* goal_mask, uint32_t flags,
                        double rowsum_tol, uint8_t* class_out) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!chain || !goal_mask || !class_out || !chain->inst_state_offset || !chain->row_ptr ||
      (chain->nnz > 0 && (!chain->col || !chain->val))) {
    set_err(ctx, "null argument");
    return RP_ERR_INVALID_ARG;
  }
  if ((flags & ~RP_PROB0_ONLY) != 0) {
    set_err(ctx, "unknown flags 0x%x", flags);
    return RP_ERR_INVALID_ARG;
  }
  const int64_t n = chain->n, nnz = chain->nnz;
  const int32_t K = chain->num_instances;
  if (n < 1 || nnz < 0 || K < 1 || K > n) {
    set_err(ctx, "bad sizes (n=%lld, nnz=%lld, K=%d)", (long long)n, (long long)nnz, K);
    return RP_ERR_INVALID_ARG;
  }
  if (n > kNoAllocMaxStates || nnz >= (int64_t)INT32_MAX) {
    set_err(ctx, "rp_classify_noalloc handles at most %lld states and 2^31-1 transitions (n=%lld, nnz=%lld)",
            (long long)kNoAllocMaxStates, (long long)n, (long long)nnz);
    return RP_ERR_TOO_LARGE;
  }
  const int64_t* off = chain->inst_state_offset;
  if (off[0] != 0 || off[K] != n) {
    set_err(ctx, "inst_state_offset must start at 0 and end at n");
    return RP_ERR_INVALID_ARG;
  }
  for (int k = 0; k < K; k++)
    if (off[k + 1] <= off[k]) {
      set_err(ctx, "inst_state_offset must be strictly increasing (instance %d)", k);
      return RP_ERR_INVALID_ARG;
    }
  if (!ctx->scratch || !ctx->flag_h) {
    set_err(ctx, "context has no no-allocation working memory or host-mapped status word");
    return RP_ERR_HIP;
  }
  const double tol = rowsum_tol > 0 ? rowsum_tol : 1e-12;
  try {
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    unsigned char* base = ctx->scratch;
    unsigned long long* bad = reinterpret_cast<unsigned long long*>(base);
    int32_t* changed = reinterpret_cast<int32_t*>(base + 8);
    int64_t* inst_off = reinterpret_cast<int64_t*>(base + 16);
    uint32_t* reach_goal = reinterpret_cast<uint32_t*>(base + kScratchHead);
    uint32_t* reach_s0 = reach_goal + n;
    // -- validation (Section 2), as rp_precompute
    const int32_t e0 = read_i32(ctx, chain->row_ptr), e1 = read_i32(ctx, chain->row_ptr + n);
    if (e0 != 0 || e1 != nnz) {
      set_err(ctx, "row %lld: %s (row_ptr[0] = %d, row_ptr[n] = %d, nnz = %lld)", (long long)n, reason_text(1), e0, e1,
              (long long)nnz);
      throw Fail{RP_ERR_BAD_CHAIN};
    }
    HIPCHK(ctx, hipMemcpyAsync(inst_off, off, sizeof(int64_t) * (size_t)(K + 1), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, launch_fill_u32(st, reinterpret_cast<uint32_t*>(bad), 2, 0xFFFFFFFFu));
    HIPCHK(ctx, launch_validate(st, n, nnz, chain->row_ptr, chain->col, chain->val, inst_off, K, tol, 0, bad));
    const uint32_t klo = (uint32_t)read_i32(ctx, reinterpret_cast<const int32_t*>(bad));
    const uint32_t khi = (uint32_t)read_i32(ctx, reinterpret_cast<const int32_t*>(bad) + 1);
    const unsigned long long key = ((unsigned long long)khi << 32) | klo;
    if (key != ~0ull) {
      set_err(ctx, "row %lld: %s", (long long)(key >> 8), reason_text((unsigned)(key & 0xFF)));
      throw Fail{RP_ERR_BAD_CHAIN};
    }
    // -- partition (Section 2.2)
    const bool prob0_only = (flags & RP_PROB0_ONLY) != 0;
    partition_searches(ctx, chain, goal_mask, prob0_only, reach_goal, reach_s0, changed, nullptr, nullptr);
    HIPCHK(ctx, launch_classes(st, n, reach_goal, prob0_only ? nullptr : reach_s0, goal_mask, prob0_only ? 1 : 0,
                               class_out, nullptr, nullptr));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return RP_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

int rp_system_destroy(rp_system* sys) {
  delete sys;
  return RP_OK;
}

int rp_system_sizes(const rp_system* s, int64_t* K, int64_t* n, int64_t* nq, int64_t* z) {
  if (!s) return RP_ERR_INVALID_ARG;
  if (K) *K = s->K;
  if (n) *n = s->n;
  if (nq) *nq = s->nq_total;
  if (z) *z = s->z;
  return RP_OK;
}

int rp_system_instance_sizes(const rp_system* s, int64_t* nq_out) {
  if (!s || !nq_out) return RP_ERR_INVALID_ARG;
  for (int k = 0; k < s->K; k++) nq_out[k] = s->nq_h[k];
  return RP_OK;
}

int rp_system_export(rp_context* ctx, const rp_system* s, int32_t* row_ptr, int32_t* col, double* val,
                     double* diag, double* rhs) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s) return RP_ERR_INVALID_ARG;
  try {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    rp_system* m = const_cast<rp_system*>(s);
    const size_t np = (size_t)s->npad, z = (size_t)s->z;
    std::vector<int32_t> rp(np + 1), cl(z), rs(np);
    std::vector<double> v(z), d(np), b(np);
    to_host(ctx, rp.data(), m->fwd.rp.p, np + 1);
    to_host(ctx, cl.data(), m->fwd.col.p, z);
    to_host(ctx, v.data(), m->fwd.v64.p, z);
    to_host(ctx, d.data(), m->d64.p, np);
    to_host(ctx, b.data(), m->b64.p, np);
    to_host(ctx, rs.data(), m->row_state.p, np);
    // padded row -> compact row
    std::vector<int32_t> comp(np, -1);
    int32_t next = 0;
    for (size_t r = 0; r < np; r++)
      if (rs[r] >= 0) comp[r] = next++;
    std::vector<int32_t> crp(1, 0), ccol;
    std::vector<double> cval, cd, cb;
    for (size_t r = 0; r < np; r++) {
      if (rs[r] < 0) continue;
      for (int32_t k = rp[r]; k < rp[r + 1]; k++) {
        ccol.push_back(comp[cl[k]]);
        cval.push_back(v[k]);
      }
      crp.push_back((int32_t)ccol.size());
      cd.push_back(d[r]);
      cb.push_back(b[r]);
    }
    if (row_ptr) to_dev(ctx, row_ptr, crp.data(), crp.size());
    if (col) to_dev(ctx, col, ccol.data(), ccol.size());
    if (val) to_dev(ctx, val, cval.data(), cval.size());
    if (diag) to_dev(ctx, diag, cd.data(), cd.size());
    if (rhs) to_dev(ctx, rhs, cb.data(), cb.size());
    return RP_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int rp_profile_enable(rp_context* ctx, int enable) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  if (!ctx->pend.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    prof_resolve(ctx);
  }
  for (auto& st : ctx->stat) st = ProfStat{};
  ctx->prof = enable != 0;
  return RP_OK;
}

int rp_profile_read(rp_context* ctx, int kernel, int64_t* launches, double* total_ms, double* alg_bytes) {
  if (!ctx || kernel < 0 || kernel >= RP_PROF_NKERNELS) return RP_ERR_INVALID_ARG;
  if (!ctx->pend.empty()) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return RP_ERR_HIP;
    prof_resolve(ctx);
  }
  if (launches) *launches = ctx->stat[kernel].launches;
  if (total_ms) *total_ms = ctx->stat[kernel].ms;
  if (alg_bytes) *alg_bytes = ctx->stat[kernel].bytes;
  return RP_OK;
}

int rp_jacobi(rp_context* ctx, rp_system* sys, const rp_opts* opts, double* x_out, rp_solve_info* info) {
  return solve_entry(ctx, sys, opts, x_out, info, 0);
}

int rp_bicgstab(rp_context* ctx, rp_system* sys, const rp_opts* opts, double* x_out, rp_solve_info* info) {
  return solve_entry(ctx, sys, opts, x_out, info, 1);
}

int rp_solve_rhs(rp_context* ctx, rp_system* s, int method, const double* rhs, const rp_opts* opts,
                 double* y_out, rp_solve_info* info) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s || !rhs || !y_out || (method != 0 && method != 1)) {
    set_err(ctx, "null system, rhs or y_out, or method not 0/1");
    return RP_ERR_INVALID_ARG;
  }
  try {
    rp_opts o;
    if (opts) o = *opts; else rp_opts_default(&o);
    check_opts(ctx, &o);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ensure_work(ctx, s);
    // right-hand side restricted to S_?, in the padded reduced layout (the
    // solve keeps its own copy; r64 is its residual workspace)
    DBuf<double> c;
    dalloc(ctx, c, (size_t)s->npad);
    HIPCHK(ctx, launch_gather_full<double>(st, s->npad, s->row_state.p, rhs, c.p));
    SolveLog log(s->K);
    solve_core(ctx, s, false, method, c.p, o, o.x0, log);
    HIPCHK(ctx, launch_scatter_full(st, s->n, s->cls.p, s->map.p, s->inst_off.p, s->K, s->x64.p, s->x64.p, nullptr,
                                    0.0, y_out));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return finish(ctx, s, log, info);
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

int rp_adjoint(rp_context* ctx, rp_system* s, int method, const double* x, const double* seed,
               const rp_opts* opts, double* lambda_out, double* grad_val_out, rp_solve_info* info) {
  if (!ctx) return RP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!s || !x || !seed || (method != 0 && method != 1)) {
    set_err(ctx, "null system, x or seed, or method not 0/1");
    return RP_ERR_INVALID_ARG;
  }
  try {
    rp_opts o;
    if (opts) o = *opts; else rp_opts_default(&o);
    o.x0 = nullptr;
    check_opts(ctx, &o);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ensure_work(ctx, s);
    if (s->nq_total > 0) ensure_transpose(ctx, s);
    // right-hand side: the seed restricted to S_?, in the padded reduced layout
    HIPCHK(ctx, launch_gather_full<double>(st, s->npad, s->row_state.p, seed, s->r64.p));
    DBuf<double> rhs;
    dalloc(ctx, rhs, (size_t)s->npad);
    HIPCHK(ctx, hipMemcpyAsync(rhs.p, s->r64.p, sizeof(double) * (size_t)s->npad, hipMemcpyDeviceToDevice, st));
    SolveLog log(s->K);
    solve_core(ctx, s, true, method, rhs.p, o, nullptr, log);
    if (lambda_out)
      HIPCHK(ctx, launch_scatter_full(st, s->n, s->cls.p, s->map.p, s->inst_off.p, s->K, s->x64.p, s->x64.p, nullptr,
                                      0.0, lambda_out));
    if (grad_val_out)
      HIPCHK(ctx, launch_gradient(st, s->n, s->prp.p, s->pcol.p, s->cls.p, s->map.p, s->x64.p, x, grad_val_out));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return finish(ctx, s, log, info);
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    set_err(ctx, "internal error");
    return RP_ERR_HIP;
  }
}

}  // extern "C"
