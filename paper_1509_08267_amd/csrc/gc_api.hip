// gc_api.hip -- the C ABI of libgc (declared in include/gc.h): handle
// management, argument checks, the round drivers and result read-back.
//
// Round drivers (GC_OPT_MODE):
//   GRAPH       (default) rounds run as captured hipGraphs of K rounds each
//               (speculate + detect launches with a device-side round base),
//               so back-to-back kernels need no host launch per round.  The
//               first call on a handle learns the round count R with one
//               4-byte read-back per chunk; because R is a function of the
//               (unchanged) graph alone, later calls queue exactly R - 1
//               rounds after round 1 and never wait on the host.  If the
//               graph was modified against the contract, vertices are left
//               uncoloured and gc_get_stats reports it.
//   CHUNKED     as GRAPH with direct launches.
//   HOST        one speculate + detect pair per round, then a read-back.
//   PERSISTENT  one cooperative launch runs every round with grid barriers.
// All drivers run the same phase code and give the same bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>

#include "gc.h"
#include "gc_internal.h"

using gc::Ctrl;
using gc::KArgs;

namespace {

thread_local std::string tl_error;

struct Pinned {  // read-back area in pinned host memory
  int32_t flag;
  int32_t pad0;
  int32_t counts[3];  // medium count, heavy count, max degree
  int32_t err[2];
  int32_t last_round;  // folded from fin by the host once a call has completed
  int32_t ncolors;
  int32_t abort;
  int32_t left;
  int32_t pad1[3];
  int32_t fin[gc::kFinishWords];  // written by the finishing kernel (layout at launch_finish)
};

// One instantiated chunk of K rounds.  The graph holds the kernel arguments
// and grid of its capture, so it is replayed only while everything the round
// kernels read from them is unchanged (options and reallocations change the
// degree lists, the flag blocks and the grid).
struct Captured {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int k = 0, lanes = 0, grid = 0;
  KArgs args{};
};

// Kernel kinds reported by gc_get_profile.
enum { kRound1 = 0, kSpecK = 1, kDetectK = 2, kFinishK = 3, kKinds = 4 };

}  // namespace

struct gc_ctx {
  int device = 0;
  int cus = 0;
  const void* rowptr = nullptr;     // the graph coloured: the caller's, or its relabelled copy
  bool rp64 = false;
  const int32_t* colidx = nullptr;
  int64_t n = 0, m = 0;
  uint32_t flags = 0;
  const void* rowptr_in = nullptr;  // the caller's CSR (borrowed) and flags
  const int32_t* colidx_in = nullptr;
  uint32_t flags_in = 0;
  int order = GC_ORDER_NATURAL;     // requested vertex order and seed
  uint64_t order_seed = 0;
  int built_order = GC_ORDER_NATURAL;  // order of the graph currently bound
  uint64_t built_seed = 0;
  void* o_rowptr = nullptr;         // device: relabelled CSR, new ids, colours by new id
  int32_t* o_colidx = nullptr;
  int32_t* o_newid = nullptr;
  int32_t* o_colors = nullptr;

  Ctrl* ctrl = nullptr;       // device
  void* state = nullptr;      // device, n * sbytes
  int sbytes = 4;             // state width (1, 2 or 4 bytes) from the max degree
  int32_t* mlist = nullptr;   // device, n
  int32_t* hlist = nullptr;   // device, n
  int32_t* dcounts = nullptr; // device, 8 ints: classify counts, validate err
  uint8_t* seen = nullptr;    // device, n * kPushColors (push algorithm), allocated on first use
  uint8_t* wide = nullptr;    // device, wide_blocks * kWideColors (push algorithm)
  int64_t wide_blocks = 0;    // blocks allocated in `wide`
  gc::PushTask* tasks = nullptr;  // device, 2 * wide_blocks: pushes queued for the grid-wide pass
  int32_t* widx = nullptr;    // device, n: wide block of each medium/heavy vertex, -1 otherwise
  int32_t* skip = nullptr;    // device, n: final-prefix offset of each row (sorted rows)
  int32_t* lst = nullptr;     // device, m: lower-neighbour lists of medium and heavy vertices
  int32_t* llen = nullptr;    // device, n: their lengths
  int32_t* part = nullptr;    // device, cus * kMaxBlocksPerCu: per-workgroup round sizes
  int epoch = 0;              // epoch of the last call's pushed flags (1..255)
  Pinned* host = nullptr;     // pinned
  int32_t* fin_dev = nullptr; // device address of host->fin
  int32_t mcount = 0, hcount = 0, maxdeg = 0;

  // options
  int mode = GC_MODE_AUTO;
  int lanes = 0;          // 0 = auto
  int medium_min = 0;     // 0 = auto (deg > medium threshold -> medium)
  int heavy_min = 4096;   // deg >= heavy_min -> heavy
  int blocks_per_cu = 8;
  int persist_per_cu = 4; // co-resident workgroups per CU of the persistent kernel
  int max_rounds = 0;
  int chunk_rounds = 16;
  int algorithm = GC_ALGO_AUTO;
  bool lists_dirty = false;

  // last colouring
  hipEvent_t done = nullptr;
  bool in_flight = false;
  bool stats_ready = false;
  int64_t known_rounds = 0;  // R of this graph once a call has completed (0 = unknown)
  int64_t partitions = 0;    // p of GC_ALGO_BLOCKS (0 = auto)
  int32_t* bslot = nullptr;  // device, nnz: ForbiddenColors slots (GC_ALGO_BLOCKS)
  uint8_t* btodo = nullptr;  // device, n

  Captured chunk;  // discovery chunk (chunk_rounds)
  Captured exact;  // R - 1 rounds, once R is known

  // profiling (GC_OPT_PROFILE): events around the kernels of a call
  bool profile = false;
  hipEvent_t pev[4] = {nullptr, nullptr, nullptr, nullptr};  // round 1 start/end, finish start/end
  hipEvent_t* rev = nullptr;  // 3 per round of rounds 2..R: spec start, spec end, detect end
  int rev_rounds = 0;         // rounds rev has room for
  int timed_rounds = 0;       // rounds 2..R timed by the last call
  bool pending_profile = false;
  double prof_ms[kKinds] = {0, 0, 0, 0};
  int64_t prof_launches[kKinds] = {0, 0, 0, 0};

  std::string err;
};

static int set_err(gc_ctx* h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
static int set_err(gc_ctx* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  tl_error = buf;
  if (h) h->err = buf;
  return code;
}

#define HIPCHECK(h, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (hipError_t)(expr);                                               \
    if (e_ != hipSuccess)                                                             \
      return set_err(h, GC_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                     __FILE__, __LINE__);                                             \
  } while (0)

#define LCHECK(h, expr)                                                                   \
  do {                                                                                    \
    int r_ = (expr);                                                                      \
    if (r_) return set_err(h, GC_EDEVICE, "%s: %s", #expr, hipGetErrorString((hipError_t)r_)); \
  } while (0)

static int auto_lanes(const gc_ctx* h) {
  if (h->lanes) return h->lanes;
  double avg = h->n ? (double)h->m / (double)h->n : 0.0;
  int L = 2;
  while (L < 32 && L * 4 <= avg) L *= 2;  // about four row entries per lane
  return L;
}

static int light_max_of(const gc_ctx* h, int L) {
  if (h->medium_min > 0) return h->medium_min;
  return std::max(8 * L, 64);
}

// Colours never exceed the degree; the largest value of the type stays unused
// so that the smallest can mark "waiting" under GC_ALGO_SEQ.
static int state_bytes(int32_t maxdeg) {
  if (maxdeg <= 126) return 1;
  if (maxdeg <= 32766) return 2;
  return 4;
}

static bool use_push(const gc_ctx* h) {
  return h->algorithm == GC_ALGO_PUSH || h->algorithm == GC_ALGO_AUTO;
}

static bool use_seq(const gc_ctx* h) { return h->algorithm == GC_ALGO_SEQ; }

// The colouring a handle computes: the speculative one (AUTO, PULL, PUSH),
// sequential First Fit (SEQ), or Algorithm 1 with p blocks.  R is a property
// of the graph and of this.
static int family_of(int algorithm) {
  return algorithm == GC_ALGO_SEQ ? 1 : algorithm == GC_ALGO_BLOCKS ? 2 : 0;
}

static int64_t partitions_of(const gc_ctx* h) {
  return h->partitions > 0 ? h->partitions : (int64_t)h->cus * 64;
}

static KArgs make_args(const gc_ctx* h, int32_t* colors, int light_max) {
  KArgs a{};
  a.rowptr = h->rowptr;
  a.colidx = h->colidx;
  a.st = h->state;
  a.colors = colors;
  a.n = (int32_t)h->n;
  a.light_max = light_max;
  a.mlist = h->mlist;
  a.mcount = h->mcount;
  a.hlist = h->hlist;
  a.hcount = h->hcount;
  a.sorted = (h->flags & GC_ROWS_SORTED) != 0;
  a.push = use_push(h) ? 1 : 0;
  a.seq = use_seq(h) ? 1 : 0;
  a.seen = h->seen;
  a.flags_by_chunk = (h->mcount + h->hcount == 0) ? 1 : 0;
  a.epoch = h->epoch;
  a.clear_seen = h->epoch == 1;
  a.wide = h->wide;
  a.wide_clear = (int32_t)h->wide_blocks;
  a.widx = h->widx;
  a.skip = h->skip;
  // wavefront- and workgroup-class conflict scans keep lists of lower neighbours not yet
  // seen final (push algorithm, sorted rows)
  a.lst = (a.push && a.sorted && !a.seq && h->mcount + h->hcount > 0) ? h->lst : nullptr;
  a.llen = a.lst ? h->llen : nullptr;
  a.part = h->part;
  // long rows of wavefront- and workgroup-class winners are pushed by a
  // grid-wide pass after each detect pass
  // (not inside the single persistent launch)
  a.tasks = (a.push && h->mcount + h->hcount > 0 && h->mode != GC_MODE_PERSISTENT) ? h->tasks
                                                                                   : nullptr;
  a.ctrl = h->ctrl;
  return a;
}

static int grid_of(const gc_ctx* h) { return std::max(1, h->cus * h->blocks_per_cu); }

// Workgroups of the round kernels: at most blocks_per_cu per CU, and no more
// than the graph can keep busy (a wavefront per 64-vertex chunk or per medium
// vertex, a workgroup per heavy vertex), so a small graph does not pay for
// dispatching thousands of idle workgroups every round.
static int round_grid(const gc_ctx* h) {
  const int64_t chunks = (h->n + gc::kWave - 1) / gc::kWave;
  const int64_t waves = std::max<int64_t>(chunks, h->mcount);
  const int64_t blocks = std::max<int64_t>((waves + gc::kWavesPerBlock - 1) / gc::kWavesPerBlock,
                                           h->hcount);
  return (int)std::max<int64_t>(1, std::min<int64_t>(grid_of(h), blocks));
}

// Build the medium and heavy lists for the current thresholds; synchronous.
static int classify(gc_ctx* h, hipStream_t s) {
  const int L = auto_lanes(h);
  const int light = light_max_of(h, L);
  const int heavy = std::max(h->heavy_min, light + 1);
  HIPCHECK(h, hipMemsetAsync(h->dcounts, 0, 3 * sizeof(int32_t), s));
  LCHECK(h, gc::launch_classify(h->rowptr, h->rp64, (int32_t)h->n, light, heavy, h->mlist, h->hlist,
                                h->dcounts, h->widx, grid_of(h), s));
  HIPCHECK(h, hipMemcpyAsync(h->host->counts, h->dcounts, 3 * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
  HIPCHECK(h, hipStreamSynchronize(s));
  h->mcount = h->host->counts[0];
  h->hcount = h->host->counts[1];
  h->maxdeg = h->host->counts[2];
  LCHECK(h, gc::launch_wide_index(h->hlist, h->hcount, h->mcount, h->widx, s));
  h->lists_dirty = false;
  return GC_OK;
}

static void drop(Captured& c) {
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  c = Captured();
}

static void free_ctx(gc_ctx* h) {
  if (!h) return;
  drop(h->chunk);
  drop(h->exact);
  for (hipEvent_t& e : h->pev)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < 3 * h->rev_rounds; ++i) (void)hipEventDestroy(h->rev[i]);
  delete[] h->rev;
  if (h->done) (void)hipEventDestroy(h->done);
  if (h->ctrl) (void)hipFree(h->ctrl);
  if (h->state) (void)hipFree(h->state);
  if (h->mlist) (void)hipFree(h->mlist);
  if (h->hlist) (void)hipFree(h->hlist);
  if (h->dcounts) (void)hipFree(h->dcounts);
  if (h->seen) (void)hipFree(h->seen);
  if (h->wide) (void)hipFree(h->wide);
  if (h->tasks) (void)hipFree(h->tasks);
  if (h->widx) (void)hipFree(h->widx);
  if (h->skip) (void)hipFree(h->skip);
  if (h->lst) (void)hipFree(h->lst);
  if (h->llen) (void)hipFree(h->llen);
  if (h->part) (void)hipFree(h->part);
  if (h->o_rowptr) (void)hipFree(h->o_rowptr);
  if (h->o_colidx) (void)hipFree(h->o_colidx);
  if (h->o_newid) (void)hipFree(h->o_newid);
  if (h->o_colors) (void)hipFree(h->o_colors);
  if (h->bslot) (void)hipFree(h->bslot);
  if (h->btodo) (void)hipFree(h->btodo);
  if (h->host) (void)hipHostFree(h->host);
  delete h;
}

extern "C" int gc_create(gc_handle* out, const void* rowptr, const int32_t* colidx, int64_t n,
                         int64_t m, uint32_t flags, void* stream) {
  if (!out) return set_err(nullptr, GC_EINVAL, "gc_create: out is NULL");
  *out = nullptr;
  if (n < 0 || m < 0) return set_err(nullptr, GC_EINVAL, "gc_create: negative n or m");
  if (n >= INT32_MAX) return set_err(nullptr, GC_ETOOBIG, "gc_create: n must be below 2^31 - 1");
  if (!(flags & GC_ROWPTR_I64) && m > INT32_MAX)
    return set_err(nullptr, GC_ETOOBIG, "gc_create: m > 2^31 - 1 needs GC_ROWPTR_I64");
  if (flags & ~(uint32_t)(GC_ROWPTR_I64 | GC_VALIDATE | GC_ROWS_SORTED))
    return set_err(nullptr, GC_EINVAL, "gc_create: unknown flag bits 0x%x", flags);
  if (!rowptr) return set_err(nullptr, GC_EINVAL, "gc_create: rowptr is NULL");
  if (m > 0 && !colidx) return set_err(nullptr, GC_EINVAL, "gc_create: colidx is NULL");

  gc_ctx* h = new (std::nothrow) gc_ctx();
  if (!h) return set_err(nullptr, GC_ENOMEM, "gc_create: out of host memory");
  h->rowptr = h->rowptr_in = rowptr;
  h->rp64 = (flags & GC_ROWPTR_I64) != 0;
  h->colidx = h->colidx_in = colidx;
  h->n = n;
  h->m = m;
  h->flags = h->flags_in = flags;
  hipStream_t s = (hipStream_t)stream;

#define CREATE_CHECK(expr)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (hipError_t)(expr);                                                         \
    if (e_ != hipSuccess) {                                                                     \
      int code_ = (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation) ? GC_ENOMEM      \
                                                                                : GC_EDEVICE;   \
      set_err(nullptr, code_, "gc_create: %s: %s", #expr, hipGetErrorString(e_));               \
      free_ctx(h);                                                                              \
      return code_;                                                                             \
    }                                                                                           \
  } while (0)

  CREATE_CHECK(hipGetDevice(&h->device));
  CREATE_CHECK(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device));
  CREATE_CHECK(hipMalloc((void**)&h->ctrl, sizeof(Ctrl)));
  CREATE_CHECK(hipMalloc((void**)&h->mlist, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)));
  CREATE_CHECK(hipMalloc((void**)&h->hlist, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)));
  CREATE_CHECK(hipMalloc((void**)&h->dcounts, 8 * sizeof(int32_t)));
  CREATE_CHECK(hipMalloc((void**)&h->widx, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)));
  CREATE_CHECK(hipMalloc((void**)&h->skip, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)));
  CREATE_CHECK(hipMalloc((void**)&h->part, (size_t)h->cus * gc::kMaxBlocksPerCu * sizeof(int32_t)));
  CREATE_CHECK(hipHostMalloc((void**)&h->host, sizeof(Pinned), hipHostMallocDefault));
  CREATE_CHECK(hipHostGetDevicePointer((void**)&h->fin_dev, h->host->fin, 0));
  CREATE_CHECK(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  memset(h->host, 0, sizeof(Pinned));

  if (flags & GC_VALIDATE) {
    int32_t init_err[2] = {INT32_MAX, -1};
    CREATE_CHECK(hipMemcpyAsync(h->dcounts + 4, init_err, sizeof init_err, hipMemcpyHostToDevice, s));
    CREATE_CHECK(gc::launch_validate(rowptr, h->rp64, colidx, (int32_t)n, m,
                                     (flags & GC_ROWS_SORTED) != 0, h->dcounts + 4, grid_of(h), s));
    CREATE_CHECK(hipMemcpyAsync(h->host->err, h->dcounts + 4, sizeof init_err,
                                hipMemcpyDeviceToHost, s));
    CREATE_CHECK(hipStreamSynchronize(s));
    int code = h->host->err[0];
    if (code != INT32_MAX) {
      static const char* what[] = {"",
                                   "rowptr[0] != 0 or rowptr[n] != m",
                                   "rowptr decreases or leaves [0, m]",
                                   "neighbour id out of range",
                                   "self-loop (a simple graph has none)",
                                   "duplicate entry in a row",
                                   "row not ascending although GC_ROWS_SORTED was given",
                                   "edge stored in one direction only (CSR not symmetric)"};
      set_err(nullptr, GC_EINVAL, "gc_create: invalid graph: %s (vertex %d)",
              (code >= 1 && code <= 7) ? what[code] : "?", h->host->err[1]);
      free_ctx(h);
      return GC_EINVAL;
    }
  }
  int rc = classify(h, s);
  if (rc) {
    tl_error = h->err;
    free_ctx(h);
    return rc;
  }
  h->sbytes = state_bytes(h->maxdeg);
  CREATE_CHECK(hipMalloc(&h->state, (size_t)std::max<int64_t>(n, 1) * h->sbytes));
  *out = h;
  return GC_OK;
}

// Wait on the host for the handle's last call (option changes and teardown).
static int ensure_idle(gc_ctx* h) {
  if (!h->in_flight) return GC_OK;
  HIPCHECK(h, hipEventSynchronize(h->done));
  h->in_flight = false;
  return GC_OK;
}

static int resolve_mode(const gc_ctx* h) {
  int mode = h->mode == GC_MODE_AUTO ? GC_MODE_GRAPH : h->mode;
  // a captured chunk cannot stop inside itself: honour a round cap by queueing
  if (mode == GC_MODE_GRAPH && h->max_rounds > 0) mode = GC_MODE_CHUNKED;
  return mode;
}

// Capture K rounds (speculate + detect, rounds relative to the device-side
// round base) and the base advance into c.
static int capture(gc_ctx* h, Captured& c, const KArgs& a, int L, int K) {
  drop(c);
  hipStream_t cs;
  HIPCHECK(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return set_err(h, GC_EDEVICE, "begin capture: %s", hipGetErrorString(e));
  }
  int rc = 0;
  for (int j = 0; j < K && !rc; ++j) {
    rc = gc::launch_round(a, h->rp64, h->sbytes, L, 0, j, true, round_grid(h), cs);
    if (!rc) rc = gc::launch_round(a, h->rp64, h->sbytes, L, 1, j, true, round_grid(h), cs);
  }
  if (!rc) rc = gc::launch_advance_base(a, K, cs);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    drop(c);
    return set_err(h, GC_EDEVICE, "capture failed: %s",
                   hipGetErrorString(rc ? (hipError_t)rc : e2));
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    drop(c);
    return set_err(h, GC_EDEVICE, "instantiate: %s", hipGetErrorString(e));
  }
  c.graph = g;
  c.exec = x;
  c.k = K;
  c.lanes = L;
  c.grid = round_grid(h);
  c.args = a;
  return GC_OK;
}

// Fields of KArgs that the captured round kernels read (the call's epoch and
// output pointer reach them through the control block and the finish kernel,
// which are launched outside the graph).
static bool usable(const Captured& c, int K, int L, int grid, const KArgs& a) {
  const KArgs& b = c.args;
  return c.exec && c.k == K && c.lanes == L && c.grid == grid && b.rowptr == a.rowptr &&
         b.colidx == a.colidx && b.st == a.st && b.n == a.n && b.light_max == a.light_max &&
         b.mlist == a.mlist && b.mcount == a.mcount && b.hlist == a.hlist &&
         b.hcount == a.hcount && b.sorted == a.sorted && b.push == a.push && b.seq == a.seq &&
         b.seen == a.seen && b.flags_by_chunk == a.flags_by_chunk && b.wide == a.wide && b.widx == a.widx && b.skip == a.skip &&
         b.lst == a.lst && b.llen == a.llen && b.part == a.part && b.tasks == a.tasks && b.ctrl == a.ctrl;
}

static float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();  // do not leave the failure for a later launch check
    return 0.f;
  }
  return ms;
}

// Room for per-round events of `rounds` rounds.
static int reserve_round_events(gc_ctx* h, int rounds) {
  if (rounds <= h->rev_rounds) return GC_OK;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[3 * (size_t)rounds]();
  if (!ev) return set_err(h, GC_ENOMEM, "profile events: host memory");
  for (int i = 0; i < 3 * h->rev_rounds; ++i) ev[i] = h->rev[i];
  for (int i = 3 * h->rev_rounds; i < 3 * rounds; ++i) {
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int j = 3 * h->rev_rounds; j < i; ++j) (void)hipEventDestroy(ev[j]);
      delete[] ev;
      return set_err(h, GC_EDEVICE, "profile events: hipEventCreate failed");
    }
  }
  delete[] h->rev;
  h->rev = ev;
  h->rev_rounds = rounds;
  return GC_OK;
}

// Add the kernel times of the finished last call to the profile totals.
static void collect_profile(gc_ctx* h) {
  if (!h->pending_profile) return;
  h->pending_profile = false;
  h->prof_ms[kRound1] += elapsed(h->pev[0], h->pev[1]);
  h->prof_launches[kRound1] += 1;
  h->prof_ms[kFinishK] += elapsed(h->pev[2], h->pev[3]);
  h->prof_launches[kFinishK] += 1;
  for (int j = 0; j < h->timed_rounds; ++j) {
    h->prof_ms[kSpecK] += elapsed(h->rev[3 * j], h->rev[3 * j + 1]);
    h->prof_ms[kDetectK] += elapsed(h->rev[3 * j + 1], h->rev[3 * j + 2]);
  }
  h->prof_launches[kSpecK] += h->timed_rounds;
  h->prof_launches[kDetectK] += h->timed_rounds;
  h->timed_rounds = 0;
}

// Bind the graph in the requested vertex order: the caller's CSR, or a
// relabelled copy built on the device (set-up work, synchronous).
static int ensure_order(gc_ctx* h, hipStream_t s) {
  if (h->order == h->built_order &&
      (h->order != GC_ORDER_RANDOM || h->order_seed == h->built_seed))
    return GC_OK;
  int rc = ensure_idle(h);
  if (rc) return rc;
  for (void* p : {h->o_rowptr, (void*)h->o_colidx, (void*)h->o_newid, (void*)h->o_colors})
    if (p) (void)hipFree(p);
  h->o_rowptr = nullptr;
  h->o_colidx = h->o_newid = h->o_colors = nullptr;
  h->rowptr = h->rowptr_in;
  h->colidx = h->colidx_in;
  h->flags = h->flags_in;
  h->built_order = GC_ORDER_NATURAL;
  h->lists_dirty = true;
  h->known_rounds = 0;
  if (h->order == GC_ORDER_NATURAL) return GC_OK;
  if (h->m > INT32_MAX)
    return set_err(h, GC_ETOOBIG, "vertex order: more than 2^31 - 1 CSR entries");
  const size_t nv = (size_t)std::max<int64_t>(h->n, 1);
  hipError_t e = hipMalloc(&h->o_rowptr, (nv + 1) * (h->rp64 ? 8 : 4));
  if (e == hipSuccess) e = hipMalloc((void**)&h->o_colidx, (size_t)std::max<int64_t>(h->m, 1) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&h->o_newid, nv * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&h->o_colors, nv * 4);
  if (e != hipSuccess) return set_err(h, GC_ENOMEM, "vertex order: %s", hipGetErrorString(e));
  LCHECK(h, gc::build_order(h->rowptr_in, h->rp64, h->colidx_in, (int32_t)h->n, h->m, h->order,
                            h->order_seed, h->o_rowptr, h->o_colidx, h->o_newid, grid_of(h), s));
  h->rowptr = h->o_rowptr;
  h->colidx = h->o_colidx;
  h->flags = h->flags_in | GC_ROWS_SORTED;  // the relabelled rows are ascending
  h->built_order = h->order;
  h->built_seed = h->order_seed;
  return GC_OK;
}

// The colours by new id go back to the caller's ids (no-op in natural order).
static int permute_back(gc_ctx* h, const int32_t* coloured, int32_t* colors_out, hipStream_t s) {
  if (coloured == colors_out || h->n == 0) return GC_OK;
  LCHECK(h, gc::launch_permute_back(h->o_newid, coloured, (int32_t)h->n, colors_out,
                                    std::min(grid_of(h), 4096), s));
  return GC_OK;
}

// Algorithm 1 with p blocks (GC_ALGO_BLOCKS): per-edge slots, p sequential
// blocks per round; the host reads the count of vertices to recolour after
// each round (R <= p).
static int color_blocks(gc_ctx* h, int32_t* colors_out, int32_t* user_out, hipStream_t s) {
  int rc = GC_OK;
  if (h->n > 0 && !h->bslot) {
    hipError_t e = hipMalloc((void**)&h->bslot, (size_t)std::max<int64_t>(h->m, 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&h->btodo, (size_t)h->n);
    if (e != hipSuccess) return set_err(h, GC_ENOMEM, "block slots: %s", hipGetErrorString(e));
  }
  h->stats_ready = false;
  KArgs a = make_args(h, colors_out, light_max_of(h, auto_lanes(h)));
  a.st = colors_out;  // the colours are the state (int32)
  a.clear_trace = 1;  // phase 2 adds each round's size into the trace
  gc::BArgs b{};
  b.rowptr = h->rowptr;
  b.colidx = h->colidx;
  b.color = colors_out;
  b.slot = h->bslot;
  b.todo = h->btodo;
  b.n = (int32_t)h->n;
  b.p = partitions_of(h);
  b.ctrl = h->ctrl;
  const int grid = round_grid(h);
  LCHECK(h, gc::launch_init(a, s));
  if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[0], s));
  if (h->n > 0) {
    LCHECK(h, gc::launch_blocks_init(b, h->rp64, grid, s));
    if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[1], s));
    for (int r = 1;; ++r) {
      b.round = r;
      if (h->profile) {  // phase 1 and phase 2 between events, as speculate and detect
        rc = reserve_round_events(h, r > h->rev_rounds ? std::max(r, 2 * h->rev_rounds) : r);
        if (rc) return rc;
        HIPCHECK(h, hipEventRecord(h->rev[3 * (r - 1)], s));
      }
      LCHECK(h, gc::launch_blocks_phase(b, h->rp64, 1, grid, s));
      if (h->profile) HIPCHECK(h, hipEventRecord(h->rev[3 * (r - 1) + 1], s));
      LCHECK(h, gc::launch_blocks_phase(b, h->rp64, 2, grid, s));
      if (h->profile) {
        HIPCHECK(h, hipEventRecord(h->rev[3 * (r - 1) + 2], s));
        h->timed_rounds = r;
      }
      HIPCHECK(h, hipMemcpyAsync(&h->host->flag, &h->ctrl->left.v, sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
      HIPCHECK(h, hipStreamSynchronize(s));
      if (!h->host->flag) break;
      if (h->max_rounds > 0 && r >= h->max_rounds) break;
      // Lemma 2: at most p rounds (p + 1 as the paper states it)
      if (r > b.p + 1) return set_err(h, GC_EDEVICE, "round %d > p + 1 = %lld: the p-block "
                                      "colouring is not converging (internal error)", r,
                                      (long long)(b.p + 1));
    }
  } else if (h->profile) {
    HIPCHECK(h, hipEventRecord(h->pev[1], s));
  }
  // a round cap can stop the loop with coloured vertices still in conflict
  if (h->n > 0 && h->host->flag) LCHECK(h, gc::launch_blocks_set_left(h->ctrl, h->host->flag, s));
  if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[2], s));
  LCHECK(h, gc::launch_finish(a, 4, h->fin_dev, s));
  if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[3], s));
  h->pending_profile = h->profile;
  rc = permute_back(h, colors_out, user_out, s);
  if (rc) return rc;
  HIPCHECK(h, hipEventRecord(h->done, s));
  h->in_flight = true;
  h->stats_ready = true;
  return rc;
}

extern "C" int gc_color(gc_handle h, int32_t* colors_out, void* stream) {
  if (!h) return set_err(nullptr, GC_EINVAL, "gc_color: NULL handle");
  if (h->n > 0 && !colors_out) return set_err(h, GC_EINVAL, "gc_color: colors_out is NULL");
  int rc = GC_OK;
  int cur = 0;
  HIPCHECK(h, hipGetDevice(&cur));
  if (cur != h->device) HIPCHECK(h, hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  // Calls on one handle are ordered: a call waits (on the device) for the
  // previous one, whose scratch it reuses.  A profiled call's events are
  // read before they are recorded again.
  if (h->in_flight && h->pending_profile) {
    rc = ensure_idle(h);
    if (rc) return rc;
    collect_profile(h);
  }
  if (h->in_flight) HIPCHECK(h, hipStreamWaitEvent(s, h->done, 0));
  rc = ensure_order(h, s);
  if (rc) return rc;
  int32_t* const user_out = colors_out;
  if (h->built_order != GC_ORDER_NATURAL) colors_out = h->o_colors;  // colours by new id
  if (h->lists_dirty) {
    rc = ensure_idle(h);
    if (rc) return rc;
    rc = classify(h, s);
    if (rc) return rc;
  }
  (void)hipGetLastError();  // launch checks below must see only this call's errors
  if (h->algorithm == GC_ALGO_BLOCKS) return color_blocks(h, colors_out, user_out, s);
  if (use_push(h)) {
    if (!h->seen && h->n > 0) {
      const size_t nv = (size_t)(h->n + gc::kWave - 1) / gc::kWave * gc::kWave;  // whole chunks
      hipError_t e = hipMalloc((void**)&h->seen, nv * gc::kPushColors);
      if (e != hipSuccess) return set_err(h, GC_ENOMEM, "colour flags: %s", hipGetErrorString(e));
      h->epoch = 0;
    }
    const int64_t blocks = (int64_t)h->mcount + h->hcount;
    if (blocks > h->wide_blocks) {
      rc = ensure_idle(h);
      if (rc) return rc;
      if (h->wide) (void)hipFree(h->wide);
      if (h->tasks) (void)hipFree(h->tasks);
      h->wide = nullptr;
      h->tasks = nullptr;
      h->wide_blocks = 0;
      hipError_t e = hipMalloc((void**)&h->wide, (size_t)blocks * gc::kWideColors);
      if (e == hipSuccess)
        e = hipMalloc((void**)&h->tasks, 2 * (size_t)blocks * sizeof(gc::PushTask));
      if (e != hipSuccess) return set_err(h, GC_ENOMEM, "wide colour flags: %s", hipGetErrorString(e));
      h->wide_blocks = blocks;
      h->epoch = 0;  // new memory: the next epoch (1) clears every flag
    }
    if (blocks > 0 && (h->flags & GC_ROWS_SORTED) && !use_seq(h) && !h->lst) {
      // lower-neighbour lists: one slot per row entry, one length per vertex
      hipError_t e = hipMalloc((void**)&h->lst, (size_t)std::max<int64_t>(h->m, 1) * sizeof(int32_t));
      if (e == hipSuccess)
        e = hipMalloc((void**)&h->llen, (size_t)std::max<int64_t>(h->n, 1) * sizeof(int32_t));
      if (e != hipSuccess) {
        if (h->lst) (void)hipFree(h->lst);
        h->lst = nullptr;
        h->llen = nullptr;
        return set_err(h, GC_ENOMEM, "lower-neighbour lists: %s", hipGetErrorString(e));
      }
    }
    // a new epoch per call marks this call's flags; flags are cleared on the
    // first call and whenever the 8-bit epoch wraps
    h->epoch = h->epoch % 255 + 1;
  }
  h->stats_ready = false;
  const int L = auto_lanes(h);
  const int light = light_max_of(h, L);
  const KArgs a = make_args(h, colors_out, light);
  const int grid = round_grid(h);
  const int mode = resolve_mode(h);

  LCHECK(h, gc::launch_init(a, s));
  if (mode == GC_MODE_PERSISTENT) {
    int maxg = 0;
    LCHECK(h, gc::persistent_max_grid(h->rp64, h->sbytes, L, &maxg));
    // persistent_max_grid bounds the grid by what the kernel's register and
    // LDS use let every CU hold at once (3 or 4 workgroups per CU); the
    // option can only lower that, and, as for the round kernels, the grid
    // stops at what the graph can keep busy: a barrier over fewer workgroups
    // is cheaper.
    int pg = std::min(std::min(maxg, h->cus * h->persist_per_cu), grid);
    if (pg < 1) return set_err(h, GC_EDEVICE, "persistent kernel cannot be resident");
    LCHECK(h, gc::launch_persistent(a, h->rp64, h->sbytes, L, h->max_rounds, pg, s));
  } else {
    if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[0], s));
    LCHECK(h, gc::launch_round1(a, h->rp64, h->sbytes, L, grid, s));
    if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[1], s));
    int r = 1;  // last round queued
    if (h->profile && h->known_rounds > 0) {
      // Profiled call with R known: rounds 2..R launched directly, each kernel
      // between two events on the caller's stream.
      const int K = (int)h->known_rounds - 1;
      rc = reserve_round_events(h, K);
      if (rc) return rc;
      for (int j = 0; j < K; ++j) {
        HIPCHECK(h, hipEventRecord(h->rev[3 * j], s));
        LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 0, 2 + j, false, grid, s));
        HIPCHECK(h, hipEventRecord(h->rev[3 * j + 1], s));
        LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 1, 2 + j, false, grid, s));
        HIPCHECK(h, hipEventRecord(h->rev[3 * j + 2], s));
      }
      h->timed_rounds = K;
    } else if (mode == GC_MODE_GRAPH && h->known_rounds > 0) {
      // R is known: queue rounds 2..R in one captured chunk, no read-back.
      const int K = (int)h->known_rounds - 1;
      if (K > 0) {
        if (!usable(h->exact, K, L, grid, a)) {
          rc = capture(h, h->exact, a, L, K);
          if (rc) return rc;
        }
        HIPCHECK(h, hipGraphLaunch(h->exact.exec, s));
      }
    } else {
      const int K = std::max(1, h->chunk_rounds);
      for (;;) {
        HIPCHECK(h, hipMemcpyAsync(&h->host->flag, &h->ctrl->more[(r + 1) % 3].v, sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        HIPCHECK(h, hipStreamSynchronize(s));
        if (!h->host->flag) break;
        if (h->max_rounds > 0 && r >= h->max_rounds) break;
        // every round colours at least the lowest uncoloured vertex (Lemma 2
        // with one vertex per block), so R <= n: more rounds mean a broken
        // invariant, reported instead of looping
        if (r > h->n) return set_err(h, GC_EDEVICE, "round %d > n = %lld: the colouring is not "
                                     "converging (internal error)", r, (long long)h->n);
        if (mode == GC_MODE_HOST) {
          ++r;
          LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 0, r, false, grid, s));
          LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 1, r, false, grid, s));
        } else if (mode == GC_MODE_CHUNKED) {
          int upto = r + K;
          if (h->max_rounds > 0) upto = std::min(upto, h->max_rounds);
          for (int q = r + 1; q <= upto; ++q) {
            LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 0, q, false, grid, s));
            LCHECK(h, gc::launch_round(a, h->rp64, h->sbytes, L, 1, q, false, grid, s));
          }
          r = upto;
        } else if (mode == GC_MODE_GRAPH) {
          if (!usable(h->chunk, K, L, grid, a)) {
            rc = capture(h, h->chunk, a, L, K);
            if (rc) return rc;
          }
          HIPCHECK(h, hipGraphLaunch(h->chunk.exec, s));
          r += K;  // rounds r+1 .. r+K ran (the round base advanced by K)
        } else {
          return set_err(h, GC_EINVAL, "unknown mode %d", mode);
        }
      }
    }
  }
  if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[2], s));
  LCHECK(h, gc::launch_finish(a, h->sbytes, h->fin_dev, s));
  if (h->profile) HIPCHECK(h, hipEventRecord(h->pev[3], s));
  h->pending_profile = h->profile && mode != GC_MODE_PERSISTENT;
  rc = permute_back(h, colors_out, user_out, s);
  if (rc) return rc;
  HIPCHECK(h, hipEventRecord(h->done, s));
  h->in_flight = true;
  h->stats_ready = true;
  return GC_OK;
}

// The finishing kernel's words, folded into the call's statistics.
static void fold_finish(gc_ctx* h) {
  Pinned* p = h->host;
  const int32_t* f = p->fin;
  p->last_round = f[0];
  p->abort = f[1];
  const int g = std::min(std::max(f[3], 0), gc::kFinishBlocks);
  int32_t nc = 0;
  int64_t left = f[2];
  for (int b = 0; b < g; ++b) {
    nc = std::max(nc, f[gc::kFinishHeader + 2 * b]);
    left += f[gc::kFinishHeader + 1 + 2 * b];
  }
  p->ncolors = nc;
  p->left = (int32_t)std::min<int64_t>(left, INT32_MAX);
}

static int wait_done(gc_ctx* h) {
  if (!h->stats_ready) return set_err(h, GC_EINVAL, "no colouring has been run on this handle");
  if (h->in_flight) {
    HIPCHECK(h, hipEventSynchronize(h->done));
    h->in_flight = false;
  }
  fold_finish(h);  // the call has completed (also when another path waited for it)
  collect_profile(h);
  if (h->host->abort) return set_err(h, GC_EDEVICE, "persistent kernel: grid barrier timed out");
  if (h->host->left) {
    if (h->max_rounds > 0 && h->host->last_round >= h->max_rounds)
      return set_err(h, GC_EROUNDS, "round cap reached with %d vertices uncoloured", h->host->left);
    h->known_rounds = 0;
    return set_err(h, GC_EINVAL, "%d vertices uncoloured after the known %d rounds: the graph "
                   "changed after gc_create", h->host->left, h->host->last_round);
  }
  if (h->max_rounds == 0) h->known_rounds = h->host->last_round;
  return GC_OK;
}

extern "C" int gc_get_stats(gc_handle h, int64_t* rounds, int32_t* num_colors) {
  if (!h) return set_err(nullptr, GC_EINVAL, "gc_get_stats: NULL handle");
  int rc = wait_done(h);
  if (rounds) *rounds = h->host->last_round;
  if (num_colors) *num_colors = h->host->ncolors;
  return rc;
}

extern "C" int gc_get_round_sizes(gc_handle h, int64_t* sizes, int64_t cap, int64_t* rounds) {
  if (!h) return set_err(nullptr, GC_EINVAL, "gc_get_round_sizes: NULL handle");
  if (cap < 0 || (cap > 0 && !sizes)) return set_err(h, GC_EINVAL, "gc_get_round_sizes: bad buffer");
  int rc = wait_done(h);
  if (rc && rc != GC_EROUNDS) return rc;
  int64_t R = h->host->last_round;
  if (rounds) *rounds = R;
  int64_t k = std::min<int64_t>(std::min<int64_t>(R, cap), gc::kTraceRounds);
  if (k > 0) {
    int32_t* tmp = new (std::nothrow) int32_t[k];
    if (!tmp) return set_err(h, GC_ENOMEM, "gc_get_round_sizes: host memory");
    hipError_t e = hipMemcpy(tmp, h->ctrl->trace, k * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      delete[] tmp;
      return set_err(h, GC_EDEVICE, "trace read-back: %s", hipGetErrorString(e));
    }
    for (int64_t i = 0; i < k; ++i) sizes[i] = tmp[i];
    delete[] tmp;
  }
  return rc;
}

extern "C" int gc_set_option(gc_handle h, int option, int64_t value) {
  if (!h) return set_err(nullptr, GC_EINVAL, "gc_set_option: NULL handle");
  int rc = ensure_idle(h);
  if (rc) return rc;
  switch (option) {
    case GC_OPT_MODE:
      if (value < GC_MODE_AUTO || value > GC_MODE_GRAPH) break;
      h->mode = (int)value;
      return GC_OK;
    case GC_OPT_LANES:
      if (value != 0 && (value < 2 || value > 64 || (value & (value - 1)))) break;
      h->lanes = (int)value;
      h->lists_dirty = true;
      return GC_OK;
    case GC_OPT_MEDIUM_DEGREE:
      if (value < 0 || value > INT32_MAX - 1) break;
      h->medium_min = (int)value;
      h->lists_dirty = true;
      return GC_OK;
    case GC_OPT_HEAVY_DEGREE:
      if (value < 1 || value > INT32_MAX) break;
      h->heavy_min = (int)value;
      h->lists_dirty = true;
      return GC_OK;
    case GC_OPT_BLOCKS_PER_CU:
      if (value < 1 || value > gc::kMaxBlocksPerCu) break;
      h->blocks_per_cu = (int)value;
      return GC_OK;
    case GC_OPT_MAX_ROUNDS:
      if (value < 0 || value > INT32_MAX) break;
      h->max_rounds = (int)value;
      return GC_OK;
    case GC_OPT_CHUNK_ROUNDS:
      if (value < 1 || value > 1024) break;
      h->chunk_rounds = (int)value;
      return GC_OK;
    case GC_OPT_PERSISTENT_BLOCKS_PER_CU:
      if (value < 1 || value > 4) break;
      h->persist_per_cu = (int)value;
      return GC_OK;
    case GC_OPT_ALGORITHM:
      if (value < GC_ALGO_AUTO || value > GC_ALGO_BLOCKS) break;
      // the round count R is a property of the graph and of the colouring
      // computed: switching to another colouring forgets it
      if (family_of((int)value) != family_of(h->algorithm)) h->known_rounds = 0;
      h->algorithm = (int)value;
      return GC_OK;
    case GC_OPT_ORDER:
      if (value < GC_ORDER_NATURAL || value > GC_ORDER_RANDOM) break;
      h->order = (int)value;
      return GC_OK;
    case GC_OPT_ORDER_SEED:
      h->order_seed = (uint64_t)value;
      return GC_OK;
    case GC_OPT_PARTITIONS:
      if (value < 0 || value > INT32_MAX) break;
      if (h->algorithm == GC_ALGO_BLOCKS) h->known_rounds = 0;
      h->partitions = value;
      return GC_OK;
    case GC_OPT_PROFILE:
      if (value < 0 || value > 1) break;
      if (value && !h->pev[0]) {
        for (hipEvent_t& e : h->pev) HIPCHECK(h, hipEventCreate(&e));
      }
      h->profile = value != 0;
      return GC_OK;
    default:
      return set_err(h, GC_EINVAL, "gc_set_option: unknown option %d", option);
  }
  return set_err(h, GC_EINVAL, "gc_set_option: value %lld out of range for option %d",
                 (long long)value, option);
}

extern "C" int gc_get_option(gc_handle h, int option, int64_t* value) {
  if (!h || !value) return set_err(h, GC_EINVAL, "gc_get_option: NULL argument");
  switch (option) {
    case GC_OPT_MODE: *value = resolve_mode(h); return GC_OK;
    case GC_OPT_LANES: *value = auto_lanes(h); return GC_OK;
    case GC_OPT_MEDIUM_DEGREE: *value = light_max_of(h, auto_lanes(h)); return GC_OK;
    case GC_OPT_HEAVY_DEGREE: *value = h->heavy_min; return GC_OK;
    case GC_OPT_BLOCKS_PER_CU: *value = h->blocks_per_cu; return GC_OK;
    case GC_OPT_MAX_ROUNDS: *value = h->max_rounds; return GC_OK;
    case GC_OPT_CHUNK_ROUNDS: *value = h->chunk_rounds; return GC_OK;
    case GC_OPT_MAX_DEGREE: *value = h->maxdeg; return GC_OK;
    case GC_OPT_MEDIUM_COUNT: *value = h->mcount; return GC_OK;
    case GC_OPT_HEAVY_COUNT: *value = h->hcount; return GC_OK;
    case GC_OPT_PERSISTENT_BLOCKS_PER_CU: *value = h->persist_per_cu; return GC_OK;
    case GC_OPT_STATE_BYTES: *value = h->sbytes; return GC_OK;
    case GC_OPT_PROFILE: *value = h->profile; return GC_OK;
    case GC_OPT_ALGORITHM:
      *value = h->algorithm == GC_ALGO_BLOCKS ? GC_ALGO_BLOCKS
               : use_seq(h)                   ? GC_ALGO_SEQ
               : use_push(h)                  ? GC_ALGO_PUSH
                                              : GC_ALGO_PULL;
      return GC_OK;
    case GC_OPT_PARTITIONS: *value = partitions_of(h); return GC_OK;
    case GC_OPT_ORDER: *value = h->order; return GC_OK;
    case GC_OPT_ORDER_SEED: *value = (int64_t)h->order_seed; return GC_OK;
    default: return set_err(h, GC_EINVAL, "gc_get_option: unknown option %d", option);
  }
}

extern "C" int gc_get_profile(gc_handle h, double* ms, int64_t* launches, int reset) {
  if (!h) return set_err(nullptr, GC_EINVAL, "gc_get_profile: NULL handle");
  int rc = ensure_idle(h);
  if (rc) return rc;
  collect_profile(h);
  for (int k = 0; k < kKinds; ++k) {
    if (ms) ms[k] = h->prof_ms[k];
    if (launches) launches[k] = h->prof_launches[k];
    if (reset) {
      h->prof_ms[k] = 0;
      h->prof_launches[k] = 0;
    }
  }
  return GC_OK;
}

extern "C" int gc_destroy(gc_handle h) {
  if (!h) return GC_OK;
  int rc = GC_OK;
  if (h->in_flight) {
    hipError_t e = hipEventSynchronize(h->done);
    if (e != hipSuccess) rc = set_err(nullptr, GC_EDEVICE, "gc_destroy: %s", hipGetErrorString(e));
  }
  free_ctx(h);
  return rc;
}

namespace gc {
void set_thread_error(const char* msg) { tl_error = msg; }
}  // namespace gc

extern "C" const char* gc_last_error(gc_handle h) {
  return h ? h->err.c_str() : tl_error.c_str();
}

extern "C" const char* gc_version(void) { return "0.2.0"; }
