// gc_batch.hip -- many independent graphs coloured in one launch.
//
// Each graph is coloured by one workgroup with exactly the rounds of the
// per-graph path (Algorithm 1 of Section 3.1 with every vertex its own
// block; the higher id of a conflicting pair is recoloured), so its colours
// are bit-identical to a gc_color call on it alone.  The batch only changes
// where the state lives and who runs it:
//   - a workgroup takes graphs from a device-side queue ordered largest
//     first (work buckets by log2 of the CSR size: longest-processing-time
//     order, so the big graphs do not finish last);
//   - a graph whose state fits the workgroup's LDS slice (n bytes at int8,
//     2n at int16, by its maximum degree) keeps it there, so every neighbour
//     colour gather of every round is an LDS read; larger graphs keep an
//     int32 state in the caller's colour array;
//   - the rounds are separated by workgroup barriers instead of grid-wide
//     ones, and each graph stops independently when its round has no loser;
//   - a graph with at least a workgroup's fair share of the batch's work
//     (and enough of it to occupy several workgroups) is coloured by a team
//     of K workgroups instead: it appears K times in the queue, the K
//     workgroups that take those entries split its chunks, its rounds are
//     separated by a barrier of the team, and each member keeps a replica of
//     the state in LDS, reloaded from the shared colour array after every
//     barrier; so a large graph no longer holds the whole launch to one
//     workgroup's speed.
// The state between rounds is the colour array itself (final colours >= 0,
// ~t for a vertex still being coloured with tentative colour t) plus the
// round count, which makes a step of a few rounds resumable: gc_batch_step
// advances each listed graph by at most max_rounds rounds.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <mutex>

#include "gc.h"
#include "gc_device.h"
#include "gc_internal.h"

namespace gc {

constexpr int kBatchBlock = 1024;         // threads per graph workgroup
constexpr int kBatchLds = 64 * 1024;      // LDS state slice per workgroup (bytes)
constexpr int kBatchWaves = kBatchBlock / kWave;
#ifndef GC_BATCH_SPEC_QUADS
#define GC_BATCH_SPEC_QUADS 3
#endif
#ifndef GC_BATCH_ENTRIES_PER_LANE
#define GC_BATCH_ENTRIES_PER_LANE 12
#endif
#ifndef GC_BATCH_MIN_LANES
#define GC_BATCH_MIN_LANES 1
#endif
constexpr int kSpecQuads = GC_BATCH_SPEC_QUADS;  // row quads per lane in flight (speculate)
// lanes per vertex: the largest power of two from kMinLanes to 16 with at
// least kEntriesPerLane entries of an average row per lane
constexpr int kEntriesPerLane = GC_BATCH_ENTRIES_PER_LANE;
constexpr int kMinLanes = GC_BATCH_MIN_LANES;
constexpr int kBuckets = 64;
constexpr int kMaxTeams = 256;          // graphs coloured by a team, per launch
constexpr int kMaxExtraTickets = 4096;  // queue entries beyond one per graph
constexpr int64_t kMinTeamWork = 65536; // work (entries + vertices) per team member
#ifndef GC_BATCH_TEAM_SHARE
#define GC_BATCH_TEAM_SHARE 20
#endif
// a graph of work w gets a team of floor(kTeamShare * w / (10 * fair share))
// workgroups when that is at least 2
constexpr uint64_t kTeamShare = GC_BATCH_TEAM_SHARE;
constexpr long kTeamSpinLimit = 1l << 25;

struct BatchCtrl {
  int32_t queue;    // next position in `order`
  int32_t tickets;  // entries of `order`: one per graph, K per team graph
  int32_t pad[62];
};

// Control words of one team (one 256-byte line each).
struct TeamCtrl {
  int32_t k;        // workgroups in the team
  int32_t joined;   // ranks handed out
  uint32_t arrive;  // barrier arrivals, counting up within the launch
  int32_t lost[3];  // "a vertex lost round r" at index r % 3
  int32_t left;     // vertices left uncoloured (summed over the team)
  int32_t maxdeg;   // maximum degree (over the team)
  int32_t abort;    // a barrier wait exceeded the spin limit
  int32_t pad[55];
};

// workspace: [BatchCtrl][teams: kMaxTeams TeamCtrl][order: T int32][slot: T int32]
//            [gk: G int32][descs: G gc_graph_desc (packed API only)], T = G + kMaxExtraTickets
__host__ __device__ constexpr size_t ws_teams_off() { return sizeof(BatchCtrl); }
__host__ __device__ constexpr size_t ws_order_off() {
  return ws_teams_off() + (size_t)kMaxTeams * sizeof(TeamCtrl);
}
__host__ __device__ constexpr size_t ws_slot_off(int64_t G) {
  return ws_order_off() + (size_t)(G + kMaxExtraTickets) * sizeof(int32_t);
}
__host__ __device__ constexpr size_t ws_gk_off(int64_t G) {
  return ws_slot_off(G) + (size_t)(G + kMaxExtraTickets) * sizeof(int32_t);
}
__host__ __device__ constexpr size_t ws_descs_off(int64_t G) {
  return (ws_gk_off(G) + (size_t)G * sizeof(int32_t) + 255) & ~(size_t)255;
}

// Descriptors of a packed batch.
__global__ void k_batch_descs(int64_t G, const int64_t* voff, const int64_t* eoff,
                              gc_graph_desc* d) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long g = tid; g < G; g += nth) {
    gc_graph_desc x;
    x.rowptr_off = voff[g] + g;
    x.colidx_off = eoff[g];
    x.color_off = voff[g];
    x.n = (int32_t)(voff[g + 1] - voff[g]);
    x.rounds = 0;
    x.active = 0;
    x.max_degree = 0;
    d[g] = x;
  }
}

// Largest-first order: one workgroup buckets the graphs by floor(log2(work))
// (batch_work) and writes them out bucket by bucket,
// largest bucket first.  A graph whose work w is at least a workgroup's fair
// share f (total work / nwg) would alone keep one workgroup busy for the
// whole launch, and longer under the load of the others: it gets a team of
// K = min(floor(2 w / f), nwg, w / kMinTeamWork) workgroups when K >= 2 and
// a team slot and K - 1 extra queue entries are left.  Its K entries are
// consecutive, with the team slot beside them (-1 for a graph of one
// workgroup).  Also resets the work queue.
// The work of a graph: its CSR entries and vertices when fresh; when it
// resumes from an earlier step (rounds > 0), the vertices it left uncoloured
// times two more than its average degree, an estimate of what its next
// rounds visit, so that the order and the teams follow the work left.
__device__ __forceinline__ uint64_t batch_work(const gc_graph_desc& x, const int32_t* rowptr_base) {
  const int64_t nnz = x.n > 0 ? rowptr_base[x.rowptr_off + x.n] : 0;
  if (x.rounds > 0 && x.n > 0 && x.active >= 0 && x.active <= x.n)
    return (uint64_t)x.active * (uint64_t)(nnz / x.n + 2) + 1;
  return (uint64_t)nnz + (uint64_t)x.n + 1;
}

__global__ __launch_bounds__(1024) void k_batch_plan(int64_t G, const gc_graph_desc* d,
                                                     const int32_t* rowptr_base, int32_t* order,
                                                     int32_t* slot, int32_t* gk, TeamCtrl* teams,
                                                     BatchCtrl* ctrl, int nwg) {
  __shared__ int hist[kBuckets];
  __shared__ int base[kBuckets];
  __shared__ unsigned long long total;
  __shared__ int nteams, extra;
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) {
    total = 0;
    nteams = 0;
    extra = 0;
  }
  __syncthreads();
  uint64_t mine = 0;
  for (long g = threadIdx.x; g < G; g += blockDim.x) mine += batch_work(d[g], rowptr_base);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mine += shfl_xor64(mine, off);
  if (lane_id() == 0 && mine) atomicAdd(&total, (unsigned long long)mine);
  __syncthreads();
  const uint64_t fair = total / (uint64_t)(nwg > 0 ? nwg : 1) + 1;
  for (long g = threadIdx.x; g < G; g += blockDim.x) {
    const uint64_t w = batch_work(d[g], rowptr_base);
    uint64_t q = kTeamShare * w / (10 * fair);
    if (q > (uint64_t)nwg) q = (uint64_t)nwg;
    if (q > w / kMinTeamWork) q = w / kMinTeamWork;
    int k = 1, s = -1;
    if (q >= 2) {
      const int ts = atomicAdd(&nteams, 1);
      const int x = atomicAdd(&extra, (int)q - 1);
      if (ts < kMaxTeams && x + (int)q - 1 <= kMaxExtraTickets) {
        k = (int)q;
        s = ts;
        TeamCtrl* t = teams + s;
        t->k = k;
        t->joined = 0;
        t->arrive = 0;
        t->lost[0] = t->lost[1] = t->lost[2] = 0;
        t->left = 0;
        t->maxdeg = 0;
        t->abort = 0;
      }
    }
    gk[g] = k | ((s + 1) << 16);
    atomicAdd(&hist[63 - __builtin_clzll(w)], k);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = kBuckets - 1; b >= 0; --b) {
      base[b] = acc;
      acc += hist[b];
    }
    ctrl->queue = 0;
    ctrl->tickets = acc;
  }
  __syncthreads();
  for (long g = threadIdx.x; g < G; g += blockDim.x) {
    const uint64_t w = batch_work(d[g], rowptr_base);
    const int k = gk[g] & 0xffff, s = (gk[g] >> 16) - 1;
    const int pos = atomicAdd(&base[63 - __builtin_clzll(w)], k);
    for (int j = 0; j < k; ++j) {
      order[pos + j] = (int32_t)g;
      slot[pos + j] = s;
    }
  }
}

struct GraphRun {
  const int32_t* rp;
  const int32_t* ci;
  int32_t* out;  // the graph's colour / state array (int32)
  int n;
  int rounds_in;
  int max_rounds;
};

// The row [b, e) read as aligned 16-byte quads: the quad holding entry b
// starts `lead` entries before it.  Every quad that holds at least one entry
// of the row lies inside the 16-byte block of an in-bounds entry, so it never
// leaves the array's last page; entries outside the row are masked.
struct Quads {
  const int4* q;
  int lead;  // entries of the first quad before b
  int len;   // lead + (e - b): entries from q[0] up to the row's end
};

__device__ __forceinline__ Quads quads_of(const int32_t* ci, int b, int e) {
  Quads r;
  r.lead = (int)(((uintptr_t)(ci + b) >> 2) & 3);
  r.q = (const int4*)(ci + b - r.lead);
  r.len = e - b + r.lead;
  return r;
}

__device__ __forceinline__ void unpack(const int4 w, int* u) {
  u[0] = w.x;
  u[1] = w.y;
  u[2] = w.z;
  u[3] = w.w;
}

// Least colour not final on any neighbour of the row [b, e), by a group of L
// lanes (gl = lane in group) with 16-byte loads, kSpecQuads quads per lane in
// flight.  Every lane returns the result.
template <typename S>
__device__ __forceinline__ int spec_quads(const int32_t* __restrict__ ci, const S* __restrict__ st,
                                          int b, int e, int L, int gl) {
  const Quads r = quads_of(ci, b, e);
  const int nq = (r.len + 3) >> 2;
  int base = 0;
  for (;;) {
    uint64_t m = 0;
    auto mark = [&](const int4 w, int idx0) {
      int u[4];
      unpack(w, u);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int idx = idx0 + j;
        if (idx >= r.lead && idx < r.len) {
          const int c = st[u[j]];
          const unsigned rel = (unsigned)c - (unsigned)base;
          if (c >= 0 && rel < 64u) m |= 1ull << rel;
        }
      }
    };
    for (int i = gl; i < nq; i += kSpecQuads * L) {
      // kSpecQuads quads per lane in flight, then their gathers
      int4 w[kSpecQuads];
#pragma unroll
      for (int j = 0; j < kSpecQuads; ++j)
        if (i + j * L < nq) w[j] = r.q[i + j * L];
#pragma unroll
      for (int j = 0; j < kSpecQuads; ++j)
        if (i + j * L < nq) mark(w[j], 4 * (i + j * L));
    }
    for (int off = L / 2; off > 0; off >>= 1) m |= shfl_xor64(m, off);
    if (m != ~0ull) return base + __builtin_ctzll(~m);
    base += 64;  // all of base..base+63 are taken: slide the window
  }
}

// Conflict scan of v (tentative colour t) over its lower neighbours, rows
// ascending, by a group of L lanes (lanes gbase .. gbase + L - 1, mask
// gmask) with 16-byte loads: each step covers L consecutive quads.  With
// `skip` (not null) the scan starts at offset *skip of the row, every lower
// neighbour before it being final, and leaves there the offset of the first
// lower neighbour seen still uncoloured, or of the point where the scan
// stopped when it saw none (the per-graph path's resume rule: final colours
// never change).  Stops at the first conflict or the first id >= v.
template <typename S>
__device__ __forceinline__ bool detect_quads(const int32_t* __restrict__ ci,
                                             const S* __restrict__ st, int b, int e, int v, int t,
                                             int L, int gl, uint64_t gmask, int gbase, int* skip) {
  const int from = skip ? *skip : 0;
  const Quads r = quads_of(ci, b + from, e);
  int first = -1;  // row offset of the first uncoloured lower neighbour seen
  for (int k0 = 0; k0 < r.len; k0 += 4 * L) {  // group-uniform
    const int k = k0 + 4 * gl;
    int u[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    if (k < r.len) unpack(r.q[k >> 2], u);
    int ja = 4, jc = 4, jp = 4;  // this lane's first uncoloured / conflict / past entry
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = k + j;
      if (idx < r.lead) continue;  // before the scan's start
      const bool in = idx < r.len;
      const bool low = in && u[j] < v;
      const int s = low ? (int)st[u[j]] : 0;
      if (low && s < 0 && ja == 4) ja = j;
      // decode, do not test the sign: a neighbour that wins in this same
      // pass flips ~t to t concurrently and must still count
      if (low && tent_of(s) == t && jc == 4) jc = j;
      if (!low && jp == 4) jp = j;
    }
    const uint64_t am = (__ballot(ja < 4) & gmask) >> gbase;
    const uint64_t cm = (__ballot(jc < 4) & gmask) >> gbase;
    const uint64_t pm = (__ballot(jp < 4) & gmask) >> gbase;
    // offsets in the row of the first such entries (rows ascend, so every
    // lower entry precedes the first past one)
    auto pos = [&](uint64_t mask, int jl) {
      const int lane = __builtin_ctzll(mask);
      const int j = __shfl(jl, gbase + lane);
      return from + k0 + 4 * lane + j - r.lead;
    };
    if (first < 0 && am) first = pos(am, ja);
    if (cm) {
      if (skip) *skip = first >= 0 ? first : pos(cm, jc);
      return true;
    }
    if (pm) {
      if (skip) *skip = first >= 0 ? first : pos(pm, jp);
      return false;
    }
  }
  if (skip) *skip = first >= 0 ? first : e - b;
  return false;
}

// One pass (speculate or detect) of one round over the graph's uncoloured
// vertices by the whole workgroup (member `rank` of a team of K; 0 of 1
// alone): each wavefront walks 64-vertex chunks, ballots the uncoloured ones
// and hands them to its groups of L lanes.  `skipv` (or null) holds each
// vertex's resume offset for the detect scans; `mirror` (or null) receives
// every state write as well (a team's shared copy).
template <typename S, bool SPEC>
__device__ __forceinline__ bool graph_pass(const GraphRun& g, S* st, int32_t* skipv, int L,
                                           int rank = 0, int K = 1, int32_t* mirror = nullptr) {
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int grp = lane / L;
  const int Gw = kWave / L;
  const uint64_t gmask = (L == kWave) ? ~0ull : (((1ull << L) - 1) << (grp * L));
  const int wave = threadIdx.x / kWave;
  bool lost = false;
  for (int ch = rank * kBatchWaves + wave; ch * kWave < g.n; ch += K * kBatchWaves) {
    const int v = ch * kWave + lane;
    bool act = false;
    int s = 0, b = 0, e = 0;
    if (v < g.n) {
      s = st[v];
      if (s < 0) {
        b = g.rp[v];
        e = g.rp[v + 1];
        act = true;
      }
    }
    const uint64_t am = __ballot(act);
    if (am == 0) continue;
    const int cnt = __popcll(am);
    for (int p = 0; p < cnt; p += Gw) {
      const int k = p + grp;
      const bool valid = k < cnt;
      const int pos = nth_set_bit(am, valid ? k : 0);
      const int vb = __shfl(b, pos);
      const int ve = __shfl(e, pos);
      const int vs = __shfl(s, pos);
      const int vv = ch * kWave + pos;
      if (valid) {  // group-uniform
        if (SPEC) {
          const int t = spec_quads<S>(g.ci, st, vb, ve, L, gl);
          if (gl == 0) {
            st[vv] = (S)~t;
            if (mirror) mirror[vv] = ~t;
          }
        } else {
          const int t = ~vs;
          int sk = skipv ? skipv[vv] : 0;
          const int sk0 = sk;
          const bool lose = detect_quads<S>(g.ci, st, vb, ve, vv, t, L, gl, gmask, grp * L,
                                            skipv ? &sk : nullptr);
          if (gl == 0) {
            if (!lose) {
              st[vv] = (S)t;
              if (mirror) mirror[vv] = t;
            }
            if (skipv && sk != sk0) skipv[vv] = sk;
            lost |= lose;
          }
        }
      }
    }
  }
  return lost;
}

// Rounds of one graph until done or max_rounds more rounds have run.
// Returns the rounds completed; *left receives the vertices still uncoloured.
// A graph whose state is in LDS keeps each vertex's resume offset in its
// colour array during the rounds (the array receives the state at the end).
template <typename S, bool IN_LDS>
__device__ __forceinline__ int run_graph(const GraphRun& g, S* st, int L, int* left) {
  __shared__ int sh_cnt;
  int32_t* const skipv = IN_LDS ? g.out : nullptr;
  bool any = false;
  int r = g.rounds_in;
  if (r == 0) {
    // round 1 in closed form (sorted rows): v keeps colour 0 iff no neighbour
    // has a lower id
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) {
      const int b = g.rp[v], e = g.rp[v + 1];
      const bool lose = e > b && g.ci[b] < v;
      st[v] = lose ? (S)-1 : (S)0;
      if (IN_LDS) skipv[v] = 0;
      any |= lose;
    }
    r = g.n > 0 ? 1 : 0;
  } else {
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) {
      const int s = g.out[v];
      if (IN_LDS) {
        st[v] = (S)s;
        skipv[v] = 0;
      }
      any |= s < 0;
    }
  }
  bool more = __syncthreads_or(any);
  // (r < n: every round colours the lowest uncoloured vertex, so R <= n;
  // the bound only stops a broken invariant from spinning forever, and the
  // graph then reports uncoloured vertices)
  while (more && r < g.n && (g.max_rounds <= 0 || r - g.rounds_in < g.max_rounds)) {
    ++r;
    graph_pass<S, true>(g, st, skipv, L);
    __syncthreads();
    const bool lost = graph_pass<S, false>(g, st, skipv, L > 4 ? L / 2 : L);
    more = __syncthreads_or(lost);
  }
  if (threadIdx.x == 0) sh_cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int v = threadIdx.x; v < g.n; v += blockDim.x) {
    const int s = st[v];
    if (IN_LDS) g.out[v] = s;
    mine += s < 0;
  }
  // (a cross-lane sum first: one LDS atomic per wave, not per thread)
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if (lane_id() == 0 && mine) atomicAdd(&sh_cnt, mine);
  __syncthreads();
  *left = sh_cnt;
  __syncthreads();
  return r;
}

// Barrier of the K workgroups of a team.  Every member runs: each holds
// one of the team's K consecutive queue entries, a workgroup takes its next
// entry only after finishing its graph, and the graphs of earlier entries
// never wait on later ones, so the members of the earliest unfinished team
// are all taken (the launch is at most two workgroups per compute unit, all
// resident).  As the persistent kernel's grid barrier: agent-scope release
// and acquire around one arrival counter; a wait beyond the spin limit sets
// the team's abort flag, after which the team's barriers return at once.
__device__ __forceinline__ bool team_barrier(TeamCtrl* tc, int K, unsigned& phase) {
  __shared__ int sh_abort;
  __syncthreads();
  if (threadIdx.x == 0) {
    ++phase;
    const unsigned target = phase * (unsigned)K;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(&tc->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ab = __hip_atomic_load(&tc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (!ab && __hip_atomic_load(&tc->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                      target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kTeamSpinLimit) {
        __hip_atomic_store(&tc->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ab = 1;
      } else if ((spins & 1023) == 0) {
        ab = __hip_atomic_load(&tc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh_abort = ab;
  }
  __syncthreads();
  return sh_abort == 0;
}

__device__ __forceinline__ int team_flag(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Start of a team's graph: each member takes every K-th vertex for round 1
// in closed form (or, on resumption, looks for vertices still uncoloured)
// and its share of the maximum degree; then the team's first barrier.  The
// shared state is the graph's colour array (int32).  "Some vertex lost round
// r" is gathered in tc->lost[r % 3]: set before the round's last barrier,
// read after it by every member (so all leave the loop together), and
// cleared by member 0 at the start of round r + 3, after every member has
// read it.
__device__ bool team_start(const GraphRun& g, TeamCtrl* tc, int rank, int K, unsigned& phase,
                           int& r) {
  int32_t* const st = g.out;
  const int t0 = rank * (int)blockDim.x + (int)threadIdx.x;
  const int tstride = K * (int)blockDim.x;
  bool any = false;
  int mx = 0;
  r = g.rounds_in;
  for (int v = t0; v < g.n; v += tstride) {
    const int b = g.rp[v], e = g.rp[v + 1];
    mx = max(mx, e - b);
    if (r == 0) {  // round 1 in closed form, as run_graph
      const bool lose = e > b && g.ci[b] < v;
      st[v] = lose ? -1 : 0;
      any |= lose;
    } else {
      any |= st[v] < 0;
    }
  }
  if (r == 0) r = g.n > 0 ? 1 : 0;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
  if (lane_id() == 0 && mx) atomicMax(&tc->maxdeg, mx);
  if (__syncthreads_or(any) && threadIdx.x == 0) atomicOr(&tc->lost[r % 3], 1);
  return team_barrier(tc, K, phase);
}

// The rounds of one graph by member `rank` of a team of K workgroups: the
// same rounds as run_graph, each member taking every K-th 64-vertex chunk,
// the passes separated by team barriers.  With IN_LDS every member keeps a
// replica of the whole state in its LDS slice, reloaded from the shared
// colour array after each barrier, and writes its vertices to both, so the
// neighbour gathers stay LDS reads; otherwise the passes work on the shared
// array.  Returns the rounds completed; *left receives the vertices still
// uncoloured (all of them if a barrier gave up).
template <typename S, bool IN_LDS>
__device__ int team_rounds(const GraphRun& g, S* lds, TeamCtrl* tc, int rank, int K, int L,
                           unsigned& phase, int r, bool ok, int* left) {
  __shared__ int sh_cnt;
  int32_t* const gst = g.out;
  S* const st = IN_LDS ? lds : (S*)gst;
  int32_t* const mirror = IN_LDS ? gst : nullptr;
  // the shared array read as aligned 16-byte quads (as quads_of: every quad
  // read holds at least one of the graph's entries), four per thread in flight
  const int lead = (int)(((uintptr_t)gst >> 2) & 3);
  const int4* const q = (const int4*)(gst - lead);
  const int nq = (g.n + lead + 3) >> 2;
  auto reload = [&]() {
    if (IN_LDS) {
      for (int i0 = threadIdx.x; i0 < nq; i0 += 4 * blockDim.x) {
        int4 w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (i0 + j * (int)blockDim.x < nq) w[j] = q[i0 + j * blockDim.x];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = i0 + j * (int)blockDim.x;
          if (i >= nq) continue;
          int u[4];
          unpack(w[j], u);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int v = 4 * i + k - lead;
            if (v >= 0 && v < g.n) lds[v] = (S)u[k];
          }
        }
      }
      __syncthreads();
    }
  };
  bool more = ok && team_flag(&tc->lost[r % 3]) != 0;
  while (more && r < g.n && (g.max_rounds <= 0 || r - g.rounds_in < g.max_rounds)) {
    ++r;
    if (rank == 0 && threadIdx.x == 0)
      __hip_atomic_store(&tc->lost[r % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    reload();
    graph_pass<S, true>(g, st, nullptr, L, rank, K, mirror);
    if (!(ok = team_barrier(tc, K, phase))) break;
    reload();
    const bool lost = graph_pass<S, false>(g, st, nullptr, L > 4 ? L / 2 : L, rank, K, mirror);
    if (__syncthreads_or(lost) && threadIdx.x == 0) atomicOr(&tc->lost[r % 3], 1);
    if (!(ok = team_barrier(tc, K, phase))) break;
    more = team_flag(&tc->lost[r % 3]) != 0;
  }
  int mine = 0;
  for (int v = rank * (int)blockDim.x + (int)threadIdx.x; v < g.n; v += K * (int)blockDim.x)
    mine += gst[v] < 0;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if (threadIdx.x == 0) sh_cnt = 0;
  __syncthreads();
  if (lane_id() == 0 && mine) atomicAdd(&sh_cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0 && sh_cnt) atomicAdd(&tc->left, sh_cnt);
  ok = team_barrier(tc, K, phase) && ok;
  *left = ok ? team_flag(&tc->left) : g.n;
  return r;
}

// A team member's whole graph: the start, then the rounds with the state
// placement run_graph would pick (by the team's maximum degree).
__device__ __forceinline__ int run_team(const GraphRun& g, char* smem, TeamCtrl* tc, int rank, int K, int L,
                        int* left) {
  unsigned phase = 0;
  int r = 0;
  const bool ok = team_start(g, tc, rank, K, phase, r);
  const int maxdeg = team_flag(&tc->maxdeg);  // complete: every member added it before the barrier
  if (maxdeg <= 127 && g.n <= kBatchLds)
    return team_rounds<int8_t, true>(g, (int8_t*)smem, tc, rank, K, L, phase, r, ok, left);
  if (maxdeg <= 32767 && 2 * g.n <= kBatchLds)
    return team_rounds<int16_t, true>(g, (int16_t*)smem, tc, rank, K, L, phase, r, ok, left);
  return team_rounds<int32_t, false>(g, nullptr, tc, rank, K, L, phase, r, ok, left);
}

__device__ __forceinline__ int dispatch_state(const GraphRun& g, int maxdeg, char* smem, int L,
                                              int* left) {
  if (maxdeg <= 127 && g.n <= kBatchLds) return run_graph<int8_t, true>(g, (int8_t*)smem, L, left);
  if (maxdeg <= 32767 && 2 * g.n <= kBatchLds)
    return run_graph<int16_t, true>(g, (int16_t*)smem, L, left);
  if (4 * g.n <= kBatchLds) return run_graph<int32_t, true>(g, (int32_t*)smem, L, left);
  return run_graph<int32_t, false>(g, g.out, L, left);
}

__global__ __launch_bounds__(kBatchBlock, 8) void k_batch_color(gc_graph_desc* d,
                                                            const int32_t* rowptr_base,
                                                            const int32_t* colidx_base,
                                                            int32_t* colors_base, int max_rounds,
                                                            const int32_t* order,
                                                            const int32_t* slot, TeamCtrl* teams,
                                                            BatchCtrl* ctrl) {
  extern __shared__ char smem[];
  __shared__ int sh_idx, sh_max, sh_rank;
  const int tickets = ctrl->tickets;
  for (;;) {
    if (threadIdx.x == 0) {
      sh_idx = atomicAdd(&ctrl->queue, 1);
      sh_max = 0;
    }
    __syncthreads();
    const int idx = sh_idx;
    if (idx >= tickets) break;  // workgroup-uniform
    const int gi = order[idx];
    const int ts = slot[idx];
    const gc_graph_desc x = d[gi];
    GraphRun g;
    g.rp = rowptr_base + x.rowptr_off;
    g.ci = colidx_base + x.colidx_off;
    g.out = colors_base + x.color_off;
    g.n = x.n;
    g.rounds_in = x.rounds;
    g.max_rounds = max_rounds;
    if (ts >= 0) {  // one member of a team (workgroup-uniform)
      TeamCtrl* tc = teams + ts;
      if (threadIdx.x == 0) sh_rank = atomicAdd(&tc->joined, 1);
      __syncthreads();
      const int rank = sh_rank, K = tc->k;
      const double avg = g.n > 0 ? (double)g.rp[g.n] / g.n : 0.0;
      int L = kMinLanes;
      while (L < 16 && 2.0 * L * kEntriesPerLane <= avg) L *= 2;
      int left = 0;
      const int rounds = run_team(g, smem, tc, rank, K, L, &left);
      if (rank == 0 && threadIdx.x == 0) {
        d[gi].rounds = rounds;
        d[gi].active = left;
        d[gi].max_degree = team_flag(&tc->maxdeg);
      }
      __syncthreads();  // sh_idx / sh_rank are rewritten for the next entry
      continue;
    }
    int mx = 0;
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) mx = max(mx, g.rp[v + 1] - g.rp[v]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
    if (lane_id() == 0 && mx) atomicMax(&sh_max, mx);
    __syncthreads();
    const int maxdeg = sh_max;
    const int64_t nnz = g.n > 0 ? (int64_t)g.rp[g.n] : 0;
    const double avg = g.n > 0 ? (double)nnz / g.n : 0.0;
    int left = 0, rounds;
    int L = kMinLanes;
    while (L < 16 && 2.0 * L * kEntriesPerLane <= avg) L *= 2;
    rounds = dispatch_state(g, maxdeg, smem, L, &left);
    if (threadIdx.x == 0) {
      d[gi].rounds = rounds;
      d[gi].active = left;
      d[gi].max_degree = maxdeg;
    }
    __syncthreads();  // sh_idx / sh_max are rewritten for the next graph
  }
}

__global__ void k_batch_rounds_out(int64_t G, const gc_graph_desc* d, int32_t* rounds_out) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long g = tid; g < G; g += nth) rounds_out[g] = d[g].rounds;
}

// Two workgroups per compute unit (two 64 KB LDS slices per 160 KB), all
// resident at once, whatever the number of graphs: a team can use workgroups
// beyond one per graph.
static int batch_grid() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
  return 2 * (cus > 0 ? cus : 1);
}

static int run_batch(int64_t G, gc_graph_desc* d, const int32_t* rpb, const int32_t* cib,
                     int32_t* colb, int max_rounds, void* ws, hipStream_t s) {
  static bool lds_set = false;
  if (!lds_set) {  // allow the 64 KB dynamic slice on top of the static LDS
    hipError_t e = hipFuncSetAttribute((const void*)k_batch_color,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLds);
    if (e != hipSuccess) return (int)e;
    lds_set = true;
  }
  BatchCtrl* ctrl = (BatchCtrl*)ws;
  TeamCtrl* teams = (TeamCtrl*)((char*)ws + ws_teams_off());
  int32_t* order = (int32_t*)((char*)ws + ws_order_off());
  int32_t* slot = (int32_t*)((char*)ws + ws_slot_off(G));
  int32_t* gk = (int32_t*)((char*)ws + ws_gk_off(G));
  const int grid = batch_grid();
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, s, G, d, rpb, order, slot, gk, teams,
                     ctrl, grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(k_batch_color, dim3(grid), dim3(kBatchBlock), kBatchLds, s, d, rpb, cib, colb,
                     max_rounds, order, slot, teams, ctrl);
  return (int)hipGetLastError();
}

}  // namespace gc

using namespace gc;

namespace {
int fail(int code, const char* msg) {
  set_thread_error(msg);
  return code;
}
}  // namespace

extern "C" size_t gc_batch_workspace_bytes(int64_t num_graphs, const int64_t* voff,
                                           const int64_t* eoff) {
  if (num_graphs < 0 || num_graphs > INT32_MAX || !voff || !eoff) return 0;
  if (voff[0] != 0 || eoff[0] != 0) return 0;
  for (int64_t g = 0; g < num_graphs; ++g) {
    const int64_t n = voff[g + 1] - voff[g], nnz = eoff[g + 1] - eoff[g];
    if (n < 0 || nnz < 0 || n >= INT32_MAX || nnz > INT32_MAX) return 0;
  }
  return ws_descs_off(num_graphs) + (size_t)num_graphs * sizeof(gc_graph_desc) + 256;
}

extern "C" int gc_color_batch(int64_t num_graphs, const int64_t* voff, const int64_t* eoff,
                              const int32_t* rowptr_local, const int32_t* colidx_local,
                              int32_t* colors_out, int32_t* rounds_out, void* workspace,
                              size_t workspace_bytes, void* stream) {
  if (num_graphs < 0 || num_graphs > INT32_MAX) return fail(GC_EINVAL, "gc_color_batch: bad num_graphs");
  if (num_graphs == 0) return GC_OK;
  if (!voff || !eoff || !rowptr_local || !workspace)
    return fail(GC_EINVAL, "gc_color_batch: NULL array");
  const size_t need = ws_descs_off(num_graphs) + (size_t)num_graphs * sizeof(gc_graph_desc) + 256;
  if (workspace_bytes < need) return fail(GC_EINVAL, "gc_color_batch: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();
  gc_graph_desc* d = (gc_graph_desc*)((char*)workspace + ws_descs_off(num_graphs));
  const int grid = (int)((num_graphs + 255) / 256 < 4096 ? (num_graphs + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_batch_descs, dim3(grid), dim3(256), 0, s, num_graphs, voff, eoff, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GC_EDEVICE, hipGetErrorString(e));
  int rc = run_batch(num_graphs, d, rowptr_local, colidx_local, colors_out, 0, workspace, s);
  if (rc) return fail(GC_EDEVICE, hipGetErrorString((hipError_t)rc));
  if (rounds_out) {
    hipLaunchKernelGGL(k_batch_rounds_out, dim3(grid), dim3(256), 0, s, num_graphs, d, rounds_out);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(GC_EDEVICE, hipGetErrorString(e));
  }
  return GC_OK;
}

// ------------------------------------------ batch without allocation --

namespace gc {

// Workspace of gc_color_batch_noalloc: a file-scope device array of
// kStaticBatchBytes, enough for kStaticBatchGraphs graphs.  Each GPU holds
// its own copy from the first launch of this library's kernels on it until
// the process ends.
constexpr int64_t kStaticBatchGraphs = GC_STATIC_BATCH_MAX_GRAPHS;
constexpr size_t kStaticBatchBytes =
    ws_descs_off(kStaticBatchGraphs) + (size_t)kStaticBatchGraphs * sizeof(gc_graph_desc) + 256;
static __device__ __align__(256) uint8_t scratch[kStaticBatchBytes];

// Device address of `scratch` on each device, looked up once per device with
// that device current (host code never passes the array's name itself).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices] = {};

static int static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace gc

extern "C" int gc_color_batch_noalloc(int64_t num_graphs, const int64_t* voff, const int64_t* eoff,
                                      const int32_t* rowptr_local, const int32_t* colidx_local,
                                      int32_t* colors_out, int32_t* rounds_out, void* stream) {
  if (num_graphs < 0) return fail(GC_EINVAL, "gc_color_batch_noalloc: bad num_graphs");
  if (num_graphs > gc::kStaticBatchGraphs)
    return fail(GC_ETOOBIG, "gc_color_batch_noalloc: more graphs than GC_STATIC_BATCH_MAX_GRAPHS");
  if (num_graphs == 0) return GC_OK;
  void* ws = nullptr;
  const int rc = gc::static_scratch(&ws);
  if (rc) return fail(GC_EDEVICE, hipGetErrorString((hipError_t)rc));
  return gc_color_batch(num_graphs, voff, eoff, rowptr_local, colidx_local, colors_out,
                        rounds_out, ws, gc::kStaticBatchBytes, stream);
}

extern "C" size_t gc_batch_step_workspace_bytes(int64_t num_graphs, int64_t total_vertices) {
  if (num_graphs < 0 || num_graphs > INT32_MAX || total_vertices < 0) return 0;
  return ws_descs_off(num_graphs) + 256;
}

extern "C" int gc_batch_step(int64_t num_graphs, gc_graph_desc* descs, const int32_t* rowptr_base,
                             const int32_t* colidx_base, int32_t* colors_base, int32_t max_rounds,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (num_graphs < 0 || num_graphs > INT32_MAX) return fail(GC_EINVAL, "gc_batch_step: bad num_graphs");
  if (num_graphs == 0) return GC_OK;
  if (!descs || !rowptr_base || !workspace) return fail(GC_EINVAL, "gc_batch_step: NULL array");
  if (max_rounds < 0) return fail(GC_EINVAL, "gc_batch_step: negative max_rounds");
  if (workspace_bytes < gc_batch_step_workspace_bytes(num_graphs, 0))
    return fail(GC_EINVAL, "gc_batch_step: workspace too small");
  (void)hipGetLastError();
  int rc = run_batch(num_graphs, descs, rowptr_base, colidx_base, colors_base, max_rounds,
                     workspace, (hipStream_t)stream);
  if (rc) return fail(GC_EDEVICE, hipGetErrorString((hipError_t)rc));
  return GC_OK;
}

// ------------------------------------------------- segment copies --

namespace gc {

// Piece p of the concatenated segments: the segment is the last one whose
// first piece is <= p (binary search, the same in every thread of the
// workgroup), and the piece covers words [q * P, min((q + 1) * P, words)) of
// it, q = p - first_piece.
__global__ __launch_bounds__(kBlock) void k_copy_segments(const gc_segment* __restrict__ seg,
                                                          int64_t count, int64_t pieces) {
  for (int64_t p = blockIdx.x; p < pieces; p += gridDim.x) {  // workgroup-uniform
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (seg[mid].first_piece <= p) lo = mid;
      else hi = mid - 1;
    }
    const gc_segment x = seg[lo];
    const int64_t start = (p - x.first_piece) * GC_COPY_PIECE_WORDS;
    if (start < 0 || start >= x.words) continue;
    const int64_t end = start + GC_COPY_PIECE_WORDS < x.words ? start + GC_COPY_PIECE_WORDS : x.words;
    const int32_t* __restrict__ src = (const int32_t*)x.src;
    int32_t* __restrict__ dst = (int32_t*)x.dst;
    for (int64_t k = start + threadIdx.x; k < end; k += blockDim.x) dst[k] = src[k];
  }
}

}  // namespace gc

extern "C" int gc_copy_segments(int64_t count, const gc_segment* segs, int64_t pieces,
                                void* stream) {
  if (count < 0 || pieces < 0) return fail(GC_EINVAL, "gc_copy_segments: negative count or pieces");
  if (count == 0 || pieces == 0) return GC_OK;
  if (!segs) return fail(GC_EINVAL, "gc_copy_segments: NULL descriptors");
  (void)hipGetLastError();
  const int grid = (int)(pieces < 4096 ? pieces : 4096);
  hipLaunchKernelGGL(gc::k_copy_segments, dim3(grid), dim3(gc::kBlock), 0, (hipStream_t)stream,
                     segs, count, pieces);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GC_EDEVICE, hipGetErrorString(e));
  return GC_OK;
}

