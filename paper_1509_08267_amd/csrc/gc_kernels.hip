// gc_kernels.hip -- gfx950 kernels of round-synchronous speculative colouring.
//
// One round (Algorithm 1 of Section 3.1 with every vertex its own block):
//   speculate  each uncoloured vertex v takes the least colour that is not
//              final on any neighbour (First Fit, Section 3);
//   detect     v loses when a lower-id neighbour also coloured this round
//              took the same colour; otherwise v's colour becomes final.
// Round 1 needs no speculate pass: nothing is final yet, so every vertex
// tries colour 0, which the initial state -1 (= ~0) already encodes.
//
// Work mapping (wave64):
//   light  deg <= light_max: a group of L lanes per vertex (L = 1..64).
//          Each wavefront walks 64 consecutive vertex ids at a time, ballots
//          the uncoloured light ones and hands them to its 64/L groups in
//          ascending order (an in-wave prefix sum over the ballot), so rows
//          are read in address order and no global worklist or append
//          atomics exist.
//   medium light_max < deg < heavy threshold: one wavefront per vertex,
//          from a static list built once per graph.
//   heavy  one 256-thread workgroup per vertex, from a static list; its
//          forbidden-colour window is a bitmask in LDS.
// The forbidden colours of a light or medium vertex are a 64-bit register
// mask per lane, OR-reduced across the group with cross-lane shuffles; the
// pick is find-first-zero.  Colours beyond the first 64 (or 4096 for heavy
// vertices) are handled by sliding the window, which only happens when a
// vertex sees that many distinct final colours.
//
// The per-vertex state is int8, int16 or int32 (template S) by maximum
// degree: a narrower state keeps the gathered array resident in the L2 of
// each XCD.  A final pass widens it into the caller's int32 colours.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "gc_device.h"
#include "gc_internal.h"

namespace gc {

enum { kSpec = 0, kDetect = 1 };

// ------------------------------------------------ per-vertex, workgroup --

struct HeavySmem {
  uint32_t bm[kHeavyWindow / 32];
  uint64_t am[4][kWavesPerBlock], cm[4][kWavesPerBlock], pm[4][kWavesPerBlock];  // detect_block_skip
  int first;
  int cnt, flag;              // detect_block_list: list length so far, conflict seen
  int wact[kWavesPerBlock];   // per-wave tallies of a detect phase
  int wlost[kWavesPerBlock];
  int wcls[kWavesPerBlock];
};

template <typename RP, typename S>
__device__ int spec_block(const int32_t* __restrict__ colidx, const S* __restrict__ st,
                          RP b, RP e, HeavySmem& sm, int base0 = 0) {
  const int tid = threadIdx.x;
  int base = base0;
  for (;;) {
    for (int w = tid; w < kHeavyWindow / 32; w += kBlock) sm.bm[w] = 0;
    if (tid == 0) sm.first = INT_MAX;
    __syncthreads();
    uint64_t m = 0;
    RP k = b + tid;
    for (; k + kBlock < e; k += 2 * kBlock) {
      int c0 = st[colidx[k]];
      int c1 = st[colidx[k + kBlock]];
      unsigned r0 = (unsigned)c0 - (unsigned)base;
      unsigned r1 = (unsigned)c1 - (unsigned)base;
      if (c0 >= 0) {
        if (r0 < 64u) m |= 1ull << r0;
        else if (r0 < (unsigned)kHeavyWindow) atomicOr(&sm.bm[r0 >> 5], 1u << (r0 & 31));
      }
      if (c1 >= 0) {
        if (r1 < 64u) m |= 1ull << r1;
        else if (r1 < (unsigned)kHeavyWindow) atomicOr(&sm.bm[r1 >> 5], 1u << (r1 & 31));
      }
    }
    if (k < e) {
      int c0 = st[colidx[k]];
      unsigned r0 = (unsigned)c0 - (unsigned)base;
      if (c0 >= 0) {
        if (r0 < 64u) m |= 1ull << r0;
        else if (r0 < (unsigned)kHeavyWindow) atomicOr(&sm.bm[r0 >> 5], 1u << (r0 & 31));
      }
    }
    m = group_or<kWave>(m);
    if (lane_id() == 0) {
      atomicOr(&sm.bm[0], (uint32_t)m);
      atomicOr(&sm.bm[1], (uint32_t)(m >> 32));
    }
    __syncthreads();
    for (int w = tid; w < kHeavyWindow / 32; w += kBlock) {
      uint32_t x = sm.bm[w];
      if (x != ~0u) atomicMin(&sm.first, w * 32 + __builtin_ctz(~x));
    }
    __syncthreads();
    int f = sm.first;
    __syncthreads();  // everyone has read first/bm before they are reused
    if (f != INT_MAX) return base + f;
    base += kHeavyWindow;
  }
}

template <typename RP, typename S>
__device__ bool detect_block(const int32_t* __restrict__ colidx, const S* __restrict__ st,
                             RP b, RP e, int v, int t, bool sorted) {
  const int tid = threadIdx.x;
  for (RP kb = b; kb < e; kb += kBlock) {
    RP k = kb + tid;
    int conf = 0, past = 0;
    if (k < e) {
      int u = colidx[k];
      if (u < v) conf = tent_of(st[u]) == t;
      else past = 1;
    } else {
      past = 1;
    }
    if (__syncthreads_or(conf)) return true;
    if (sorted && __syncthreads_or(past)) return false;
  }
  return false;
}

// detect_lane_skip's scan for one vertex by the whole block (sorted rows), four
// entries per thread in flight: a step covers 1,024 entries as four
// sub-ranges of 256 visited in order.  The waves' ballots of "uncoloured",
// "conflict" and "past the lower prefix" meet in LDS, and every thread reads
// the first set position of each.  Every thread returns the same result and
// *skip.
template <typename RP, typename S>
__device__ bool detect_block_skip(const int32_t* __restrict__ colidx, const S* __restrict__ st,
                                  RP b, RP e, int v, int t, int* skip, HeavySmem& sm) {
  const int tid = threadIdx.x;
  const int wv = tid / kWave;
  int first = -1;
  for (RP kb = b + *skip; kb < e; kb += 4 * kBlock) {
    int u[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const RP k = kb + j * kBlock + tid;
      u[j] = k < e ? colidx[k] : INT32_MAX;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool low = u[j] < v;
      const uint64_t am = __ballot(low && s[j] < 0);
      const uint64_t cm = __ballot(low && tent_of(s[j]) == t);
      const uint64_t pm = __ballot(!low);
      if (lane_id() == 0) {
        sm.am[j][wv] = am;
        sm.cm[j][wv] = cm;
        sm.pm[j][wv] = pm;
      }
    }
    __syncthreads();
    int fa = -1, fc = -1, fp = -1;  // positions within the step, sub-range major
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < kWavesPerBlock; ++i) {
        const int pos = j * kBlock + i * kWave;
        if (fa < 0 && sm.am[j][i]) fa = pos + __builtin_ctzll(sm.am[j][i]);
        if (fc < 0 && sm.cm[j][i]) fc = pos + __builtin_ctzll(sm.cm[j][i]);
        if (fp < 0 && sm.pm[j][i]) fp = pos + __builtin_ctzll(sm.pm[j][i]);
      }
    __syncthreads();  // the masks are rewritten next step
    const int off = (int)(kb - b);
    // rows ascend, so lower entries (uncoloured or conflicting) all precede
    // the first past entry
    if (first < 0 && fa >= 0) first = off + fa;
    if (fc >= 0) {
      *skip = first >= 0 ? first : off + fc;
      return true;
    }
    if (fp >= 0) {
      *skip = first >= 0 ? first : off + fp;
      return false;
    }
  }
  *skip = first >= 0 ? first : (int)(e - b);
  return false;
}

// detect_wave_list's scan for a heavy vertex by the whole block: the list
// first, one entry per thread per step, then the row from *skip, a step of
// 1,024 entries as four sub-ranges of 256 in row order (as in
// detect_block_skip).  List order carries no meaning, so each wave claims its
// slots with one LDS atomic; a barrier between a step's reads and its writes
// keeps the in-place compaction of the list from overwriting an entry not yet
// read.  Every thread returns the same result, *skip and *len.
template <typename RP, typename S>
__device__ bool detect_block_list(const int32_t* __restrict__ colidx, const S* __restrict__ st,
                                  int32_t* lst, RP b, RP e, int v, int t, int* skip, int* len,
                                  HeavySmem& sm) {
  const int tid = threadIdx.x;
  const int wv = tid / kWave;
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1;
  const int n0 = *len;
  if (tid == 0) {
    sm.cnt = 0;
    sm.flag = 0;
  }
  __syncthreads();
  for (int i0 = 0; i0 < n0; i0 += kBlock) {  // block-uniform
    const int i = i0 + tid;
    const int u = i < n0 ? lst[i] : -1;
    const int sv = u >= 0 ? (int)st[u] : 0;
    const bool keep = u >= 0 && sv < 0;
    const uint64_t km = __ballot(keep);
    const uint64_t cb = __ballot(u >= 0 && tent_of(sv) == t);
    __syncthreads();  // the step's entries are all read before any is rewritten
    int base = 0;
    if (lane == 0) {
      if (km) base = atomicAdd(&sm.cnt, __popcll(km));
      if (cb) sm.flag = 1;
    }
    base = __shfl(base, 0);
    if (keep) lst[base + __popcll(km & below)] = u;
  }
  __syncthreads();
  bool lose = sm.flag != 0;
  if (!lose) {
    int stop = -1;
    for (RP kb = b + *skip; kb < e; kb += 4 * kBlock) {  // block-uniform
      int u[4], sv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const RP k = kb + j * kBlock + tid;
        u[j] = k < e ? colidx[k] : INT32_MAX;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) sv[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool low = u[j] < v;
        const uint64_t cm = __ballot(low && tent_of(sv[j]) == t);
        const uint64_t pm = __ballot(!low);
        if (lane == 0) {
          sm.cm[j][wv] = cm;
          sm.pm[j][wv] = pm;
        }
      }
      __syncthreads();
      int fc = -1, fp = -1;  // positions within the step, sub-range major
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) {
          const int pos = j * kBlock + w * kWave;
          if (fc < 0 && sm.cm[j][w]) fc = pos + __builtin_ctzll(sm.cm[j][w]);
          if (fp < 0 && sm.pm[j][w]) fp = pos + __builtin_ctzll(sm.pm[j][w]);
        }
      // rows ascend, so a conflict precedes the first past entry or there is none
      const int P = fc >= 0 ? fc : fp >= 0 ? fp : 4 * kBlock;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool keep = u[j] < v && sv[j] < 0 && j * kBlock + tid < P;
        const uint64_t km = __ballot(keep);
        int base = 0;
        if (lane == 0 && km) base = atomicAdd(&sm.cnt, __popcll(km));
        base = __shfl(base, 0);
        if (keep) lst[base + __popcll(km & below)] = u[j];
      }
      __syncthreads();  // the masks are rewritten next step
      if (P < 4 * kBlock) {
        stop = (int)(kb - b) + P;
        lose = fc >= 0;
        break;
      }
    }
    *skip = stop >= 0 ? stop : (int)(e - b);
  }
  *len = sm.cnt;
  __syncthreads();  // cnt and flag are reset for the next vertex
  return lose;
}

// ---------------------------------------------------------- one phase --

// Per-thread tallies of a phase, reduced per block at the end.
struct Tally {
  int active;  // uncoloured vertices this thread's group/wave/block led
  int lost;    // of which lost (detect only)
  int cls;     // classes of the losers: 1 light, 2 medium, 4 heavy
};

template <typename RP, typename S, int L, int PHASE>
__device__ void light_phase(const KArgs& a, long wave_gid, long nwaves, Tally& tl) {
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int grp = lane / L;
  constexpr int G = kWave / L;
  const uint64_t gmask = (L == kWave) ? ~0ull : (((1ull << L) - 1) << (grp * L));
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  S* __restrict__ st = (S*)a.st;
  const bool sorted = a.sorted != 0;
  const bool push = a.push != 0;
  const int epoch = push ? a.ctrl->epoch.v : 0;
  const bool seq = a.seq != 0;
  const long nchunks = ((long)a.n + kWave - 1) / kWave;
  for (long ch = wave_gid; ch < nchunks; ch += nwaves) {
    const int v = (int)(ch * kWave) + lane;
    if (PHASE == kDetect && seq) {
      // id-priority schedule: every vertex picked this round (any degree
      // class) commits; the others keep waiting
      if (v < a.n) {
        const int s0 = st[v];
        if (s0 < 0) {
          if (s0 != waiting_state<S>()) st[v] = (S)~s0;
          else tl.lost += 1;  // (the class flags are not used by this schedule)
          tl.active += 1;
        }
      }
      continue;
    }
    bool act = false;
    int s = 0;
    RP b = 0, e = 0;
    if (v < a.n) {
      s = st[v];
      if (PHASE == kSpec && push && s < 0 && !a.flags_by_chunk) {
        // pushed flags: the least colour absent from the final neighbours is
        // the first colour not flagged, unless all of 0..31 are taken; those
        // vertices (light ones here) scan their row from colour 32
        const uint32_t m = taken_colours(a.seen, v, epoch);
        if (m != ~0u) {
          st[v] = (S)~__builtin_ctz(~m);
          s = 0;
        }
      }
    }
    if (PHASE == kSpec && push && a.flags_by_chunk) {
      // the same from the chunk's colour rows, eight rows in flight per
      // step, until every uncoloured vertex of the chunk has found a colour
      // not flagged
      const uint8_t* row = a.seen + (size_t)ch * kPushColors * kWave + lane;
      int t = -1;
      const bool need = v < a.n && s < 0;
      for (int c0 = 0; c0 < kPushColors && __ballot(need && t < 0); c0 += 8) {
        int f[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = row[(size_t)(c0 + j) * kWave];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (t < 0 && f[j] != epoch) t = c0 + j;
      }
      if (need && t >= 0) {
        st[v] = (S)~t;
        s = 0;
      }
    }
    if (v < a.n) {
      if (s < 0) {
        b = rp[v];
        e = rp[v + 1];
        act = (e - b) <= (RP)a.light_max;
      }
    }
    const uint64_t am = __ballot(act);
    if (am == 0) continue;
    if (PHASE == kDetect && sorted) {
      // sorted rows: each lane scans for its own vertex (most scans stop
      // within a few entries), then the chunk's winners push together.  A
      // chunk with at most kSparseChunk uncoloured vertices (the later rounds)
      // gives each of them a group of 64 / 2^ceil(log2 count) lanes instead.
      const int t = ~s;
      RP pb = 0;
      int len = 0;
      const int cnt = __popcll(am);
      if (cnt <= kSparseChunk) {  // wave-uniform
        const int GL = kWave >> (cnt <= 1 ? 0 : 32 - __builtin_clz((unsigned)cnt - 1));
        const int g = lane / GL;
        const bool valid = g < cnt;
        const int pos = nth_set_bit(am, valid ? g : 0);
        const RP vb = shfl_any<RP>(b, pos);
        const RP ve = shfl_any<RP>(e, pos);
        const int vt = __shfl(t, pos);
        const int vv = (int)(ch * kWave) + pos;
        int sk = 0, lose = 0;
        if (valid) {  // group-uniform
          const int sk0 = a.skip[vv];
          sk = sk0;
          const uint64_t gmask = GL == kWave ? ~0ull : ((1ull << GL) - 1) << (g * GL);
          lose = detect_group4_skip<RP, S>(a.colidx, st, vb, ve, vv, vt, GL, lane % GL, gmask,
                                           g * GL, &sk);
          if (lane % GL == 0 && sk != sk0) a.skip[vv] = sk;
        }
        // back to the owning lanes: the vertex of lane v is the rank-th active one
        const int src = act ? __popcll(am & ((1ull << lane) - 1)) * GL : 0;
        const int osk = __shfl(sk, src);
        const int olose = __shfl(lose, src);
        if (act) {
          if (!olose) {
            st[v] = (S)t;
            pb = b + osk;
            len = (int)(e - pb);
          }
          tl.lost += olose;
          tl.cls |= olose;
          tl.active += 1;
        }
      } else if (act) {
        const int sk0 = a.skip[v];
        int sk = sk0;
        const bool lose = detect_lane_skip<RP, S>(a.colidx, st, b, e, v, t, &sk);
        if (sk != sk0) a.skip[v] = sk;
        if (!lose) {
          st[v] = (S)t;
          pb = b + sk;
          len = (int)(e - pb);
        }
        tl.lost += lose;
        tl.cls |= (int)lose;
        tl.active += 1;
      }
      // every entry is pushed, final neighbours included: their flags are
      // never read again, and a state gather per entry costs more than the
      // extra stores (measured)
      if (push) push_flat<RP, S, false>(a, st, pb, len, t, epoch);
      continue;
    }
    const int cnt = __popcll(am);
    for (int p = 0; p < cnt; p += G) {  // wave-uniform
      const int k = p + grp;
      const bool valid = k < cnt;
      const int pos = nth_set_bit(am, valid ? k : 0);
      const RP vb = shfl_any<RP>(b, pos);
      const RP ve = shfl_any<RP>(e, pos);
      const int vs = shfl_any<int32_t>(s, pos);
      const int vv = (int)(ch * kWave) + pos;
      if (valid) {  // group-uniform
        if (PHASE == kSpec && seq) {
          // ready once every lower neighbour is final; then the least colour
          // absent from the final neighbours is the least absent from the
          // lower ones (a higher neighbour cannot be final before v)
          int sk = sorted ? a.skip[vv] : 0;
          const bool ready =
              ready_group<RP, S, L>(a.colidx, st, vb, ve, vv, gl, gmask, grp * L, sorted, &sk);
          if (sorted && gl == 0) a.skip[vv] = sk;
          if (ready) {
            const int t = spec_group<RP, S, L>(a.colidx, st, vb, ve, gl, 0);
            if (gl == 0) st[vv] = (S)~t;
          }
        } else if (PHASE == kSpec) {
          int t = spec_group<RP, S, L>(a.colidx, st, vb, ve, gl, push ? kPushColors : 0);
          if (gl == 0) st[vv] = (S)~t;
        } else {
          // unsorted rows (sorted ones took the lane scan above): the whole
          // row is scanned from its start
          const int t = ~vs;
          const bool lose = detect_group<RP, S, L>(a.colidx, st, vb, ve, vv, t, gl, gmask, false);
          if (gl == 0) {
            if (!lose) st[vv] = (S)t;
            tl.lost += lose;
            tl.cls |= (int)lose;
          }
          if (push && !lose) push_colour<RP, S>(a, st, vb, ve, t, epoch, gl, L);
        }
        if (gl == 0) tl.active += 1;
      }
    }
  }
}

// Queue a winner's pushes (colour t to the row entries [b, e)) for the
// grid-wide push pass.  One 64-bit atomic hands out the task slot (high
// half) and its first piece (low half), so the tasks' first pieces ascend
// with their slots.
__device__ __forceinline__ void queue_push(const KArgs& a, int64_t b, int64_t e, int t) {
  const uint64_t pieces = (uint64_t)((e - b + kPieceEntries - 1) / kPieceEntries);
  const uint64_t old = atomicAdd((unsigned long long*)&a.ctrl->tasks, (1ull << 32) | pieces);
  PushTask x;
  x.b = b;
  x.e = e;
  x.t = t;
  x.first = (int32_t)(old & 0xffffffffu);
  a.tasks[old >> 32] = x;
}

template <typename RP, typename S, int PHASE>
__device__ void medium_phase(const KArgs& a, long wave_gid, long nwaves, Tally& tl) {
  const int lane = lane_id();
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  S* __restrict__ st = (S*)a.st;
  if (PHASE == kDetect && a.seq) return;  // the light pass commits every vertex
  const int epoch = a.push ? a.ctrl->epoch.v : 0;
  // A wave owns list entries wave_gid, wave_gid + nwaves, ...; it reads 64 of
  // them and their states at once and works only on the uncoloured ones, so
  // a round with few uncoloured medium vertices costs one load per lane, not
  // a chain of dependent loads per entry.
  for (long base = wave_gid; base < a.mcount; base += nwaves * kWave) {
    const long i = base + (long)lane * nwaves;
    int v = 0, s = 0;
    bool act = false;
    if (i < a.mcount) {
      v = a.mlist[i];
      s = st[v];
      act = s < 0;
      // with pushed flags a vertex with a free colour among 0..31 takes the
      // first one here (the light pass, which reads every vertex's flags,
      // may do the same: it writes the same value, and it is skipped once
      // no light vertex is left); only the vertices whose colours 0..31 are
      // all taken scan their row below (from colour 32)
      if (PHASE == kSpec && a.push && act) {
        const uint32_t m = taken_colours(a.seen, v, epoch);
        if (m != ~0u) {
          st[v] = (S)~__builtin_ctz(~m);
          act = false;
        }
      }
    }
    uint64_t am = __ballot(act);
    while (am) {  // wave-uniform
      const int pos = __builtin_ctzll(am);
      am &= am - 1;
      const int vv = __shfl(v, pos);
      const int vs = __shfl(s, pos);
      const RP b = rp[vv], e = rp[vv + 1];
      if (PHASE == kSpec && a.seq) {
        int sk = a.sorted ? a.skip[vv] : 0;
        const bool ready = ready_group<RP, S, kWave>(a.colidx, st, b, e, vv, lane, ~0ull, 0,
                                                     a.sorted != 0, &sk);
        if (a.sorted && lane == 0) a.skip[vv] = sk;
        if (ready) {
          const int t = spec_group<RP, S, kWave>(a.colidx, st, b, e, lane, 0);
          if (lane == 0) st[vv] = (S)~t;
        }
      } else if (PHASE == kSpec) {
        int t = -1;
        if (a.push) t = first_free_wide(a.wide, a.widx[vv], epoch);
        if (t < 0)
          t = spec_group<RP, S, kWave>(a.colidx, st, b, e, lane,
                                       a.push ? kPushColors + kWideColors : 0);
        if (lane == 0) st[vv] = (S)~t;
      } else {
        const int t = ~vs;
        bool lose;
        RP pb = b;
        int ln = 0;
        if (a.lst) {
          int sk = a.skip[vv];
          ln = a.llen[vv];
          const int sk0 = sk, ln0 = ln;
          lose = detect_wave_list<RP, S>(a.colidx, st, a.lst + b, b, e, vv, t, lane, &sk, &ln);
          if (lane == 0 && sk != sk0) a.skip[vv] = sk;
          if (lane == 0 && ln != ln0) a.llen[vv] = ln;
          pb = b + sk;
        } else if (a.sorted) {
          int sk = a.skip[vv];
          lose = detect_wave4_skip<RP, S>(a.colidx, st, b, e, vv, t, lane, &sk);
          if (lane == 0) a.skip[vv] = sk;
          pb = b + sk;
        } else {
          lose = detect_group<RP, S, kWave>(a.colidx, st, b, e, vv, t, lane, ~0ull, false);
        }
        if (lane == 0) {
          if (!lose) st[vv] = (S)t;
          tl.lost += lose;
          tl.cls |= lose ? 2 : 0;
        }
        if (a.push && !lose) {
          // with a list, its entries are the lower neighbours still uncoloured and
          // the row from pb holds the higher ones
          if (ln > 0) {
            if (a.tasks && ln > kDeferRow) {
              if (lane == 0) queue_push(a, (int64_t)b, (int64_t)b + ln, t | kFromList);
            } else {
              // the list entries were written by other lanes of this wave
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
              push_colour_ids<RP, S>(a, a.lst, st, b, b + ln, t, epoch, lane, kWave);
            }
          }
          if (a.tasks && e - pb > (RP)kDeferRow) {
            // a long row: the push pass after this one spreads it over the grid
            if (lane == 0) queue_push(a, pb, e, t);
          } else {
            push_colour<RP, S>(a, st, pb, e, t, epoch, lane, kWave);
          }
        }
      }
      if (lane == 0) tl.active += 1;
    }
  }
}

// Is every lower-id neighbour of v final?  Whole block (heavy vertices).
// Unsorted rows: the whole row, one entry per thread per step.
template <typename RP, typename S>
__device__ bool ready_block(const int32_t* __restrict__ colidx, const S* __restrict__ st,
                            RP b, RP e, int v) {
  for (RP kb = b; kb < e; kb += kBlock) {
    const RP k = kb + threadIdx.x;
    int wait = 0;
    if (k < e) {
      const int u = colidx[k];
      wait = u < v && st[u] < 0;
    }
    if (__syncthreads_or(wait)) return false;
  }
  return true;
}

// The same on sorted rows with the resume offset of the conflict scans:
// from b + skip, four entries per thread per step (sub-ranges of 256 in
// order).  Returns 2 * (new offset) + (1 if no lower neighbour is left that
// is not final): the new offset is that of the first lower neighbour not yet
// final, or where the lower prefix ends.  Every thread returns the same.
// (The masks live in the function's own LDS arrays: taking the shared
// HeavySmem by reference here made the gfx950 backend reject the code.)
template <typename RP, typename S>
__device__ __forceinline__ int ready_block_skip(const int32_t* __restrict__ colidx,
                                                const S* __restrict__ st, RP b, RP e, int v,
                                                int skip) {
  __shared__ uint64_t wmask[4][kWavesPerBlock], pmask[4][kWavesPerBlock];
  const int tid = threadIdx.x;
  const int wv = tid / kWave;
  for (RP kb = b + skip; kb < e; kb += 4 * kBlock) {
    int u[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const RP k = kb + j * kBlock + tid;
      u[j] = k < e ? colidx[k] : INT32_MAX;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t wm = __ballot(u[j] < v && s[j] < 0);
      const uint64_t pm = __ballot(u[j] >= v);
      if (lane_id() == 0) {
        wmask[j][wv] = wm;
        pmask[j][wv] = pm;
      }
    }
    __syncthreads();
    int fw = -1, fp = -1;  // positions within the step, sub-range major
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < kWavesPerBlock; ++i) {
        const int pos = j * kBlock + i * kWave;
        if (fw < 0 && wmask[j][i]) fw = pos + __builtin_ctzll(wmask[j][i]);
        if (fp < 0 && pmask[j][i]) fp = pos + __builtin_ctzll(pmask[j][i]);
      }
    __syncthreads();  // the masks are rewritten next step
    const int off = (int)(kb - b);
    if (fw >= 0) return 2 * (off + fw);  // lower entries all precede the first past entry
    if (fp >= 0) return 2 * (off + fp) + 1;
  }
  return 2 * (int)(e - b) + 1;
}

template <typename RP, typename S, int PHASE>
__device__ void heavy_phase(const KArgs& a, long blk, long nblk, Tally& tl, HeavySmem& sm) {
  if (PHASE == kDetect && a.seq) return;  // the light pass commits every vertex
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  S* __restrict__ st = (S*)a.st;
  for (long i = blk; i < a.hcount; i += nblk) {
    const int v = a.hlist[i];
    const int s = st[v];
    // with pushed flags a vertex with a free colour among 0..31 takes the
    // first one (as in the medium pass)
    const uint32_t m =
        PHASE == kSpec && a.push && s < 0 ? taken_colours(a.seen, v, a.ctrl->epoch.v) : ~0u;
    const bool skip = m != ~0u;
    __syncthreads();  // the commit below happens after every thread read s
    if (skip && threadIdx.x == 0) st[v] = (S)~__builtin_ctz(~m);
    if (s >= 0 || skip) continue;  // block-uniform
    const RP b = rp[v], e = rp[v + 1];
    if (PHASE == kSpec && a.seq) {
      bool ready;
      if (a.sorted) {
        const int r2 = ready_block_skip<RP, S>(a.colidx, st, b, e, v, a.skip[v]);
        ready = r2 & 1;
        __syncthreads();  // every thread has read the old offset
        if (threadIdx.x == 0) a.skip[v] = r2 >> 1;
      } else {
        ready = ready_block<RP, S>(a.colidx, st, b, e, v);
      }
      if (ready) {
        const int t = spec_block<RP, S>(a.colidx, st, b, e, sm, 0);
        if (threadIdx.x == 0) st[v] = (S)~t;
      }
    } else if (PHASE == kSpec) {
      int t = -1;
      if (a.push) {
        if (threadIdx.x < kWave) {
          const int f = first_free_wide(a.wide, a.widx[v], a.ctrl->epoch.v);
          if (threadIdx.x == 0) sm.first = f;
        }
        __syncthreads();
        t = sm.first;
        __syncthreads();
      }
      if (t < 0)
        t = spec_block<RP, S>(a.colidx, st, b, e, sm, a.push ? kPushColors + kWideColors : 0);
      if (threadIdx.x == 0) st[v] = (S)~t;
    } else {
      const int t = ~s;
      bool lose;
      RP pb = b;
      int ln = 0;
      if (a.lst) {
        int sk = a.skip[v];
        ln = a.llen[v];
        lose = detect_block_list<RP, S>(a.colidx, st, a.lst + b, b, e, v, t, &sk, &ln, sm);
        if (threadIdx.x == 0) {
          a.skip[v] = sk;
          a.llen[v] = ln;
        }
        pb = b + sk;
      } else if (a.sorted) {
        int sk = a.skip[v];
        lose = detect_block_skip<RP, S>(a.colidx, st, b, e, v, t, &sk, sm);
        if (threadIdx.x == 0) a.skip[v] = sk;
        pb = b + sk;
      } else {
        lose = detect_block<RP, S>(a.colidx, st, b, e, v, t, false);
      }
      if (threadIdx.x == 0) {
        if (!lose) st[v] = (S)t;
        tl.lost += lose;
        tl.cls |= lose ? 4 : 0;
      }
      if (a.push && !lose) {
        // with a list, its entries are the lower neighbours still uncoloured
        // and the row from pb holds the higher ones
        if (ln > 0) {
          if (a.tasks && ln > kDeferRow) {
            if (threadIdx.x == 0) queue_push(a, (int64_t)b, (int64_t)b + ln, t | kFromList);
          } else {
            push_colour_ids<RP, S>(a, a.lst, st, b, b + ln, t, a.ctrl->epoch.v, threadIdx.x,
                                   kBlock);
          }
        }
        if (a.tasks && e - pb > (RP)kDeferRow) {
          // a hub's long row: its pushes are spread over the whole grid by
          // the pass that follows, instead of one workgroup walking it
          if (threadIdx.x == 0) queue_push(a, pb, e, t);
        } else {
          push_colour<RP, S>(a, st, pb, e, t, a.ctrl->epoch.v, threadIdx.x, kBlock);
        }
      }
    }
    if (threadIdx.x == 0) tl.active += 1;
  }
}

// Round q's flags start clear; the detect pass of round q - 1 sets them.
__device__ __forceinline__ void clear_round_flags(const KArgs& a, int q) {
  a.ctrl->more[q % 3].v = 0;
  ClassLine& c = a.ctrl->cls[q % 3];
  c.light = 0;
  c.medium = 0;
  c.heavy = 0;
}

// Detect publishes, per block: whether round r + 1 has work
// (more[(r+1) % 3]), r as the last non-empty round, and |U_r| in the trace.
__device__ void publish_detect(const KArgs& a, int r, const Tally& tl, HeavySmem& sm) {
  // per-wave sums by cross-lane reduction, then one slot per wave in LDS
  // (same-address LDS atomics from every lane used to serialise here)
  int act = tl.active, lost = tl.lost, cls = tl.cls;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    act += __shfl_xor(act, off);
    lost += __shfl_xor(lost, off);
    cls |= __shfl_xor(cls, off);
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    sm.wact[w] = act;
    sm.wlost[w] = lost;
    sm.wcls[w] = cls;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    act = lost = cls = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
      act += sm.wact[i];
      lost += sm.wlost[i];
      cls |= sm.wcls[i];
    }
    // Flags shared by every block are read before they are written: a
    // block stores only what it does not already see, so the stores of
    // some 1,500 blocks to one line do not queue up at the end of the pass.
    // (Slot (r + 1) % 3 was cleared by the previous detect pass.)
    if (lost && !a.ctrl->more[(r + 1) % 3].v) a.ctrl->more[(r + 1) % 3].v = 1;
    // the classes that keep uncoloured vertices into round r + 1 (only
    // graphs with several classes read them)
    if (a.mcount + a.hcount > 0 && a.seq == 0 && cls) {
      ClassLine& c = a.ctrl->cls[(r + 1) % 3];
      if ((cls & 1) && !c.light) c.light = 1;
      if ((cls & 2) && !c.medium) c.medium = 1;
      if ((cls & 4) && !c.heavy) c.heavy = 1;
    }
    if (act && a.ctrl->last_round.v < r) a.ctrl->last_round.v = r;
    // the round's size: one count per workgroup with a plain store, folded
    // by the next pass (same-address device atomics from every workgroup
    // would queue up at the end of the pass)
    a.part[blockIdx.x] = act;
    if (blockIdx.x == 0) {
      a.ctrl->pend.v = r;
      a.ctrl->pend_grid.v = (int)gridDim.x;
    }
  }
}

// Sum of the per-workgroup counts of the last detect pass into the round
// trace.  Run by every thread of one workgroup, after the kernel boundary (or
// grid barrier) that follows that pass.
__device__ void fold_trace(const KArgs& a) {
  __shared__ int sh[kWavesPerBlock];
  const int r = a.ctrl->pend.v;
  if (r == 0) return;
  const int g = a.ctrl->pend_grid.v;
  int sum = 0;
  for (int i = threadIdx.x; i < g; i += blockDim.x) sum += a.part[i];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWavesPerBlock; ++w) sum += sh[w];
    if (r - 1 < kTraceRounds) a.ctrl->trace[r - 1] = sum;
    a.ctrl->pend.v = 0;
  }
  __syncthreads();
}

// A whole phase of round r over every uncoloured vertex, by one block of a
// grid of nblk blocks.  Detect also clears more[(r+2) % 3] for the round
// after next.
template <typename RP, typename S, int L, int PHASE>
__device__ void phase(const KArgs& a, int r, long blk, long nblk, HeavySmem& sm) {
  Tally tl{0, 0, 0};
  if (PHASE == kDetect && blk == 0 && threadIdx.x == 0) clear_round_flags(a, r + 2);
  // A degree class with no uncoloured vertex left is skipped (on power-law
  // graphs the light vertices are all final long before the hubs: walking
  // their chunks would cost every later pass the same fixed time).  The
  // id-priority schedule visits every class every round.
  // A graph of light vertices only needs no flags (its light class is busy
  // whenever the round is), and reading them would put a dependent load in
  // front of every pass.
  const bool mixed = a.mcount + a.hcount > 0 && a.seq == 0;
  const ClassLine* c = mixed ? &a.ctrl->cls[r % 3] : nullptr;
  if (a.hcount > 0 && (!mixed || c->heavy)) heavy_phase<RP, S, PHASE>(a, blk, nblk, tl, sm);
  const long wave_gid = blk * kWavesPerBlock + threadIdx.x / kWave;
  const long nwaves = nblk * kWavesPerBlock;
  if (a.mcount > 0 && (!mixed || c->medium)) medium_phase<RP, S, PHASE>(a, wave_gid, nwaves, tl);
  if (!mixed || c->light) light_phase<RP, S, L, PHASE>(a, wave_gid, nwaves, tl);
  if (PHASE == kDetect) publish_detect(a, r, tl, sm);
}

// ------------------------------------------------------------- kernels --

template <typename RP, typename S, int L, int PHASE>
__global__ __launch_bounds__(kBlock) void k_phase(KArgs a, int round, int from_base) {
  __shared__ HeavySmem sm;
  const int r = from_base ? a.ctrl->round_base.v + round : round;
  if (PHASE == kSpec && blockIdx.x == 0) {
    fold_trace(a);
    // the previous round's push pass has run
    if (threadIdx.x == 0) *(uint64_t*)&a.ctrl->tasks = 0;
  }
  if (!a.ctrl->more[r % 3].v) {
    if (PHASE == kDetect && blockIdx.x == 0 && threadIdx.x == 0) clear_round_flags(a, r + 2);
    return;
  }
  phase<RP, S, L, PHASE>(a, r, blockIdx.x, gridDim.x, sm);
}

// The grid-wide push pass after a detect pass: the queued tasks' rows are
// cut into pieces of kPieceEntries entries, one workgroup per piece (four
// entries per thread in flight); each entry marks colour t taken for a
// neighbour that is still uncoloured, as push_colour does.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_push_tasks(KArgs a) {
  const uint64_t packed = *(const uint64_t*)&a.ctrl->tasks;
  const int count = (int)(packed >> 32);
  const int64_t pieces = (int64_t)(packed & 0xffffffffu);
  if (count == 0) return;
  const S* __restrict__ st = (const S*)a.st;
  const int epoch = a.ctrl->epoch.v;
  for (int64_t p = blockIdx.x; p < pieces; p += gridDim.x) {  // workgroup-uniform
    int lo = 0, hi = count - 1;  // the last task whose first piece is <= p
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (a.tasks[mid].first <= p) lo = mid;
      else hi = mid - 1;
    }
    const PushTask x = a.tasks[lo];
    const int t = x.t & ~kFromList;
    const int32_t* __restrict__ ids = (x.t & kFromList) ? a.lst : a.colidx;
    const int64_t k0 = x.b + (p - x.first) * (int64_t)kPieceEntries;
    const int64_t k1 = k0 + kPieceEntries < x.e ? k0 + kPieceEntries : x.e;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 4 * kBlock) {
      int u[4], sv[4], w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = k + j * kBlock < k1 ? ids[k + j * kBlock] : -1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sv[j] = u[j] >= 0 ? (int)st[u[j]] : 0;
        w[j] = u[j] >= 0 && t >= kPushColors ? a.widx[u[j]] : -1;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (u[j] < 0 || sv[j] >= 0) continue;
        if (t < kPushColors) a.seen[flag_index(a, u[j], t)] = (uint8_t)epoch;
        else if (t < kPushColors + kWideColors && w[j] >= 0)
          a.wide[(size_t)w[j] * kWideColors + (t - kPushColors)] = (uint8_t)epoch;
      }
    }
  }
}

// Round 1 in closed form for sorted rows: nothing is final, so every vertex
// tries colour 0 and v keeps it exactly when no neighbour has a lower id,
// i.e. when its first (smallest) neighbour is above v.  One lane per vertex
// writes the whole state array, so no initialisation pass is needed.
template <typename RP, typename S>
__global__ __launch_bounds__(kBlock) void k_round1_sorted(KArgs a) {
  __shared__ HeavySmem sm;
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  S* __restrict__ st = (S*)a.st;
  Tally tl{0, 0, 0};
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long v = tid; v < a.n; v += nth) {
    const RP b = rp[v], e = rp[v + 1];
    const bool lose = e > b && a.colidx[b] < v;
    st[v] = lose ? (S)-1 : (S)0;
    a.skip[v] = 0;
    if (a.llen) a.llen[v] = 0;
    tl.lost += lose;
    tl.cls |= lose ? 7 : 0;  // (any class may have lost: the closed form does not tell)
    tl.active += 1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) clear_round_flags(a, 3);
  publish_detect(a, 1, tl, sm);
}

// Round 1 in closed form with pushes (sorted rows, push algorithm, no heavy
// vertices): as
// k_round1_sorted, and each winner marks colour 0 taken for all of its
// neighbours, every one of which has a lower neighbour (the winner) and so
// loses round 1.  Chunks of 64 vertices per wave; the winners of a chunk
// push together.
template <typename RP, typename S>
__global__ __launch_bounds__(kBlock) void k_round1_sorted_push(KArgs a) {
  __shared__ HeavySmem sm;
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  S* __restrict__ st = (S*)a.st;
  const int epoch = a.ctrl->epoch.v;
  Tally tl{0, 0, 0};
  const long wave_gid = blockIdx.x * (long)kWavesPerBlock + threadIdx.x / kWave;
  const long nwaves = (long)gridDim.x * kWavesPerBlock;
  const long nchunks = ((long)a.n + kWave - 1) / kWave;
  for (long ch = wave_gid; ch < nchunks; ch += nwaves) {
    const int v = (int)(ch * kWave) + lane_id();
    RP pb = 0;
    int len = 0;
    if (v < a.n) {
      const RP b = rp[v], e = rp[v + 1];
      const bool lose = e > b && a.colidx[b] < v;
      st[v] = lose ? (S)-1 : (S)0;
      a.skip[v] = 0;
      if (a.llen) a.llen[v] = 0;
      tl.lost += lose;
      tl.cls |= lose ? 7 : 0;  // (any class may have lost: the closed form does not tell)
      tl.active += 1;
      if (!lose) {
        pb = b;
        len = (int)(e - b);
      }
    }
    push_flat<RP, S, false>(a, st, pb, len, 0, epoch);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) clear_round_flags(a, 3);
  publish_detect(a, 1, tl, sm);
}

// Unsorted rows: initialise every vertex to "tentative 0"; the general
// detect phase then runs round 1.
template <typename S>
__global__ void k_fill_tent0(KArgs a) {
  S* __restrict__ st = (S*)a.st;
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  const S init = (S)(a.seq ? waiting_state<S>() : -1);
  for (long v = tid; v < a.n; v += nth) {
    st[v] = init;
    a.skip[v] = 0;
    if (a.llen) a.llen[v] = 0;
  }
}

__global__ void k_init(KArgs a) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  // round sizes: every round the colouring runs stores its own; only the
  // p-block passes add into them
  if (a.clear_trace)
    for (long i = tid; i < kTraceRounds; i += nth) a.ctrl->trace[i] = 0;
  if (a.push && a.clear_seen) {
    uint4* p = (uint4*)a.seen;  // kPushColors bytes per vertex = 2 x 16 bytes
    const long nv = ((long)a.n + kWave - 1) / kWave * kWave;  // whole chunks
    for (long i = tid; i < 2l * nv; i += nth) p[i] = make_uint4(0, 0, 0, 0);
    uint4* q = (uint4*)a.wide;  // kWideColors = 30 x 16 bytes per block
    const long nw = (long)a.wide_clear * (kWideColors / 16);
    for (long i = tid; i < nw; i += nth) q[i] = make_uint4(0, 0, 0, 0);
  }
  if (tid == 0) {
    a.ctrl->more[0].v = 0;
    a.ctrl->more[1].v = a.n > 0;  // round 1 has work iff there are vertices
    a.ctrl->more[2].v = 0;
    for (int q = 0; q < 3; ++q) {
      const int on = q == 1 && a.n > 0;  // round 1: every class may have vertices
      a.ctrl->cls[q].light = on;
      a.ctrl->cls[q].medium = on;
      a.ctrl->cls[q].heavy = on;
    }
    a.ctrl->last_round.v = 0;
    a.ctrl->round_base.v = 2;
    a.ctrl->pend.v = 0;
    a.ctrl->bar.v = 0;
    a.ctrl->abort.v = 0;
    a.ctrl->left.v = 0;
    *(uint64_t*)&a.ctrl->tasks = 0;
    a.ctrl->epoch.v = a.epoch;
  }
}

__global__ void k_advance_base(Ctrl* c, int by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->round_base.v += by;
}

__device__ __forceinline__ void store_system(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Widening pass and statistics: the state becomes the caller's int32
// colours, and each workgroup reports the largest colour and the uncoloured
// count of its vertices straight into pinned host memory (layout at
// launch_finish).  Each thread takes 16 bytes of state (16, 8 or 4
// vertices): one 16-byte load, and 16-byte stores when both arrays are
// 16-byte aligned (VEC).  No device atomics: the host folds the
// per-workgroup pairs.
template <typename S, bool VEC>
__global__ __launch_bounds__(kBlock) void k_finish(KArgs a, int32_t* out) {
  __shared__ int sh_max[kWavesPerBlock], sh_left[kWavesPerBlock];
  if (blockIdx.x == 0) fold_trace(a);  // the last detect pass's round size
  constexpr int V = 16 / (int)sizeof(S);
  const S* __restrict__ st = (const S*)a.st;
  int mx = -1, left = 0;
  const long nth = (long)gridDim.x * blockDim.x;
  const long ngroups = ((long)a.n + V - 1) / V;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < ngroups; g += nth) {
    const long v0 = g * V;
    int s[V];
    if (VEC && v0 + V <= a.n) {
      const uint4 w = *(const uint4*)(st + v0);
      S x[V];
      __builtin_memcpy(x, &w, sizeof w);
#pragma unroll
      for (int q = 0; q < V; ++q) s[q] = x[q];
#pragma unroll
      for (int q = 0; q < V; q += 4)
        *(int4*)(a.colors + v0 + q) = make_int4(s[q], s[q + 1], s[q + 2], s[q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) s[q] = v0 + q < a.n ? (int)st[v0 + q] : 0;
#pragma unroll
      for (int q = 0; q < V; ++q)
        if (v0 + q < a.n) a.colors[v0 + q] = s[q];
    }
#pragma unroll
    for (int q = 0; q < V; ++q)
      if (v0 + q < a.n) {
        mx = s[q] > mx ? s[q] : mx;
        left += s[q] < 0;
      }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const int om = __shfl_xor(mx, off);
    mx = om > mx ? om : mx;
    left += __shfl_xor(left, off);
  }
  if (lane_id() == 0) {
    sh_max[threadIdx.x / kWave] = mx;
    sh_left[threadIdx.x / kWave] = left;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWavesPerBlock; ++w) {
      mx = sh_max[w] > mx ? sh_max[w] : mx;
      left += sh_left[w];
    }
    store_system(&out[kFinishHeader + 2 * blockIdx.x], mx + 1);
    store_system(&out[kFinishHeader + 1 + 2 * blockIdx.x], left);
    if (blockIdx.x == 0) {
      store_system(&out[0], a.ctrl->last_round.v);
      store_system(&out[1], a.ctrl->abort.v);
      store_system(&out[2], a.ctrl->left.v);
      store_system(&out[3], (int32_t)gridDim.x);
    }
  }
}

// Grid-wide barrier of a co-resident (cooperative) grid.  Arrivals count up
// monotonically; each block waits for epoch * gridDim.x.  Release/acquire at
// agent scope make every block's writes visible across the XCDs' L2s.  A
// wait that exceeds the spin limit sets ctrl->abort, and every later
// barrier returns at once, so the kernel always drains.
__device__ __forceinline__ bool grid_barrier(Ctrl* c, unsigned& epoch) {
  __shared__ int sh_abort;
  __syncthreads();
  if (threadIdx.x == 0) {
    ++epoch;
    const unsigned target = epoch * gridDim.x;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add((unsigned*)&c->bar.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ab = __hip_atomic_load(&c->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (!ab && __hip_atomic_load((unsigned*)&c->bar.v, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1l << 25)) {
        __hip_atomic_store(&c->abort.v, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ab = 1;
      } else if ((spins & 1023) == 0) {
        ab = __hip_atomic_load(&c->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    sh_abort = ab;
  }
  __syncthreads();
  return sh_abort == 0;
}

// The whole colouring in one launch: round 1 (detect only, from the state
// -1 everywhere), then rounds of speculate / barrier / detect / barrier until
// a round has no losers.
template <typename RP, typename S, int L>
__global__ __launch_bounds__(kBlock) void k_persistent(KArgs a, int max_rounds) {
  __shared__ HeavySmem sm;
  unsigned epoch = 0;
  {
    S* __restrict__ st = (S*)a.st;
    const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long nth = (long)gridDim.x * blockDim.x;
    const S init = (S)(a.seq ? waiting_state<S>() : -1);
    for (long v = tid; v < a.n; v += nth) {
      st[v] = init;
      a.skip[v] = 0;
      if (a.llen) a.llen[v] = 0;
    }
  }
  if (!grid_barrier(a.ctrl, epoch)) return;
  if (a.seq) {
    phase<RP, S, L, kSpec>(a, 1, blockIdx.x, gridDim.x, sm);
    if (!grid_barrier(a.ctrl, epoch)) return;
  }
  phase<RP, S, L, kDetect>(a, 1, blockIdx.x, gridDim.x, sm);
  if (!grid_barrier(a.ctrl, epoch)) return;
  // (r <= n: R <= n by Lemma 2 with one vertex per block; the bound only
  // keeps a broken invariant from looping forever)
  for (int r = 2; r <= a.n && (max_rounds <= 0 || r <= max_rounds); ++r) {
    const int more = __hip_atomic_load(&a.ctrl->more[r % 3].v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    if (!more) break;  // grid-uniform: read after a barrier, written before it
    if (blockIdx.x == 0) fold_trace(a);
    phase<RP, S, L, kSpec>(a, r, blockIdx.x, gridDim.x, sm);
    if (!grid_barrier(a.ctrl, epoch)) return;
    phase<RP, S, L, kDetect>(a, r, blockIdx.x, gridDim.x, sm);
    if (!grid_barrier(a.ctrl, epoch)) return;
  }
}

// ------------------------------------------------------ graph set-up --

// Degree classes: medium (light_max < deg < heavy_min) and heavy
// (deg >= heavy_min) vertex lists; counts[2] receives the maximum degree.
template <typename RP>
__global__ void k_classify(const RP* rowptr, int32_t n, int32_t light_max, int32_t heavy_min,
                           int32_t* mlist, int32_t* hlist, int32_t* counts, int32_t* widx) {
  __shared__ int sh_max;
  if (threadIdx.x == 0) sh_max = 0;
  __syncthreads();
  int mx = 0;
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long v = tid; v < n; v += nth) {
    RP d = rowptr[v + 1] - rowptr[v];
    int di = d > (RP)INT_MAX ? INT_MAX : (int)d;
    mx = di > mx ? di : mx;
    int w = -1;  // wide block: medium i -> i; heavy j -> mcount + j (set afterwards)
    if (di > light_max) {
      if (di >= heavy_min) hlist[atomicAdd(&counts[1], 1)] = (int)v;
      else mlist[w = atomicAdd(&counts[0], 1)] = (int)v;
    }
    widx[v] = w;
  }
  atomicMax(&sh_max, mx);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&counts[2], sh_max);
}

// ------------------------------------------------------ host launchers --

template <typename RP, typename S, int L>
static int launch_round_t(const KArgs& a, int phase_id, int round, bool from_base, int grid,
                          hipStream_t s) {
  if (phase_id == kSpec)
    hipLaunchKernelGGL((k_phase<RP, S, L, kSpec>), dim3(grid), dim3(kBlock), 0, s, a, round,
                       (int)from_base);
  else {
    hipLaunchKernelGGL((k_phase<RP, S, L, kDetect>), dim3(grid), dim3(kBlock), 0, s, a, round,
                       (int)from_base);
    if (a.tasks) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return (int)e;
      hipLaunchKernelGGL((k_push_tasks<S>), dim3(grid), dim3(kBlock), 0, s, a);
    }
  }
  return (int)hipGetLastError();
}

template <typename RP, typename S, int L>
static int launch_round1_t(const KArgs& a, int grid, hipStream_t s) {
  if (a.sorted && !a.push && !a.seq) {
    hipLaunchKernelGGL((k_round1_sorted<RP, S>), dim3(grid), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
  }
  // (a heavy winner would push its whole row from one wavefront: those
  // graphs take the general round-1 pass, whose heavy path uses a workgroup)
  if (a.sorted && a.push && a.hcount == 0) {
    hipLaunchKernelGGL((k_round1_sorted_push<RP, S>), dim3(grid), dim3(kBlock), 0, s, a);
    return (int)hipGetLastError();
  }
  hipLaunchKernelGGL((k_fill_tent0<S>), dim3(grid), dim3(kBlock), 0, s, a);
  int rc = (int)hipGetLastError();
  if (rc) return rc;
  if (a.seq) {  // round 1 picks the vertices with no lower neighbour
    rc = launch_round_t<RP, S, L>(a, kSpec, 1, false, grid, s);
    if (rc) return rc;
  }
  return launch_round_t<RP, S, L>(a, kDetect, 1, false, grid, s);
}

template <typename RP, typename S, int L>
static int launch_persistent_t(const KArgs& a, int max_rounds, int grid, hipStream_t s) {
  KArgs aa = a;
  int mr = max_rounds;
  void* args[] = {&aa, &mr};
  return (int)hipLaunchCooperativeKernel((const void*)&k_persistent<RP, S, L>, dim3(grid),
                                         dim3(kBlock), args, 0, s);
}

// Workgroups of `kernel` (kBlock threads, no dynamic LDS) that one compute
// unit of a gfx950 can hold at once, from the kernel's own register and LDS
// use: a SIMD's register file holds 512 registers per lane, allocated to a
// wave in granules of 8 (architectural and accumulation registers together),
// and runs at most 8 waves; a CU has 4 SIMDs and 160 KB of LDS.  Returns 0
// when the attributes cannot be read.
static int resident_blocks_per_cu(const void* kernel) {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, kernel) != hipSuccess || fa.numRegs <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  const int regs = (fa.numRegs + 7) / 8 * 8;
  const int waves_per_simd = std::min(8, 512 / regs);
  int blocks = waves_per_simd * 4 / kWavesPerBlock;
  if (fa.sharedSizeBytes > 0) blocks = std::min<int>(blocks, (int)((160u << 10) / fa.sharedSizeBytes));
  return blocks;
}

// Grid of the cooperative kernel: every workgroup must be resident at once,
// or a grid barrier waits for one that never starts.  The occupancy query
// alone is not trusted for that: on gfx950 it admitted 8 workgroups per CU of
// a kernel whose 120-152 registers per lane allow only 3-4 waves per SIMD
// (the barrier then timed out).  The grid is the smaller of the two bounds.
template <typename RP, typename S, int L>
static int persistent_grid_t(int* grid_out) {
  int dev = 0, per_cu = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  const void* kernel = (const void*)&k_persistent<RP, S, L>;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
  if (e != hipSuccess) return (int)e;
  const int derived = resident_blocks_per_cu(kernel);
  per_cu = derived > 0 ? std::min(per_cu, derived) : std::min(per_cu, 1);
  *grid_out = per_cu * cus;
  return 0;
}

// Dispatch on (rowptr width, state width, lanes) to the template instances.
#define GC_DISPATCH_L(RP, S, FN, ...)                \
  switch (lanes) {                                   \
    case 2: return FN<RP, S, 2>(__VA_ARGS__);        \
    case 4: return FN<RP, S, 4>(__VA_ARGS__);        \
    case 8: return FN<RP, S, 8>(__VA_ARGS__);        \
    case 16: return FN<RP, S, 16>(__VA_ARGS__);      \
    case 32: return FN<RP, S, 32>(__VA_ARGS__);      \
    case 64: return FN<RP, S, 64>(__VA_ARGS__);      \
    default: return (int)hipErrorInvalidValue;       \
  }

#define GC_DISPATCH_S(RP, FN, ...)                                        \
  switch (sbytes) {                                                       \
    case 1: { GC_DISPATCH_L(RP, int8_t, FN, __VA_ARGS__) }                \
    case 2: { GC_DISPATCH_L(RP, int16_t, FN, __VA_ARGS__) }               \
    case 4: { GC_DISPATCH_L(RP, int32_t, FN, __VA_ARGS__) }               \
    default: return (int)hipErrorInvalidValue;                            \
  }

#define GC_DISPATCH(FN, ...)                                        \
  do {                                                              \
    if (rp64) { GC_DISPATCH_S(int64_t, FN, __VA_ARGS__) }           \
    else { GC_DISPATCH_S(int32_t, FN, __VA_ARGS__) }                \
  } while (0)

int launch_round(const KArgs& a, bool rp64, int sbytes, int lanes, int phase_id, int round,
                 bool round_from_base, int grid, void* stream) {
  GC_DISPATCH(launch_round_t, a, phase_id, round, round_from_base, grid, (hipStream_t)stream);
}

int launch_round1(const KArgs& a, bool rp64, int sbytes, int lanes, int grid, void* stream) {
  GC_DISPATCH(launch_round1_t, a, grid, (hipStream_t)stream);
}

int launch_persistent(const KArgs& a, bool rp64, int sbytes, int lanes, int max_rounds, int grid,
                      void* stream) {
  GC_DISPATCH(launch_persistent_t, a, max_rounds, grid, (hipStream_t)stream);
}

int persistent_max_grid(bool rp64, int sbytes, int lanes, int* grid_out) {
  GC_DISPATCH(persistent_grid_t, grid_out);
}

int launch_init(const KArgs& a, void* stream) {
  hipLaunchKernelGGL(k_init, dim3(a.push && a.clear_seen ? 1024 : 64), dim3(kBlock), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_advance_base(const KArgs& a, int by, void* stream) {
  hipLaunchKernelGGL(k_advance_base, dim3(1), dim3(64), 0, (hipStream_t)stream, a.ctrl, by);
  return (int)hipGetLastError();
}

int launch_finish(const KArgs& a, int sbytes, int32_t* out, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (sbytes != 1 && sbytes != 2 && sbytes != 4) return (int)hipErrorInvalidValue;
  // 16 bytes of state per thread, at most kFinishBlocks workgroups
  const long per = (16l / sbytes) * kBlock;
  const int grid = (int)std::max<long>(1, std::min<long>(kFinishBlocks, ((long)a.n + per - 1) / per));
  const bool vec = ((uintptr_t)a.st % 16 == 0) && ((uintptr_t)a.colors % 16 == 0);
#define GC_FINISH(S_)                                                                     \
  if (vec) hipLaunchKernelGGL((k_finish<S_, true>), dim3(grid), dim3(kBlock), 0, s, a, out); \
  else hipLaunchKernelGGL((k_finish<S_, false>), dim3(grid), dim3(kBlock), 0, s, a, out)
  if (sbytes == 1) GC_FINISH(int8_t);
  else if (sbytes == 2) GC_FINISH(int16_t);
  else GC_FINISH(int32_t);
#undef GC_FINISH
  return (int)hipGetLastError();
}

int launch_classify(const void* rowptr, bool rp64, int32_t n, int32_t light_max, int32_t heavy_min,
                    int32_t* mlist, int32_t* hlist, int32_t* counts, int32_t* widx, int grid,
                    void* stream) {
  if (rp64)
    hipLaunchKernelGGL(k_classify<int64_t>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       (const int64_t*)rowptr, n, light_max, heavy_min, mlist, hlist, counts, widx);
  else
    hipLaunchKernelGGL(k_classify<int32_t>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       (const int32_t*)rowptr, n, light_max, heavy_min, mlist, hlist, counts, widx);
  return (int)hipGetLastError();
}

__global__ void k_wide_index(const int32_t* hlist, int32_t hcount, int32_t mcount, int32_t* widx) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long j = tid; j < hcount; j += nth) widx[hlist[j]] = mcount + (int)j;
}

int launch_wide_index(const int32_t* hlist, int32_t hcount, int32_t mcount, int32_t* widx,
                      void* stream) {
  if (hcount <= 0) return 0;
  hipLaunchKernelGGL(k_wide_index, dim3((hcount + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     (hipStream_t)stream, hlist, hcount, mcount, widx);
  return (int)hipGetLastError();
}

}  // namespace gc
