// gc_device.h -- device helpers shared by the per-graph and batched kernels:
// cross-lane reductions for wave64 and the per-vertex speculate / detect
// work of a group of L lanes.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "gc_internal.h"

namespace gc {

// ------------------------------------------------------------ helpers --

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int mask) {
  int lo = __shfl_xor((int)(uint32_t)x, mask);
  int hi = __shfl_xor((int)(uint32_t)(x >> 32), mask);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <typename T>
__device__ __forceinline__ T shfl_any(T x, int src);
template <>
__device__ __forceinline__ int32_t shfl_any<int32_t>(int32_t x, int src) {
  return __shfl(x, src);
}
template <>
__device__ __forceinline__ int64_t shfl_any<int64_t>(int64_t x, int src) {
  int lo = __shfl((int)(uint32_t)x, src);
  int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int L>
__device__ __forceinline__ uint64_t group_or(uint64_t m) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) m |= shfl_xor64(m, off);
  return m;
}

// position of the k-th (0-based) set bit of m; k < popcount(m)
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    int c = __popcll((m >> pos) & ((1ull << w) - 1));
    if (k >= c) {
      k -= c;
      pos += w;
    }
  }
  return pos;
}

// tentative colour carried by a state word (final colours decode to themselves)
__device__ __forceinline__ int tent_of(int s) { return s < 0 ? ~s : s; }

// ------------------------------------------- per-vertex work, L lanes --

// Least colour not final on any neighbour of the row [b, e), computed by a
// group of L lanes (gl = lane in group).  Every lane returns the result.
template <typename RP, typename S, int L>
__device__ __forceinline__ int spec_group(const int32_t* __restrict__ colidx,
                                          const S* __restrict__ st, RP b, RP e,
                                          int gl, int base0 = 0) {
  int base = base0;
  for (;;) {
    uint64_t m = 0;
    RP k = b + gl;
    for (; k + L < e; k += 2 * L) {  // two gathers in flight per lane
      int u0 = colidx[k];
      int u1 = colidx[k + L];
      int c0 = st[u0];
      int c1 = st[u1];
      unsigned r0 = (unsigned)c0 - (unsigned)base;
      unsigned r1 = (unsigned)c1 - (unsigned)base;
      if (c0 >= 0 && r0 < 64u) m |= 1ull << r0;
      if (c1 >= 0 && r1 < 64u) m |= 1ull << r1;
    }
    if (k < e) {
      int c0 = st[colidx[k]];
      unsigned r0 = (unsigned)c0 - (unsigned)base;
      if (c0 >= 0 && r0 < 64u) m |= 1ull << r0;
    }
    m = group_or<L>(m);
    if (m != ~0ull) return base + __builtin_ctzll(~m);
    base += 64;  // all of base..base+63 are taken: slide the window
  }
}

// Position of v's flag for colour c (< kPushColors) in KArgs::seen.  By
// vertex: v's 32 bytes are consecutive.  By chunk: a 64-vertex chunk's 2 KB
// are 32 rows of 64 bytes, row c holding colour c of every vertex of the
// chunk, so a wavefront reads one colour of its whole chunk with one
// coalesced load, a speculate pass reads only the rows up to the largest
// colour its chunk needs (the by-vertex block costs a whole 32-byte sector
// per vertex), and the pushes of one colour to a chunk meet in one row.  The
// by-chunk layout is used only without medium and heavy vertices, whose
// passes read one vertex's 32 flags on their own.
__device__ __forceinline__ size_t flag_index(const KArgs& a, int v, int c) {
  return a.flags_by_chunk
             ? ((size_t)(v / kWave) * kPushColors + c) * kWave + (size_t)(v % kWave)
             : (size_t)v * kPushColors + c;
}

// A vertex that has just committed colour t marks t as taken for its
// neighbours (row [b, e)) that are still uncoloured: byte t of the
// neighbour's flag block gets the call's epoch (t < 32), or byte t - 32 of
// its wide block when it has one (32 <= t < 512; only vertices of degree
// above the light bound can ever need such a colour).  Plain byte stores:
// concurrent writers touch different bytes or write the same value.  A
// neighbour that is already final needs nothing, which the state read skips
// (about half of all entries).  A group of `step` lanes.  The neighbour ids
// are ids[b .. e): the row itself (push_colour) or a list of some of its
// entries (a wavefront-class vertex's lower-neighbour list).
template <typename RP, typename S>
__device__ __forceinline__ void push_colour_ids(const KArgs& a, const int32_t* __restrict__ ids,
                                                const S* __restrict__ st, RP b, RP e, int t,
                                                int epoch, int gl, int step) {
  // four entries per lane in flight: the neighbour ids, then their states,
  // then the stores
  if (t < kPushColors) {
    RP k = b + gl;
    for (; k + 3 * (RP)step < e; k += 4 * (RP)step) {
      int u[4], s[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = ids[k + j * step];
#pragma unroll
      for (int j = 0; j < 4; ++j) s[j] = st[u[j]];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (s[j] < 0) a.seen[flag_index(a, u[j], t)] = (uint8_t)epoch;
    }
    for (; k < e; k += step) {
      const int u = ids[k];
      if (st[u] < 0) a.seen[flag_index(a, u, t)] = (uint8_t)epoch;
    }
  } else if (t < kPushColors + kWideColors) {
    // the same with the neighbour's wide-block index gathered beside its
    // state (both depend only on the neighbour id)
    const int c = t - kPushColors;
    RP k = b + gl;
    for (; k + 3 * (RP)step < e; k += 4 * (RP)step) {
      int u[4], s[4], w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = ids[k + j * step];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s[j] = st[u[j]];
        w[j] = a.widx[u[j]];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (w[j] >= 0 && s[j] < 0) a.wide[(size_t)w[j] * kWideColors + c] = (uint8_t)epoch;
    }
    for (; k < e; k += step) {
      const int u = ids[k];
      const int w = a.widx[u];
      if (w >= 0 && st[u] < 0) a.wide[(size_t)w * kWideColors + c] = (uint8_t)epoch;
    }
  }
}

template <typename RP, typename S>
__device__ __forceinline__ void push_colour(const KArgs& a, const S* __restrict__ st, RP b, RP e,
                                            int t, int epoch, int gl, int step) {
  push_colour_ids<RP, S>(a, a.colidx, st, b, e, t, epoch, gl, step);
}

// First colour in 32..511 not flagged in wide block w, or -1 when all are
// taken; computed by one wavefront (every lane returns the result).
__device__ __forceinline__ int first_free_wide(const uint8_t* wide, int w, int epoch) {
  const int lane = lane_id();
  constexpr int per_lane = (kWideColors + kWave - 1) / kWave;  // 8 bytes
  int first = INT32_MAX;
  const uint8_t* p = wide + (size_t)w * kWideColors;
#pragma unroll
  for (int j = 0; j < per_lane; ++j) {
    const int c = lane * per_lane + j;
    if (c < kWideColors && p[c] != (uint8_t)epoch && c < first) first = c;
  }
  // wave minimum
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(first, off);
    first = o < first ? o : first;
  }
  return first == INT32_MAX ? -1 : kPushColors + first;
}

// Bit c of the result is set when byte c of v's flag block equals epoch
// (a neighbour of v has final colour c), for c < kPushColors = 32.  The
// by-vertex flag layout.
__device__ __forceinline__ uint32_t taken_colours(const uint8_t* seen, int v, int epoch) {
  const uint4* p = (const uint4*)(seen + (size_t)v * kPushColors);
  const uint4 x = p[0], y = p[1];
  const uint32_t w[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      m |= (uint32_t)(((w[i] >> (8 * j)) & 0xffu) == (uint32_t)epoch) << (4 * i + j);
  return m;
}

// detect_lane_skip's scan for one vertex by a whole wavefront with four
// entries per lane in flight: each step covers 256 entries as four
// sub-ranges of 64, visited in order, so the first uncoloured entry, the
// first conflict and the end of the lower prefix are found in row order.
template <typename RP, typename S>
__device__ __forceinline__ bool detect_wave4_skip(const int32_t* __restrict__ colidx,
                                                  const S* __restrict__ st, RP b, RP e, int v,
                                                  int t, int lane, int* skip) {
  int first = -1;
  for (RP kb = b + *skip; kb < e; kb += 4 * kWave) {
    int u[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const RP k = kb + j * kWave + lane;
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
      const int base = (int)(kb - b) + j * kWave;
      if (first < 0 && am) first = base + __builtin_ctzll(am);
      if (cm) {
        *skip = first >= 0 ? first : base + __builtin_ctzll(cm);
        return true;
      }
      if (pm) {
        *skip = first >= 0 ? first : base + __builtin_ctzll(pm);
        return false;
      }
    }
  }
  *skip = first >= 0 ? first : (int)(e - b);
  return false;
}

// A wavefront-class vertex's conflict scan over a list of its lower
// neighbours (sorted rows, pushed colours).  lst (deg(v) entries, parallel to
// v's row) holds in its first *len entries lower neighbours that were still
// uncoloured when last seen; every lower neighbour before row offset *skip is
// final or on the list.  The list is read whole (the final entries it sheds
// are the point: a hub's lower prefix interleaves many final neighbours with
// a few uncoloured ones, which a resume offset alone cannot pass) and
// compacted in place, then the row is read from *skip, 256 entries per step as
// four sub-ranges of 64 in row order, adding the uncoloured lower neighbours
// it passes to the list.  The row part stops at a conflict (left unread at
// *skip, not listed) or at the first id >= v (*skip then points there, where
// a winner's pushes to its higher neighbours start).  Returns whether a
// lower neighbour carries tentative colour t.  Compaction is safe in place:
// an entry is written at or below the position it was read from, after the
// whole step's entries are in registers.
template <typename RP, typename S>
__device__ __forceinline__ bool detect_wave_list(const int32_t* __restrict__ colidx,
                                                 const S* __restrict__ st, int32_t* lst, RP b,
                                                 RP e, int v, int t, int lane, int* skip,
                                                 int* len) {
  const uint64_t below = (1ull << lane) - 1;
  const int n0 = *len;
  int w = 0;
  bool lose = false;
  for (int i0 = 0; i0 < n0; i0 += 2 * kWave) {
    int u[2], s[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = i0 + j * kWave + lane;
      u[j] = i < n0 ? lst[i] : -1;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) s[j] = u[j] >= 0 ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      // decode, do not test the sign, for the conflict (as in the row scans)
      lose |= __ballot(u[j] >= 0 && tent_of(s[j]) == t) != 0;
      const bool keep = u[j] >= 0 && s[j] < 0;
      const uint64_t km = __ballot(keep);
      const int dst = w + __popcll(km & below);
      if (keep && dst != i0 + j * kWave + lane) lst[dst] = u[j];
      w += __popcll(km);
    }
  }
  if (lose) {
    *len = w;
    return true;
  }
  for (RP kb = b + *skip; kb < e; kb += 4 * kWave) {
    int u[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const RP k = kb + j * kWave + lane;
      u[j] = k < e ? colidx[k] : INT32_MAX;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool low = u[j] < v;
      const uint64_t cm = __ballot(low && tent_of(s[j]) == t);
      const uint64_t stop = cm | __ballot(!low);
      const int p = stop ? __builtin_ctzll(stop) : kWave;  // lanes before p are passed
      const bool keep = low && s[j] < 0 && lane < p;
      const uint64_t km = __ballot(keep);
      if (keep) lst[w + __popcll(km & below)] = u[j];
      w += __popcll(km);
      if (stop) {
        *skip = (int)(kb - b) + j * kWave + p;
        *len = w;
        return (cm >> p) & 1;
      }
    }
  }
  *skip = (int)(e - b);
  *len = w;
  return false;
}

// detect_wave4_skip's scan by a group of GL lanes (lanes gbase ..
// gbase + GL - 1, mask gmask; GL a power of two up to 64) for one vertex:
// each step covers 4 * GL entries as four sub-ranges of GL, visited in order.
// Used where a chunk holds few uncoloured vertices, so that a long lower
// prefix is not walked four entries at a time by a single lane.
template <typename RP, typename S>
__device__ __forceinline__ bool detect_group4_skip(const int32_t* __restrict__ colidx,
                                                   const S* __restrict__ st, RP b, RP e, int v,
                                                   int t, int GL, int gl, uint64_t gmask,
                                                   int gbase, int* skip) {
  int first = -1;
  for (RP kb = b + *skip; kb < e; kb += 4 * GL) {  // group-uniform
    int u[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const RP k = kb + j * GL + gl;
      u[j] = k < e ? colidx[k] : INT32_MAX;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool low = u[j] < v;
      const uint64_t am = (__ballot(low && s[j] < 0) & gmask) >> gbase;
      const uint64_t cm = (__ballot(low && tent_of(s[j]) == t) & gmask) >> gbase;
      const uint64_t pm = (__ballot(!low) & gmask) >> gbase;
      const int base = (int)(kb - b) + j * GL;
      if (first < 0 && am) first = base + __builtin_ctzll(am);
      if (cm) {
        *skip = first >= 0 ? first : base + __builtin_ctzll(cm);
        return true;
      }
      if (pm) {
        *skip = first >= 0 ? first : base + __builtin_ctzll(pm);
        return false;
      }
    }
  }
  *skip = first >= 0 ? first : (int)(e - b);
  return false;
}

// Conflict scan with a resume offset (sorted rows), by one lane for its own
// vertex: starting at b + *skip, does a lower-id neighbour of v that is still
// uncoloured carry tentative colour t?  The scan stops at the first conflict
// or at the first neighbour id >= v.  On return *skip is the offset of the
// first still-uncoloured lower neighbour seen, or of the point where the scan
// ended when it saw none: every lower neighbour before it is final, and final
// colours never change, so later rounds (and the winner's pushes) may start
// there.  Two entries in flight: neighbour ids first, then the states of the
// lower ones.
template <typename RP, typename S>
__device__ __forceinline__ bool detect_lane_skip(const int32_t* __restrict__ colidx,
                                                 const S* __restrict__ st, RP b, RP e, int v,
                                                 int t, int* skip) {
  int first = -1;
  for (RP k = b + *skip; k < e; k += 2) {
    int u[2], s[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) u[j] = k + j < e ? colidx[k + j] : INT32_MAX;
#pragma unroll
    for (int j = 0; j < 2; ++j) s[j] = u[j] < v ? (int)st[u[j]] : 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int off = (int)(k - b) + j;
      if (u[j] >= v) {  // past the lower prefix (or the row's end)
        *skip = first >= 0 ? first : off;
        return false;
      }
      if (first < 0 && s[j] < 0) first = off;
      // decode, do not test the sign: a neighbour that wins in this same pass
      // flips ~t to t concurrently and must still count; final colours of
      // earlier rounds never equal t
      if (tent_of(s[j]) == t) {
        *skip = first >= 0 ? first : off;
        return true;
      }
    }
  }
  *skip = first >= 0 ? first : (int)(e - b);
  return false;
}

// The pushes of several winners of one wave, spread over all 64 lanes: lane i
// contributes the row segment [pb, pb + len) of its own winner (len = 0 for
// none) with colour t.  The segments are concatenated in lane order; entry j
// of the concatenation belongs to the last lane whose exclusive prefix is
// <= j, found by binary search over the prefixes with cross-lane reads.
// Each lane keeps four entries in flight.  Stores as in push_colour; without
// CHECK_STATE every entry is taken to be still uncoloured (the caller knows).
template <typename RP, typename S, bool CHECK_STATE = true>
__device__ __forceinline__ void push_flat(const KArgs& a, const S* __restrict__ st, RP pb, int len,
                                          int t, int epoch) {
  const int lane = lane_id();
  int incl = len;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int total = __shfl(incl, kWave - 1);
  if (total == 0) return;  // wave-uniform
  const int excl = incl - len;
  for (int j0 = 0; j0 < total; j0 += 4 * kWave) {
    int u[4], tt[4];
    bool ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + q * kWave + lane;
      ok[q] = j < total;
      int lo = 0;
#pragma unroll
      for (int w = 32; w > 0; w >>= 1) {
        const int mid = lo + w;
        const int pm = __shfl(excl, mid < kWave ? mid : kWave - 1);
        if (mid < kWave && pm <= j) lo = mid;
      }
      const RP ob = shfl_any<RP>(pb, lo);
      const int oe = __shfl(excl, lo);
      tt[q] = __shfl(t, lo);
      u[q] = ok[q] ? a.colidx[ob + (j - oe)] : 0;
    }
    int s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = ok[q] && CHECK_STATE ? (int)st[u[q]] : -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!ok[q] || s[q] >= 0) continue;
      if (tt[q] < kPushColors) {
        a.seen[flag_index(a, u[q], tt[q])] = (uint8_t)epoch;
      } else if (tt[q] < kPushColors + kWideColors) {
        const int w = a.widx[u[q]];
        if (w >= 0) a.wide[(size_t)w * kWideColors + (tt[q] - kPushColors)] = (uint8_t)epoch;
      }
    }
  }
}

// The state value of a vertex that is not yet ready under the id-priority
// schedule: the smallest value of the state type (colours and ~colour stay
// above it, since colours never exceed the degree and the state width
// leaves one value spare).
template <typename S>
__device__ __forceinline__ int waiting_state() {
  return sizeof(S) == 1 ? -128 : sizeof(S) == 2 ? -32768 : INT32_MIN;
}

// Is every lower-id neighbour of v final?  Group of L lanes.  With sorted
// rows the scan starts at *skip, stops at the first id >= v, and leaves in
// *skip the offset of the first lower neighbour that is not final (or where
// it ended): every lower neighbour before it is final for good.
template <typename RP, typename S, int L>
__device__ __forceinline__ bool ready_group(const int32_t* __restrict__ colidx,
                                            const S* __restrict__ st, RP b, RP e, int v, int gl,
                                            uint64_t gmask, int gbase, bool sorted, int* skip) {
  for (RP kb = b + (sorted ? *skip : 0); kb < e; kb += L) {
    const RP k = kb + gl;
    bool wait = false, past = false;
    if (k < e) {
      const int u = colidx[k];
      if (u < v) wait = st[u] < 0;
      else past = true;
    } else {
      past = true;
    }
    const uint64_t wm = (__ballot(wait) & gmask) >> gbase;
    if (wm) {
      if (sorted) *skip = (int)(kb - b) + __builtin_ctzll(wm);
      return false;
    }
    if (sorted) {
      const uint64_t pm = (__ballot(past) & gmask) >> gbase;
      if (pm) {
        *skip = (int)(kb - b) + __builtin_ctzll(pm);
        return true;
      }
    }
  }
  if (sorted) *skip = (int)(e - b);
  return true;
}

// Does a lower-id neighbour of v carry tentative colour t?  Group of L lanes.
// With sorted rows the scan stops at the first neighbour id >= v.
template <typename RP, typename S, int L>
__device__ __forceinline__ bool detect_group(const int32_t* __restrict__ colidx,
                                             const S* __restrict__ st, RP b, RP e,
                                             int v, int t, int gl, uint64_t gmask, bool sorted) {
  for (RP kb = b; kb < e; kb += L) {
    RP k = kb + gl;
    bool conf = false, past = false;
    if (k < e) {
      int u = colidx[k];
      if (u < v) {
        conf = tent_of(st[u]) == t;
      } else {
        past = true;
      }
    } else {
      past = true;
    }
    if (__ballot(conf) & gmask) return true;
    if (sorted && (__ballot(past) & gmask)) return false;
  }
  return false;
}

}  // namespace gc
