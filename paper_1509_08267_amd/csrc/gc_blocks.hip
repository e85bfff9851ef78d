// gc_blocks.hip -- Algorithm 1 of Section 3.1 with p blocks, read literally
// (GC_ALGO_BLOCKS).
//
// The vertices are split into p blocks of consecutive ids (block(v) =
// floor(v p / n)).  Every vertex keeps a ForbiddenColors slot per CSR entry.
// A round is
//   phase 1: each block colours its vertices still to colour, in increasing
//            id order, each with the least colour absent from its slots, and
//            writes that colour into the slot for it of every neighbour in the
//            same block;
//   phase 2: each such vertex with neighbours in other blocks copies their
//            current colours into its slots for them, and is recoloured next
//            round when one of them, in a higher-numbered block, has its
//            colour (the paper's "the vertex in the lower partition is
//            recoloured").
// Mapping: one wavefront per block in phase 1 (a block is sequential by
// definition; the wavefront searches each row for the least absent colour
// together), one wavefront per 64 consecutive vertices in phase 2, a kernel
// boundary per barrier.
//
// The slot for a neighbour in the same block always equals that
// neighbour's current colour (it is written whenever the neighbour is
// coloured, and both start at -1), so phase 1 reads the colour array for
// those entries and the slot array holds only entries whose neighbour lies
// in another block.  A colour written for a vertex is read by later vertices
// of its block in the same wavefront: a workgroup-scope fence orders the
// write before those reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gc_device.h"
#include "gc_internal.h"

namespace gc {

// first id of block b: the least v with floor(v p / n) == b
__device__ __forceinline__ int block_start(long b, int n, long p) {
  return (int)((b * (long)n + p - 1) / p);
}

template <typename RP>
__global__ __launch_bounds__(kBlock) void k_blk_init(BArgs a) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long v = tid; v < a.n; v += nth) {
    a.color[v] = -1;
    a.todo[v] = 1;
  }
  const long nnz = a.n > 0 ? (long)((const RP*)a.rowptr)[a.n] : 0;
  for (long k = tid; k < nnz; k += nth) a.slot[k] = -1;
}

template <typename RP>
__global__ __launch_bounds__(kBlock) void k_blk_phase1(BArgs a) {
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  const int lane = lane_id();
  const long wave_gid = blockIdx.x * (long)kWavesPerBlock + threadIdx.x / kWave;
  const long nwaves = (long)gridDim.x * kWavesPerBlock;
  for (long b = wave_gid; b < a.p; b += nwaves) {
    const int v0 = block_start(b, a.n, a.p), v1 = block_start(b + 1, a.n, a.p);
    for (int v = v0; v < v1; ++v) {  // wave-uniform
      if (!a.todo[v]) continue;
      const RP rb = rp[v], re = rp[v + 1];
      int c = 0;
      for (int base = 0;; base += kWave) {  // least colour absent from the slots
        uint64_t m = 0;
        for (RP k = rb + lane; k < re; k += kWave) {
          const int u = a.colidx[k];
          const int s = (u >= v0 && u < v1) ? a.color[u] : a.slot[k];
          const unsigned r = (unsigned)s - (unsigned)base;
          if (s >= 0 && r < 64u) m |= 1ull << r;
        }
        m = group_or<kWave>(m);
        if (m != ~0ull) {
          c = base + __builtin_ctzll(~m);
          break;
        }
      }
      if (lane == 0) a.color[v] = c;
      // later vertices of this block (same wavefront) read this colour
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
  }
}

// Phase 2 by 64-vertex chunks: the rows of a chunk's pending vertices are
// consecutive in colidx, so the wavefront streams them as one segmented
// list (coalesced reads of colidx, coalesced slot writes); entry j belongs to
// the last lane whose exclusive prefix is <= j (binary search over the
// prefixes with cross-lane reads), and the conflicts of the chunk meet in a
// 64-bit mask, bit i for lane i's vertex.
template <typename RP>
__global__ __launch_bounds__(kBlock) void k_blk_phase2(BArgs a) {
  __shared__ int sh_active, sh_lost;
  const RP* __restrict__ rp = (const RP*)a.rowptr;
  if (threadIdx.x == 0) {
    sh_active = 0;
    sh_lost = 0;
  }
  __syncthreads();
  int active = 0, lost = 0;
  const int lane = lane_id();
  const long wave_gid = blockIdx.x * (long)kWavesPerBlock + threadIdx.x / kWave;
  const long nwaves = (long)gridDim.x * kWavesPerBlock;
  const long nchunks = ((long)a.n + kWave - 1) / kWave;
  for (long ch = wave_gid; ch < nchunks; ch += nwaves) {
    const int v = (int)(ch * kWave) + lane;
    const bool pend = v < a.n && a.todo[v];
    RP b = 0;
    int len = 0, v0 = 0, v1 = 0, cv = 0;
    if (pend) {
      b = rp[v];
      len = (int)(rp[v + 1] - b);
      const long blk = (long)v * a.p / a.n;
      v0 = block_start(blk, a.n, a.p);
      v1 = block_start(blk + 1, a.n, a.p);
      cv = a.color[v];
    }
    if (__ballot(pend) == 0) continue;
    int incl = len;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    const int total = __shfl(incl, kWave - 1);
    const int excl = incl - len;
    uint64_t lm = 0;
    for (int j0 = 0; j0 < total; j0 += 4 * kWave) {
      int u[4], o[4], ov1[4], ocv[4];
      bool ok[4], foreign[4];
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
        o[q] = lo;
        const RP ob = shfl_any<RP>(b, lo);
        const int oe = __shfl(excl, lo);
        const int ov0 = __shfl(v0, lo);
        ov1[q] = __shfl(v1, lo);
        ocv[q] = __shfl(cv, lo);
        u[q] = ok[q] ? a.colidx[ob + (j - oe)] : 0;
        foreign[q] = ok[q] && (u[q] < ov0 || u[q] >= ov1[q]);
        if (foreign[q]) {
          const int cu = a.color[u[q]];
          a.slot[ob + (j - oe)] = cu;
          if (cu == ocv[q] && u[q] >= ov1[q]) lm |= 1ull << o[q];  // higher block
        }
      }
    }
    lm = group_or<kWave>(lm);
    if (pend) {
      const bool lose = (lm >> lane) & 1;
      a.todo[v] = lose;
      active += 1;
      lost += lose;
    }
  }
  if (active) atomicAdd(&sh_active, active);
  if (lost) atomicAdd(&sh_lost, lost);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (sh_lost) atomicAdd(&a.ctrl->left.v, sh_lost);
    if (sh_active) {
      a.ctrl->last_round.v = a.round;
      if (a.round - 1 < kTraceRounds) atomicAdd(&a.ctrl->trace[a.round - 1], sh_active);
    }
  }
}

__global__ void k_blk_clear_left(Ctrl* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->left.v = 0;
}

template <typename RP>
static int launch_blocks_phase_t(const BArgs& a, int phase, int grid, hipStream_t s) {
  if (phase == 1) {
    hipLaunchKernelGGL(k_blk_clear_left, dim3(1), dim3(64), 0, s, a.ctrl);
    // enough wavefronts for one per block, capped by the grid of the round kernels
    const long waves = a.p;
    const int g1 = (int)std::min<long>((waves + kWavesPerBlock - 1) / kWavesPerBlock, (long)grid);
    hipLaunchKernelGGL((k_blk_phase1<RP>), dim3(std::max(1, g1)), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_blk_phase2<RP>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return (int)hipGetLastError();
}

__global__ void k_blk_set_left(Ctrl* c, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->left.v = value;
}

int launch_blocks_set_left(Ctrl* c, int value, void* stream) {
  hipLaunchKernelGGL(k_blk_set_left, dim3(1), dim3(64), 0, (hipStream_t)stream, c, value);
  return (int)hipGetLastError();
}

int launch_blocks_init(const BArgs& a, bool rp64, int grid, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (rp64) hipLaunchKernelGGL((k_blk_init<int64_t>), dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_blk_init<int32_t>), dim3(grid), dim3(kBlock), 0, s, a);
  return (int)hipGetLastError();
}

int launch_blocks_phase(const BArgs& a, bool rp64, int phase, int grid, void* stream) {
  return rp64 ? launch_blocks_phase_t<int64_t>(a, phase, grid, (hipStream_t)stream)
              : launch_blocks_phase_t<int32_t>(a, phase, grid, (hipStream_t)stream);
}

}  // namespace gc
