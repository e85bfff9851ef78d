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
// together), one lane per vertex in phase 2, a kernel boundary per barrier.
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
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long vl = tid; vl < a.n; vl += nth) {
    const int v = (int)vl;
    if (!a.todo[v]) continue;
    const long b = (long)v * a.p / a.n;
    const int v0 = block_start(b, a.n, a.p), v1 = block_start(b + 1, a.n, a.p);
    const int cv = a.color[v];
    bool lose = false;
    for (RP k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = a.colidx[k];
      if (u >= v0 && u < v1) continue;  // same block
      const int cu = a.color[u];
      a.slot[k] = cu;
      lose |= cu == cv && u >= v1;  // u in a higher-numbered block
    }
    a.todo[v] = lose;
    active += 1;
    lost += lose;
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
static int launch_blocks_round_t(const BArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_blk_clear_left, dim3(1), dim3(64), 0, s, a.ctrl);
  // enough wavefronts for one per block, capped by the grid of the round kernels
  const long waves = a.p;
  const int g1 = (int)std::min<long>((waves + kWavesPerBlock - 1) / kWavesPerBlock, (long)grid);
  hipLaunchKernelGGL((k_blk_phase1<RP>), dim3(std::max(1, g1)), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((k_blk_phase2<RP>), dim3(grid), dim3(kBlock), 0, s, a);
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

int launch_blocks_round(const BArgs& a, bool rp64, int grid, void* stream) {
  return rp64 ? launch_blocks_round_t<int64_t>(a, grid, (hipStream_t)stream)
              : launch_blocks_round_t<int32_t>(a, grid, (hipStream_t)stream);
}

}  // namespace gc
