// gc_order.hip -- relabelling a graph by a vertex order before colouring.
//
// Orders (GC_OPT_ORDER): largest degree first (ties by id), and a seeded
// random order by the splitmix64 generator's output at step v + 1 from the
// seed (Steele, Lea and Flood, 2014; Jones and Plassmann's random order).
// Vertex sigma[i] becomes vertex i.  Everything runs on the device:
//   1. a radix sort of (key, id) pairs gives sigma;
//   2. newid[sigma[i]] = i and the new degrees; an exclusive scan gives the
//      new row pointers;
//   3. every CSR entry (v, u) becomes the key (newid[v] << b) | newid[u]
//      (b = bits of n); one radix sort over all entries orders them by new
//      row and, within a row, by new neighbour id, so the new rows come out
//      ascending; the low b bits are the new column ids.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>

#include "gc.h"
#include "gc_internal.h"

namespace gc {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename RP>
__global__ void k_order_keys(const RP* rowptr, int32_t n, int kind, uint64_t seed, uint64_t* keys,
                             int32_t* ids) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long v = tid; v < n; v += nth) {
    uint64_t key;
    if (kind == GC_ORDER_LARGEST_FIRST) {
      const uint64_t deg = (uint64_t)(rowptr[v + 1] - rowptr[v]);
      key = ((0xFFFFFFFFull - deg) << 32) | (uint64_t)v;
    } else {
      key = splitmix64_mix(seed + (uint64_t)(v + 1) * kGamma);
    }
    keys[v] = key;
    ids[v] = (int32_t)v;
  }
}

template <typename RP>
__global__ void k_order_newid(const RP* rowptr, const int32_t* sigma, int32_t n, int32_t* newid,
                              RP* deg2) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long i = tid; i < n; i += nth) {
    const int32_t v = sigma[i];
    newid[v] = (int32_t)i;
    deg2[i] = rowptr[v + 1] - rowptr[v];
  }
  if (tid == 0) deg2[n] = 0;
}

// one thread per CSR entry; its row by binary search over rowptr
template <typename RP>
__global__ void k_order_edge_keys(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t nnz,
                                  const int32_t* newid, int bits, uint64_t* ekeys) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long k = tid; k < nnz; k += nth) {
    int32_t lo = 0, hi = n - 1;  // the row v with rowptr[v] <= k < rowptr[v + 1]
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if ((long)rowptr[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    ekeys[k] = ((uint64_t)newid[lo] << bits) | (uint64_t)newid[colidx[k]];
  }
}

__global__ void k_order_cols(const uint64_t* sorted, int64_t nnz, uint64_t mask, int32_t* colidx2) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long k = tid; k < nnz; k += nth) colidx2[k] = (int32_t)(sorted[k] & mask);
}

__global__ void k_permute_back(const int32_t* newid, const int32_t* coloured, int32_t n,
                               int32_t* out) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long v = tid; v < n; v += nth) out[v] = coloured[newid[v]];
}

struct Scratch {  // device temporaries of one build, freed on every exit
  void* p[6] = {};
  ~Scratch() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};

template <typename RP>
int build_t(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t nnz, int kind,
            uint64_t seed, RP* rowptr2, int32_t* colidx2, int32_t* newid, int grid, hipStream_t s) {
  Scratch t;
  uint64_t *keys = nullptr, *keys2 = nullptr;
  int32_t *ids = nullptr, *sigma = nullptr;
  hipError_t e;
  const size_t nv = (size_t)(n > 0 ? n : 1);
  if ((e = hipMalloc((void**)&keys, 2 * nv * sizeof(uint64_t))) != hipSuccess) return (int)e;
  t.p[0] = keys;
  keys2 = keys + nv;
  if ((e = hipMalloc((void**)&ids, 2 * nv * sizeof(int32_t))) != hipSuccess) return (int)e;
  t.p[1] = ids;
  sigma = ids + nv;
  hipLaunchKernelGGL((k_order_keys<RP>), dim3(grid), dim3(256), 0, s, rowptr, n, kind, seed, keys,
                     ids);
  size_t tb = 0;
  if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, keys2, ids, sigma, (int)n, 0, 64,
                                              s)) != hipSuccess)
    return (int)e;
  void* temp = nullptr;
  if ((e = hipMalloc(&temp, tb > 0 ? tb : 1)) != hipSuccess) return (int)e;
  t.p[2] = temp;
  if ((e = hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, keys2, ids, sigma, (int)n, 0, 64,
                                              s)) != hipSuccess)
    return (int)e;
  // new ids, new degrees (deg2 has n + 1 entries, the last 0), new row pointers
  RP* deg2 = nullptr;
  if ((e = hipMalloc((void**)&deg2, (nv + 1) * sizeof(RP))) != hipSuccess) return (int)e;
  t.p[3] = deg2;
  hipLaunchKernelGGL((k_order_newid<RP>), dim3(grid), dim3(256), 0, s, rowptr, sigma, n, newid,
                     deg2);
  size_t sb = 0;
  if ((e = hipcub::DeviceScan::ExclusiveSum(nullptr, sb, deg2, rowptr2, (int)n + 1, s)) !=
      hipSuccess)
    return (int)e;
  void* stemp = nullptr;
  if ((e = hipMalloc(&stemp, sb > 0 ? sb : 1)) != hipSuccess) return (int)e;
  t.p[4] = stemp;
  if ((e = hipcub::DeviceScan::ExclusiveSum(stemp, sb, deg2, rowptr2, (int)n + 1, s)) !=
      hipSuccess)
    return (int)e;
  if (nnz > 0) {
    int bits = 1;
    while (bits < 31 && (1ll << bits) < (long long)n) ++bits;
    uint64_t* ek = nullptr;
    if ((e = hipMalloc((void**)&ek, 2 * (size_t)nnz * sizeof(uint64_t))) != hipSuccess) return (int)e;
    t.p[5] = ek;
    uint64_t* ek2 = ek + nnz;
    hipLaunchKernelGGL((k_order_edge_keys<RP>), dim3(grid), dim3(256), 0, s, rowptr, colidx, n, nnz,
                       newid, bits, ek);
    size_t eb = 0;
    if ((e = hipcub::DeviceRadixSort::SortKeys(nullptr, eb, ek, ek2, (int)nnz, 0, 2 * bits, s)) !=
        hipSuccess)
      return (int)e;
    if (eb > tb) {  // reuse the first sort's temporary when large enough
      (void)hipFree(temp);
      t.p[2] = nullptr;
      if ((e = hipMalloc(&temp, eb)) != hipSuccess) return (int)e;
      t.p[2] = temp;
      tb = eb;
    }
    if ((e = hipcub::DeviceRadixSort::SortKeys(temp, tb, ek, ek2, (int)nnz, 0, 2 * bits, s)) !=
        hipSuccess)
      return (int)e;
    hipLaunchKernelGGL(k_order_cols, dim3(grid), dim3(256), 0, s, ek2, nnz,
                       (uint64_t)((1ull << bits) - 1), colidx2);
  }
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  // the temporaries are freed on return: the stream must be done with them
  return (int)hipStreamSynchronize(s);
}

}  // namespace

int build_order(const void* rowptr, bool rp64, const int32_t* colidx, int32_t n, int64_t nnz,
                int kind, uint64_t seed, void* rowptr2, int32_t* colidx2, int32_t* newid, int grid,
                void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return rp64 ? build_t<int64_t>((const int64_t*)rowptr, colidx, n, nnz, kind, seed,
                                 (int64_t*)rowptr2, colidx2, newid, grid, s)
              : build_t<int32_t>((const int32_t*)rowptr, colidx, n, nnz, kind, seed,
                                 (int32_t*)rowptr2, colidx2, newid, grid, s);
}

int launch_permute_back(const int32_t* newid, const int32_t* coloured, int32_t n, int32_t* out,
                        int grid, void* stream) {
  hipLaunchKernelGGL(k_permute_back, dim3(grid), dim3(256), 0, (hipStream_t)stream, newid,
                     coloured, n, out);
  return (int)hipGetLastError();
}

}  // namespace gc
