// gc_validate.hip -- the CSR checks of gc_create (GC_VALIDATE).
//
// The colouring needs a simple undirected graph (§2.1): row pointers that
// rise from 0 to the entry count, neighbour ids in range, no self-loops, no
// repeated entries, and every edge stored in both directions.  Rows given as
// ascending are checked in place (adjacent entries, and a binary search in
// the neighbour's row for the reverse edge).  Other rows are checked the
// same way on an ascending copy: one radix sort of (row, neighbour) keys
// over all entries orders every row without changing its contents, so the
// whole check costs O(m log m) whatever the degrees are, where comparing
// each entry with the rest of its row would cost O(sum of squared degrees)
// (seconds for one hub of 10^5 entries).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>

#include "gc.h"
#include "gc_internal.h"

namespace gc {

namespace {

// err[0] receives the smallest failing check code (0 = fine), err[1] the
// vertex where one failure of that code was seen:
//   1 rowptr[0] != 0 or rowptr[n] != m     2 rowptr decreases
//   3 neighbour id out of range             4 self-loop
//   5 duplicate entry in a row              6 row not ascending (sorted mode)
//   7 edge (v, u) without (u, v)
// Without SORTED a row's entries are compared pairwise (the fallback when
// an ascending copy cannot be made).
template <typename RP, bool SORTED>
__global__ void k_validate(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t m,
                           int32_t* err) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  auto fail = [&](int code, long where) {
    int old = atomicMin(&err[0], code);
    if (code <= old) err[1] = (int)where;
  };
  if (tid == 0 && (rowptr[0] != 0 || (int64_t)rowptr[n] != m)) fail(1, 0);
  for (long v = tid; v < n; v += nth) {
    RP b = rowptr[v], e = rowptr[v + 1];
    if (e < b || b < 0 || (int64_t)e > m) {
      fail(2, v);
      continue;
    }
    for (RP k = b; k < e; ++k) {
      int u = colidx[k];
      if (u < 0 || u >= n) {
        fail(3, v);
        continue;
      }
      if (u == v) fail(4, v);
      if (k > b) {
        int p = colidx[k - 1];
        if (p == u) fail(5, v);
        else if (SORTED && p > u) fail(6, v);
      }
      if (!SORTED) {
        for (RP j = b; j < k; ++j)
          if (colidx[j] == u) fail(5, v);
      }
      // symmetry: v must appear in row u
      RP ub = rowptr[u], ue = rowptr[u + 1];
      if (ue < ub || ub < 0 || (int64_t)ue > m) continue;  // reported at u
      bool found = false;
      if (SORTED) {
        RP lo = ub, hi = ue;
        while (lo < hi) {
          RP mid = lo + (hi - lo) / 2;
          if (colidx[mid] < v) lo = mid + 1;
          else hi = mid;
        }
        found = lo < ue && colidx[lo] == v;
      } else {
        for (RP j = ub; j < ue && !found; ++j) found = colidx[j] == v;
      }
      if (!found) fail(7, v);
    }
  }
}

// The sort key of entry k: its row in the high word (the last row whose
// pointer is <= k, by binary search; any row when the pointers are broken,
// which the check then reports as code 1 or 2), its neighbour id in the low
// word.  Ids out of range sort after every valid id of the row.
template <typename RP>
__global__ void k_entry_keys(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t nnz,
                             uint64_t* keys) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long k = tid; k < nnz; k += nth) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if ((long)rowptr[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    keys[k] = ((uint64_t)(uint32_t)lo << 32) | (uint64_t)(uint32_t)colidx[k];
  }
}

__global__ void k_low_words(const uint64_t* keys, int64_t nnz, int32_t* out) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nth = (long)gridDim.x * blockDim.x;
  for (long k = tid; k < nnz; k += nth) out[k] = (int32_t)(uint32_t)keys[k];
}

struct Temps {  // device temporaries, freed on every exit
  void* p[3] = {};
  ~Temps() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};

// Unsorted rows: the checks on an ascending copy.  Returns 0 when the copy
// was checked, 1 when it could not be made (too many entries for one sort,
// or no memory for it), or a HIP error.
template <typename RP>
int validate_sorted_copy(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t m,
                         int32_t* err, int grid, hipStream_t s) {
  if (m > INT32_MAX || m == 0 || n < 1) return 1;
  Temps t;
  uint64_t* keys = nullptr;
  if (hipMalloc((void**)&keys, 2 * (size_t)m * sizeof(uint64_t)) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  t.p[0] = keys;
  uint64_t* keys2 = keys + m;
  int bits = 1;
  while (bits < 31 && (1ll << bits) < (long long)n) ++bits;
  size_t tb = 0;
  hipError_t e;
  if ((e = hipcub::DeviceRadixSort::SortKeys(nullptr, tb, keys, keys2, (int)m, 0, 32 + bits, s)) !=
      hipSuccess)
    return (int)e;
  void* temp = nullptr;
  int32_t* copy = nullptr;
  if (hipMalloc(&temp, tb > 0 ? tb : 1) != hipSuccess ||
      (t.p[1] = temp, hipMalloc((void**)&copy, (size_t)m * sizeof(int32_t))) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  t.p[2] = copy;
  hipLaunchKernelGGL((k_entry_keys<RP>), dim3(grid), dim3(256), 0, s, rowptr, colidx, n, m, keys);
  if ((e = hipcub::DeviceRadixSort::SortKeys(temp, tb, keys, keys2, (int)m, 0, 32 + bits, s)) !=
      hipSuccess)
    return (int)e;
  hipLaunchKernelGGL(k_low_words, dim3(grid), dim3(256), 0, s, keys2, m, copy);
  hipLaunchKernelGGL((k_validate<RP, true>), dim3(grid), dim3(256), 0, s, rowptr, copy, n, m, err);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  // the temporaries are freed on return: the stream must be done with them
  return (int)hipStreamSynchronize(s);
}

template <typename RP>
int validate_t(const RP* rowptr, const int32_t* colidx, int32_t n, int64_t m, bool sorted,
               int32_t* err, int grid, hipStream_t s) {
  if (!sorted) {
    const int rc = validate_sorted_copy<RP>(rowptr, colidx, n, m, err, grid, s);
    if (rc != 1) return rc;
    hipLaunchKernelGGL((k_validate<RP, false>), dim3(grid), dim3(256), 0, s, rowptr, colidx, n, m,
                       err);
  } else {
    hipLaunchKernelGGL((k_validate<RP, true>), dim3(grid), dim3(256), 0, s, rowptr, colidx, n, m,
                       err);
  }
  return (int)hipGetLastError();
}

}  // namespace

int launch_validate(const void* rowptr, bool rp64, const int32_t* colidx, int32_t n, int64_t m,
                    bool sorted, int32_t* err, int grid, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  return rp64 ? validate_t<int64_t>((const int64_t*)rowptr, colidx, n, m, sorted, err, grid, s)
              : validate_t<int32_t>((const int32_t*)rowptr, colidx, n, m, sorted, err, grid, s);
}

}  // namespace gc
