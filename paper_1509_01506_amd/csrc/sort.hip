// Ordering of the matches that a single-pass find appends in no particular
// order: keys (end position << 24 | pattern id) sorted ascending, which is
// the output order (ascending end position, ties by ascending pattern id),
// then split into the caller's position and pattern arrays.  Up to
// kSmallSort keys are sorted by one block in LDS; more by a device radix sort
// (rocPRIM).  A translation unit of its own: rocPRIM is heavy to compile.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <cstdint>

namespace coex {

constexpr uint32_t kSmallSort = 4096;

// One block of 1024 threads: bitonic sort of n <= kSmallSort keys in LDS
// (padded with ~0), then the split into positions (counted from the
// sequence's first base, buffer position `first`) and pattern ids.
__global__ __launch_bounds__(1024) void k_sort_small(const uint64_t* keys, uint64_t n, int64_t* pos, uint32_t* pat,
                                                     uint64_t first) {
  __shared__ uint64_t k[kSmallSort];
  uint32_t m = 1;
  while (m < n) m <<= 1;
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) k[i] = i < n ? keys[i] : ~0ull;
  __syncthreads();
  for (uint32_t size = 2; size <= m; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const uint64_t x = k[i], y = k[j];
          if ((x > y) == up) {
            k[i] = y;
            k[j] = x;
          }
        }
      }
      __syncthreads();
    }
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    pos[i] = (int64_t)((k[i] >> 24) - first);
    if (pat) pat[i] = (uint32_t)(k[i] & 0xFFFFFFu);
  }
}

__global__ void k_split_keys(const uint64_t* keys, uint64_t n, int64_t* pos, uint32_t* pat, uint64_t first) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    pos[i] = (int64_t)((keys[i] >> 24) - first);
    if (pat) pat[i] = (uint32_t)(keys[i] & 0xFFFFFFu);
  }
}

// Per-pattern counts of n matches from their pattern ids: per-block LDS
// histograms added to the zeroed counts (n_pat <= kIdHist), else global
// atomics.  ids NULL: a one-pattern automaton, every match is pattern 0.
constexpr uint32_t kIdHist = 4096;

__global__ void k_zero_counts(uint64_t* counts, uint32_t n_pat) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_pat; i += gridDim.x * blockDim.x) counts[i] = 0;
}

__global__ __launch_bounds__(256) void k_count_ids(const uint32_t* ids, uint64_t n, uint32_t n_pat,
                                                   uint64_t* counts) {
  __shared__ uint32_t h[kIdHist];
  if (!ids) {
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[0] = n;
    return;
  }
  const bool local = n_pat <= kIdHist;
  if (local) {
    for (uint32_t i = threadIdx.x; i < n_pat; i += blockDim.x) h[i] = 0;
    __syncthreads();
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t id = ids[i];
    if (id >= n_pat) continue;  // never: ids come from the automaton's output sets
    if (local) atomicAdd(h + id, 1u);
    else atomicAdd(reinterpret_cast<unsigned long long*>(counts + id), 1ull);
  }
  if (local) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_pat; i += blockDim.x)
      if (h[i]) atomicAdd(reinterpret_cast<unsigned long long*>(counts + i), (unsigned long long)h[i]);
  }
}

// counts_dev[0..n_pat) from the n pattern ids of a find (ids NULL: one
// pattern, or no match at all).  Asynchronous.
int counts_from_ids(const uint32_t* ids, uint64_t n, uint32_t n_pat, uint64_t* counts, hipStream_t st) {
  if (n_pat == 0) return 0;
  if (ids || n_pat > 1) hipLaunchKernelGGL(k_zero_counts, dim3((n_pat + 255) / 256), dim3(256), 0, st, counts, n_pat);
  if (!ids && n_pat > 1) return hipGetLastError() == hipSuccess ? 0 : -1;  // no ids kept: no match
  const uint64_t want = (n + 255) / 256;
  const uint32_t blocks = (uint32_t)(want == 0 ? 1 : (want < 1024 ? want : 1024));
  hipLaunchKernelGGL(k_count_ids, dim3(ids ? blocks : 1u), dim3(256), 0, st, ids, n, n_pat, counts);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Temporary bytes the radix sort needs for up to `cap` keys.
size_t sort_temp_bytes(uint64_t cap) {
  if (cap <= kSmallSort) return 0;
  size_t bytes = 0;
  if (rocprim::radix_sort_keys(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr, (size_t)cap, 0, 64) !=
      hipSuccess)
    return 0;
  return bytes;
}

// keys[0..n) -> pos/pat in order; `tmp` holds n keys, `temp` the sort's
// temporary storage (sort_temp_bytes(cap) bytes, cap >= n); key positions
// are buffer positions, `first` the one of the sequence's first base.
// Asynchronous.
int sort_match_keys(const uint64_t* keys, uint64_t* tmp, uint64_t n, void* temp, size_t temp_bytes, int64_t* pos,
                    uint32_t* pat, uint64_t first, hipStream_t st) {
  if (n == 0) return 0;
  if (n <= kSmallSort) {
    hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(1024), 0, st, keys, n, pos, pat, first);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  size_t bytes = temp_bytes;
  if (rocprim::radix_sort_keys(temp, bytes, keys, tmp, (size_t)n, 0, 64, st) != hipSuccess) return -1;
  const uint32_t blocks = (uint32_t)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_split_keys, dim3(blocks), dim3(256), 0, st, tmp, n, pos, pat, first);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace coex
