// Node tiles and their halos for the LDS-staged gather kernels.
//
// Nodes are cut into tiles of kTileNodes consecutive nodes (Morton order makes
// a tile a compact patch). The halo of a tile is the sorted set of distinct
// neighbour indices of its rows. The stage and filter kernels load the halo's
// field values into LDS once per tile and then read every neighbour value
// from LDS through a 16-bit position in the halo, which also halves the
// per-edge index stream (2 instead of 4 bytes).
//
// One workgroup builds one tile: the row entries are inserted into an LDS
// hash set, the distinct indices are sorted (bitonic sort in LDS), and every
// entry's position in the sorted halo is found by binary search.
#include <climits>

#include "common.hpp"

namespace labfm {
namespace {

constexpr int kTileNodes = LABFM_TILE_NODES;
constexpr int kHaloMax = LABFM_TILE_HALO_MAX;
constexpr int kHashCap = 2 * kHaloMax;  // load factor <= 1/2
constexpr int kThreads = 256;
constexpr int kEmpty = -1;

__device__ __forceinline__ unsigned hash_slot(int j) {
  return (static_cast<unsigned>(j) * 2654435761u) >> (32 - 11);  // kHashCap = 2^11
}
static_assert(kHashCap == 2048, "hash_slot assumes 2^11 slots");

__global__ void __launch_bounds__(kThreads)
build_tiles_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col, int n,
                   int* __restrict__ halo_count, int* __restrict__ halo_idx,
                   unsigned short* __restrict__ lcol, int* __restrict__ max_halo,
                   int* __restrict__ overflow) {
  __shared__ int table[kHashCap];
  __shared__ int list[kHashCap];
  __shared__ int s_count;
  __shared__ int s_full;
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const int t0 = t * kTileNodes;
  const int t1 = min(n, t0 + kTileNodes);
  const int e0 = row_ptr[t0], e1 = row_ptr[t1];
  for (int k = tid; k < kHashCap; k += kThreads) {
    table[k] = kEmpty;
    list[k] = INT_MAX;
  }
  if (tid == 0) {
    s_count = 0;
    s_full = 0;
  }
  __syncthreads();
  // insert every neighbour index (linear probing; duplicates stop at their slot)
  for (int e = e0 + tid; e < e1; e += kThreads) {
    const int j = col[e];
    unsigned sl = hash_slot(j);
    for (int probe = 0; probe < kHashCap; ++probe) {
      const int prev = atomicCAS(&table[sl], kEmpty, j);
      if (prev == kEmpty) {
        const int pos = atomicAdd(&s_count, 1);
        if (pos < kHaloMax) {
          list[pos] = j;
        } else {
          s_full = 1;
        }
        break;
      }
      if (prev == j) break;
      sl = (sl + 1) & (kHashCap - 1);
    }
  }
  __syncthreads();
  const int count = s_count;
  if (s_full || count > kHaloMax) {
    if (tid == 0) {
      atomicMax(overflow, 1);
      halo_count[t] = 0;
    }
    return;
  }
  // bitonic sort of list[0 .. kHaloMax) ascending (unused entries are INT_MAX)
  for (int size = 2; size <= kHaloMax; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = tid; k < kHaloMax; k += kThreads) {
        const int p = k ^ stride;
        if (p > k) {
          const bool up = (k & size) == 0;
          const int a = list[k], b = list[p];
          if ((a > b) == up) {
            list[k] = b;
            list[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int k = tid; k < count; k += kThreads)
    halo_idx[static_cast<long long>(t) * kHaloMax + k] = list[k];
  if (tid == 0) {
    halo_count[t] = count;
    atomicMax(max_halo, count);
  }
  // position of every entry in the sorted halo
  for (int e = e0 + tid; e < e1; e += kThreads) {
    const int j = col[e];
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (list[mid] < j) {
        lo = mid + 1;
      } else {
        hi = mid;
      }
    }
    lcol[e] = static_cast<unsigned short>(lo);
  }
}

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" int32_t labfm_tile_count(int32_t n) {
  return n > 0 ? (n + kTileNodes - 1) / kTileNodes : 0;
}

extern "C" size_t labfm_tiles_workspace_bytes(void) { return 256; }

extern "C" int labfm_build_tiles(const int32_t* row_ptr, const int32_t* col, int32_t n,
                                 int64_t nnz, int32_t* halo_count, int32_t* halo_idx,
                                 uint16_t* lcol, int32_t* max_halo_out, void* workspace,
                                 size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0 && row_ptr && halo_count && halo_idx && max_halo_out,
                "build_tiles: bad arguments");
  LABFM_REQUIRE(nnz >= 0 && (nnz == 0 || (col && lcol)), "build_tiles: bad CSR arguments");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_tiles_workspace_bytes(), "build_tiles");
  hipStream_t st = as_stream(stream_);
  const int ntiles = labfm_tile_count(n);
  int* d = static_cast<int*>(workspace);
  hipError_t e = hipMemsetAsync(d, 0, 2 * sizeof(int), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(build_tiles_kernel, dim3(ntiles), dim3(kThreads), 0, st, row_ptr, col, n,
                       halo_count, halo_idx, lcol, d, d + 1);
    e = hipGetLastError();
  }
  int h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  LABFM_HIP(e);
  *max_halo_out = h[0];
  if (h[1]) {
    set_error("build_tiles: a tile's halo exceeds %d nodes", kHaloMax);
    return LABFM_ERR_CAPACITY;
  }
  return LABFM_OK;
}
