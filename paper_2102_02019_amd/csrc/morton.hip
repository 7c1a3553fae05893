// Morton (Z-order) permutation of a node set: the binning that gives the
// stencil search and the gather kernels their locality (nodes close in space
// close in memory). Each node's cell (ix, iy) = (floor(x / cell),
// floor(y / cell)), clamped to the grid, gets the key with x's bits in the
// even and y's bits in the odd positions; a stable radix sort of the keys
// (rocPRIM) carries the node indices along.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <rocprim/device/device_radix_sort.hpp>

#include "common.hpp"

namespace labfm {
namespace {

// the bits of a (< 2^21) moved to the even positions of a 64-bit word
__device__ __forceinline__ unsigned long long spread_bits(unsigned long long a) {
  a &= 0x00000000FFFFFFFFull;
  a = (a | (a << 16)) & 0x0000FFFF0000FFFFull;
  a = (a | (a << 8)) & 0x00FF00FF00FF00FFull;
  a = (a | (a << 4)) & 0x0F0F0F0F0F0F0F0Full;
  a = (a | (a << 2)) & 0x3333333333333333ull;
  a = (a | (a << 1)) & 0x5555555555555555ull;
  return a;
}

// clamped before the conversion (a NaN position goes to cell 0)
__device__ __forceinline__ long long cell_of(double p, double cell, long long nc) {
  const double f = floor(p / cell);
  if (!(f >= 0.0)) return 0;
  if (f >= static_cast<double>(nc)) return nc - 1;
  return static_cast<long long>(f);
}

__global__ void morton_key_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                  int n, double cell, long long ncx, long long ncy,
                                  unsigned long long* __restrict__ key, int* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long ix = static_cast<unsigned long long>(cell_of(x[i], cell, ncx));
  const unsigned long long iy = static_cast<unsigned long long>(cell_of(y[i], cell, ncy));
  key[i] = spread_bits(ix) | (spread_bits(iy) << 1);
  idx[i] = i;
}

}  // namespace
}  // namespace labfm

using namespace labfm;

namespace {

// Bytes of rocPRIM's radix sort of n (64-bit key, int) pairs over bits
// [0, end_bit).
size_t morton_sort_bytes(int32_t n, unsigned end_bit) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, static_cast<unsigned long long*>(nullptr),
                                  static_cast<unsigned long long*>(nullptr),
                                  static_cast<int*>(nullptr), static_cast<int*>(nullptr),
                                  static_cast<size_t>(n), 0u, end_bit, hipStream_t{});
  return bytes;
}

// Workspace layout: keys in, keys out (n each), node indices (n), then the
// sort's storage (sized for the widest key, 42 bits).
size_t morton_keys_bytes(int32_t n) {
  return align256((2 * sizeof(unsigned long long) + sizeof(int)) * static_cast<size_t>(n));
}

}  // namespace

extern "C" size_t labfm_morton_workspace_bytes(int32_t n) {
  if (n <= 0) return 0;
  size_t sort = 0;
  for (unsigned b = 1; b <= 42; ++b) sort = std::max(sort, morton_sort_bytes(n, b));
  return morton_keys_bytes(n) + align256(std::max<size_t>(sort, 1));
}

extern "C" int labfm_morton_order(const double* x, const double* y, int32_t n, labfm_box box,
                                  double cell, int32_t* perm, void* workspace,
                                  size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0 && x && y && perm, "morton_order: null or empty argument");
  LABFM_REQUIRE(cell > 0.0 && std::isfinite(cell), "morton_order: cell must be positive");
  LABFM_REQUIRE(box.Lx > 0.0 && box.Ly > 0.0, "morton_order: box sides must be positive");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_morton_workspace_bytes(n), "morton_order");
  const double fx = std::ceil(box.Lx / cell), fy = std::ceil(box.Ly / cell);
  LABFM_REQUIRE(fx <= 2097152.0 && fy <= 2097152.0,
                "morton_order: at most 2^21 cells per axis (cell too small for the box)");
  const long long ncx = std::max(1LL, static_cast<long long>(fx));
  const long long ncy = std::max(1LL, static_cast<long long>(fy));
  int bits = 0;
  while ((1LL << bits) < std::max(ncx, ncy)) ++bits;
  const unsigned end_bit = static_cast<unsigned>(std::max(2 * bits, 1));
  hipStream_t st = as_stream(stream_);

  const size_t nn = static_cast<size_t>(n);
  unsigned long long* k_in = static_cast<unsigned long long*>(workspace);
  unsigned long long* k_out = k_in + nn;
  int* idx = reinterpret_cast<int*>(k_out + nn);
  void* sort_tmp = static_cast<char*>(workspace) + morton_keys_bytes(n);
  size_t bytes = workspace_bytes - morton_keys_bytes(n);
  hipLaunchKernelGGL(morton_key_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, y, n, cell,
                     ncx, ncy, k_in, idx);
  LABFM_LAUNCHED();
  LABFM_HIP(rocprim::radix_sort_pairs(sort_tmp, bytes, k_in, k_out, idx,
                                      reinterpret_cast<int*>(perm), n, 0u, end_bit, st));
  LABFM_HIP(hipStreamSynchronize(st));
  return LABFM_OK;
}
