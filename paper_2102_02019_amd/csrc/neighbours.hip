// Stencil search: N_i = { j != i : |r_ji| <= 2 h_i } (stencil definition of
// the paper's LABFM section), as CSR with ascending j per row.
//
// Nodes are binned into a uniform cell grid whose cells are at least
// 2 max(h) wide (cell counts and their scan give each cell's start; a stable
// radix sort of the cell indices lists each cell's nodes in ascending order),
// so every neighbour of a node lies in the 3x3 block of cells around it. A count pass sizes each row, a scan turns counts into row
// offsets, and a fill pass walks the candidate cells as a k-way merge of
// their (ascending) node lists so that each row comes out sorted without a
// separate sort. The distance test rounds every product and sum separately
// (no fused multiply-add), so the lists are reproducible bit for bit by any
// IEEE-754 double implementation of the same test.
#include <algorithm>
#include <climits>
#include <cmath>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "common.hpp"

namespace labfm {
namespace {

struct Grid {
  int ncx, ncy;
  double wx, wy;  // cell widths
  double Lx, Ly;
  int px, py;     // periodic flags
};

__device__ __forceinline__ int cell_coord(double p, double w, int nc) {
  int c = static_cast<int>(floor(p / w));
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Candidate cell coordinates along one axis (at most 3, all distinct).
__device__ __forceinline__ int axis_candidates(int c, int nc, int periodic, int* out) {
  int k = 0;
  if (periodic) {
    if (nc >= 3) {
      out[k++] = (c + nc - 1) % nc;
      out[k++] = c;
      out[k++] = (c + 1) % nc;
    } else {
      for (int a = 0; a < nc; ++a) out[k++] = a;
    }
  } else {
    for (int a = c - 1; a <= c + 1; ++a)
      if (a >= 0 && a < nc) out[k++] = a;
  }
  return k;
}

// |r_ji| <= 2 h_i with separately rounded products and sum (contraction into
// an FMA is switched off here).
__device__ __forceinline__ bool within(double xi, double yi, double xj, double yj, double r2,
                                       const Grid& g) {
#pragma clang fp contract(off)
  const double dx = wrap_axis(xj - xi, g.Lx, g.px);
  const double dy = wrap_axis(yj - yi, g.Ly, g.py);
  const double d2 = dx * dx + dy * dy;
  return d2 <= r2;
}

// max over h ignoring NaN (fmax), from 0
struct FMax {
  __host__ __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct ToI64 {
  __host__ __device__ long long operator()(int v) const { return static_cast<long long>(v); }
};

__global__ void bin_count_kernel(const double* __restrict__ x, const double* __restrict__ y, int n,
                                 Grid g, int* __restrict__ cell_of, int* __restrict__ cell_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_coord(x[i], g.wx, g.ncx);
  const int cy = cell_coord(y[i], g.wy, g.ncy);
  const int c = cy * g.ncx + cx;
  cell_of[i] = c;
  atomicAdd(&cell_count[c], 1);
}

struct Candidates {
  int cells[9];
  int count;
};

__device__ __forceinline__ Candidates candidate_cells(int cell, const Grid& g) {
  int xs[3], ys[3];
  const int cx = cell % g.ncx, cy = cell / g.ncx;
  const int nx = axis_candidates(cx, g.ncx, g.px, xs);
  const int ny = axis_candidates(cy, g.ncy, g.py, ys);
  Candidates c;
  c.count = 0;
  for (int b = 0; b < ny; ++b)
    for (int a = 0; a < nx; ++a) c.cells[c.count++] = ys[b] * g.ncx + xs[a];
  return c;
}

__global__ void count_kernel(const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ h, int n, Grid g,
                             const int* __restrict__ cell_of, const int* __restrict__ cell_start,
                             const int* __restrict__ cell_nodes, int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i];
  const double r = 2.0 * h[i];
  const double r2 = r * r;  // a lone product: rounded once
  const Candidates cand = candidate_cells(cell_of[i], g);
  int cnt = 0;
  for (int c = 0; c < cand.count; ++c) {
    const int b = cell_start[cand.cells[c]], e = cell_start[cand.cells[c] + 1];
    for (int k = b; k < e; ++k) {
      const int j = cell_nodes[k];
      if (j != i && within(xi, yi, x[j], y[j], r2, g)) ++cnt;
    }
  }
  counts[i] = cnt;
}

__global__ void fill_kernel(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ h, int n, Grid g,
                            const int* __restrict__ cell_of, const int* __restrict__ cell_start,
                            const int* __restrict__ cell_nodes, const int* __restrict__ row_ptr,
                            int* __restrict__ col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i];
  const double r = 2.0 * h[i];
  const double r2 = r * r;  // a lone product: rounded once
  const Candidates cand = candidate_cells(cell_of[i], g);
  int cur[9], end[9], head[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    if (c < cand.count) {
      cur[c] = cell_start[cand.cells[c]];
      end[c] = cell_start[cand.cells[c] + 1];
    } else {
      cur[c] = 0;
      end[c] = 0;
    }
    head[c] = (cur[c] < end[c]) ? cell_nodes[cur[c]] : INT_MAX;
  }
  int out = row_ptr[i];
  const int stop = row_ptr[i + 1];
  while (true) {
    // smallest head among the candidate cells (cells are disjoint)
    int best = 0;
#pragma unroll
    for (int c = 1; c < 9; ++c)
      if (head[c] < head[best]) best = c;
    const int j = head[best];
    if (j == INT_MAX) break;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      if (c == best) {
        ++cur[c];
        head[c] = (cur[c] < end[c]) ? cell_nodes[cur[c]] : INT_MAX;
      }
    }
    if (j != i && within(xi, yi, x[j], y[j], r2, g)) {
      if (out < stop) col[out] = j;
      ++out;
    }
  }
}


// Sizes of the search's workspace for n nodes: the cell table has at most
// 4n + 65 entries (see the cell-count cap below), and one temporary storage
// area serves every rocPRIM reduction, scan and sort of the search.
size_t neighbours_temp_bytes(int32_t n) {
  const size_t nscan = 4 * static_cast<size_t>(n) + 65;
  size_t tb_max = 0, tb_sum = 0, tb_scan = 0, tb_sort = 0;
  hipStream_t st{};
  (void)rocprim::reduce(nullptr, tb_max, static_cast<const double*>(nullptr),
                        static_cast<double*>(nullptr), 0.0, static_cast<size_t>(n), FMax(), st);
  (void)rocprim::reduce(nullptr, tb_sum,
                        rocprim::make_transform_iterator(static_cast<const int*>(nullptr), ToI64()),
                        static_cast<long long*>(nullptr), 0LL, static_cast<size_t>(n),
                        rocprim::plus<long long>(), st);
  (void)rocprim::exclusive_scan(nullptr, tb_scan, static_cast<const int*>(nullptr),
                                static_cast<int*>(nullptr), 0, nscan, rocprim::plus<int>(), st);
  for (unsigned b = 1; b <= 31; ++b) {
    size_t t = 0;
    (void)rocprim::radix_sort_pairs(nullptr, t, static_cast<const int*>(nullptr),
                                    static_cast<int*>(nullptr), rocprim::counting_iterator<int>(0),
                                    static_cast<int*>(nullptr), static_cast<size_t>(n), 0u, b, st);
    tb_sort = std::max(tb_sort, t);
  }
  return align256(std::max(std::max(tb_max, tb_sort), std::max(tb_sum, tb_scan)));
}

// the per-node and per-cell integer arrays (cell table at its cap)
size_t neighbours_table_bytes(int32_t n) {
  const size_t ncell_max = 4 * static_cast<size_t>(n) + 64;
  return align256(sizeof(int) * (static_cast<size_t>(n) * 4 + 1 + 2 * (ncell_max + 1)));
}

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" size_t labfm_neighbours_workspace_bytes(int32_t n) {
  if (n <= 0) return 0;
  return 256 + neighbours_temp_bytes(n) + neighbours_table_bytes(n);
}

extern "C" int labfm_build_neighbours(const double* x, const double* y, const double* h,
                                      int32_t n, labfm_box box, int32_t* row_ptr, int32_t* col,
                                      int64_t capacity, int64_t* nnz_out, void* workspace,
                                      size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0, "build_neighbours: n must be positive (got %d)", n);
  LABFM_REQUIRE(x && y && h && row_ptr && nnz_out, "build_neighbours: null pointer argument");
  LABFM_REQUIRE(box.Lx > 0.0 && box.Ly > 0.0, "build_neighbours: box sides must be positive");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_neighbours_workspace_bytes(n),
                  "build_neighbours");
  hipStream_t st = as_stream(stream_);

  // workspace: [0, 256) the two reduction results, then the rocPRIM
  // temporary storage, then the integer tables
  size_t tbytes = neighbours_temp_bytes(n);
  char* base = static_cast<char*>(workspace);
  double* d_hmax = reinterpret_cast<double*>(base);
  long long* d_total = reinterpret_cast<long long*>(base + 16);
  void* d_temp = base + 256;

  LABFM_HIP(rocprim::reduce(d_temp, tbytes, h, d_hmax, 0.0, static_cast<size_t>(n), FMax(), st));
  double hmax = 0.0;
  LABFM_HIP(hipMemcpyAsync(&hmax, d_hmax, sizeof(double), hipMemcpyDeviceToHost, st));
  LABFM_HIP(hipStreamSynchronize(st));
  LABFM_REQUIRE(std::isfinite(hmax) && hmax > 0.0, "build_neighbours: max(h) must be positive");
  if (box.periodic_x)
    LABFM_REQUIRE(4.0 * hmax < box.Lx, "build_neighbours: periodic Lx must exceed 4 max(h)");
  if (box.periodic_y)
    LABFM_REQUIRE(4.0 * hmax < box.Ly, "build_neighbours: periodic Ly must exceed 4 max(h)");

  // Cells strictly wider than the largest stencil diameter.
  const double reach = 2.0 * hmax * (1.0 + 1e-9);
  Grid g;
  g.ncx = static_cast<int>(std::fmax(1.0, std::floor(box.Lx / reach)));
  g.ncy = static_cast<int>(std::fmax(1.0, std::floor(box.Ly / reach)));
  // keep the cell table modest for very small stencils
  while (static_cast<long long>(g.ncx) * g.ncy > 4LL * n + 64) {
    g.ncx = (g.ncx + 1) / 2;
    g.ncy = (g.ncy + 1) / 2;
  }
  g.wx = box.Lx / g.ncx;
  g.wy = box.Ly / g.ncy;
  g.Lx = box.Lx;
  g.Ly = box.Ly;
  g.px = box.periodic_x ? 1 : 0;
  g.py = box.periodic_y ? 1 : 0;
  const int ncell = g.ncx * g.ncy;

  int* cell_of = reinterpret_cast<int*>(base + 256 + tbytes);
  int* cell_nodes = cell_of + n;
  int* counts = cell_nodes + n;              // n + 1 (the last stays 0)
  int* cell_count = counts + n + 1;          // ncell + 1 (the last stays 0)
  int* cell_start = cell_count + ncell + 1;  // ncell + 1
  int* sorted_cell = cell_start + ncell + 1;  // n (the radix sort's keys out)

  const int T = 256;
  LABFM_HIP(hipMemsetAsync(cell_count, 0, sizeof(int) * (ncell + 1), st));
  hipLaunchKernelGGL(bin_count_kernel, dim3(blocks_for(n, T)), dim3(T), 0, st, x, y, n, g,
                     cell_of, cell_count);
  LABFM_LAUNCHED();
  LABFM_HIP(rocprim::exclusive_scan(d_temp, tbytes, cell_count, cell_start, 0,
                                    static_cast<size_t>(ncell) + 1, rocprim::plus<int>(), st));
  // node indices ordered by cell, ascending within a cell (stable sort)
  unsigned end_bit = 1;
  while (end_bit < 31 && (1LL << end_bit) < ncell) ++end_bit;
  LABFM_HIP(rocprim::radix_sort_pairs(d_temp, tbytes, static_cast<const int*>(cell_of), sorted_cell,
                                      rocprim::counting_iterator<int>(0), cell_nodes,
                                      static_cast<size_t>(n), 0u, end_bit, st));
  hipLaunchKernelGGL(count_kernel, dim3(blocks_for(n, T)), dim3(T), 0, st, x, y, h, n, g, cell_of,
                     cell_start, cell_nodes, counts);
  LABFM_LAUNCHED();
  LABFM_HIP(hipMemsetAsync(counts + n, 0, sizeof(int), st));
  // the total in 64 bits (an int32 offset past INT_MAX is reported below)
  LABFM_HIP(rocprim::reduce(d_temp, tbytes, rocprim::make_transform_iterator(
                                static_cast<const int*>(counts), ToI64()),
                            d_total, 0LL, static_cast<size_t>(n), rocprim::plus<long long>(), st));
  LABFM_HIP(rocprim::exclusive_scan(d_temp, tbytes, counts, row_ptr, 0,
                                    static_cast<size_t>(n) + 1, rocprim::plus<int>(), st));
  long long total = 0;
  LABFM_HIP(hipMemcpyAsync(&total, d_total, sizeof(long long), hipMemcpyDeviceToHost, st));
  LABFM_HIP(hipStreamSynchronize(st));
  *nnz_out = total;
  if (total > INT_MAX) {
    set_error("build_neighbours: %lld entries exceed the int32 CSR index range", total);
    return LABFM_ERR_UNSUPPORTED;
  }
  if (col == nullptr || capacity < total) {
    set_error("build_neighbours: col capacity %lld < nnz %lld", (long long)capacity, total);
    return LABFM_ERR_CAPACITY;
  }
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n, T)), dim3(T), 0, st, x, y, h, n, g, cell_of,
                     cell_start, cell_nodes, row_ptr, col);
  LABFM_LAUNCHED();
  return LABFM_OK;
}
