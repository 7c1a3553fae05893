// Boundary operators of LABFM (section "Boundaries", table tab:boundaries,
// Appendix A): finite differences along the 5-node orthogonal strip columns
// for the wall-normal derivative, one-dimensional LABFM along the strip rows
// for the tangential derivative, rotated into d/dx, d/dy; at wall nodes a
// tangential filter operator and its calibration.
//
// One 64-lane wavefront per (column, level) item, levels 0..2. The lanes walk
// the node's CSR row twice: first to accumulate the 4 x 4 one-dimensional
// moment matrix (then summed across the wave and solved redundantly by every
// lane, partial pivoting), then to write the weights of every entry of the
// row, so the row's x and y weights are replaced as a whole.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.hpp"

namespace labfm {
namespace {

constexpr int kDepth = LABFM_STRIP_DEPTH;
constexpr int kTan = 4;                  // order of the 1D LABFM along the rows
constexpr double kSameWall = 0.5;        // cos 60 degrees
constexpr int kWaves = 4;                // wavefronts per 256-thread workgroup

// 5-point first-difference coefficients (times 12 s) of the nodes i0..i4 of a
// column, for the node at level q: one-sided, asymmetric and centred.
__constant__ double kFirstDiff[3][kDepth] = {
    {-25.0, 48.0, -36.0, 16.0, -3.0},
    {-3.0, -10.0, 18.0, -6.0, 1.0},
    {1.0, -8.0, 0.0, 8.0, -1.0},
};

__device__ __forceinline__ double psi_wendland(double q) {
  if (q >= 2.0) return 0.0;
  const double t = 1.0 - 0.5 * q;
  return (t * t) * (t * t) * (1.0 + 2.0 * q);
}

// ABF values W^k = psi(|z|) He_k(z), k = 1..4 (probabilists' Hermite).
__device__ __forceinline__ void abf_1d(double z, double W[kTan]) {
  const double p = psi_wendland(fabs(z));
  double hm = 1.0, hk = z;  // He_0, He_1
  W[0] = p * hk;
#pragma unroll
  for (int k = 1; k < kTan; ++k) {
    const double hn = z * hk - k * hm;  // He_{k+1}
    hm = hk;
    hk = hn;
    W[k] = p * hk;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void strip_map_kernel(const int* __restrict__ column, const double* __restrict__ normal,
                                 int count, signed char* __restrict__ level,
                                 int* __restrict__ colidx, double* __restrict__ wall_normal) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
#pragma unroll
  for (int q = 0; q < kDepth; ++q) {
    const int i = column[kDepth * k + q];
    level[i] = static_cast<signed char>(q);
    colidx[i] = k;
  }
  const int i0 = column[kDepth * k];
  wall_normal[2 * static_cast<long long>(i0)] = normal[2 * k];
  wall_normal[2 * static_cast<long long>(i0) + 1] = normal[2 * k + 1];
}

struct BoundaryArgs {
  const double *x, *y, *h, *s;
  int n;
  double Lx, Ly;
  int px, py;
  const int *row_ptr, *col;
  long long nnz;
  const int* column;
  const double* normal;
  int count;
  const signed char* level;
  const int* colidx;
  double* w;
  float* w32;
  float* mom32;
  double* kappa;
  signed char* status;
};

__global__ void __launch_bounds__(64 * kWaves) boundary_weights_kernel(BoundaryArgs a) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (item >= 3 * a.count) return;  // whole waves leave together
  const int k = item / 3;
  const int q = item - 3 * k;
  const int i = a.column[kDepth * k + q];
  const double nx = a.normal[2 * k], ny = a.normal[2 * k + 1];
  const double tx = -ny, ty = nx;
  const double hi = a.h[i];
  const double xi0 = a.x[i], yi0 = a.y[i];
  const int e0 = a.row_ptr[i], e1 = a.row_ptr[i + 1];

  // 1. moment matrix M[r][c] = sum_j (z^(r+1)/(r+1)!) W^(c+1)(z) over B_i
  double M[kTan][kTan];
#pragma unroll
  for (int r = 0; r < kTan; ++r)
#pragma unroll
    for (int c = 0; c < kTan; ++c) M[r][c] = 0.0;
  for (int e = e0 + lane; e < e1; e += 64) {
    const int j = a.col[e];
    if (a.level[j] != q) continue;
    const int kj = a.colidx[j];
    if (a.normal[2 * kj] * nx + a.normal[2 * kj + 1] * ny <= kSameWall) continue;
    const double dx = wrap_axis(a.x[j] - xi0, a.Lx, a.px);
    const double dy = wrap_axis(a.y[j] - yi0, a.Ly, a.py);
    const double z = (dx * tx + dy * ty) / hi;
    double W[kTan];
    abf_1d(z, W);
    double mono = 1.0;
#pragma unroll
    for (int r = 0; r < kTan; ++r) {
      mono = mono * z / (r + 1);
#pragma unroll
      for (int c = 0; c < kTan; ++c) M[r][c] += mono * W[c];
    }
  }
#pragma unroll
  for (int r = 0; r < kTan; ++r)
#pragma unroll
    for (int c = 0; c < kTan; ++c) M[r][c] = wave_sum(M[r][c]);

  // 2. M Psi = C for C = h^-1 e_1 and (wall nodes) h^-4 e_4; every lane
  // eliminates the same 4 x 4 system with partial pivoting
  double R[kTan][2];
#pragma unroll
  for (int r = 0; r < kTan; ++r) {
    R[r][0] = (r == 0) ? 1.0 / hi : 0.0;
    R[r][1] = (r == kTan - 1) ? 1.0 / (hi * hi * hi * hi) : 0.0;
  }
  bool singular = false;
#pragma unroll
  for (int p = 0; p < kTan; ++p) {
    int piv = p;
    double big = fabs(M[p][p]);
#pragma unroll
    for (int r = p + 1; r < kTan; ++r) {
      if (fabs(M[r][p]) > big) {
        big = fabs(M[r][p]);
        piv = r;
      }
    }
    if (!(big > 0.0)) singular = true;
#pragma unroll
    for (int r = p + 1; r < kTan; ++r) {
      if (r == piv) {
#pragma unroll
        for (int c = 0; c < kTan; ++c) {
          const double t = M[p][c];
          M[p][c] = M[r][c];
          M[r][c] = t;
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double t = R[p][c];
          R[p][c] = R[r][c];
          R[r][c] = t;
        }
      }
    }
    const double inv = 1.0 / M[p][p];
#pragma unroll
    for (int r = p + 1; r < kTan; ++r) {
      const double f = M[r][p] * inv;
#pragma unroll
      for (int c = p; c < kTan; ++c) M[r][c] -= f * M[p][c];
      R[r][0] -= f * R[p][0];
      R[r][1] -= f * R[p][1];
    }
  }
  double P1[kTan], P4[kTan];
#pragma unroll
  for (int r = kTan - 1; r >= 0; --r) {
    double s1 = R[r][0], s4 = R[r][1];
#pragma unroll
    for (int c = r + 1; c < kTan; ++c) {
      s1 -= M[r][c] * P1[c];
      s4 -= M[r][c] * P4[c];
    }
    P1[r] = s1 / M[r][r];
    P4[r] = s4 / M[r][r];
  }

  // 3. the column's nodes: all four others must be in the stencil
  int hits = 0;
  for (int e = e0 + lane; e < e1; e += 64) {
    const int j = a.col[e];
#pragma unroll
    for (int kk = 0; kk < kDepth; ++kk)
      if (kk != q && j == a.column[kDepth * k + kk]) ++hits;
  }
  hits = wave_sum_int(hits);
  const bool ok = !singular && hits == kDepth - 1;

  // 4. weights of every entry of the row
  const double inv12s = 1.0 / (12.0 * a.s[a.column[kDepth * k]]);
  const double kf = 2.0 * M_PI / (3.0 * a.s[i]);
  double f0 = 0.0;
  for (int e = e0 + lane; e < e1; e += 64) {
    const int j = a.col[e];
    double wxi = 0.0;
#pragma unroll
    for (int kk = 0; kk < kDepth; ++kk)
      if (kk != q && j == a.column[kDepth * k + kk]) wxi = kFirstDiff[q][kk] * inv12s;
    const double dx = wrap_axis(a.x[j] - xi0, a.Lx, a.px);
    const double dy = wrap_axis(a.y[j] - yi0, a.Ly, a.py);
    double weta = 0.0, whyp = 0.0;
    if (a.level[j] == q) {
      const int kj = a.colidx[j];
      if (a.normal[2 * kj] * nx + a.normal[2 * kj + 1] * ny > kSameWall) {
        double W[kTan];
        abf_1d((dx * tx + dy * ty) / hi, W);
#pragma unroll
        for (int c = 0; c < kTan; ++c) {
          weta += W[c] * P1[c];
          whyp += W[c] * P4[c];
        }
      }
    }
    double wx = nx * wxi + tx * weta;
    double wy = ny * wxi + ty * weta;
    if (!ok) {
      wx = 0.0;
      wy = 0.0;
      whyp = 0.0;
    }
    a.w[LABFM_OP_X * a.nnz + e] = wx;
    a.w[LABFM_OP_Y * a.nnz + e] = wy;
    if (a.w32) {
      a.w32[LABFM_OP_X * w32_stride(a.nnz) + e] = static_cast<float>(wx);
      a.w32[LABFM_OP_Y * w32_stride(a.nnz) + e] = static_cast<float>(wy);
    }
    if (q == 0) {
      a.w[LABFM_OP_L * a.nnz + e] = 0.0;
      a.w[LABFM_OP_XX * a.nnz + e] = 0.0;
      a.w[LABFM_OP_XY * a.nnz + e] = 0.0;
      a.w[LABFM_OP_HYP * a.nnz + e] = whyp;
      if (a.w32) {
        a.w32[LABFM_OP_L * w32_stride(a.nnz) + e] = 0.0f;
        a.w32[LABFM_OP_XX * w32_stride(a.nnz) + e] = 0.0f;
        a.w32[LABFM_OP_XY * w32_stride(a.nnz) + e] = 0.0f;
        a.w32[LABFM_OP_HYP * w32_stride(a.nnz) + e] = static_cast<float>(whyp);
      }
      f0 += (1.0 - cos(kf * dx) * cos(kf * dy)) * whyp;
    }
  }
  f0 = wave_sum(f0);
  if (lane != 0) return;
  signed char st = a.status[i];
  if (singular) {
    st = LABFM_NODE_SINGULAR;
  } else if (hits != kDepth - 1) {
    st = LABFM_NODE_FEW_NEIGHBOURS;
  } else if (q == 0) {
    st = LABFM_NODE_OK;
  }
  if (q == 0) {
    double kap = 0.0;
    if (ok && std::isfinite(f0) && f0 != 0.0) {
      kap = 2.0 / (3.0 * f0);
    } else if (ok) {
      st = LABFM_NODE_BAD_FILTER;
    }
    a.kappa[i] = kap;
    if (a.mom32) {
      // the second-derivative operators of a wall node are zero
#pragma unroll
      for (int r = 0; r < kMoments; ++r) a.mom32[static_cast<long long>(r) * a.n + i] = 0.0f;
    }
  }
  a.status[i] = st;
}

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" size_t labfm_boundary_workspace_bytes(int32_t n) {
  return n > 0 ? align256((sizeof(int) + 1) * static_cast<size_t>(n) + 16) : 0;
}

extern "C" int labfm_boundary_weights(const double* x, const double* y, const double* h,
                                      const double* s, int32_t n, labfm_box box,
                                      const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                                      const labfm_strips* strips, double* w, float* w32,
                                      float* mom32, double* kappa, int8_t* status,
                                      double* wall_normal, void* workspace,
                                      size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0 && x && y && h && s && row_ptr && (col || nnz == 0) && strips && w &&
                    kappa && status && wall_normal,
                "boundary_weights: null or empty argument");
  LABFM_REQUIRE(strips->count >= 0, "boundary_weights: negative column count");
  LABFM_REQUIRE(strips->count == 0 || (strips->column && strips->normal),
                "boundary_weights: null column or normal array");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_boundary_workspace_bytes(n),
                  "boundary_weights");
  hipStream_t st = as_stream(stream_);
  const int count = strips->count;

  // host check of the columns: indices in range, no node twice, unit normals
  std::vector<int32_t> hcol(static_cast<size_t>(kDepth) * count);
  std::vector<double> hnrm(2 * static_cast<size_t>(count));
  if (count > 0) {
    LABFM_HIP(hipMemcpyAsync(hcol.data(), strips->column, sizeof(int32_t) * hcol.size(),
                             hipMemcpyDeviceToHost, st));
    LABFM_HIP(hipMemcpyAsync(hnrm.data(), strips->normal, sizeof(double) * hnrm.size(),
                             hipMemcpyDeviceToHost, st));
    LABFM_HIP(hipStreamSynchronize(st));
  }
  std::vector<char> seen(static_cast<size_t>(n), 0);
  for (size_t t = 0; t < hcol.size(); ++t) {
    const int32_t i = hcol[t];
    LABFM_REQUIRE(i >= 0 && i < n, "boundary_weights: column node %d outside 0..%d", i, n - 1);
    LABFM_REQUIRE(!seen[i], "boundary_weights: node %d appears in two columns", i);
    seen[i] = 1;
  }
  for (int k = 0; k < count; ++k) {
    const double len = std::hypot(hnrm[2 * k], hnrm[2 * k + 1]);
    LABFM_REQUIRE(std::fabs(len - 1.0) < 1e-12, "boundary_weights: normal %d is not unit", k);
  }

  int* colidx = static_cast<int*>(workspace);
  signed char* level = reinterpret_cast<signed char*>(colidx + n);
  LABFM_HIP(hipMemsetAsync(level, 0xFF, static_cast<size_t>(n), st));  // -1: off the strips
  LABFM_HIP(hipMemsetAsync(colidx, 0, sizeof(int) * static_cast<size_t>(n), st));
  LABFM_HIP(hipMemsetAsync(wall_normal, 0, 2 * sizeof(double) * static_cast<size_t>(n), st));
  if (count == 0) return LABFM_OK;
  hipLaunchKernelGGL(strip_map_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st,
                     strips->column, strips->normal, count, level, colidx, wall_normal);
  LABFM_LAUNCHED();

  BoundaryArgs a;
  a.x = x;
  a.y = y;
  a.h = h;
  a.s = s;
  a.n = n;
  a.Lx = box.Lx;
  a.Ly = box.Ly;
  a.px = box.periodic_x ? 1 : 0;
  a.py = box.periodic_y ? 1 : 0;
  a.row_ptr = row_ptr;
  a.col = col;
  a.nnz = nnz;
  a.column = strips->column;
  a.normal = strips->normal;
  a.count = count;
  a.level = level;
  a.colidx = colidx;
  a.w = w;
  a.w32 = w32;
  a.mom32 = mom32;
  a.kappa = kappa;
  a.status = reinterpret_cast<signed char*>(status);
  const long long items = 3LL * count;
  hipLaunchKernelGGL(boundary_weights_kernel, dim3(blocks_for(items, kWaves)), dim3(64 * kWaves),
                     0, st, a);
  LABFM_LAUNCHED();
  return LABFM_OK;
}
