// LABFM in a Lagrangian frame (section "Conclusions": node positions advanced
// by the same time integration as the flow). Every Runge-Kutta stage builds
// the stencils and weights at its own positions (labfm_build_neighbours,
// labfm_build_weights) and then runs one gather kernel that evaluates the
// material rates of eq. icns (no u . grad terms) and advances positions and
// fields in the two-register form. After each step the filter uses weights
// at the new positions, which also serve the next step's first stage.
//
// Registers (x, y, ln rho, u, v): the caller's state Q and three workspace
// registers, rotated so that no launch writes what it gathers and Q keeps
// the last completed step until the filter writes the new one:
//   stage 1: gather Q,  q in Q  -> q to Ya, Y to Yb
//   stage 2: gather Yb, q in Ya -> q to Ya, Y to Yc
//   stage 3: gather Yc, q in Ya -> q to Ya, Y to Yb
//   stage 4: gather Yb, q in Ya -> q to Ya
//   filter:  weights at Ya's positions; Ya -> Q
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "gather.hpp"

namespace labfm {
namespace {

constexpr int kStatusKinds = 5;  // LABFM_NODE_OK .. LABFM_NODE_BAD_ORDER

struct Reg {
  double* x;
  double* y;
  double* f;  // [ln rho | u | v], 3n
};

__device__ __forceinline__ double fold(double p, double L) {
  if (p >= L) return p - L;
  if (p < 0.0) return p + L;
  return p;
}

// One RK stage of the extended system. Y is gathered; qin/qout may be the
// same register (each node reads its own entries before writing them).
template <int LPN>
__global__ void __launch_bounds__(256)
lagr_stage_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col,
                  const double* __restrict__ w, long long nnz, Reg Y, Reg qin, Reg qout,
                  Reg Yout, double dta, double dtb, Flow fl, double Lx, double Ly, int n) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;  // whole LPN groups leave together
  const long long n2 = 2 * static_cast<long long>(n);
  const double* Yl = Y.f;
  const double* Yu = Y.f + n;
  const double* Yv = Y.f + n2;
  const double li = Yl[node], ui = Yu[node], vi = Yv[node];
  double s[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = 0.0;
  const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
  for (int e = e0 + sub; e < e1; e += LPN) {
    const int j = col[e];
    const double a = w[e], b = w[nnz + e], c = w[2 * nnz + e], d = w[3 * nnz + e],
                 f = w[4 * nnz + e];
    const double dl = Yl[j] - li, du = Yu[j] - ui, dv = Yv[j] - vi;
    s[0] += a * dl;
    s[1] += b * dl;
    s[2] += a * du;
    s[3] += b * du;
    s[4] += c * du;
    s[5] += d * du;
    s[6] += f * du;
    s[7] += a * dv;
    s[8] += b * dv;
    s[9] += c * dv;
    s[10] += d * dv;
    s[11] += f * dv;
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = group_sum<LPN>(s[k]);
  if (sub != 0) return;
  const double Lxs = s[0], Lys = s[1], Ux = s[2], Uy = s[3], UL = s[4], Uxx = s[5], Uxy = s[6];
  const double Vx = s[7], Vy = s[8], VL = s[9], Vxx = s[10], Vxy = s[11];
  const double nu = fl.mu / exp(li);
  const double third = 1.0 / 3.0;
  // material rates: eq. icns without the convective terms; dr/dt = u
  const double rl = -(Ux + Vy);
  const double ru = -fl.c2 * Lxs + nu * (UL + third * (Uxx + Vxy)) + fl.gx;
  const double rv = -fl.c2 * Lys + nu * (VL + third * ((VL - Vxx) + Uxy)) + fl.gy;
  const double r[5] = {ui, vi, rl, ru, rv};
  const double q[5] = {qin.x[node], qin.y[node], qin.f[node], qin.f[n + node],
                       qin.f[n2 + node]};
  if (Yout.x) {
    Yout.x[node] = fold(q[0] + dta * r[0], Lx);
    Yout.y[node] = fold(q[1] + dta * r[1], Ly);
    Yout.f[node] = q[2] + dta * r[2];
    Yout.f[n + node] = q[3] + dta * r[3];
    Yout.f[n2 + node] = q[4] + dta * r[4];
  }
  qout.x[node] = fold(q[0] + dtb * r[0], Lx);
  qout.y[node] = fold(q[1] + dtb * r[1], Ly);
  qout.f[node] = q[2] + dtb * r[2];
  qout.f[n + node] = q[3] + dtb * r[3];
  qout.f[n2 + node] = q[4] + dtb * r[4];
}

hipError_t launch_lagr_stage(int lpn, const int* row_ptr, const int* col, const double* w,
                             long long nnz, const Reg& Y, const Reg& qin, const Reg& qout,
                             const Reg& Yout, double dta, double dtb, const Flow& fl, double Lx,
                             double Ly, int n, hipStream_t st) {
  const unsigned grid = blocks_for(static_cast<long long>(n) * lpn, 256);
  switch (lpn) {
    case 4:
      hipLaunchKernelGGL(lagr_stage_kernel<4>, dim3(grid), dim3(256), 0, st, row_ptr, col, w, nnz,
                         Y, qin, qout, Yout, dta, dtb, fl, Lx, Ly, n);
      break;
    case 8:
      hipLaunchKernelGGL(lagr_stage_kernel<8>, dim3(grid), dim3(256), 0, st, row_ptr, col, w, nnz,
                         Y, qin, qout, Yout, dta, dtb, fl, Lx, Ly, n);
      break;
    default:
      hipLaunchKernelGGL(lagr_stage_kernel<16>, dim3(grid), dim3(256), 0, st, row_ptr, col, w,
                         nnz, Y, qin, qout, Yout, dta, dtb, fl, Lx, Ly, n);
      break;
  }
  return hipGetLastError();
}

// Adds the per-node statuses of one build to counts[LABFM_NODE_*] (statuses
// outside 0..4 are not written by the build).
__global__ void __launch_bounds__(256)
count_status_kernel(const int8_t* __restrict__ status, int n, unsigned long long* counts) {
  __shared__ unsigned int c[kStatusKinds];
  if (threadIdx.x < kStatusKinds) c[threadIdx.x] = 0u;
  __syncthreads();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = status[i];
    if (v >= 0 && v < kStatusKinds) atomicAdd(&c[v], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kStatusKinds && c[threadIdx.x] != 0u)
    atomicAdd(&counts[threadIdx.x], static_cast<unsigned long long>(c[threadIdx.x]));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t reg, rowptr, col, w, kappa, status, counts, setup, total;
};

Layout layout_of(int32_t n, int64_t cap) {
  Layout L;
  L.reg = align_up(sizeof(double) * 5 * static_cast<size_t>(n));
  L.rowptr = align_up(sizeof(int32_t) * (static_cast<size_t>(n) + 1));
  L.col = align_up(sizeof(int32_t) * static_cast<size_t>(cap));
  L.w = align_up(sizeof(double) * 6 * static_cast<size_t>(cap));
  L.kappa = align_up(sizeof(double) * static_cast<size_t>(n));
  L.status = align_up(static_cast<size_t>(n));
  L.counts = align_up(sizeof(unsigned long long) * kStatusKinds);
  // the stencil search's and the weight build's workspaces (one after the
  // other on the stream, so they share one area)
  L.setup = align_up(std::max(labfm_neighbours_workspace_bytes(n), labfm_build_workspace_bytes(n)));
  L.total = 3 * L.reg + L.rowptr + L.col + L.w + L.kappa + L.status + L.counts + L.setup;
  return L;
}

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" size_t labfm_lagrangian_workspace_bytes(int32_t n, int64_t nnz_capacity) {
  if (n <= 0 || nnz_capacity < 0) return 0;
  return layout_of(n, nnz_capacity).total;
}

extern "C" int labfm_lagrangian_step(double* x, double* y, double* q, const double* h,
                                     const double* s, const int8_t* order_m, int32_t n,
                                     labfm_box box, const labfm_rk_params* prm, int32_t n_steps,
                                     int64_t nnz_capacity, void* workspace,
                                     size_t workspace_bytes, labfm_lagrangian_stats* stats,
                                     void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0 && x && y && q && h && s && order_m && prm && workspace,
                "lagrangian_step: null or empty argument");
  LABFM_REQUIRE(n_steps >= 0 && nnz_capacity > 0, "lagrangian_step: bad step count or capacity");
  LABFM_REQUIRE(prm->dt > 0.0 && prm->c2 > 0.0 && prm->mu >= 0.0,
                "lagrangian_step: dt and c2 must be positive, mu non-negative");
  if (!box.periodic_x || !box.periodic_y) {
    set_error("lagrangian_step: moving nodes need a periodic box on both axes");
    return LABFM_ERR_UNSUPPORTED;
  }
  const Layout L = layout_of(n, nnz_capacity);
  LABFM_REQUIRE(workspace_bytes >= L.total, "lagrangian_step: workspace of %zu bytes required",
                L.total);
  hipStream_t st = as_stream(stream_);
  char* base = static_cast<char*>(workspace);
  auto reg_at = [&](size_t off) {
    double* p = reinterpret_cast<double*>(base + off);
    return Reg{p, p + n, p + 2 * static_cast<size_t>(n)};
  };
  const Reg Q{x, y, q};
  const Reg Ya = reg_at(0), Yb = reg_at(L.reg), Yc = reg_at(2 * L.reg);
  size_t off = 3 * L.reg;
  int32_t* row_ptr = reinterpret_cast<int32_t*>(base + off);
  off += L.rowptr;
  int32_t* col = reinterpret_cast<int32_t*>(base + off);
  off += L.col;
  double* w = reinterpret_cast<double*>(base + off);
  off += L.w;
  double* kappa = reinterpret_cast<double*>(base + off);
  off += L.kappa;
  int8_t* status = reinterpret_cast<int8_t*>(base + off);
  off += L.status;
  unsigned long long* counts = reinterpret_cast<unsigned long long*>(base + off);
  off += L.counts;
  void* setup_ws = base + off;
  LABFM_HIP(hipMemsetAsync(counts, 0, sizeof(unsigned long long) * kStatusKinds, st));
  const unsigned count_grid =
      static_cast<unsigned>(std::min<long long>(1024, (static_cast<long long>(n) + 255) / 256));

  labfm_lagrangian_stats local{};
  labfm_lagrangian_stats& sx = stats ? *stats : local;
  sx = labfm_lagrangian_stats{};
  long long nnz = 0;
  // stencils and weights at the positions of register R
  auto build = [&](const Reg& R) -> int {
    const auto t0 = std::chrono::steady_clock::now();
    int64_t got = 0;
    int r = labfm_build_neighbours(R.x, R.y, h, n, box, row_ptr, col, nnz_capacity, &got,
                                   setup_ws, L.setup, stream_);
    if (r == LABFM_ERR_CAPACITY) {
      set_error("lagrangian_step: %lld stencil entries exceed the capacity %lld",
                static_cast<long long>(got), static_cast<long long>(nnz_capacity));
      return r;
    }
    if (r != LABFM_OK) return r;
    nnz = got;
    r = labfm_build_weights(R.x, R.y, h, s, order_m, n, box, row_ptr, col, nnz, 0x3F, w,
                            nullptr, nullptr, kappa, nullptr, status, setup_ws, L.setup,
                            stream_);
    if (r != LABFM_OK) return r;
    hipLaunchKernelGGL(count_status_kernel, dim3(count_grid), dim3(256), 0, st, status, n,
                       counts);
    if (hipGetLastError() != hipSuccess) {
      set_error("lagrangian_step: status count launch failed");
      return LABFM_ERR_HIP;
    }
    // the build's kernels run asynchronously after its sizing step; wait
    // for them so that build_ms covers them
    LABFM_HIP(hipStreamSynchronize(st));
    const auto t1 = std::chrono::steady_clock::now();
    sx.builds += 1;
    sx.build_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (got > sx.max_nnz) sx.max_nnz = got;
    return LABFM_OK;
  };
  // node builds per status, summed over the call's builds, into the stats
  auto read_counts = [&]() -> hipError_t {
    unsigned long long hc[kStatusKinds];
    const hipError_t e = hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) return e2;
    for (int k = 0; k < kStatusKinds; ++k) sx.node_status[k] = static_cast<int64_t>(hc[k]);
    return hipSuccess;
  };
  hipEvent_t ev[2];
  LABFM_HIP(hipEventCreate(&ev[0]));
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    set_error("lagrangian_step: hipEventCreate failed");
    return LABFM_ERR_HIP;
  }
  struct Events {
    hipEvent_t* e;
    ~Events() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  // times the kernels enqueued by fn (the next build's synchronisation, or
  // the final one, completes them)
  auto timed = [&](auto fn) -> hipError_t {
    hipError_t e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    sx.stage_ms += ms;
    return e;
  };

  const Flow fl{prm->c2, prm->mu, prm->gx, prm->gy};
  const double dt = prm->dt;
  const Reg none{nullptr, nullptr, nullptr};
  const Reg G[4] = {Q, Yb, Yc, Yb};
  const Reg Qin[4] = {Q, Ya, Ya, Ya};
  const Reg Yo[4] = {Yb, Yc, Yb, none};
  const size_t field_bytes = sizeof(double) * static_cast<size_t>(n);
  // the steps; every early exit (a capacity error) still reports the
  // statuses of the builds done so far
  auto advance = [&]() -> int {
    if (n_steps > 0) {
      if (int r = build(Q)) return r;
    }
    for (int step = 0; step < n_steps; ++step) {
      for (int k = 0; k < 4; ++k) {
        if (k > 0) {
          if (int r = build(G[k])) return r;
        }
        const double K = static_cast<double>(nnz) / n;
        const int lpn = K > 48.0 ? 16 : (K > 12.0 ? 8 : 4);
        const double dta = (k < 3) ? dt * kA[k] : 0.0;
        LABFM_HIP(timed([&] {
          return launch_lagr_stage(lpn, row_ptr, col, w, nnz, G[k], Qin[k], Ya, Yo[k], dta,
                                   dt * kB[k], fl, box.Lx, box.Ly, n, st);
        }));
      }
      // weights at the new positions: the filter's, and the next first stage's
      if (int r = build(Ya)) return r;
      LABFM_HIP(hipMemcpyAsync(Q.x, Ya.x, field_bytes, hipMemcpyDeviceToDevice, st));
      LABFM_HIP(hipMemcpyAsync(Q.y, Ya.y, field_bytes, hipMemcpyDeviceToDevice, st));
      if (prm->filter) {
        labfm_operators ops{};
        ops.n = n;
        ops.nnz = nnz;
        ops.row_ptr = row_ptr;
        ops.col = col;
        ops.w = w;
        ops.kappa = kappa;
        const LaunchCfg fc = cfg_for(LABFM_KERNEL_FILTER, LABFM_F64, n, nnz);
        LABFM_HIP(timed([&] { return launch_filter<F64>(fc, &ops, w, Ya.f, Q.f, st); }));
      } else {
        LABFM_HIP(hipMemcpyAsync(Q.f, Ya.f, 3 * field_bytes, hipMemcpyDeviceToDevice, st));
      }
      sx.steps_done = step + 1;
    }
    return LABFM_OK;
  };
  const int adv = advance();
  const hipError_t cerr = read_counts();
  if (adv != LABFM_OK) return adv;
  LABFM_HIP(cerr);
  if (n_steps > 0 && prm->check_finite) {
    std::vector<double> hq(3 * static_cast<size_t>(n));
    LABFM_HIP(hipMemcpy(hq.data(), q, 3 * field_bytes, hipMemcpyDeviceToHost));
    for (double v : hq) {
      if (!std::isfinite(v)) {
        set_error("lagrangian_step: non-finite state");
        return LABFM_ERR_NONFINITE;
      }
    }
  }
  return LABFM_OK;
}
