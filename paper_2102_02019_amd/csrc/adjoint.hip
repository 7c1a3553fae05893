// Reverse mode (adjoint) of the filtered RK3(2)4[2R+]C time loop of the
// isothermal Navier-Stokes equations, float64.
//
// With A_d = [w^d_ij] - diag(S^d_i) (S^d_i = sum_j w^d_ij) every operator is
// L^d = A_d, so its transpose acts as
//     (A_d^T g)_j = sum_{i : j in N_i} w^d_ij g_i - S^d_j g_j,
// a gather over the transposed stencils (the edges i -> j grouped by j, in
// ascending i, with their own copy of the weights): no atomics touch
// floating-point data and every result is bitwise reproducible.
//
// One step q -> filter(q + dt sum_i b_i F_i), Y_i = q + dt sum_{j<i} a_ij F_j,
// F_i = R(Y_i), is reversed as
//     qbar' = qbar + A_hyp^T (kappa qbar)                       (filter)
//     Fbar_i = dt (b_i P_i + a_{i+1,i} Ybar_{i+1}),  Ybar_i = J_R(Y_i)^T Fbar_i
//     with P_4 = P_3 = qbar', P_2 = P_3 + Ybar_4, P_1 = P_2 + Ybar_3,
//     qbar = P_1 + Ybar_2 + Ybar_1,
// which uses the two-register structure of the scheme (a_ij = b_j for
// j < i - 1). J_R^T is applied in two kernels: a forward gather at Y_i that
// forms the twelve operator-sum adjoints g and the pointwise terms, then a
// transposed gather of g. States are checkpointed every ckpt_every steps and
// each segment is recomputed once before it is reversed.
#include <climits>

#include "gather.hpp"

namespace labfm {
namespace {

constexpr int kAdjLpn = 16;

// ----------------------------------------------------------- transpose build

__global__ void tcount_kernel(const int* __restrict__ col, long long nnz, int* __restrict__ cnt) {
  for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < nnz;
       e += static_cast<long long>(gridDim.x) * blockDim.x)
    atomicAdd(&cnt[col[e]], 1);
}

constexpr int kScan = 1024;
__global__ void __launch_bounds__(kScan)
tscan_kernel(const int* __restrict__ in, int* __restrict__ out, int n) {
  __shared__ long long sh[kScan];
  long long carry = 0;
  for (int base = 0; base < n; base += kScan) {
    const int i = base + threadIdx.x;
    const long long v = (i < n) ? static_cast<long long>(in[i]) : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScan; off <<= 1) {
      const long long t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) out[i] = static_cast<int>(carry + sh[threadIdx.x] - v);
    carry += sh[kScan - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = static_cast<int>(carry);
}

__global__ void tfill_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col, int n,
                             const int* __restrict__ tptr, int* __restrict__ cursor,
                             int* __restrict__ tsrc, int* __restrict__ tslot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    const int j = col[e];
    const int pos = tptr[j] + atomicAdd(&cursor[j], 1);
    tsrc[pos] = i;
    tslot[pos] = e;
  }
}

// Orders each transposed row by source node (insertion sort, a few tens of
// entries), which makes the layout independent of the fill's thread order.
__global__ void tsort_kernel(const int* __restrict__ tptr, int n, int* __restrict__ tsrc,
                             int* __restrict__ tslot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b = tptr[j], e = tptr[j + 1];
  for (int k = b + 1; k < e; ++k) {
    const int s = tsrc[k], sl = tslot[k];
    int p = k - 1;
    while (p >= b && tsrc[p] > s) {
      tsrc[p + 1] = tsrc[p];
      tslot[p + 1] = tslot[p];
      --p;
    }
    tsrc[p + 1] = s;
    tslot[p + 1] = sl;
  }
}

__global__ void tweights_kernel(const double* __restrict__ w, const int* __restrict__ tslot,
                                long long nnz, double* __restrict__ tw) {
  for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < nnz;
       e += static_cast<long long>(gridDim.x) * blockDim.x) {
    const int s = tslot[e];
#pragma unroll
    for (int d = 0; d < LABFM_NUM_OPS; ++d) tw[d * nnz + e] = w[d * nnz + s];
  }
}

// ------------------------------------------------------------ adjoint kernels

// Forward operator sums at Y and the pointwise part of J_R^T: with
// Rbar = dtb P + dta Ynext (Ynext may be null), writes the twelve operator-sum
// adjoints g[node][k] (l_x, l_y, u_x, u_y, Lu, u_xx, u_xy, v_x, v_y, Lv,
// v_xx, v_xy; node-major, so the transposed gather reads a source node's
// twelve values from one or two cache lines) and the pointwise adjoints
// loc[f][node] of (ln rho, u, v).
template <int LPN>
__global__ void __launch_bounds__(256)
adj_forward_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col,
                   const double* __restrict__ w, long long nnz, const double* __restrict__ Y,
                   const double* __restrict__ P, const double* __restrict__ Ynext, double dtb,
                   double dta, Flow fl, int n, double* __restrict__ g, double* __restrict__ loc) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;
  const long long n2 = 2 * static_cast<long long>(n);
  const double li = Y[node], ui = Y[n + node], vi = Y[n2 + node];
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int e = row_ptr[node] + sub; e < row_ptr[node + 1]; e += LPN) {
    const int j = col[e];
    const double dl = Y[j] - li, du = Y[n + j] - ui, dv = Y[n2 + j] - vi;
    const double a = w[e], b = w[nnz + e], c = w[2 * nnz + e], d = w[3 * nnz + e],
                 f = w[4 * nnz + e];
    acc[0] = fma(a, dl, acc[0]);
    acc[1] = fma(b, dl, acc[1]);
    acc[2] = fma(a, du, acc[2]);
    acc[3] = fma(b, du, acc[3]);
    acc[4] = fma(c, du, acc[4]);
    acc[5] = fma(d, du, acc[5]);
    acc[6] = fma(f, du, acc[6]);
    acc[7] = fma(a, dv, acc[7]);
    acc[8] = fma(b, dv, acc[8]);
    acc[9] = fma(c, dv, acc[9]);
    acc[10] = fma(d, dv, acc[10]);
    acc[11] = fma(f, dv, acc[11]);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = group_sum<LPN>(acc[k]);
  if (sub != 0) return;
  const double lx = acc[0], ly = acc[1], ux = acc[2], uy = acc[3], uL = acc[4], uxx = acc[5];
  const double uxy = acc[6], vx = acc[7], vy = acc[8], vL = acc[9], vxx = acc[10], vxy = acc[11];
  double rl = dtb * P[node], ru = dtb * P[n + node], rv = dtb * P[n2 + node];
  if (Ynext) {
    rl += dta * Ynext[node];
    ru += dta * Ynext[n + node];
    rv += dta * Ynext[n2 + node];
  }
  const double nu = fl.mu / exp(li);
  const double third = 1.0 / 3.0;
  double* gn = g + 12LL * node;
  // R_l = -(u l_x + v l_y) - (u_x + v_y)
  // R_u = -(u u_x + v u_y) - c2 l_x + nu (Lu + (u_xx + v_xy)/3) + gx
  // R_v = -(u v_x + v v_y) - c2 l_y + nu (4/3 Lv - v_xx/3 + u_xy/3) + gy
  gn[0] = -ui * rl - fl.c2 * ru;
  gn[1] = -vi * rl - fl.c2 * rv;
  gn[2] = -rl - ui * ru;
  gn[3] = -vi * ru;
  gn[4] = nu * ru;
  gn[5] = nu * ru * third;
  gn[6] = nu * rv * third;
  gn[7] = -ui * rv;
  gn[8] = -rl - vi * rv;
  gn[9] = 4.0 * third * nu * rv;
  gn[10] = -nu * rv * third;
  gn[11] = nu * ru * third;
  // d nu / d ln rho = -nu
  loc[node] = -nu * (ru * (uL + third * (uxx + vxy)) + rv * (vL + third * ((vL - vxx) + uxy)));
  loc[n + node] = -rl * lx - ru * ux - rv * vx;
  loc[n2 + node] = -rl * ly - ru * uy - rv * vy;
}

// Transposed gather of g: Ybar_j = loc_j + sum_{i -> j} w^d_ij g_d(i) - S^d_j g_d(j),
// then P_j += Pupd_j when Pupd is set (g node-major, g[i][d]).
template <int LPN>
__global__ void __launch_bounds__(256)
adj_transpose_kernel(const int* __restrict__ tptr, const int* __restrict__ tsrc,
                     const double* __restrict__ tw, long long nnz,
                     const double* __restrict__ rowsum, const double* __restrict__ g,
                     const double* __restrict__ loc, int n, double* __restrict__ Ybar,
                     double* __restrict__ P, const double* __restrict__ Pupd) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;
  double sl = 0.0, su = 0.0, sv = 0.0;
  for (int e = tptr[node] + sub; e < tptr[node + 1]; e += LPN) {
    const int i = tsrc[e];
    const double a = tw[e], b = tw[nnz + e], c = tw[2 * nnz + e], d = tw[3 * nnz + e],
                 f = tw[4 * nnz + e];
    const double* gi = g + 12LL * i;
    sl = fma(a, gi[0], sl);
    sl = fma(b, gi[1], sl);
    su = fma(a, gi[2], su);
    su = fma(b, gi[3], su);
    su = fma(c, gi[4], su);
    su = fma(d, gi[5], su);
    su = fma(f, gi[6], su);
    sv = fma(a, gi[7], sv);
    sv = fma(b, gi[8], sv);
    sv = fma(c, gi[9], sv);
    sv = fma(d, gi[10], sv);
    sv = fma(f, gi[11], sv);
  }
  sl = group_sum<LPN>(sl);
  su = group_sum<LPN>(su);
  sv = group_sum<LPN>(sv);
  if (sub != 0) return;
  const long long n2 = 2 * static_cast<long long>(n);
  const double* S = rowsum;  // S[d * n + node]
  const double* gj = g + 12LL * node;
  const double dl = S[node] * gj[0] + S[n + node] * gj[1];
  const double du = S[node] * gj[2] + S[n + node] * gj[3] + S[2 * n + node] * gj[4] +
                    S[3 * n + node] * gj[5] + S[4 * n + node] * gj[6];
  const double dv = S[node] * gj[7] + S[n + node] * gj[8] + S[2 * n + node] * gj[9] +
                    S[3 * n + node] * gj[10] + S[4 * n + node] * gj[11];
  Ybar[node] = loc[node] + (sl - dl);
  Ybar[n + node] = loc[n + node] + (su - du);
  Ybar[n2 + node] = loc[n2 + node] + (sv - dv);
  if (Pupd) {
    P[node] += Pupd[node];
    P[n + node] += Pupd[n + node];
    P[n2 + node] += Pupd[n2 + node];
  }
}

// Filter adjoint: out = qbar + A_hyp^T (kappa qbar), per field.
template <int LPN>
__global__ void __launch_bounds__(256)
adj_filter_kernel(const int* __restrict__ tptr, const int* __restrict__ tsrc,
                  const double* __restrict__ twhyp, const double* __restrict__ Shyp,
                  const double* __restrict__ kappa, const double* __restrict__ qbar, int n,
                  double* __restrict__ out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;
  const long long n2 = 2 * static_cast<long long>(n);
  double sl = 0.0, su = 0.0, sv = 0.0;
  for (int e = tptr[node] + sub; e < tptr[node + 1]; e += LPN) {
    const int i = tsrc[e];
    const double a = twhyp[e] * kappa[i];
    sl = fma(a, qbar[i], sl);
    su = fma(a, qbar[n + i], su);
    sv = fma(a, qbar[n2 + i], sv);
  }
  sl = group_sum<LPN>(sl);
  su = group_sum<LPN>(su);
  sv = group_sum<LPN>(sv);
  if (sub != 0) return;
  const double ks = Shyp[node] * kappa[node];
  out[node] = qbar[node] + (sl - ks * qbar[node]);
  out[n + node] = qbar[n + node] + (su - ks * qbar[n + node]);
  out[n2 + node] = qbar[n2 + node] + (sv - ks * qbar[n2 + node]);
}

__global__ void add3_kernel(const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ out, long long len) {
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    out[i] = a[i] + b[i];
}

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" size_t labfm_transpose_workspace_bytes(int32_t n, int64_t nnz) {
  if (n <= 0 || nnz < 0) return 0;
  return align256(sizeof(int) * (2 * (static_cast<size_t>(n) + 1) + static_cast<size_t>(nnz) + 1));
}

extern "C" int labfm_build_transpose(const labfm_operators* ops, int32_t* tptr, int32_t* tsrc,
                                     double* tw, void* workspace, size_t workspace_bytes,
                                     void* stream_) {
  clear_error();
  LABFM_REQUIRE(ops && ops->n > 0 && ops->row_ptr && ops->w && tptr && tsrc && tw,
                "build_transpose: bad arguments");
  const int n = ops->n;
  const long long nnz = ops->nnz;
  LABFM_REQUIRE(nnz == 0 || ops->col, "build_transpose: missing col");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_transpose_workspace_bytes(n, nnz),
                  "build_transpose");
  hipStream_t st = as_stream(stream_);
  int* tmp = static_cast<int*>(workspace);
  int* cnt = tmp;
  int* cursor = cnt + n + 1;
  int* tslot = cursor + n + 1;
  const int T = 256;
  const unsigned ge = static_cast<unsigned>(std::min<long long>(65535, ceil_div(nnz + 1, T)));
  hipError_t e = hipMemsetAsync(tmp, 0, sizeof(int) * 2 * (static_cast<size_t>(n) + 1), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(tcount_kernel, dim3(ge), dim3(T), 0, st, ops->col, nnz, cnt);
    hipLaunchKernelGGL(tscan_kernel, dim3(1), dim3(kScan), 0, st, cnt, tptr, n);
    hipLaunchKernelGGL(tfill_kernel, dim3(blocks_for(n, T)), dim3(T), 0, st, ops->row_ptr,
                       ops->col, n, tptr, cursor, tsrc, tslot);
    hipLaunchKernelGGL(tsort_kernel, dim3(blocks_for(n, T)), dim3(T), 0, st, tptr, n, tsrc, tslot);
    hipLaunchKernelGGL(tweights_kernel, dim3(ge), dim3(T), 0, st, ops->w, tslot, nnz, tw);
    e = hipGetLastError();
  }
  LABFM_HIP(e);
  return LABFM_OK;
}

extern "C" size_t labfm_adjoint_workspace_bytes(int32_t n, int32_t n_steps, int32_t ckpt_every) {
  if (n <= 0 || n_steps < 0 || ckpt_every <= 0) return 0;
  const long long nck = ceil_div(n_steps, ckpt_every) + 1;
  // checkpoints, one recomputed segment, and 45 n doubles of registers
  const long long doubles = 3LL * n * (nck + ckpt_every) + 45LL * n;
  return static_cast<size_t>(doubles) * sizeof(double) + 256;
}

extern "C" int labfm_rk_adjoint(const double* q0, const double* qbar_end, double* qbar_0,
                                const labfm_operators* ops, const labfm_transpose* tr,
                                const labfm_rk_params* prm, int32_t n_steps, int32_t ckpt_every,
                                void* workspace, size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(ops && ops->n > 0 && ops->w && ops->row_ptr && ops->kappa,
                "rk_adjoint: float64 operators with kappa required");
  if (ops->wall_normal) {
    set_error("rk_adjoint: operators with wall nodes are not supported");
    return LABFM_ERR_UNSUPPORTED;
  }
  LABFM_REQUIRE(tr && tr->tptr && tr->tsrc && tr->tw && tr->rowsum,
                "rk_adjoint: transposed stencils and row sums required");
  LABFM_REQUIRE(q0 && qbar_end && qbar_0 && prm, "rk_adjoint: null argument");
  LABFM_REQUIRE(n_steps >= 0 && ckpt_every > 0, "rk_adjoint: bad step counts");
  LABFM_REQUIRE(prm->dt > 0.0, "rk_adjoint: dt must be positive");
  const int n = ops->n;
  const size_t need = labfm_adjoint_workspace_bytes(n, n_steps, ckpt_every);
  LABFM_REQUIRE(workspace && workspace_bytes >= need, "rk_adjoint: workspace of %zu bytes required",
                need);
  hipStream_t st = as_stream(stream_);
  const long long N3 = 3LL * n;
  const size_t b3 = sizeof(double) * N3;
  const long long nck = ceil_div(n_steps, ckpt_every) + 1;
  double* ws = static_cast<double*>(workspace);
  double* ck = ws;
  double* seg = ck + nck * N3;
  double* Y2 = seg + static_cast<long long>(ckpt_every) * N3;
  double* Y3 = Y2 + N3;
  double* Y4 = Y3 + N3;
  double* qs = Y4 + N3;
  double* Ra = qs + N3;
  double* Rb = Ra + N3;
  double* qbar = Rb + N3;
  double* P = qbar + N3;
  double* Ba = P + N3;
  double* Bb = Ba + N3;
  double* g = Bb + N3;
  double* loc = g + 12LL * n;

  const Flow fl{prm->c2, prm->mu, prm->gx, prm->gy};
  const double dt = prm->dt;
  StepPlan plan;
  plan.ops = ops;
  plan.w = ops->w;
  plan.prec = LABFM_F64;
  plan.stage_cfg = cfg_for(LABFM_KERNEL_STAGE, LABFM_F64, n, ops->nnz);
  plan.filter_cfg = cfg_for(LABFM_KERNEL_FILTER, LABFM_F64, n, ops->nnz);
  plan.fl = fl;
  plan.dt = dt;
  plan.filter = prm->filter;
  plan.Ya = Ra;
  plan.Yb = Rb;
  const LaunchCfg scfg = plan.stage_cfg;
  const long long nnz = ops->nnz;
  const unsigned grid = blocks_for(static_cast<long long>(n) * kAdjLpn, 256);
  const unsigned gadd = static_cast<unsigned>(std::min<long long>(4096, ceil_div(N3, 256)));

  // forward pass, keeping a checkpoint every ckpt_every steps
  LABFM_HIP(hipMemcpyAsync(seg, q0, b3, hipMemcpyDeviceToDevice, st));
  for (int k = 0; k < n_steps; ++k) {
    if (k % ckpt_every == 0)
      LABFM_HIP(hipMemcpyAsync(ck + (k / ckpt_every) * N3, seg, b3, hipMemcpyDeviceToDevice, st));
    plan.Q = seg;
    LABFM_HIP(enqueue_step<F64>(plan, st, nullptr));
  }

  LABFM_HIP(hipMemcpyAsync(qbar, qbar_end, b3, hipMemcpyDeviceToDevice, st));
  for (long long s = ceil_div(n_steps, ckpt_every) - 1; s >= 0; --s) {
    const int k0 = static_cast<int>(s * ckpt_every);
    const int k1 = std::min(n_steps, k0 + ckpt_every);
    // recompute the segment's states q_k0 .. q_{k1-1}
    LABFM_HIP(hipMemcpyAsync(seg, ck + s * N3, b3, hipMemcpyDeviceToDevice, st));
    for (int k = k0 + 1; k < k1; ++k) {
      double* dst = seg + static_cast<long long>(k - k0) * N3;
      LABFM_HIP(hipMemcpyAsync(dst, dst - N3, b3, hipMemcpyDeviceToDevice, st));
      plan.Q = dst;
      LABFM_HIP(enqueue_step<F64>(plan, st, nullptr));
    }
    for (int k = k1 - 1; k >= k0; --k) {
      const double* q = seg + static_cast<long long>(k - k0) * N3;
      // stage values Y2, Y3, Y4 of this step
      LABFM_HIP(launch_stage<F64>(scfg, ops, ops->w, q, q, qs, Y2, dt * kA[0], dt * kB[0], fl, st));
      LABFM_HIP(launch_stage<F64>(scfg, ops, ops->w, Y2, qs, qs, Y3, dt * kA[1], dt * kB[1], fl, st));
      LABFM_HIP(launch_stage<F64>(scfg, ops, ops->w, Y3, qs, qs, Y4, dt * kA[2], dt * kB[2], fl, st));
      // filter adjoint: P = qbar + A_hyp^T (kappa qbar)
      if (prm->filter) {
        hipLaunchKernelGGL(adj_filter_kernel<kAdjLpn>, dim3(grid), dim3(256), 0, st, tr->tptr,
                           tr->tsrc, tr->tw + LABFM_OP_HYP * nnz, tr->rowsum + LABFM_OP_HYP * n,
                           ops->kappa, qbar, n, P);
        LABFM_LAUNCHED();
      } else {
        LABFM_HIP(hipMemcpyAsync(P, qbar, b3, hipMemcpyDeviceToDevice, st));
      }
      // stages 4 .. 1 (index i = 3 .. 0): Ybar_4 -> Ba, Ybar_3 -> Bb,
      // Ybar_2 -> Ba, Ybar_1 -> Bb. Stage index i reads P and Ybar_{i+1};
      // its transposed gather then folds Ybar_{i+1} into P for stage i-1
      // (P_2 = P_3 + Ybar_4, P_1 = P_2 + Ybar_3, and Ybar_2 last).
      const double* Ys[4] = {q, Y2, Y3, Y4};
      double* out[4] = {Bb, Ba, Bb, Ba};
      for (int i = 3; i >= 0; --i) {
        const double* ynext = (i == 3) ? nullptr : out[i + 1];
        const double dta = (i == 3) ? 0.0 : dt * kA[i];
        hipLaunchKernelGGL(adj_forward_kernel<kAdjLpn>, dim3(grid), dim3(256), 0, st,
                           ops->row_ptr, ops->col, ops->w, nnz, Ys[i], P, ynext, dt * kB[i], dta,
                           fl, n, g, loc);
        LABFM_LAUNCHED();
        hipLaunchKernelGGL(adj_transpose_kernel<kAdjLpn>, dim3(grid), dim3(256), 0, st, tr->tptr,
                           tr->tsrc, tr->tw, nnz, tr->rowsum, g, loc, n, out[i], P, ynext);
        LABFM_LAUNCHED();
      }
      // qbar = P_1 + Ybar_2 + Ybar_1 (P holds P_1 + Ybar_2 after the last fold)
      hipLaunchKernelGGL(add3_kernel, dim3(gadd), dim3(256), 0, st, P, out[0], qbar, N3);
      LABFM_LAUNCHED();
    }
  }
  LABFM_HIP(hipMemcpyAsync(qbar_0, qbar, b3, hipMemcpyDeviceToDevice, st));
  return LABFM_OK;
}
