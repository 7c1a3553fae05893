#pragma once
// Gather kernels shared by the forward and adjoint entry points: operator
// application (eq. general_do), the fused Runge-Kutta stage of the isothermal
// Navier-Stokes equations (eq. icns), the filter pass, the time step
// (eq. dt) and the RK3(2)4[2R+]C step sequence.
//
// Gather layout: G = 64 / LPN nodes per wavefront, LPN lanes per node. The
// lanes of a node walk its CSR row with stride LPN, so each weight array is
// read in contiguous LPN-wide runs and consecutive nodes (Morton order) read
// consecutive rows; the field values phi_j are gathered through the cache.
// Partial sums are combined with a butterfly over the LPN lanes. No atomics
// touch floating-point data, so every result is bitwise reproducible.
//
// Precision policies:
//   F64      float64 weights, differences and sums.
//   F32Comp  float32 weights; phi_j - phi_i formed in float64 and split into
//            a float32 pair hi + lo; each product w*hi split exactly with an
//            FMA (TwoProd), w*lo added to its error term, and the products
//            summed with TwoSum, the error terms accumulated separately
//            (Dot2 of Ogita, Rump & Oishi 2005); each lane's pair is carried
//            into float64 and the lanes' partials summed in float64. (A single
//            float32 difference would carry a rounding error of order
//            eps32 |grad phi| h into every product, i.e. eps32 |grad phi| / h
//            into a second derivative, whatever the summation.)
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace labfm {

// Process-wide launch shapes ([kernel][precision]; lanes_per_node 0 selects
// the built-in choice) and the timing events, created once and reused.
extern std::mutex g_cfg_mutex;
extern labfm_launch_config g_cfg[3][3];
extern std::mutex g_event_mutex;
extern std::vector<hipEvent_t> g_events;

namespace {

// --------------------------------------------------------------------------
// precision policies
// --------------------------------------------------------------------------

struct F64 {
  using W = double;
  static constexpr bool kMomentFix = false;
  struct Acc {
    double s;
    __device__ __forceinline__ void zero() { s = 0.0; }
    __device__ __forceinline__ void add(double w, double d) { s = fma(w, d, s); }
    template <int width>
    __device__ __forceinline__ double reduce() {
      return group_sum<width>(s);
    }
  };
  using D = double;
  __device__ __forceinline__ static D diff(double pj, double pi) { return pj - pi; }
};

// Error-free transformations need every operation rounded on its own, so
// floating-point contraction into FMAs is switched off inside them.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

struct F32Comp {
  using W = float;
  static constexpr bool kMomentFix = true;
  struct Acc {
    float s, c;
    __device__ __forceinline__ void zero() {
      s = 0.0f;
      c = 0.0f;
    }
    __device__ __forceinline__ void add(float w, float2 d) {
#pragma clang fp contract(off)
      const float p = w * d.x;
      // w*hi = p + (its exact error); w*lo is second order and rounded once
      const float ep = fmaf(w, d.y, fmaf(w, d.x, -p));
      float t, es;
      two_sum(s, p, t, es);
      s = t;
      c = c + (es + ep);
    }
    // The lane's compensated pair is carried into float64 (s + c rounded
    // once at float64 precision) and the lanes' partials are summed in
    // float64: on this GPU that costs fewer instructions than combining the
    // pairs with TwoSum in float32, and its rounding (eps64) lies far below
    // the Dot2 error of each partial.
    template <int width>
    __device__ __forceinline__ double reduce() {
      return group_sum<width>(static_cast<double>(s) + static_cast<double>(c));
    }
  };
  using D = float2;  // (hi, lo) of the float64 difference
  __device__ __forceinline__ static D diff(double pj, double pi) {
    const double d = pj - pi;
    const float hi = static_cast<float>(d);
    return make_float2(hi, static_cast<float>(d - static_cast<double>(hi)));
  }
};

// float32 weights, float64 differences and sums: the product of a float32
// weight and a float64 difference is rounded once, as in F64.
struct F32W {
  using W = float;
  static constexpr bool kMomentFix = true;
  using Acc = F64::Acc;
  using D = double;
  __device__ __forceinline__ static D diff(double pj, double pi) { return pj - pi; }
};

// Row stride of a policy's weight array: nnz for the float64 weights, the
// padded w32_stride(nnz) for the float32 copy.
template <class P>
__host__ __device__ constexpr long long wstride(long long nnz) {
  return std::is_same<typename P::W, float>::value ? w32_stride(nnz) : nnz;
}

// Float32 weights break the first-moment conditions sum_j w_ji r_ji = 0 of
// the second-derivative operators by rounding; the float32 precisions remove
// the resulting leak of the gradient, grad(phi)_i . mu^d_i, with the stored
// first moments mu of the rounded weights (rows (L,x) (L,y) (xx,x) (xx,y)
// (xy,x) (xy,y) of mom, each of length n).
__device__ __forceinline__ void moment_fix(const float* __restrict__ mom, int node, int n,
                                           double gx, double gy, double& dL, double& dxx,
                                           double& dxy) {
  const long long nn = n;
  dL -= gx * static_cast<double>(mom[node]) + gy * static_cast<double>(mom[nn + node]);
  dxx -= gx * static_cast<double>(mom[2 * nn + node]) + gy * static_cast<double>(mom[3 * nn + node]);
  dxy -= gx * static_cast<double>(mom[4 * nn + node]) + gy * static_cast<double>(mom[5 * nn + node]);
}

// --------------------------------------------------------------------------
// launch variants
// --------------------------------------------------------------------------

// Bit flags of a gather kernel's variant (labfm_launch_config.flags).
constexpr int kXcdOrder = LABFM_LAUNCH_XCD_ORDER;   // contiguous node ranges per XCD
constexpr int kStreaming = LABFM_LAUNCH_STREAMING;  // non-temporal weight/index loads

// The dispatcher hands workgroups to the 8 XCDs round-robin. With the XCD
// order flag, workgroup b works on logical tile xcd_tile(b) so that each XCD
// gets one contiguous run of tiles (a compact, Morton-ordered region whose
// gathered field values then stay in that XCD's L2).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
  const unsigned q = nb / kXcds, r = nb % kXcds;
  const unsigned x = b % kXcds, k = b / kXcds;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <int FL>
__device__ __forceinline__ int first_thread() {
  const unsigned b = (FL & kXcdOrder) ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  return static_cast<int>(b * blockDim.x + threadIdx.x);
}

// Loads of data that is read once per launch (weights, column indices).
template <int FL, class T>
__device__ __forceinline__ T stream_load(const T* p) {
  if constexpr ((FL & kStreaming) != 0) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

// Edges per lane whose loads are issued together in the gather loops.
__host__ __device__ constexpr int unroll_of(int lpn) { return lpn >= 32 ? 3 : (lpn >= 16 ? 3 : 4); }

// --------------------------------------------------------------------------
// operator application
// --------------------------------------------------------------------------

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
apply_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col,
             const typename P::W* __restrict__ w, const float* __restrict__ mom, long long nnz,
             unsigned mask, const double* __restrict__ phi, double* __restrict__ out, int n) {
  const int gid = first_thread<FL>();
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;  // whole LPN groups exit together
  constexpr unsigned kSecond = (1u << LABFM_OP_L) | (1u << LABFM_OP_XX) | (1u << LABFM_OP_XY);
  constexpr unsigned kFirst = (1u << LABFM_OP_X) | (1u << LABFM_OP_Y);
  // the moment correction needs the x and y sums
  const unsigned need = (P::kMomentFix && (mask & kSecond)) ? (mask | kFirst) : mask;
  const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
  const double pi = phi[node];
  typename P::Acc acc[LABFM_NUM_OPS];
#pragma unroll
  for (int d = 0; d < LABFM_NUM_OPS; ++d) acc[d].zero();
  constexpr int U = unroll_of(LPN);
  if (e1 > e0) {
    for (int base = e0 + sub; base < e1; base += U * LPN) {
      int ee[U];
      bool ok[U];
      typename P::D dj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * LPN;
        ok[u] = e < e1;
        ee[u] = ok[u] ? e : e1 - 1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) dj[u] = P::diff(phi[stream_load<FL>(col + ee[u])], pi);
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        if (need & (1u << d)) {
          typename P::W wv[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            wv[u] = stream_load<FL>(w + d * wstride<P>(nnz) + ee[u]);
#pragma unroll
          for (int u = 0; u < U; ++u) acc[d].add(ok[u] ? wv[u] : typename P::W(0), dj[u]);
        }
      }
    }
  }
  double v[LABFM_NUM_OPS];
#pragma unroll
  for (int d = 0; d < LABFM_NUM_OPS; ++d)
    v[d] = (need & (1u << d)) ? acc[d].template reduce<LPN>() : 0.0;
  if (sub != 0) return;
  if constexpr (P::kMomentFix) {
    if (mask & kSecond)
      moment_fix(mom, node, n, v[LABFM_OP_X], v[LABFM_OP_Y], v[LABFM_OP_L], v[LABFM_OP_XX],
                 v[LABFM_OP_XY]);
  }
  int k = 0;
#pragma unroll
  for (int d = 0; d < LABFM_NUM_OPS; ++d) {
    if (mask & (1u << d)) {
      out[static_cast<long long>(k) * n + node] = v[d];
      ++k;
    }
  }
}

// --------------------------------------------------------------------------
// fused Runge-Kutta stage
// --------------------------------------------------------------------------

struct Flow {
  double c2, mu, gx, gy;
};

// Wall normal of a node, or (0, 0) off the walls and when wn is null.
__device__ __forceinline__ bool wall_node(const double* wn, int node, double& nx, double& ny) {
  if (!wn) return false;
  nx = wn[2 * static_cast<long long>(node)];
  ny = wn[2 * static_cast<long long>(node) + 1];
  return nx != 0.0 || ny != 0.0;
}

// d(ln rho)/dt at a no-slip wall node (eq. lodilnro with L2 = 0 and the
// incoming wave L4 = L1 + 2 rho c g.n). Along the normal xi, with
// dp/dxi = c^2 rho d(ln rho)/dxi, -(L4 + L1)/(rho c^2) reduces to
// (c - u_xi)(l_xi - (du_xi/dxi)/c) - 2 g.n / c; the tangential (eta) terms
// follow.
__device__ __forceinline__ double wall_lnrho_rate(double nx, double ny, double ui, double vi,
                                                  double Lx, double Ly, double Ux, double Uy,
                                                  double Vx, double Vy, const Flow& fl) {
  const double c = sqrt(fl.c2);
  const double tx = -ny, ty = nx;
  const double l_xi = nx * Lx + ny * Ly;
  const double l_eta = tx * Lx + ty * Ly;
  const double u_xi = nx * ui + ny * vi;
  const double u_eta = tx * ui + ty * vi;
  const double dxi_uxi = nx * (nx * Ux + ny * Uy) + ny * (nx * Vx + ny * Vy);
  const double deta_ueta = tx * (tx * Ux + ty * Uy) + ty * (tx * Vx + ty * Vy);
  return (c - u_xi) * (l_xi - dxi_uxi / c) - 2.0 * (fl.gx * nx + fl.gy * ny) / c -
         u_eta * l_eta - deta_ueta;
}

// Right-hand side of eq. icns at one node from its operator sums
// D = (l_x, l_y, u_x, u_y, Lu, u_xx, u_xy, v_x, v_y, Lv, v_xx, v_xy), and the
// two-register update: Y' = q + dta F (when Yout is set), q <- q + dtb F.
// 4/3 u_xx + u_yy = L u + u_xx/3 and 4/3 v_yy + v_xx = L v + v_yy/3 with
// v_yy = L v - v_xx. qin == nullptr evaluates the right-hand side alone.
// Wall nodes (wn set and non-zero there) hold their velocity and take the
// wall equation for ln rho.
__device__ __forceinline__ void stage_update(int node, int n, double li, double ui, double vi,
                                             const double* D, const double* qin, double* qout,
                                             double* Yout, double dta, double dtb,
                                             const Flow& fl, const double* wn) {
  const double Lx = D[0], Ly = D[1], Ux = D[2], Uy = D[3], UL = D[4], Uxx = D[5], Uxy = D[6];
  const double Vx = D[7], Vy = D[8], VL = D[9], Vxx = D[10], Vxy = D[11];
  const double nu = fl.mu / exp(li);
  const double third = 1.0 / 3.0;
  double rl = -(ui * Lx + vi * Ly) - (Ux + Vy);
  double ru = -(ui * Ux + vi * Uy) - fl.c2 * Lx + nu * (UL + third * (Uxx + Vxy)) + fl.gx;
  double rv = -(ui * Vx + vi * Vy) - fl.c2 * Ly + nu * (VL + third * ((VL - Vxx) + Uxy)) + fl.gy;
  double nx, ny;
  if (wall_node(wn, node, nx, ny)) {
    rl = wall_lnrho_rate(nx, ny, ui, vi, Lx, Ly, Ux, Uy, Vx, Vy, fl);
    ru = 0.0;
    rv = 0.0;
  }
  const long long n2 = 2 * static_cast<long long>(n);
  const double ql = qin ? qin[node] : 0.0;
  const double qu = qin ? qin[n + node] : 0.0;
  const double qv = qin ? qin[n2 + node] : 0.0;
  if (Yout) {
    Yout[node] = ql + dta * rl;
    Yout[n + node] = qu + dta * ru;
    Yout[n2 + node] = qv + dta * rv;
  }
  qout[node] = ql + dtb * rl;
  qout[n + node] = qu + dtb * ru;
  qout[n2 + node] = qv + dtb * rv;
}

// Stage of the two-register scheme. Y (gathered) holds the stage value, q the
// solution. With F = R(Y):  Y' = q + dta F  (skipped when Yout is null),
// q <- q + dtb F. qin and qout may be the same buffer; Y is never written.
template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
rk_stage_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col,
                const typename P::W* __restrict__ w, const float* __restrict__ mom,
                long long nnz, const double* Y,
                const double* qin, double* qout, double* Yout, double dta, double dtb, Flow fl,
                int n, const double* __restrict__ wn) {
  const int gid = first_thread<FL>();
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;
  const double* Yl = Y;
  const double* Yu = Y + n;
  const double* Yv = Y + 2 * static_cast<long long>(n);
  const double li = Yl[node], ui = Yu[node], vi = Yv[node];
  const long long wst = wstride<P>(nnz);
  const typename P::W* wx = w + 0 * wst;
  const typename P::W* wy = w + 1 * wst;
  const typename P::W* wL = w + 2 * wst;
  const typename P::W* wxx = w + 3 * wst;
  const typename P::W* wxy = w + 4 * wst;
  typename P::Acc lx, ly, ux, uy, uL, uxx, uxy, vx, vy, vL, vxx, vxy;
  lx.zero(); ly.zero();
  ux.zero(); uy.zero(); uL.zero(); uxx.zero(); uxy.zero();
  vx.zero(); vy.zero(); vL.zero(); vxx.zero(); vxy.zero();
  // Edges are taken U per lane at a time: all index, weight and field loads
  // of the U edges are issued before any is used. Lanes past the row's end
  // re-read its last entry (a valid address) with zero weights.
  constexpr int U = unroll_of(LPN);
  using W = typename P::W;
  using D = typename P::D;
  const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
  if (e1 > e0) {
    for (int base = e0 + sub; base < e1; base += U * LPN) {
      int ee[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * LPN;
        ok[u] = e < e1;
        ee[u] = ok[u] ? e : e1 - 1;
      }
      int jj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) jj[u] = stream_load<FL>(col + ee[u]);
      W a[U], b[U], c[U], d[U], f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = stream_load<FL>(wx + ee[u]);
        b[u] = stream_load<FL>(wy + ee[u]);
        c[u] = stream_load<FL>(wL + ee[u]);
        d[u] = stream_load<FL>(wxx + ee[u]);
        f[u] = stream_load<FL>(wxy + ee[u]);
      }
      double gl[U], gu[U], gv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        gl[u] = Yl[jj[u]];
        gu[u] = Yu[jj[u]];
        gv[u] = Yv[jj[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const W z = W(0);
        const W au = ok[u] ? a[u] : z, bu = ok[u] ? b[u] : z, cu = ok[u] ? c[u] : z;
        const W du_ = ok[u] ? d[u] : z, fu = ok[u] ? f[u] : z;
        const D dl = P::diff(gl[u], li);
        const D du = P::diff(gu[u], ui);
        const D dv = P::diff(gv[u], vi);
        lx.add(au, dl);
        ly.add(bu, dl);
        ux.add(au, du);
        uy.add(bu, du);
        uL.add(cu, du);
        uxx.add(du_, du);
        uxy.add(fu, du);
        vx.add(au, dv);
        vy.add(bu, dv);
        vL.add(cu, dv);
        vxx.add(du_, dv);
        vxy.add(fu, dv);
      }
    }
  }
  const double Lx = lx.template reduce<LPN>(), Ly = ly.template reduce<LPN>();
  const double Ux = ux.template reduce<LPN>(), Uy = uy.template reduce<LPN>();
  const double UL = uL.template reduce<LPN>(), Uxx = uxx.template reduce<LPN>();
  const double Uxy = uxy.template reduce<LPN>();
  const double Vx = vx.template reduce<LPN>(), Vy = vy.template reduce<LPN>();
  const double VL = vL.template reduce<LPN>(), Vxx = vxx.template reduce<LPN>();
  const double Vxy = vxy.template reduce<LPN>();
  if (sub != 0) return;
  double sums[12] = {Lx, Ly, Ux, Uy, UL, Uxx, Uxy, Vx, Vy, VL, Vxx, Vxy};
  if constexpr (P::kMomentFix) {
    moment_fix(mom, node, n, sums[2], sums[3], sums[4], sums[5], sums[6]);
    moment_fix(mom, node, n, sums[7], sums[8], sums[9], sums[10], sums[11]);
  }
  stage_update(node, n, li, ui, vi, sums, qin, qout, Yout, dta, dtb, fl, wn);
}

// --------------------------------------------------------------------------
// filter: phi <- phi + kappa_i L^hyp_i(phi) for the three fields
// --------------------------------------------------------------------------

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
filter_kernel(const int* __restrict__ row_ptr, const int* __restrict__ col,
              const typename P::W* __restrict__ whyp, const double* __restrict__ kappa,
              const double* __restrict__ in, double* __restrict__ out, int n,
              const double* __restrict__ wn) {
  const int gid = first_thread<FL>();
  const int node = gid / LPN;
  const int sub = gid % LPN;
  if (node >= n) return;
  const long long n2 = 2 * static_cast<long long>(n);
  const double li = in[node], ui = in[n + node], vi = in[n2 + node];
  typename P::Acc al, au, av;
  al.zero();
  au.zero();
  av.zero();
  const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
  constexpr int U = unroll_of(LPN);
  if (e1 > e0) {
    for (int base = e0 + sub; base < e1; base += U * LPN) {
      int ee[U], jj[U];
      bool ok[U];
      typename P::W a[U];
      double gl[U], gu[U], gv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * LPN;
        ok[u] = e < e1;
        ee[u] = ok[u] ? e : e1 - 1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        jj[u] = stream_load<FL>(col + ee[u]);
        a[u] = stream_load<FL>(whyp + ee[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        gl[u] = in[jj[u]];
        gu[u] = in[n + jj[u]];
        gv[u] = in[n2 + jj[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const typename P::W wu = ok[u] ? a[u] : typename P::W(0);
        al.add(wu, P::diff(gl[u], li));
        au.add(wu, P::diff(gu[u], ui));
        av.add(wu, P::diff(gv[u], vi));
      }
    }
  }
  const double sl = al.template reduce<LPN>();
  const double su = au.template reduce<LPN>();
  const double sv = av.template reduce<LPN>();
  if (sub != 0) return;
  const double k = kappa[node];
  double nx, ny;
  const bool wall = wall_node(wn, node, nx, ny);  // the wall velocity is imposed
  out[node] = li + k * sl;
  out[n + node] = wall ? ui : ui + k * su;
  out[n2 + node] = wall ? vi : vi + k * sv;
}

// --------------------------------------------------------------------------
// LDS-staged (tiled) stage and filter kernels
// --------------------------------------------------------------------------

// One workgroup per tile of LABFM_TILE_NODES nodes. The gathered register's
// values at the tile's halo are first copied into LDS (three arrays of hmax
// doubles, dynamic shared memory); the tile's nodes are then processed
// 256/LPN at a time, every neighbour value read from LDS through its 16-bit
// halo position.
struct Tiles {
  const int* count;
  const int* idx;
  const unsigned short* lcol;
  int hmax;
};

template <int FL>
__device__ __forceinline__ int tile_of_block() {
  return static_cast<int>((FL & kXcdOrder) ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
}

__device__ __forceinline__ void load_halo(const Tiles& tl, int t, const double* Y, int n,
                                          double* sl, double* su, double* sv) {
  const int hc = tl.count[t];
  const int* idx = tl.idx + static_cast<long long>(t) * LABFM_TILE_HALO_MAX;
  const long long n2 = 2 * static_cast<long long>(n);
  for (int k = threadIdx.x; k < hc; k += blockDim.x) {
    const int g = idx[k];
    sl[k] = Y[g];
    su[k] = Y[n + g];
    sv[k] = Y[n2 + g];
  }
  __syncthreads();
}

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
rk_stage_tiled_kernel(const int* __restrict__ row_ptr, Tiles tl,
                      const typename P::W* __restrict__ w, const float* __restrict__ mom,
                      long long nnz, const double* Y,
                      const double* qin, double* qout, double* Yout, double dta, double dtb,
                      Flow fl, int n, const double* __restrict__ wn) {
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, Y, n, sl, su, sv);
  const long long wst = wstride<P>(nnz);
  const typename P::W* wx = w + 0 * wst;
  const typename P::W* wy = w + 1 * wst;
  const typename P::W* wL = w + 2 * wst;
  const typename P::W* wxx = w + 3 * wst;
  const typename P::W* wxy = w + 4 * wst;
  constexpr int NPR = 256 / LPN;  // nodes per round
  constexpr int U = unroll_of(LPN);
  using W = typename P::W;
  using D = typename P::D;
  const int sub = threadIdx.x % LPN;
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;  // whole LPN groups stop together
    const double li = Y[node], ui = Y[n + node], vi = Y[2 * static_cast<long long>(n) + node];
    typename P::Acc lx, ly, ux, uy, uL, uxx, uxy, vx, vy, vL, vxx, vxy;
    lx.zero(); ly.zero();
    ux.zero(); uy.zero(); uL.zero(); uxx.zero(); uxy.zero();
    vx.zero(); vy.zero(); vL.zero(); vxx.zero(); vxy.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    if (e1 > e0) {
      for (int base = e0 + sub; base < e1; base += U * LPN) {
        int ee[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * LPN;
          ok[u] = e < e1;
          ee[u] = ok[u] ? e : e1 - 1;
        }
        int jj[U];
        W a[U], b[U], c[U], d[U], f[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          jj[u] = stream_load<FL>(tl.lcol + ee[u]);
          a[u] = stream_load<FL>(wx + ee[u]);
          b[u] = stream_load<FL>(wy + ee[u]);
          c[u] = stream_load<FL>(wL + ee[u]);
          d[u] = stream_load<FL>(wxx + ee[u]);
          f[u] = stream_load<FL>(wxy + ee[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const W z = W(0);
          const W au = ok[u] ? a[u] : z, bu = ok[u] ? b[u] : z, cu = ok[u] ? c[u] : z;
          const W du_ = ok[u] ? d[u] : z, fu = ok[u] ? f[u] : z;
          const D dl = P::diff(sl[jj[u]], li);
          const D du = P::diff(su[jj[u]], ui);
          const D dv = P::diff(sv[jj[u]], vi);
          lx.add(au, dl);
          ly.add(bu, dl);
          ux.add(au, du);
          uy.add(bu, du);
          uL.add(cu, du);
          uxx.add(du_, du);
          uxy.add(fu, du);
          vx.add(au, dv);
          vy.add(bu, dv);
          vL.add(cu, dv);
          vxx.add(du_, dv);
          vxy.add(fu, dv);
        }
      }
    }
    double Dv[12] = {lx.template reduce<LPN>(),  ly.template reduce<LPN>(),
                           ux.template reduce<LPN>(),  uy.template reduce<LPN>(),
                           uL.template reduce<LPN>(),  uxx.template reduce<LPN>(),
                           uxy.template reduce<LPN>(), vx.template reduce<LPN>(),
                           vy.template reduce<LPN>(),  vL.template reduce<LPN>(),
                           vxx.template reduce<LPN>(), vxy.template reduce<LPN>()};
    if (sub == 0) {
      if constexpr (P::kMomentFix) {
        moment_fix(mom, node, n, Dv[2], Dv[3], Dv[4], Dv[5], Dv[6]);
        moment_fix(mom, node, n, Dv[7], Dv[8], Dv[9], Dv[10], Dv[11]);
      }
      stage_update(node, n, li, ui, vi, Dv, qin, qout, Yout, dta, dtb, fl, wn);
    }
  }
}

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
filter_tiled_kernel(const int* __restrict__ row_ptr, Tiles tl,
                    const typename P::W* __restrict__ whyp, const double* __restrict__ kappa,
                    const double* __restrict__ in, double* __restrict__ out, int n,
                    const double* __restrict__ wn) {
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, in, n, sl, su, sv);
  constexpr int NPR = 256 / LPN;
  constexpr int U = unroll_of(LPN);
  const int sub = threadIdx.x % LPN;
  const long long n2 = 2 * static_cast<long long>(n);
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;
    const double li = in[node], ui = in[n + node], vi = in[n2 + node];
    typename P::Acc al, au, av;
    al.zero();
    au.zero();
    av.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    if (e1 > e0) {
      for (int base = e0 + sub; base < e1; base += U * LPN) {
        int ee[U], jj[U];
        bool ok[U];
        typename P::W a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * LPN;
          ok[u] = e < e1;
          ee[u] = ok[u] ? e : e1 - 1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          jj[u] = stream_load<FL>(tl.lcol + ee[u]);
          a[u] = stream_load<FL>(whyp + ee[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const typename P::W wu = ok[u] ? a[u] : typename P::W(0);
          al.add(wu, P::diff(sl[jj[u]], li));
          au.add(wu, P::diff(su[jj[u]], ui));
          av.add(wu, P::diff(sv[jj[u]], vi));
        }
      }
    }
    const double rl = al.template reduce<LPN>();
    const double ru = au.template reduce<LPN>();
    const double rv = av.template reduce<LPN>();
    if (sub == 0) {
      const double k = kappa[node];
      double nx, ny;
      const bool wall = wall_node(wn, node, nx, ny);
      out[node] = li + k * rl;
      out[n + node] = wall ? ui : ui + k * ru;
      out[n2 + node] = wall ? vi : vi + k * rv;
    }
  }
}

// --------------------------------------------------------------------------
// tiled kernels with packed edge loads
// --------------------------------------------------------------------------

// Each lane loads two consecutive edges of every weight array with one load
// (16 bytes of float64 or 8 bytes of float32 weights) and their two halo
// slots with one 4-byte load, halving the memory instructions per edge.
// Pairs start at even edges; the edge of a pair outside the node's row
// contributes nothing and reads no halo value. Needs a weight base aligned to
// the pair size (checked by the launcher); with an odd nnz the stage kernel
// loads the two misaligned arrays edge by edge and the filter (whose one
// array is then misaligned) keeps its single-edge loads.
template <class W>
struct PairOf;
template <>
struct PairOf<double> {
  using VT = double2;
};
template <>
struct PairOf<float> {
  using VT = float2;
};
// Pairs per lane in flight (measured on MI355X at K ~ 90: 3 for float64,
// 2 for float32 weights in the stage; 3 in the filter). The components are
// selected inline where they are used: through a helper taking the pair by
// reference the compiler split some 16-byte loads into two. kUse: the
// float32-weight, float64-sum policy runs faster with its single-edge loads
// (143 against 150 us per stage at K ~ 90), the others with pairs (float64
// 220 -> 204 us, Dot2 174 -> 157 us).
template <class P>
struct Packed {
  static constexpr bool kUse = !std::is_same<P, F32W>::value;
  static constexpr int V = 2;
  static constexpr int kStageU = std::is_same<typename P::W, double>::value ? 3 : 2;
  static constexpr int kFilterU = 3;
  using VT = typename PairOf<typename P::W>::VT;
  using IT = unsigned;
  __device__ __forceinline__ static int slot(IT j, int h) {
    return static_cast<int>(h ? (j >> 16) : (j & 0xFFFFu));
  }
};

template <int LPN, int FL, class P, bool ODD>
__global__ void __launch_bounds__(256)
rk_stage_tiled_packed_kernel(const int* __restrict__ row_ptr, Tiles tl,
                             const typename P::W* __restrict__ w, const float* __restrict__ mom,
                             long long nnz, const double* Y, const double* qin, double* qout,
                             double* Yout, double dta, double dtb, Flow fl, int n,
                             const double* __restrict__ wn) {
  using K = Packed<P>;
  using W = typename P::W;
  using D = typename P::D;
  constexpr int V = K::V;
  constexpr int U = K::kStageU;
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, Y, n, sl, su, sv);
  // with an odd nnz the arrays of operators 1 and 3 (y, xx) start half a pair
  // off alignment: their two edges are loaded one by one
  const long long wst = wstride<P>(nnz);
  const typename K::VT* wx = reinterpret_cast<const typename K::VT*>(w + 0 * wst);
  const typename K::VT* wy = reinterpret_cast<const typename K::VT*>(w + 1 * wst);
  const typename K::VT* wL = reinterpret_cast<const typename K::VT*>(w + 2 * wst);
  const typename K::VT* wxx = reinterpret_cast<const typename K::VT*>(w + 3 * wst);
  const typename K::VT* wxy = reinterpret_cast<const typename K::VT*>(w + 4 * wst);
  const W* wy1 = w + 1 * wst;
  const W* wxx1 = w + 3 * wst;
  const typename K::IT* lc = reinterpret_cast<const typename K::IT*>(tl.lcol);
  constexpr int NPR = 256 / LPN;
  const int sub = threadIdx.x % LPN;
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;  // whole LPN groups stop together
    const double li = Y[node], ui = Y[n + node], vi = Y[2 * static_cast<long long>(n) + node];
    typename P::Acc lx, ly, ux, uy, uL, uxx, uxy, vx, vy, vL, vxx, vxy;
    lx.zero(); ly.zero();
    ux.zero(); uy.zero(); uL.zero(); uxx.zero(); uxy.zero();
    vx.zero(); vy.zero(); vL.zero(); vxx.zero(); vxy.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    const int g0 = e0 / V, g1 = (e1 + V - 1) / V;
    for (int gb = g0 + sub; gb < g1; gb += U * LPN) {
      int gg[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int g = gb + u * LPN;
        ok[u] = g < g1;
        gg[u] = ok[u] ? g : g1 - 1;
      }
      typename K::IT jj[U];
      typename K::VT a[U], b[U], c[U], d[U], f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long e2 = 2LL * gg[u];
        if constexpr (ODD) {
          // the last pair of the array has no second slot
          jj[u] = (e2 + 1 < nnz) ? lc[gg[u]] : static_cast<typename K::IT>(tl.lcol[e2]);
          b[u].x = wy1[e2];
          b[u].y = wy1[e2 + 1];
          d[u].x = wxx1[e2];
          d[u].y = wxx1[e2 + 1];
        } else {
          jj[u] = lc[gg[u]];
          b[u] = wy[gg[u]];
          d[u] = wxx[gg[u]];
        }
        a[u] = wx[gg[u]];
        c[u] = wL[gg[u]];
        f[u] = wxy[gg[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int h = 0; h < V; ++h) {
          const int e = gg[u] * V + h;
          const bool v = ok[u] && e >= e0 && e < e1;
          const int j = v ? K::slot(jj[u], h) : 0;
          const W z = W(0);
          const W aw = v ? (h ? a[u].y : a[u].x) : z, bw = v ? (h ? b[u].y : b[u].x) : z;
          const W cw = v ? (h ? c[u].y : c[u].x) : z, dw = v ? (h ? d[u].y : d[u].x) : z;
          const W fw = v ? (h ? f[u].y : f[u].x) : z;
          // edges outside the row read no halo value (slot 0 may be unset)
          const D dl = P::diff(v ? sl[j] : li, li);
          const D du = P::diff(v ? su[j] : ui, ui);
          const D dv = P::diff(v ? sv[j] : vi, vi);
          lx.add(aw, dl);
          ly.add(bw, dl);
          ux.add(aw, du);
          uy.add(bw, du);
          uL.add(cw, du);
          uxx.add(dw, du);
          uxy.add(fw, du);
          vx.add(aw, dv);
          vy.add(bw, dv);
          vL.add(cw, dv);
          vxx.add(dw, dv);
          vxy.add(fw, dv);
        }
      }
    }
    double Dv[12] = {lx.template reduce<LPN>(),  ly.template reduce<LPN>(),
                     ux.template reduce<LPN>(),  uy.template reduce<LPN>(),
                     uL.template reduce<LPN>(),  uxx.template reduce<LPN>(),
                     uxy.template reduce<LPN>(), vx.template reduce<LPN>(),
                     vy.template reduce<LPN>(),  vL.template reduce<LPN>(),
                     vxx.template reduce<LPN>(), vxy.template reduce<LPN>()};
    if (sub == 0) {
      if constexpr (P::kMomentFix) {
        moment_fix(mom, node, n, Dv[2], Dv[3], Dv[4], Dv[5], Dv[6]);
        moment_fix(mom, node, n, Dv[7], Dv[8], Dv[9], Dv[10], Dv[11]);
      }
      stage_update(node, n, li, ui, vi, Dv, qin, qout, Yout, dta, dtb, fl, wn);
    }
  }
}

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
filter_tiled_packed_kernel(const int* __restrict__ row_ptr, Tiles tl,
                           const typename P::W* __restrict__ whyp,
                           const double* __restrict__ kappa, const double* __restrict__ in,
                           double* __restrict__ out, int n, const double* __restrict__ wn) {
  using K = Packed<P>;
  using W = typename P::W;
  constexpr int V = K::V;
  constexpr int U = K::kFilterU;
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, in, n, sl, su, sv);
  const typename K::VT* wh = reinterpret_cast<const typename K::VT*>(whyp);
  const typename K::IT* lc = reinterpret_cast<const typename K::IT*>(tl.lcol);
  constexpr int NPR = 256 / LPN;
  const int sub = threadIdx.x % LPN;
  const long long n2 = 2 * static_cast<long long>(n);
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;
    const double li = in[node], ui = in[n + node], vi = in[n2 + node];
    typename P::Acc al, au, av;
    al.zero();
    au.zero();
    av.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    const int g0 = e0 / V, g1 = (e1 + V - 1) / V;
    for (int gb = g0 + sub; gb < g1; gb += U * LPN) {
      int gg[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int g = gb + u * LPN;
        ok[u] = g < g1;
        gg[u] = ok[u] ? g : g1 - 1;
      }
      typename K::IT jj[U];
      typename K::VT a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        jj[u] = lc[gg[u]];
        a[u] = wh[gg[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int h = 0; h < V; ++h) {
          const int e = gg[u] * V + h;
          const bool v = ok[u] && e >= e0 && e < e1;
          const int j = v ? K::slot(jj[u], h) : 0;
          const W aw = v ? (h ? a[u].y : a[u].x) : W(0);
          al.add(aw, P::diff(v ? sl[j] : li, li));
          au.add(aw, P::diff(v ? su[j] : ui, ui));
          av.add(aw, P::diff(v ? sv[j] : vi, vi));
        }
      }
    }
    const double rl = al.template reduce<LPN>();
    const double ru = au.template reduce<LPN>();
    const double rv = av.template reduce<LPN>();
    if (sub == 0) {
      const double k = kappa[node];
      double nx, ny;
      const bool wall = wall_node(wn, node, nx, ny);  // the wall velocity is imposed
      out[node] = li + k * rl;
      out[n + node] = wall ? ui : ui + k * ru;
      out[n2 + node] = wall ? vi : vi + k * rv;
    }
  }
}

// --------------------------------------------------------------------------
// tiled kernels with quad edge loads (float32 weights)
// --------------------------------------------------------------------------

// The rows of the float32 weight copy start on 128-byte boundaries (stride
// w32_stride(nnz)), so a lane loads four consecutive edges of every weight
// array with one 16-byte load and their four 16-bit halo slots with one
// 8-byte load. With 8 lanes per node a load instruction covers 128
// contiguous bytes of each node's row, a whole cache line: with 8-byte pairs
// (two half-line requests per line) the float32 stage moved 1.35x its
// algorithmic bytes at K ~ 90, with quads about 1.05x. Quads start at edges
// 4g; the edges of a quad outside the node's row contribute nothing and read
// no halo value. The last quad of the slot array may run past nnz: its slots
// are then read one by one.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int quad_slot(u32x2 j, int h) {
  const unsigned word = (h < 2) ? j.x : j.y;
  return static_cast<int>((h & 1) ? (word >> 16) : (word & 0xFFFFu));
}

// Halo slots of edges 4g..4g+3 (those at or past nnz read as 0).
__device__ __forceinline__ u32x2 quad_slots(const unsigned short* __restrict__ lcol, long long g,
                                            long long nnz) {
  const long long e = 4 * g;
  if (e + 4 <= nnz) return reinterpret_cast<const u32x2*>(lcol)[g];
  unsigned s[4] = {0u, 0u, 0u, 0u};
  for (int h = 0; h < 4; ++h)
    if (e + h < nnz) s[h] = lcol[e + h];
  return u32x2{s[0] | (s[1] << 16), s[2] | (s[3] << 16)};
}

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
rk_stage_tiled_quad_kernel(const int* __restrict__ row_ptr, Tiles tl,
                           const float* __restrict__ w, const float* __restrict__ mom,
                           long long nnz, const double* Y, const double* qin, double* qout,
                           double* Yout, double dta, double dtb, Flow fl, int n,
                           const double* __restrict__ wn) {
  static_assert(std::is_same<typename P::W, float>::value, "quads are float32 weights");
  using D = typename P::D;
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, Y, n, sl, su, sv);
  const long long wst = w32_stride(nnz);
  const f32x4* wx = reinterpret_cast<const f32x4*>(w + 0 * wst);
  const f32x4* wy = reinterpret_cast<const f32x4*>(w + 1 * wst);
  const f32x4* wL = reinterpret_cast<const f32x4*>(w + 2 * wst);
  const f32x4* wxx = reinterpret_cast<const f32x4*>(w + 3 * wst);
  const f32x4* wxy = reinterpret_cast<const f32x4*>(w + 4 * wst);
  constexpr int NPR = 256 / LPN;
  const int sub = threadIdx.x % LPN;
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;  // whole LPN groups stop together
    const double li = Y[node], ui = Y[n + node], vi = Y[2 * static_cast<long long>(n) + node];
    typename P::Acc lx, ly, ux, uy, uL, uxx, uxy, vx, vy, vL, vxx, vxy;
    lx.zero(); ly.zero();
    ux.zero(); uy.zero(); uL.zero(); uxx.zero(); uxy.zero();
    vx.zero(); vy.zero(); vL.zero(); vxx.zero(); vxy.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    const int g0 = e0 / 4, g1 = (e1 + 3) / 4;
    for (int g = g0 + sub; g < g1; g += LPN) {
      const u32x2 jj = quad_slots(tl.lcol, g, nnz);
      const f32x4 a = stream_load<FL>(wx + g), b = stream_load<FL>(wy + g);
      const f32x4 c = stream_load<FL>(wL + g), d = stream_load<FL>(wxx + g);
      const f32x4 f = stream_load<FL>(wxy + g);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int e = 4 * g + h;
        const bool v = e >= e0 && e < e1;
        const int j = v ? quad_slot(jj, h) : 0;
        const float aw = v ? a[h] : 0.0f, bw = v ? b[h] : 0.0f, cw = v ? c[h] : 0.0f;
        const float dw = v ? d[h] : 0.0f, fw = v ? f[h] : 0.0f;
        // edges outside the row read no halo value (slot 0 may be unset)
        const D dl = P::diff(v ? sl[j] : li, li);
        const D du = P::diff(v ? su[j] : ui, ui);
        const D dv = P::diff(v ? sv[j] : vi, vi);
        lx.add(aw, dl);
        ly.add(bw, dl);
        ux.add(aw, du);
        uy.add(bw, du);
        uL.add(cw, du);
        uxx.add(dw, du);
        uxy.add(fw, du);
        vx.add(aw, dv);
        vy.add(bw, dv);
        vL.add(cw, dv);
        vxx.add(dw, dv);
        vxy.add(fw, dv);
      }
    }
    double Dv[12] = {lx.template reduce<LPN>(),  ly.template reduce<LPN>(),
                     ux.template reduce<LPN>(),  uy.template reduce<LPN>(),
                     uL.template reduce<LPN>(),  uxx.template reduce<LPN>(),
                     uxy.template reduce<LPN>(), vx.template reduce<LPN>(),
                     vy.template reduce<LPN>(),  vL.template reduce<LPN>(),
                     vxx.template reduce<LPN>(), vxy.template reduce<LPN>()};
    if (sub == 0) {
      moment_fix(mom, node, n, Dv[2], Dv[3], Dv[4], Dv[5], Dv[6]);
      moment_fix(mom, node, n, Dv[7], Dv[8], Dv[9], Dv[10], Dv[11]);
      stage_update(node, n, li, ui, vi, Dv, qin, qout, Yout, dta, dtb, fl, wn);
    }
  }
}

template <int LPN, int FL, class P>
__global__ void __launch_bounds__(256)
filter_tiled_quad_kernel(const int* __restrict__ row_ptr, Tiles tl,
                         const float* __restrict__ whyp, long long nnz,
                         const double* __restrict__ kappa, const double* __restrict__ in,
                         double* __restrict__ out, int n, const double* __restrict__ wn) {
  static_assert(std::is_same<typename P::W, float>::value, "quads are float32 weights");
  extern __shared__ double lds[];
  double* sl = lds;
  double* su = lds + tl.hmax;
  double* sv = lds + 2 * tl.hmax;
  const int t = tile_of_block<FL>();
  load_halo(tl, t, in, n, sl, su, sv);
  const f32x4* wh = reinterpret_cast<const f32x4*>(whyp);
  constexpr int NPR = 256 / LPN;
  const int sub = threadIdx.x % LPN;
  const long long n2 = 2 * static_cast<long long>(n);
#pragma unroll 1
  for (int r = 0; r < (LABFM_TILE_NODES + NPR - 1) / NPR; ++r) {
    const int local = r * NPR + threadIdx.x / LPN;
    if (local >= LABFM_TILE_NODES) break;  // a tile smaller than a pass
    const int node = t * LABFM_TILE_NODES + local;
    if (node >= n) break;
    const double li = in[node], ui = in[n + node], vi = in[n2 + node];
    typename P::Acc al, au, av;
    al.zero();
    au.zero();
    av.zero();
    const int e0 = row_ptr[node], e1 = row_ptr[node + 1];
    const int g0 = e0 / 4, g1 = (e1 + 3) / 4;
    for (int g = g0 + sub; g < g1; g += LPN) {
      const u32x2 jj = quad_slots(tl.lcol, g, nnz);
      const f32x4 a = stream_load<FL>(wh + g);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int e = 4 * g + h;
        const bool v = e >= e0 && e < e1;
        const int j = v ? quad_slot(jj, h) : 0;
        const float aw = v ? a[h] : 0.0f;
        al.add(aw, P::diff(v ? sl[j] : li, li));
        au.add(aw, P::diff(v ? su[j] : ui, ui));
        av.add(aw, P::diff(v ? sv[j] : vi, vi));
      }
    }
    const double rl = al.template reduce<LPN>();
    const double ru = au.template reduce<LPN>();
    const double rv = av.template reduce<LPN>();
    if (sub == 0) {
      const double k = kappa[node];
      double nx, ny;
      const bool wall = wall_node(wn, node, nx, ny);  // the wall velocity is imposed
      out[node] = li + k * rl;
      out[n + node] = wall ? ui : ui + k * ru;
      out[n2 + node] = wall ? vi : vi + k * rv;
    }
  }
}

// --------------------------------------------------------------------------
// time step and finiteness check
// --------------------------------------------------------------------------

constexpr int kRedThreads = 256;

__global__ void __launch_bounds__(kRedThreads)
dt_partial_kernel(const double* __restrict__ q, const double* __restrict__ s, int n, double c,
                  double mu, double conv_coef, double visc_coef, double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  double m = INFINITY;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double u = q[n + i], v = q[2 * static_cast<long long>(n) + i];
    const double speed = sqrt(u * u + v * v);
    const double conv = conv_coef * s[i] / (speed + c);
    const double visc = visc_coef * s[i] * s[i] * exp(q[i]) / mu;
    m = fmin(m, fmin(conv, visc));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kRedThreads)
min_final_kernel(const double* __restrict__ partial, int m, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double v = INFINITY;
  for (int i = threadIdx.x; i < m; i += blockDim.x) v = fmin(v, partial[i]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void nonfinite_kernel(const double* __restrict__ q, long long len, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    bad |= !isfinite(q[i]);
  if (__any(bad) && (threadIdx.x % 64) == 0) atomicOr(flag, 1);
}

// --------------------------------------------------------------------------
// launch helpers
// --------------------------------------------------------------------------

constexpr int kThreads = 256;

struct LaunchCfg {
  int lpn;    // lanes per node: 4, 8, 16 or 32
  int flags;  // kXcdOrder | kStreaming
};

// Calls fn(integral_constant<LPN>, integral_constant<FLAGS>) for a config.
template <class Fn>
hipError_t with_cfg(LaunchCfg c, Fn&& fn) {
  using std::integral_constant;
#define LABFM_CFG_CASE(L, F)                                  \
  case (L) * 8 + (F):                                          \
    fn(integral_constant<int, L>{}, integral_constant<int, F>{}); \
    break;
#define LABFM_CFG_LPN(L) \
  LABFM_CFG_CASE(L, 0) LABFM_CFG_CASE(L, 1) LABFM_CFG_CASE(L, 2) LABFM_CFG_CASE(L, 3)
  switch (c.lpn * 8 + c.flags) {
    LABFM_CFG_LPN(4)
    LABFM_CFG_LPN(8)
    LABFM_CFG_LPN(16)
    LABFM_CFG_LPN(32)
    default:
      return hipErrorInvalidValue;
  }
#undef LABFM_CFG_LPN
#undef LABFM_CFG_CASE
  return hipGetLastError();
}

bool valid_cfg(const labfm_launch_config& c) {
  return (c.lanes_per_node == 4 || c.lanes_per_node == 8 || c.lanes_per_node == 16 ||
          c.lanes_per_node == 32) &&
         c.flags >= 0 && c.flags <= 3;
}

// Default variant from the mean row length K (measured on MI355X at K ~ 90,
// tiled kernels: 16 lanes per node for the stage, 8 for the filter pass);
// overridden per kernel and precision by labfm_set_launch_config or
// labfm_tune.
LaunchCfg default_cfg(int kernel, labfm_prec prec, int n, long long nnz) {
  const double k = n > 0 ? static_cast<double>(nnz) / n : 0.0;
  int lpn = k > 48.0 ? 16 : (k > 12.0 ? 8 : 4);
  if (kernel == LABFM_KERNEL_FILTER && k > 48.0) lpn = 8;
  // stage on 32-node tiles: 8 lanes per node (float64: two passes of 32
  // nodes per workgroup, 197 us against 200 us for 16 at 262,144 nodes,
  // K = 90; float32: the quad loads then cover whole 128-byte lines)
  if (kernel == LABFM_KERNEL_STAGE && k > 48.0) lpn = 8;
  return LaunchCfg{lpn, 0};
}

int prec_slot(labfm_prec p) { return p == LABFM_F64 ? 0 : (p == LABFM_F32_COMP ? 1 : 2); }

LaunchCfg cfg_for(int kernel, labfm_prec prec, int n, long long nnz) {
  std::lock_guard<std::mutex> lock(g_cfg_mutex);
  const labfm_launch_config& c = g_cfg[kernel][prec_slot(prec)];
  if (c.lanes_per_node == 0) return default_cfg(kernel, prec, n, nnz);
  return LaunchCfg{c.lanes_per_node, c.flags};
}

template <class P>
hipError_t launch_apply(LaunchCfg cfg, const labfm_operators* o, const typename P::W* w,
                        unsigned mask, const double* phi, double* out, hipStream_t st) {
  const int n = o->n;
  const unsigned grid = blocks_for(static_cast<long long>(n) * cfg.lpn, kThreads);
  return with_cfg(cfg, [&](auto L, auto F) {
    hipLaunchKernelGGL((apply_kernel<decltype(L)::value, decltype(F)::value, P>), dim3(grid),
                       dim3(kThreads), 0, st, o->row_ptr, o->col, w, o->mom32,
                       static_cast<long long>(o->nnz), mask, phi, out, n);
  });
}

Tiles tiles_of(const labfm_operators* o) {
  const labfm_tiles* t = o->tiles;
  return Tiles{t->halo_count, t->halo_idx, t->lcol, t->max_halo > 0 ? t->max_halo : 1};
}

// The packed tiled kernels apply when every weight array and the halo
// slots are aligned for their pair loads: an even nnz and a weight base
// aligned to two weights.
template <class P>
bool packable(const labfm_operators* o, const void* w, bool odd_ok) {
  if (!Packed<P>::kUse) return false;
  const uintptr_t wb = reinterpret_cast<uintptr_t>(w);
  const uintptr_t lb = reinterpret_cast<uintptr_t>(o->tiles->lcol);
  return (odd_ok || o->nnz % 2 == 0) && wb % (2 * sizeof(typename P::W)) == 0 && lb % 4 == 0;
}

// The quad kernels apply to the float32 weights when the weight base is
// aligned to 16 bytes (rows then are, at the padded stride) and the halo
// slots to 8 bytes.
template <class P>
bool quadable(const labfm_operators* o, const void* w) {
  if (!std::is_same<typename P::W, float>::value) return false;
  const uintptr_t wb = reinterpret_cast<uintptr_t>(w);
  const uintptr_t lb = reinterpret_cast<uintptr_t>(o->tiles->lcol);
  return wb % 16 == 0 && lb % 8 == 0;
}

template <class P>
hipError_t launch_stage(LaunchCfg cfg, const labfm_operators* o, const typename P::W* w,
                        const double* Y, const double* qin, double* qout, double* Yout, double dta,
                        double dtb, const Flow& fl, hipStream_t st) {
  const int n = o->n;
  if constexpr (std::is_same<typename P::W, float>::value) {
    if (o->tiles && quadable<P>(o, w)) {
      const Tiles tl = tiles_of(o);
      const size_t shmem = 3 * sizeof(double) * tl.hmax;
      return with_cfg(cfg, [&](auto L, auto F) {
        hipLaunchKernelGGL(
            (rk_stage_tiled_quad_kernel<decltype(L)::value, decltype(F)::value, P>),
            dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, w, o->mom32,
            static_cast<long long>(o->nnz), Y, qin, qout, Yout, dta, dtb, fl, n, o->wall_normal);
      });
    }
  }
  if (o->tiles && packable<P>(o, w, true)) {
    const Tiles tl = tiles_of(o);
    const size_t shmem = 3 * sizeof(double) * tl.hmax;
    const bool odd = (o->nnz % 2) != 0;
    return with_cfg(cfg, [&](auto L, auto F) {
      if (odd) {
        hipLaunchKernelGGL(
            (rk_stage_tiled_packed_kernel<decltype(L)::value, decltype(F)::value, P, true>),
            dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, w, o->mom32,
            static_cast<long long>(o->nnz), Y, qin, qout, Yout, dta, dtb, fl, n, o->wall_normal);
      } else {
        hipLaunchKernelGGL(
            (rk_stage_tiled_packed_kernel<decltype(L)::value, decltype(F)::value, P, false>),
            dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, w, o->mom32,
            static_cast<long long>(o->nnz), Y, qin, qout, Yout, dta, dtb, fl, n, o->wall_normal);
      }
    });
  }
  if (o->tiles) {
    const Tiles tl = tiles_of(o);
    const size_t shmem = 3 * sizeof(double) * tl.hmax;
    return with_cfg(cfg, [&](auto L, auto F) {
      hipLaunchKernelGGL((rk_stage_tiled_kernel<decltype(L)::value, decltype(F)::value, P>),
                         dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, w,
                         o->mom32, static_cast<long long>(o->nnz), Y, qin, qout, Yout, dta, dtb,
                         fl, n, o->wall_normal);
    });
  }
  const unsigned grid = blocks_for(static_cast<long long>(n) * cfg.lpn, kThreads);
  return with_cfg(cfg, [&](auto L, auto F) {
    hipLaunchKernelGGL((rk_stage_kernel<decltype(L)::value, decltype(F)::value, P>), dim3(grid),
                       dim3(kThreads), 0, st, o->row_ptr, o->col, w, o->mom32,
                       static_cast<long long>(o->nnz), Y, qin, qout, Yout, dta, dtb, fl, n,
                       o->wall_normal);
  });
}

template <class P>
hipError_t launch_filter(LaunchCfg cfg, const labfm_operators* o, const typename P::W* w,
                         const double* in, double* out, hipStream_t st) {
  const int n = o->n;
  const typename P::W* whyp = w + LABFM_OP_HYP * wstride<P>(o->nnz);
  if constexpr (std::is_same<typename P::W, float>::value) {
    if (o->tiles && quadable<P>(o, w)) {
      const Tiles tl = tiles_of(o);
      const size_t shmem = 3 * sizeof(double) * tl.hmax;
      return with_cfg(cfg, [&](auto L, auto F) {
        hipLaunchKernelGGL((filter_tiled_quad_kernel<decltype(L)::value, decltype(F)::value, P>),
                           dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl,
                           whyp, static_cast<long long>(o->nnz), o->kappa, in, out, n,
                           o->wall_normal);
      });
    }
  }
  if (o->tiles && packable<P>(o, w, false)) {
    const Tiles tl = tiles_of(o);
    const size_t shmem = 3 * sizeof(double) * tl.hmax;
    return with_cfg(cfg, [&](auto L, auto F) {
      hipLaunchKernelGGL((filter_tiled_packed_kernel<decltype(L)::value, decltype(F)::value, P>),
                         dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, whyp,
                         o->kappa, in, out, n, o->wall_normal);
    });
  }
  if (o->tiles) {
    const Tiles tl = tiles_of(o);
    const size_t shmem = 3 * sizeof(double) * tl.hmax;
    return with_cfg(cfg, [&](auto L, auto F) {
      hipLaunchKernelGGL((filter_tiled_kernel<decltype(L)::value, decltype(F)::value, P>),
                         dim3(o->tiles->ntiles), dim3(kThreads), shmem, st, o->row_ptr, tl, whyp,
                         o->kappa, in, out, n, o->wall_normal);
    });
  }
  const unsigned grid = blocks_for(static_cast<long long>(n) * cfg.lpn, kThreads);
  return with_cfg(cfg, [&](auto L, auto F) {
    hipLaunchKernelGGL((filter_kernel<decltype(L)::value, decltype(F)::value, P>), dim3(grid),
                       dim3(kThreads), 0, st, o->row_ptr, o->col, whyp, o->kappa, in, out, n,
                       o->wall_normal);
  });
}

// Calls fn(policy{}, weights) with the arithmetic policy of a precision.
template <class Fn>
hipError_t with_prec(labfm_prec prec, const labfm_operators* o, Fn&& fn) {
  switch (prec) {
    case LABFM_F64:
      return fn(F64{}, o->w);
    case LABFM_F32_COMP:
      return fn(F32Comp{}, o->w32);
    case LABFM_F32W:
      return fn(F32W{}, o->w32);
  }
  return hipErrorInvalidValue;
}

bool known_prec(labfm_prec p) {
  return p == LABFM_F64 || p == LABFM_F32_COMP || p == LABFM_F32W;
}

// RK3(2)4[2R+]C (Kennedy, Carpenter & Lewis 2000): sub-diagonal a_{i+1,i}
// and weights b_i of the two-register form.
constexpr double kA[3] = {11847461282814.0 / 36547543011857.0,
                          3943225443063.0 / 7078155732230.0,
                          -346793006927.0 / 4029903576067.0};
constexpr double kB[4] = {1017324711453.0 / 9774461848756.0,
                          8237718856693.0 / 13685301971492.0,
                          57731312506979.0 / 19404895981398.0,
                          -101169746363290.0 / 37734290219643.0};

// Kernel sequence of one full step. Registers rotate between the caller's
// state Q and workspace buffers Ya, Yb so that no launch writes a buffer it
// gathers from and no copy is needed:
//   stage 1: gather Q,  q in Q  -> q to Ya, Y to Yb
//   stage 2: gather Yb, q in Ya -> q to Ya, Y to Q
//   stage 3: gather Q,  q in Ya -> q to Ya, Y to Yb
//   stage 4: gather Yb, q in Ya -> q to Ya
//   filter:  gather Ya          -> Q        (or a copy Ya -> Q without filter)
struct StepPlan {
  const labfm_operators* ops;
  const void* w;
  labfm_prec prec;
  LaunchCfg stage_cfg, filter_cfg;
  Flow fl;
  double dt;
  int filter;
  double* Q;
  double* Ya;
  double* Yb;
};

// Event marks around the launches of a step when timing is requested: one
// mark before every launch and one after the last, so the time of launch k
// is mark[k+1] - mark[k] (launches on one stream run back to back).
struct Marks {
  hipEvent_t* ev;
  int count;
};

template <class P>
hipError_t enqueue_step(const StepPlan& p, hipStream_t st, Marks* mk) {
  const auto* w = static_cast<const typename P::W*>(p.w);
  const long long bytes = 3LL * p.ops->n * sizeof(double);
  double* const Ys[4] = {p.Yb, p.Q, p.Yb, nullptr};
  const double* const G[4] = {p.Q, p.Yb, p.Q, p.Yb};
  const double* const Qin[4] = {p.Q, p.Ya, p.Ya, p.Ya};
  hipError_t e = hipSuccess;
  for (int s = 0; s < 4 && e == hipSuccess; ++s) {
    const double dta = (s < 3) ? p.dt * kA[s] : 0.0;
    if (mk) e = hipEventRecord(mk->ev[mk->count++], st);
    if (e == hipSuccess)
      e = launch_stage<P>(p.stage_cfg, p.ops, w, G[s], Qin[s], p.Ya, Ys[s], dta, p.dt * kB[s],
                          p.fl, st);
  }
  if (e != hipSuccess) return e;
  if (p.filter) {
    if (mk) e = hipEventRecord(mk->ev[mk->count++], st);
    if (e == hipSuccess) e = launch_filter<P>(p.filter_cfg, p.ops, w, p.Ya, p.Q, st);
  } else {
    if (mk) e = hipEventRecord(mk->ev[mk->count++], st);
    if (e == hipSuccess) e = hipMemcpyAsync(p.Q, p.Ya, bytes, hipMemcpyDeviceToDevice, st);
  }
  if (mk && e == hipSuccess) e = hipEventRecord(mk->ev[mk->count++], st);
  return e;
}

hipError_t enqueue_step_any(const StepPlan& p, hipStream_t st, Marks* mk) {
  return with_prec(p.prec, p.ops, [&](auto pol, const auto*) {
    return enqueue_step<decltype(pol)>(p, st, mk);
  });
}

hipError_t reserve_events(size_t count) {
  while (g_events.size() < count) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    g_events.push_back(e);
  }
  return hipSuccess;
}

int check_ops(const labfm_operators* o, labfm_prec prec, const char* who) {
  LABFM_REQUIRE(o, "%s: null operators", who);
  LABFM_REQUIRE(o->n > 0 && o->nnz >= 0 && o->row_ptr && (o->col || o->nnz == 0),
                "%s: incomplete operator description", who);
  LABFM_REQUIRE(known_prec(prec), "%s: unknown precision %d", who, (int)prec);
  if (prec == LABFM_F64) LABFM_REQUIRE(o->w, "%s: float64 weights required", who);
  if (prec != LABFM_F64)
    LABFM_REQUIRE(o->w32 && o->mom32, "%s: float32 weights and their first moments required",
                  who);
  if (o->tiles) {
    const labfm_tiles* t = o->tiles;
    LABFM_REQUIRE(t->ntiles == labfm_tile_count(o->n) && t->halo_count && t->halo_idx &&
                      (t->lcol || o->nnz == 0) && t->max_halo >= 0 &&
                      t->max_halo <= LABFM_TILE_HALO_MAX,
                  "%s: inconsistent tiles", who);
  }
  return LABFM_OK;
}

}  // namespace
}  // namespace labfm
