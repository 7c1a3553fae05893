// Weight construction (sections "LABFM" and "New ABFs" of the paper, eqs.
// disc_form, lsys, w_abf and hermite; filter calibration of section "Spatial
// filtering").
//
// One 64-lane wavefront builds one node:
//   1. basis tables: for 16 neighbours at a time, four lanes per neighbour
//      evaluate x^a/a!, y^b/b!, psi He_a(x), He_b(y) (scaled offsets, a,b <= m)
//      into LDS;
//   2. moment matrix M~ = sum_j X~_j (outer) W_j, n x n with n = (m^2+3m)/2,
//      accumulated with FP64 MFMA (v_mfma_f64_16x16x4f64): the moment index
//      is tiled by 16, the neighbour index is the MFMA's K dimension;
//   3. LU factorisation with partial pivoting (largest magnitude, first index
//      on ties) of [M~ | C~] in LDS, applied to the six right-hand sides;
//   4. back substitution for Psi^d;
//   5. per neighbour (one lane each), w^d_j = W_j . Psi^d for the six
//      operators, the filter sum F_0 and the row sums, reduced across the
//      wave.
// Hermite ABFs use the probabilists' polynomials He_a(x/h), which equal the
// paper's H_a(x/(h sqrt 2)) / sqrt(2^a).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>
#include <type_traits>

#include "common.hpp"
#include "tune_cache.hpp"

namespace labfm {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kChunk = 16;  // neighbours per basis-table chunk

// Output rows of an op_mask build: 3 bits per operator (labfm_op order) give
// the row of w, w32 and rowsum that holds it; kNoRow marks an operator that
// is not written (its weights are still formed, the filter's for kappa).
constexpr int kNoRow = 7;
__host__ __device__ constexpr int op_row(unsigned rows, int d) {
  return static_cast<int>((rows >> (3 * d)) & 7u);
}
constexpr unsigned rows_of_mask(unsigned op_mask) {
  unsigned rows = 0;
  int r = 0;
  for (int d = 0; d < LABFM_NUM_OPS; ++d)
    rows |= static_cast<unsigned>((op_mask >> d) & 1u ? r++ : kNoRow) << (3 * d);
  return rows;
}
static_assert(rows_of_mask(0x3F) == (0u | 1u << 3 | 2u << 6 | 3u << 9 | 4u << 12 | 5u << 15),
              "the full mask keeps the labfm_op rows");

// (a, b) exponents of moment index p (degree-major, decreasing power of x).
__device__ __forceinline__ void exponents_of(int p, int& a, int& b) {
  int d = 1;
  while ((d + 1) * (d + 2) / 2 - 1 <= p) ++d;
  b = p - (d * (d + 1) / 2 - 1);
  a = d - b;
}

__device__ __forceinline__ int index_of(int a, int b) {
  const int d = a + b;
  return d * (d + 1) / 2 - 1 + b;
}

__device__ __forceinline__ double wendland_c2(double q) {
  if (q >= 2.0) return 0.0;
  const double t = 1.0 - 0.5 * q;
  const double t2 = t * t;
  return t2 * t2 * (1.0 + 2.0 * q);
}

template <int MMAX>
struct Shape {
  static constexpr int NMAX = moments_of(MMAX);
  static constexpr int NB = (NMAX + 15) / 16;   // 16-wide MFMA tiles per side
  static constexpr int LDA = (NMAX + 6) | 1;     // row stride of [M | C] (odd)
  static constexpr int TW = MMAX + 1;            // one basis table's length
  static constexpr int TABLE = 4 * TW + 1;       // four tables per neighbour and a zero
  static constexpr int ZERO = 4 * TW;            // the zero entry of a neighbour's tables
  static constexpr int HW = 2 * TW + 1;          // per-lane Hermite row (odd)
};

template <int MMAX>
__global__ void __launch_bounds__(64)
build_weights_kernel(const double* __restrict__ x, const double* __restrict__ y,
                     const double* __restrict__ hh, const double* __restrict__ ss,
                     const int8_t* __restrict__ order, int nnodes, labfm_box box,
                     const int* __restrict__ row_ptr, const int* __restrict__ col, long long nnz,
                     double* __restrict__ w, float* __restrict__ w32,
                     float* __restrict__ mom32, double* __restrict__ kappa,
                     double* __restrict__ rowsum, int8_t* __restrict__ status, unsigned rows) {
  using S = Shape<MMAX>;
  __shared__ double A[S::NMAX * S::LDA];
  __shared__ double T[kChunk * S::TABLE];
  __shared__ double H[64 * S::HW];
  __shared__ int s_flag;

  const int i = blockIdx.x;
  if (i >= nnodes) return;
  const int lane = threadIdx.x;
  const int m = order[i];
  const int e0 = row_ptr[i];
  const int K = row_ptr[i + 1] - e0;

  if (m < 1 || m > MMAX) {
    for (int k = lane; k < K; k += 64)
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const int r = op_row(rows, d);
        if (r == kNoRow) continue;
        w[r * nnz + e0 + k] = 0.0;
        if (w32) w32[r * w32_stride(nnz) + e0 + k] = 0.0f;
      }
    if (lane == 0) {
      kappa[i] = 0.0;
      status[i] = LABFM_NODE_BAD_ORDER;
      if (rowsum)
        for (int d = 0; d < LABFM_NUM_OPS; ++d)
          if (op_row(rows, d) != kNoRow) rowsum[op_row(rows, d) * (long long)nnodes + i] = 0.0;
      if (mom32)
        for (int k = 0; k < kMoments; ++k) mom32[k * (long long)nnodes + i] = 0.0f;
    }
    return;
  }
  const int n = moments_of(m);
  const double xi = x[i], yi = y[i], h = hh[i], s = ss[i];
  const int px = box.periodic_x, py = box.periodic_y;

  // ---- 1+2: basis tables and MFMA assembly of M~ -------------------------
  int pa[S::NB], pb[S::NB];  // exponents of this lane's row/column in each tile
#pragma unroll
  for (int P = 0; P < S::NB; ++P) {
    const int p = P * 16 + (lane & 15);
    if (p < n) {
      exponents_of(p, pa[P], pb[P]);
    } else {
      pa[P] = -1;
      pb[P] = -1;
    }
  }
  double4_t acc[S::NB][S::NB];
#pragma unroll
  for (int P = 0; P < S::NB; ++P)
#pragma unroll
    for (int Q = 0; Q < S::NB; ++Q) acc[P][Q] = double4_t{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < K; k0 += kChunk) {
    {
      const int kk = lane >> 2, t = lane & 3;
      const int k = k0 + kk;
      double* tab = &T[kk * S::TABLE + t * S::TW];
      if (k < K) {
        const int j = col[e0 + k];
        const double dx = wrap_axis(x[j] - xi, box.Lx, px);
        const double dy = wrap_axis(y[j] - yi, box.Ly, py);
        const double xs = dx / h, ys = dy / h;
        const double z = (t == 0 || t == 2) ? xs : ys;
        if (t < 2) {
          // z^a / a!
          double v = 1.0;
          tab[0] = 1.0;
#pragma unroll
          for (int a = 1; a <= MMAX; ++a) {
            v = v * z / static_cast<double>(a);
            tab[a] = v;
          }
        } else {
          // probabilists' Hermite He_a(z); the x table carries psi
          const double psi = (t == 2) ? wendland_c2(sqrt(xs * xs + ys * ys)) : 1.0;
          double h0 = 1.0, h1 = z;
          tab[0] = psi;
          tab[1] = psi * z;
#pragma unroll
          for (int a = 1; a < MMAX; ++a) {
            const double h2 = z * h1 - static_cast<double>(a) * h0;
            h0 = h1;
            h1 = h2;
            tab[a + 1] = psi * h2;
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a <= MMAX; ++a) tab[a] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kChunk / 4; ++ks) {
      const double* tk = &T[(ks * 4 + (lane >> 4)) * S::TABLE];
      double av[S::NB], bv[S::NB];
#pragma unroll
      for (int P = 0; P < S::NB; ++P) {
        if (pa[P] >= 0) {
          av[P] = tk[pa[P]] * tk[S::TW + pb[P]];
          bv[P] = tk[2 * S::TW + pa[P]] * tk[3 * S::TW + pb[P]];
        } else {
          av[P] = 0.0;
          bv[P] = 0.0;
        }
      }
#pragma unroll
      for (int P = 0; P < S::NB; ++P)
#pragma unroll
        for (int Q = 0; Q < S::NB; ++Q)
          acc[P][Q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[P], bv[Q], acc[P][Q], 0, 0, 0);
    }
    __syncthreads();
  }
  // element v of lane l holds D[l/16 + 4v][l%16] of its 16x16 tile
#pragma unroll
  for (int P = 0; P < S::NB; ++P)
#pragma unroll
    for (int Q = 0; Q < S::NB; ++Q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = P * 16 + (lane >> 4) + 4 * v;
        const int c = Q * 16 + (lane & 15);
        if (r < n && c < n) A[r * S::LDA + c] = acc[P][Q][v];
      }
  // right-hand sides C~^d = C^d h^-(a+b)
  for (int r = lane; r < n; r += 64)
#pragma unroll
    for (int d = 0; d < LABFM_NUM_OPS; ++d) A[r * S::LDA + S::NMAX + d] = 0.0;
  __syncthreads();
  if (lane == 0) {
    const double h1 = 1.0 / h, h2 = 1.0 / (h * h);
    const int C0 = S::NMAX;
    A[0 * S::LDA + C0 + LABFM_OP_X] = h1;
    A[1 * S::LDA + C0 + LABFM_OP_Y] = h1;
    if (m >= 2) {
      A[index_of(2, 0) * S::LDA + C0 + LABFM_OP_L] = h2;
      A[index_of(0, 2) * S::LDA + C0 + LABFM_OP_L] = h2;
      A[index_of(2, 0) * S::LDA + C0 + LABFM_OP_XX] = h2;
      A[index_of(1, 1) * S::LDA + C0 + LABFM_OP_XY] = h2;
    }
    const int mp = (m % 2 == 0) ? m : m - 1;
    if (mp >= 2) {
      double hp = 1.0;
      for (int k = 0; k < mp; ++k) hp *= h;
      const int half = mp / 2;
      double binom = 1.0;
      for (int p = 0; p <= half; ++p) {
        A[index_of(2 * p, mp - 2 * p) * S::LDA + C0 + LABFM_OP_HYP] = binom / hp;
        binom = binom * static_cast<double>(half - p) / static_cast<double>(p + 1);
      }
    }
    s_flag = 0;
  }
  __syncthreads();

  // ---- 3: LU with partial pivoting on [M~ | C~] -----------------------------
  // columns of the augmented matrix: 0..n-1 (M~) and NMAX..NMAX+5 (C~)
  int st = (K < n) ? LABFM_NODE_FEW_NEIGHBOURS : LABFM_NODE_OK;
  bool singular = false;
  for (int c = 0; c < n; ++c) {
    // pivot: largest |A[r][c]|, r >= c, smallest r on ties
    double best = -1.0;
    int bi = n;
    for (int r = c + lane; r < n; r += 64) {
      const double v = fabs(A[r * S::LDA + c]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (!(best > 0.0)) {  // zero pivot (or a non-finite column)
      singular = true;
      break;
    }
    // swap rows c and bi over the columns still in play
    if (bi != c) {
      for (int jj = c + lane; jj < n; jj += 64) {
        const double t0 = A[c * S::LDA + jj];
        A[c * S::LDA + jj] = A[bi * S::LDA + jj];
        A[bi * S::LDA + jj] = t0;
      }
      if (lane < LABFM_NUM_OPS) {
        const int jj = S::NMAX + lane;
        const double t0 = A[c * S::LDA + jj];
        A[c * S::LDA + jj] = A[bi * S::LDA + jj];
        A[bi * S::LDA + jj] = t0;
      }
    }
    __syncthreads();
    const double piv = A[c * S::LDA + c];
    // multipliers l_r = A[r][c] / pivot, kept in column c
    for (int r = c + 1 + lane; r < n; r += 64) A[r * S::LDA + c] = A[r * S::LDA + c] / piv;
    __syncthreads();
    // trailing update, one lane per column (M~ columns c+1..n-1 and the RHS)
    const int width = (n - c - 1) + LABFM_NUM_OPS;
    for (int t = lane; t < width; t += 64) {
      const int jj = (t < n - c - 1) ? (c + 1 + t) : (S::NMAX + t - (n - c - 1));
      const double ucj = A[c * S::LDA + jj];
      int r = c + 1;
      for (; r + 3 < n; r += 4) {
        const double l0 = A[r * S::LDA + c], l1 = A[(r + 1) * S::LDA + c];
        const double l2 = A[(r + 2) * S::LDA + c], l3 = A[(r + 3) * S::LDA + c];
        A[r * S::LDA + jj] -= l0 * ucj;
        A[(r + 1) * S::LDA + jj] -= l1 * ucj;
        A[(r + 2) * S::LDA + jj] -= l2 * ucj;
        A[(r + 3) * S::LDA + jj] -= l3 * ucj;
      }
      for (; r < n; ++r) A[r * S::LDA + jj] -= A[r * S::LDA + c] * ucj;
    }
    __syncthreads();
  }

  if (singular) {
    for (int k = lane; k < K; k += 64)
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const int r = op_row(rows, d);
        if (r == kNoRow) continue;
        w[r * nnz + e0 + k] = 0.0;
        if (w32) w32[r * w32_stride(nnz) + e0 + k] = 0.0f;
      }
    if (lane == 0) {
      kappa[i] = 0.0;
      status[i] = LABFM_NODE_SINGULAR;
      if (rowsum)
        for (int d = 0; d < LABFM_NUM_OPS; ++d)
          if (op_row(rows, d) != kNoRow) rowsum[op_row(rows, d) * (long long)nnodes + i] = 0.0;
      if (mom32)
        for (int k = 0; k < kMoments; ++k) mom32[k * (long long)nnodes + i] = 0.0f;
    }
    return;
  }

  // ---- 4: back substitution U Psi = C' (in place in the RHS columns) ------
  for (int c = n - 1; c >= 0; --c) {
    if (lane < LABFM_NUM_OPS) {
      const int jj = S::NMAX + lane;
      A[c * S::LDA + jj] = A[c * S::LDA + jj] / A[c * S::LDA + c];
    }
    __syncthreads();
    for (int t = lane; t < c * LABFM_NUM_OPS; t += 64) {
      const int r = t / LABFM_NUM_OPS, d = t - r * LABFM_NUM_OPS;
      const int jj = S::NMAX + d;
      A[r * S::LDA + jj] -= A[r * S::LDA + c] * A[c * S::LDA + jj];
    }
    __syncthreads();
  }

  // ---- 5: weights, filter calibration, row sums ----------------------------
  // one lane per neighbour; its Hermite values go to its own LDS row so the
  // loop over moments can index them at run time
  double* hx = &H[lane * S::HW];
  double* hy = hx + (MMAX + 1);
  const double kf = 2.0 * M_PI / (3.0 * s);
  double f0 = 0.0;
  double rs[LABFM_NUM_OPS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double mo[kMoments] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 64) {
    const int k = k0 + lane;
    if (k < K) {
      const int j = col[e0 + k];
      const double dx = wrap_axis(x[j] - xi, box.Lx, px);
      const double dy = wrap_axis(y[j] - yi, box.Ly, py);
      const double xs = dx / h, ys = dy / h;
      const double psi = wendland_c2(sqrt(xs * xs + ys * ys));
      {
        double a0 = 1.0, a1 = xs, b0 = 1.0, b1 = ys;
        hx[0] = 1.0;
        hy[0] = 1.0;
        hx[1] = xs;
        hy[1] = ys;
        for (int a = 1; a < m; ++a) {
          const double a2 = xs * a1 - static_cast<double>(a) * a0;
          const double b2 = ys * b1 - static_cast<double>(a) * b0;
          a0 = a1;
          a1 = a2;
          b0 = b1;
          b1 = b2;
          hx[a + 1] = a2;
          hy[a + 1] = b2;
        }
      }
      double wd[LABFM_NUM_OPS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int p = 0;
      for (int deg = 1; deg <= m; ++deg) {
        for (int b = 0; b <= deg; ++b, ++p) {
          const double Wq = hx[deg - b] * hy[b];
          const double* psi_row = &A[p * S::LDA + S::NMAX];
#pragma unroll
          for (int d = 0; d < LABFM_NUM_OPS; ++d) wd[d] += Wq * psi_row[d];
        }
      }
      const long long e = e0 + k;
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const double v = psi * wd[d];
        const int r = op_row(rows, d);
        if (r != kNoRow) {
          w[r * nnz + e] = v;
          if (w32) w32[r * w32_stride(nnz) + e] = static_cast<float>(v);
        }
        rs[d] += v;
      }
#pragma unroll
      for (int d = LABFM_OP_L; d <= LABFM_OP_XY; ++d) {
        const double v32 = static_cast<double>(static_cast<float>(psi * wd[d]));
        mo[2 * (d - LABFM_OP_L)] += v32 * dx;
        mo[2 * (d - LABFM_OP_L) + 1] += v32 * dy;
      }
      const double phi = 1.0 - cos(kf * dx) * cos(kf * dy);
      f0 += phi * (psi * wd[LABFM_OP_HYP]);
    }
  }
  f0 = group_sum<64>(f0);
#pragma unroll
  for (int d = 0; d < LABFM_NUM_OPS; ++d) rs[d] = group_sum<64>(rs[d]);
#pragma unroll
  for (int k = 0; k < kMoments; ++k) mo[k] = group_sum<64>(mo[k]);
  if (lane == 0) {
    if (mom32)
#pragma unroll
      for (int k = 0; k < kMoments; ++k) mom32[k * (long long)nnodes + i] = static_cast<float>(mo[k]);
    const bool bad = !isfinite(f0) || f0 == 0.0;
    kappa[i] = bad ? 0.0 : 2.0 / (3.0 * f0);
    if (st == LABFM_NODE_OK && bad) st = LABFM_NODE_BAD_FILTER;
    status[i] = static_cast<int8_t>(st);
    if (rowsum)
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d)
        if (op_row(rows, d) != kNoRow) rowsum[op_row(rows, d) * (long long)nnodes + i] = rs[d];
  }
}

// ---------------------------------------------------------------------------
// Four wavefronts per node
// ---------------------------------------------------------------------------
//
// The same steps with a 256-thread workgroup per node: wave 0 builds the
// basis tables of 16 neighbours at a time; the four waves share the MFMA tiles
// of M~ (tile t goes to wave t mod 4); the LU's trailing updates, the back
// substitution and the weights run over all 256 threads; per-node sums are
// reduced in a fixed order (bitwise reproducible). Used one workgroup per
// node, or persistently: workgroups take node indices from a work list
// (heaviest orders first) through an atomic counter until it is exhausted.

struct BuildArgs {
  const double* x;
  const double* y;
  const double* h;
  const double* s;
  const int8_t* order;
  int n;
  labfm_box box;
  const int* row_ptr;
  const int* col;
  long long nnz;
  double* w;
  float* w32;
  float* mom32;
  double* kappa;
  double* rowsum;
  int8_t* status;
  unsigned rows;  // output row of each operator (op_row)
  // the rows kernel skips nodes whose flag is 0 (the stencil optimiser's
  // passes); null: every node is built
  const int8_t* active = nullptr;
};

constexpr int kBlock = 256;

template <int MMAX>
struct BlockSmem {
  using S = Shape<MMAX>;
  // [M | C] from the end of the assembly to the end of the back substitution.
  // Before it (assembly) and after it (weights) the same storage holds the
  // basis tables of 16 neighbours (T) and, in the weights phase, the
  // per-neighbour-slot partial sums (part: 6 row sums, F0, and at 8..13 the
  // first moments of the float32 weights). This keeps a workgroup of m = 10
  // within a quarter of the CU's LDS (four resident).
  static constexpr int kAliased = kChunk * S::TABLE + kChunk * 16 + 4 * kChunk;
  static constexpr int kSize = S::NMAX * S::LDA > kAliased ? S::NMAX * S::LDA : kAliased;
  double A[kSize];
  double psi[S::NMAX * LABFM_NUM_OPS];  // the solution, copied out of A
  int qa[S::NMAX], qb[S::NMAX];
  unsigned long long key[3];  // pivot keys of three consecutive columns
  double rinv;                 // 1 / pivot of the pair's first column (LU)
  int next;
  __device__ double* T() { return A; }
  __device__ double* part() { return A + kChunk * S::TABLE; }
  // weights phase: offsets and filter cosines of the chunk's neighbours
  __device__ double* nb() { return A + kChunk * S::TABLE + kChunk * 16; }
};

// Coordinates of one neighbour per table lane, fetched ahead of their chunk:
// the column index two chunks ahead and the coordinates one chunk ahead, so
// that no dependent global load sits between a chunk's barrier and its
// tables (the LDS-only barriers leave these loads in flight).
struct NbrPrefetch {
  int j2;          // column index of the lane's neighbour two chunks ahead (-1: none)
  double x1, y1;   // coordinates of its neighbour one chunk ahead
  bool v1;
  __device__ void init(const BuildArgs& g, int e0, int K, int kk) {
    v1 = kk < K;
    const int j = v1 ? g.col[e0 + kk] : 0;
    x1 = v1 ? g.x[j] : 0.0;
    y1 = v1 ? g.y[j] : 0.0;
    j2 = (kChunk + kk < K) ? g.col[e0 + kChunk + kk] : -1;
  }
  // this chunk's coordinates (false: no neighbour); issues the next loads
  __device__ bool advance(const BuildArgs& g, int e0, int K, int k0, int kk, double& xj,
                          double& yj) {
    xj = x1;
    yj = y1;
    const bool v = v1;
    v1 = j2 >= 0;
    x1 = v1 ? g.x[j2] : 0.0;
    y1 = v1 ? g.y[j2] : 0.0;
    const int k3 = k0 + 2 * kChunk + kk;
    j2 = (k3 < K) ? g.col[e0 + k3] : -1;
    return v;
  }
};

// Every value that steers control flow around a barrier is made wave-uniform
// with readfirstlane (all lanes hold the same value): with conditions the
// compiler cannot prove uniform, it may structure the loops so that the
// waves of the workgroup pass through different sequences of barriers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier that orders LDS only: the workgroup shares no global
// data within a node (positions are read-only, each weight is written by one
// thread), so outstanding global loads and stores stay in flight across it
// (a full __syncthreads waits for all of them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// a / b for 0 <= a <= 256 and 1 <= b <= 128 (no integer divide instruction):
// (a + 1/2) / b is at least 1/(2b) away from an integer, far more than the
// float32 rounding of (a + 1/2) * rcp(b).
__device__ __forceinline__ int small_div(int a, int b) {
  return static_cast<int>((static_cast<float>(a) + 0.5f) *
                          __builtin_amdgcn_rcpf(static_cast<float>(b)));
}

// Pivot key of a candidate a at row r: the bits of |a| (ordered like the
// values, |a| >= 0) with the 7 lowest mantissa bits replaced by 127 - r, so
// the largest key is the largest |a| and, among values equal to 2^-45
// relative, the first row. Rows are < 128 (n <= 65).
__device__ __forceinline__ unsigned long long pivot_key(double a, int r) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(fabs(a)));
  return (b & ~0x7Full) | static_cast<unsigned long long>(static_cast<unsigned>(127 - r));
}

// Assembles [M~ | C~] of node i (order m, n moments, K neighbours from e0,
// stencil scale h) in sm.A: basis tables of 16-neighbour chunks in LDS and
// the moment matrix M~ = sum_j X~_j W_j^T on the FP64 matrix cores, then the
// right-hand sides C~^d = C^d h^-(a+b) of the six operators. Ends with a
// barrier.
template <int MMAX>
__device__ void assemble_system(const BuildArgs& g, int i, int m, int n, int e0, int K, double h,
                                BlockSmem<MMAX>& sm, int tid) {
  using S = Shape<MMAX>;
  constexpr int TPW = (S::NB * S::NB + 3) / 4;  // MFMA tiles per wave
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nb = (n + 15) / 16;
  const double xi = g.x[i], yi = g.y[i];
  const int px = g.box.periodic_x, py = g.box.periodic_y;
  for (int p = tid; p < n; p += kBlock) exponents_of(p, sm.qa[p], sm.qb[p]);
  // the zero entries (operands of moment indices beyond n); the tables
  // written below stop short of them
  for (int k = tid; k < kChunk; k += kBlock) sm.T()[k * S::TABLE + S::ZERO] = 0.0;
  lds_barrier();

  // ---- basis tables and MFMA assembly --------------------------------------
  int tP[TPW], tQ[TPW];
  // LDS offsets of this lane's A and B operands in a neighbour's tables
  // (the zero entry for a moment index beyond n: the operand is 0 * 0)
  int oa[TPW], ob[TPW], oc[TPW], od[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int t = wave + 4 * k;
    tP[k] = (t < nb * nb) ? t / nb : -1;
    tQ[k] = (t < nb * nb) ? t % nb : -1;
    const int p = tP[k] * 16 + (lane & 15);
    const int q = tQ[k] * 16 + (lane & 15);
    const bool pok = tP[k] >= 0 && p < n, qok = tQ[k] >= 0 && q < n;
    oa[k] = pok ? sm.qa[p] : S::ZERO;
    ob[k] = pok ? S::TW + sm.qb[p] : S::ZERO;
    oc[k] = qok ? 2 * S::TW + sm.qa[q] : S::ZERO;
    od[k] = qok ? 3 * S::TW + sm.qb[q] : S::ZERO;
  }
  const double hinv = 1.0 / h;
  double4_t acc[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) acc[k] = double4_t{0.0, 0.0, 0.0, 0.0};
  // table lanes: lanes 0..31 of wavefronts 0 and 1, two per neighbour (x and
  // y); wavefront 0 writes the Hermite tables, wavefront 1 the monomial ones,
  // so the two kinds are computed side by side rather than one after the other
  const bool tab_lane = tid < 128 && lane < 32;
  NbrPrefetch pf;
  if (tab_lane) pf.init(g, e0, K, lane >> 1);
  for (int k0 = 0; k0 < K; k0 += kChunk) {
    if (tab_lane) {
      const int kk = lane >> 1, t = (lane & 1) + (wave == 0 ? 2 : 0);
      double xj, yj;
      const bool have = pf.advance(g, e0, K, k0, kk, xj, yj);
      double* tab = &sm.T()[kk * S::TABLE + t * S::TW];
      if (have) {
        const double dx = wrap_axis(xj - xi, g.box.Lx, px);
        const double dy = wrap_axis(yj - yi, g.box.Ly, py);
        const double xs = dx * hinv, ys = dy * hinv;
        const double z = (t == 0 || t == 2) ? xs : ys;
        if (t < 2) {
          double v = 1.0;
          tab[0] = 1.0;
#pragma unroll
          for (int a = 1; a <= MMAX; ++a) {
            v = v * z * (1.0 / static_cast<double>(a));  // z^a / a!
            tab[a] = v;
          }
        } else {
          const double psi = (t == 2) ? wendland_c2(sqrt(xs * xs + ys * ys)) : 1.0;
          double h0 = 1.0, h1 = z;
          tab[0] = psi;
          tab[1] = psi * z;
#pragma unroll
          for (int a = 1; a < MMAX; ++a) {
            const double h2 = z * h1 - static_cast<double>(a) * h0;
            h0 = h1;
            h1 = h2;
            tab[a + 1] = psi * h2;
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a <= MMAX; ++a) tab[a] = 0.0;
      }
    }
    lds_barrier();
#pragma unroll
    for (int ks = 0; ks < kChunk / 4; ++ks) {
      const double* tk = &sm.T()[(ks * 4 + (lane >> 4)) * S::TABLE];
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        if (tP[k] >= 0) {  // wave-uniform
          const double av = tk[oa[k]] * tk[ob[k]];
          const double bv = tk[oc[k]] * tk[od[k]];
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[k], 0, 0, 0);
        }
      }
    }
    lds_barrier();
  }
  // element v of lane l holds D[l/16 + 4v][l%16] of its tile
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    if (tP[k] >= 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = tP[k] * 16 + (lane >> 4) + 4 * v;
        const int c = tQ[k] * 16 + (lane & 15);
        if (r < n && c < n) sm.A[r * S::LDA + c] = acc[k][v];
      }
    }
  }
  for (int t = tid; t < n * LABFM_NUM_OPS; t += kBlock)
    sm.A[(t / LABFM_NUM_OPS) * S::LDA + S::NMAX + t % LABFM_NUM_OPS] = 0.0;
  lds_barrier();
  if (tid == 0) {
    const double h1 = 1.0 / h, h2 = 1.0 / (h * h);
    const int C0 = S::NMAX;
    sm.A[0 * S::LDA + C0 + LABFM_OP_X] = h1;
    sm.A[1 * S::LDA + C0 + LABFM_OP_Y] = h1;
    if (m >= 2) {
      sm.A[index_of(2, 0) * S::LDA + C0 + LABFM_OP_L] = h2;
      sm.A[index_of(0, 2) * S::LDA + C0 + LABFM_OP_L] = h2;
      sm.A[index_of(2, 0) * S::LDA + C0 + LABFM_OP_XX] = h2;
      sm.A[index_of(1, 1) * S::LDA + C0 + LABFM_OP_XY] = h2;
    }
    const int mp = (m % 2 == 0) ? m : m - 1;
    if (mp >= 2) {
      double hp = 1.0;
      for (int k = 0; k < mp; ++k) hp *= h;
      const int half = mp / 2;
      double binom = 1.0;
      for (int p = 0; p <= half; ++p) {
        sm.A[index_of(2 * p, mp - 2 * p) * S::LDA + C0 + LABFM_OP_HYP] = binom / hp;
        binom = binom * static_cast<double>(half - p) / static_cast<double>(p + 1);
      }
    }
  }
  lds_barrier();

}

// LU with partial pivoting of [M~ | C~] in sm.A and back substitution: the
// solution Psi^d is left in the right-hand-side columns. Returns true (the
// same in every thread) for a zero or non-finite pivot column. Ends with a
// barrier.
template <int MMAX>
__device__ bool factor_solve(int n, BlockSmem<MMAX>& sm, int tid) {
  using S = Shape<MMAX>;
  bool singular = false;
  // ---- LU with partial pivoting on [M~ | C~] --------------------------------
  // Columns are eliminated in pairs (c, c+1), with the arithmetic of two
  // single-column steps in their order:
  //   A: the pivot of column c is known (its key); rows c and bi swap, and
  //      wavefront 0 applies step c to column c+1 alone (one row per lane),
  //      proposing the pivot of column c+1 (LDS atomic max of the keys);
  //   B: rows c+1 and bi1 swap, and every thread applies steps c and c+1 to
  //      its column of the rest (columns c+2.. and the right-hand sides):
  //      a <- a - l_c u_c, then a <- a - l_{c+1} u_{c+1}, with u_{c+1} the
  //      pivot row after step c, which each thread forms for its column.
  //      Column c+2 (the next pivot column) is done by wavefront 0, one row
  //      per lane, which also proposes its pivot.
  // Each half ends with a barrier (and a swap adds one), so the barriers are
  // as many as with single columns while the bulk update, and its fixed
  // cost, runs once per pair. Row c+1 after step c is written to a staging
  // row (sm.psi, unused until the solution is copied out) and moved into A
  // during the next pair, since its old values are read throughout B. The
  // multipliers are not kept (the right-hand sides are eliminated along).
  // Key slots: the sub-step for column s reads key[s % 3], clears
  // key[(s + 2) % 3] and proposes into key[(s + 1) % 3].
  if (tid < 3) sm.key[tid] = 0ull;
  lds_barrier();
  for (int r = tid; r < n; r += kBlock) atomicMax(&sm.key[0], pivot_key(sm.A[r * S::LDA], r));
  lds_barrier();
  double* stage = sm.psi;
  int staged = -1;  // row whose step-c values wait in the staging row, or -1
  for (int c = 0; c < n; c += 2) {
    const unsigned long long kc = uniform64(sm.key[c % 3]);
    const unsigned long long vb = kc & ~0x7Full;
    if (vb == 0ull || vb >= 0x7FF0000000000000ull) {  // zero or non-finite column
      singular = true;
      break;
    }
    const int bi = 127 - static_cast<int>(kc & 0x7Full);
    if (tid == 0) sm.key[(c + 2) % 3] = 0ull;
    // the previous pair's row c-1 (columns c.. and the right-hand sides) by
    // wavefronts 1-3; rows >= c are all that this pair touches
    if (staged >= 0 && tid >= 64) {
      const int w1 = (n - c) + LABFM_NUM_OPS;
      for (int t = tid - 64; t < w1; t += kBlock - 64) {
        const int jj = (t < n - c) ? (c + t) : (S::NMAX + t - (n - c));
        sm.A[staged * S::LDA + jj] = stage[t];
      }
    }
    const int width = (n - c) + LABFM_NUM_OPS;  // columns c..n-1 and the RHS
    if (bi != c) {
      for (int t = tid; t < width; t += kBlock) {
        const int jj = (t < n - c) ? (c + t) : (S::NMAX + t - (n - c));
        const double t0 = sm.A[c * S::LDA + jj];
        sm.A[c * S::LDA + jj] = sm.A[bi * S::LDA + jj];
        sm.A[bi * S::LDA + jj] = t0;
      }
      lds_barrier();
    }
    if (c + 1 == n) {  // last column alone: nothing below it
      staged = -1;
      lds_barrier();
      break;
    }
    // ---- A: column c+1 (rows c+1..n-1, at most 64: one per lane of wave 0);
    // wavefront 0 also forms 1 / pivot for the other wavefronts
    if (tid < 64) {
      const double inv = 1.0 / sm.A[c * S::LDA + c];
      if (tid == 0) sm.rinv = inv;
      const int r = c + 1 + tid;
      if (r < n) {
        const double v = fma(-(sm.A[r * S::LDA + c] * inv), sm.A[c * S::LDA + c + 1],
                             sm.A[r * S::LDA + c + 1]);
        sm.A[r * S::LDA + c + 1] = v;
        atomicMax(&sm.key[(c + 1) % 3], pivot_key(v, r));
      }
    }
    lds_barrier();
    const double inv0 = sm.rinv;
    // ---- B: pivot of column c+1, then both steps on the rest
    const int c1 = c + 1;
    const unsigned long long kc1 = uniform64(sm.key[c1 % 3]);
    const unsigned long long vb1 = kc1 & ~0x7Full;
    if (vb1 == 0ull || vb1 >= 0x7FF0000000000000ull) {
      singular = true;
      break;
    }
    const int bi1 = 127 - static_cast<int>(kc1 & 0x7Full);
    if (tid == 0) sm.key[(c1 + 2) % 3] = 0ull;
    if (bi1 != c1) {
      for (int t = tid; t < width; t += kBlock) {
        const int jj = (t < n - c) ? (c + t) : (S::NMAX + t - (n - c));
        const double t0 = sm.A[c1 * S::LDA + jj];
        sm.A[c1 * S::LDA + jj] = sm.A[bi1 * S::LDA + jj];
        sm.A[bi1 * S::LDA + jj] = t0;
      }
      lds_barrier();
    }
    const double inv1 = 1.0 / sm.A[c1 * S::LDA + c1];
    const double l01 = sm.A[c1 * S::LDA + c] * inv0;  // row c+1's multiplier in step c
    const int nc = n - c - 2;                          // matrix columns right of c+1
    // column c+2, the next pivot column, by wavefront 0 (one row per lane,
    // at most 63), with the pivot proposals; the rest of the pass has none
    if (nc > 0) {
      const int r = c + 2 + tid;
      if (r < n) {
        const int j = c + 2;
        const double u0 = sm.A[c * S::LDA + j];
        const double u1 = fma(-l01, u0, sm.A[c1 * S::LDA + j]);
        if (tid == 0) stage[0] = u1;
        const double x = fma(-(sm.A[r * S::LDA + c] * inv0), u0, sm.A[r * S::LDA + j]);
        const double v = fma(-(sm.A[r * S::LDA + c1] * inv1), u1, x);
        sm.A[r * S::LDA + j] = v;
        atomicMax(&sm.key[(c1 + 1) % 3], pivot_key(v, r));
      }
    }
    // columns c+3.. and the right-hand sides: slot t of the pair's columns
    // (t < nc: column c+2+t, else right-hand side t-nc), t from off
    const int off = nc > 0 ? 1 : 0;
    const int W = nc + LABFM_NUM_OPS - off;
    const int groups = small_div(kBlock, W);
    const int rg = small_div(tid, W);
    if (rg < groups) {
      const int t = tid - rg * W + off;
      const int jj = (t < nc) ? (c + 2 + t) : (S::NMAX + t - nc);
      const double u0 = sm.A[c * S::LDA + jj];
      const double u1 = fma(-l01, u0, sm.A[c1 * S::LDA + jj]);
      if (rg == 0) stage[t] = u1;
      int r = c + 2 + rg;
#pragma unroll 1
      for (; r + groups < n; r += 2 * groups) {
        const int r1 = r + groups;
        const double a0 = sm.A[r * S::LDA + c], b0 = sm.A[r * S::LDA + c1];
        const double x0 = sm.A[r * S::LDA + jj];
        const double a1 = sm.A[r1 * S::LDA + c], b1 = sm.A[r1 * S::LDA + c1];
        const double x1 = sm.A[r1 * S::LDA + jj];
        sm.A[r * S::LDA + jj] = fma(-(b0 * inv1), u1, fma(-(a0 * inv0), u0, x0));
        sm.A[r1 * S::LDA + jj] = fma(-(b1 * inv1), u1, fma(-(a1 * inv0), u0, x1));
      }
      if (r < n) {
        const double x = fma(-(sm.A[r * S::LDA + c] * inv0), u0, sm.A[r * S::LDA + jj]);
        sm.A[r * S::LDA + jj] = fma(-(sm.A[r * S::LDA + c1] * inv1), u1, x);
      }
    }
    staged = c1;
    lds_barrier();
  }
  if (!singular && staged >= 0) {
    // the last pair's row c+1 (columns from n and the right-hand sides)
    const int c = staged + 1;
    const int w1 = (n - c) + LABFM_NUM_OPS;
    for (int t = tid; t < w1; t += kBlock) {
      const int jj = (t < n - c) ? (c + t) : (S::NMAX + t - (n - c));
      sm.A[staged * S::LDA + jj] = stage[t];
    }
    lds_barrier();
  }
  if (!singular) {
  // ---- back substitution ----------------------------------------------------
  // Rows c and c-1 per pass: six threads solve row c, apply it to row c-1
  // and solve that; then the rows above take both updates, in the order of
  // two single-row passes (half the barriers).
  for (int c = n - 1; c >= 0; c -= 2) {
    if (tid < LABFM_NUM_OPS) {
      const int jj = S::NMAX + tid;
      const double p = sm.A[c * S::LDA + jj] / sm.A[c * S::LDA + c];
      sm.A[c * S::LDA + jj] = p;
      if (c >= 1) {
        double x = sm.A[(c - 1) * S::LDA + jj];
        x -= sm.A[(c - 1) * S::LDA + c] * p;
        sm.A[(c - 1) * S::LDA + jj] = x / sm.A[(c - 1) * S::LDA + c - 1];
      }
    }
    lds_barrier();
    for (int t = tid; t < (c - 1) * LABFM_NUM_OPS; t += kBlock) {
      const int r = t / LABFM_NUM_OPS, d = t - r * LABFM_NUM_OPS;
      const int jj = S::NMAX + d;
      double v = sm.A[r * S::LDA + jj];
      v -= sm.A[r * S::LDA + c] * sm.A[c * S::LDA + jj];
      v -= sm.A[r * S::LDA + c - 1] * sm.A[(c - 1) * S::LDA + jj];
      sm.A[r * S::LDA + jj] = v;
    }
    lds_barrier();
  }

  }
  return singular;
}

template <int MMAX>
__device__ void build_node_block(int i_in, const BuildArgs& g, BlockSmem<MMAX>& sm, int tid) {
  using S = Shape<MMAX>;
  const int lane = tid & 63;
  const int i = uniform(i_in);
  const int m = uniform(g.order[i]);
  const int e0 = uniform(g.row_ptr[i]);
  const int K = uniform(g.row_ptr[i + 1]) - e0;
  // one exit: every path below ends at the final barrier, and every branch
  // around a barrier depends on wave-uniform values only
  const bool valid = (m >= 1 && m <= MMAX);
  bool singular = false;
  if (valid) {
  const int n = moments_of(m);
  const double xi = g.x[i], yi = g.y[i], h = g.h[i], s = g.s[i];
  const int px = g.box.periodic_x, py = g.box.periodic_y;
  const double hinv = 1.0 / h;
  assemble_system<MMAX>(g, i, m, n, e0, K, h, sm, tid);
  int st = (K < n) ? LABFM_NODE_FEW_NEIGHBOURS : LABFM_NODE_OK;
  singular = factor_solve<MMAX>(n, sm, tid);
  if (!singular) {

  // ---- weights, filter calibration, row sums --------------------------------
  // the solution leaves A, whose storage the tables and sums take over
  for (int t = tid; t < n * LABFM_NUM_OPS; t += kBlock)
    sm.psi[t] = sm.A[(t / LABFM_NUM_OPS) * S::LDA + S::NMAX + t % LABFM_NUM_OPS];
  lds_barrier();
  // threads 0..191: neighbour slot k = t/12, operator d = (t/2)%6, half = t%2
  const int slot = tid / 12, dop = (tid / 2) % 6, half = tid & 1;
  const double kf = 2.0 * M_PI / (3.0 * s);
  double rs = 0.0, f0 = 0.0, mx = 0.0, my = 0.0;
  double* nbx = sm.nb();  // [0, 16): dx, [16, 32): dy, [32, 48): cos(kf dx), [48, 64): cos(kf dy)
  // table lanes as in the assembly: wavefront 0 writes the psi He_a and He_b
  // tables, wavefront 1 each neighbour's offsets and filter cosines
  const bool tab_lane = tid < 128 && lane < 32;
  NbrPrefetch pf;
  if (tab_lane) pf.init(g, e0, K, lane >> 1);
  for (int k0 = 0; k0 < K; k0 += kChunk) {
    if (tab_lane) {
      const int kk = lane >> 1, t = (lane & 1) + (tid < 64 ? 2 : 0);
      double xj, yj;
      const bool have = pf.advance(g, e0, K, k0, kk, xj, yj);
      double* tab = &sm.T()[kk * S::TABLE + t * S::TW];
      const double dx = have ? wrap_axis(xj - xi, g.box.Lx, px) : 0.0;
      const double dy = have ? wrap_axis(yj - yi, g.box.Ly, py) : 0.0;
      if (t < 2) {
        const double d = (t == 0) ? dx : dy;
        nbx[t * kChunk + kk] = d;
        nbx[(2 + t) * kChunk + kk] = have ? cos(kf * d) : 1.0;
      } else {
        if (have) {
          const double xs = dx * hinv, ys = dy * hinv;
          const double z = (t == 2) ? xs : ys;
          const double psi = (t == 2) ? wendland_c2(sqrt(xs * xs + ys * ys)) : 1.0;
          double h0 = 1.0, h1 = z;
          tab[0] = psi;
          tab[1] = psi * z;
#pragma unroll
          for (int a = 1; a < MMAX; ++a) {
            const double h2 = z * h1 - static_cast<double>(a) * h0;
            h0 = h1;
            h1 = h2;
            tab[a + 1] = psi * h2;
          }
        } else {
#pragma unroll
          for (int a = 0; a <= MMAX; ++a) tab[a] = 0.0;
        }
      }
    }
    lds_barrier();
    if (tid < 12 * kChunk) {
      const int k = k0 + slot;
      const double* tk = &sm.T()[slot * S::TABLE];
      double acc = 0.0;
#pragma unroll 4
      for (int q = half; q < n; q += 2)
        acc += (tk[2 * S::TW + sm.qa[q]] * tk[3 * S::TW + sm.qb[q]]) *
               sm.psi[q * LABFM_NUM_OPS + dop];
      acc += __shfl_xor(acc, 1);
      if (k < K) {
        if (half == 0) {
          const long long e = e0 + k;
          const int r = op_row(g.rows, dop);
          if (r != kNoRow) {
            g.w[r * g.nnz + e] = acc;
            if (g.w32) g.w32[r * w32_stride(g.nnz) + e] = static_cast<float>(acc);
          }
          if (dop == LABFM_OP_HYP) {
            f0 += (1.0 - nbx[2 * kChunk + slot] * nbx[3 * kChunk + slot]) * acc;
          } else if (dop >= LABFM_OP_L && dop <= LABFM_OP_XY) {
            const double v32 = static_cast<double>(static_cast<float>(acc));
            mx += v32 * nbx[slot];
            my += v32 * nbx[kChunk + slot];
          }
        }
        rs += acc;
      }
    }
    lds_barrier();
  }
  // deterministic reduction over the 16 neighbour slots
  if (tid < 12 * kChunk && half == 0) {
    sm.part()[slot * 16 + dop] = rs;
    if (dop == LABFM_OP_HYP) sm.part()[slot * 16 + 6] = f0;
    if (dop >= LABFM_OP_L && dop <= LABFM_OP_XY) {
      sm.part()[slot * 16 + 8 + 2 * (dop - LABFM_OP_L)] = mx;
      sm.part()[slot * 16 + 9 + 2 * (dop - LABFM_OP_L)] = my;
    }
  }
  lds_barrier();
  if (tid >= 8 && tid < 8 + kMoments && g.mom32) {
    double v = 0.0;
    for (int k = 0; k < kChunk; ++k) v += sm.part()[k * 16 + tid];
    g.mom32[(tid - 8) * (long long)g.n + i] = static_cast<float>(v);
  }
  if (tid < 7) {
    double v = 0.0;
    for (int k = 0; k < kChunk; ++k) v += sm.part()[k * 16 + tid];
    if (tid < 6) {
      if (g.rowsum && op_row(g.rows, tid) != kNoRow)
        g.rowsum[op_row(g.rows, tid) * (long long)g.n + i] = v;
    } else {
      const bool bad = !isfinite(v) || v == 0.0;
      g.kappa[i] = bad ? 0.0 : 2.0 / (3.0 * v);
      if (st == LABFM_NODE_OK && bad) st = LABFM_NODE_BAD_FILTER;
      g.status[i] = static_cast<int8_t>(st);
    }
  }
  }  // !singular
  }  // valid
  if (!valid || singular) {
    for (int k = tid; k < K; k += kBlock)
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const int r = op_row(g.rows, d);
        if (r == kNoRow) continue;
        g.w[r * g.nnz + e0 + k] = 0.0;
        if (g.w32) g.w32[r * w32_stride(g.nnz) + e0 + k] = 0.0f;
      }
    if (tid == 0) {
      g.kappa[i] = 0.0;
      g.status[i] = valid ? LABFM_NODE_SINGULAR : LABFM_NODE_BAD_ORDER;
      if (g.rowsum)
        for (int d = 0; d < LABFM_NUM_OPS; ++d)
          if (op_row(g.rows, d) != kNoRow) g.rowsum[op_row(g.rows, d) * (long long)g.n + i] = 0.0;
      if (g.mom32)
        for (int k = 0; k < kMoments; ++k) g.mom32[k * (long long)g.n + i] = 0.0f;
    }
  }
  lds_barrier();
}

// one workgroup per node of the list (or per node when list is null)
// Waves per SIMD for the workgroup-per-node kernel (measured): m = 8 runs
// eight workgroups per CU (its LDS just fits eight; 64 VGPRs, a few values
// spilled at the phase boundaries), m = 4 and 6 seven (at eight their spills
// cost more than the extra workgroup brings), m = 10 is bounded by its LDS
// (four workgroups).
template <int MMAX>
constexpr int block_waves() {
  return MMAX == 8 ? 8 : (MMAX < 8 ? 7 : 4);
}

template <int MMAX>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(block_waves<MMAX>())))
build_block_kernel(BuildArgs g, const int* __restrict__ list, int count) {
  __shared__ BlockSmem<MMAX> sm;
  const int k = blockIdx.x;
  if (k >= count) return;
  build_node_block<MMAX>(list ? list[k] : k, g, sm, threadIdx.x);
}

// Waves per SIMD that the workgroup-per-node kernel reaches for each MMAX (by
// its register and LDS use). The loop of the persistent kernel keeps more
// values live, and without this bound the register allocator would give it
// one resident workgroup per CU less.
template <int MMAX>
constexpr int persistent_waves() {
  return MMAX <= 8 ? 6 : 4;
}

// persistent: workgroups take list entries through *counter until exhausted
template <int MMAX>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(persistent_waves<MMAX>())))
build_persistent_kernel(BuildArgs g, const int* __restrict__ list, int count, int* counter) {
  __shared__ BlockSmem<MMAX> sm;
  for (;;) {
    if (threadIdx.x == 0) sm.next = atomicAdd(counter, 1);
    lds_barrier();
    const int k = uniform(sm.next);
    if (k >= count) break;  // the same value for every thread of the workgroup
    // ends with a barrier, so sm.next is read by all before it is rewritten
    // the thread index passes through an empty asm statement in every
    // iteration, so nothing derived from it is kept live across nodes (which
    // would cost registers and occupancy)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    build_node_block<MMAX>(list[k], g, sm, tid);
  }
}

// ---------------------------------------------------------------------------
// One wavefront per node, the system's rows in registers (orders 1..10)
// ---------------------------------------------------------------------------
//
// For n <= 64 moments the whole augmented system [M~ | C~] fits one row per
// lane: lane r keeps row r (n + 6 doubles, padded to an even count) in
// registers, so the factorisation needs no workgroup barrier and no LDS
// traffic for the trailing updates. Order 10 has n = 65: the pivot row of
// column 0 is chosen from the first 16-column strip of M~, before the rows
// reach the lanes, and kept in LDS; the other 64 rows fill the lanes, column
// 0 is eliminated with the row from LDS, and the 64 remaining columns run on
// 64 lanes as for the lower orders. Per node:
//   1. the basis tables of 16 neighbours at a time in LDS and M~ on the FP64
//      matrix cores, exactly as in the workgroup kernel (one wavefront
//      accumulates every 16x16 tile);
//   2. M~ goes to row-per-lane registers through LDS, one 16-column strip at
//      a time (a strip's accumulators die as its columns arrive); every lane
//      forms its own row of C~ from its monomial's exponents;
//   3. LU with partial pivoting, rows never swapped: at column c the pivot is
//      the row (lane) not yet used with the largest |a_rc|, compared exactly:
//      the high words of |a| (sign, exponent and 20 mantissa bits) are
//      reduced over the wave with DPP and read lanes, and only when several
//      rows share the largest high word are their low words reduced too; of
//      equal magnitudes the lowest lane wins. The
//      pivot row reaches the other lanes through scalar registers (v_readlane)
//      and the lanes not yet used subtract l_r = a_rc / u_cc times it (the
//      multiplier from the reciprocal of the pivot, as LAPACK's unblocked
//      factorisation forms it: a hardware reciprocal and one Newton step).
//      The right-hand sides are eliminated along. (Broadcasting the rows
//      through LDS instead makes every lane pull every value: 64 x 8 bytes per
//      value through the CU's shared LDS data path, which then bounds the
//      kernel.)
//   4. back substitution from the last column: every lane reads y_c and
//      1/u_cc from the pivot lane of column c (a ballot) and subtracts
//      (u_rc / u_cc) y_c from its right-hand sides; at the end each lane
//      forms its own x = y / u_cc and writes it into Psi in LDS;
//   5. one lane per neighbour: w^d_j = psi_j sum_q He_a(x_j) He_b(y_j) Psi^d_q
//      (Psi read from LDS a row at a time: there the reads cost less than
//      reading each row out of its lane, measured), then the float32 copy,
//      the filter calibration sum, the row sums and the first moments,
//      reduced over the wave in a fixed order. A last pass over at most 32
//      neighbours gives each neighbour two lanes, one per three operators.
// The register arrays are indexed by compile-time constants only (every loop
// over columns is unrolled), so the order is a template parameter.

template <int M>
struct RowShape {
  static constexpr int N = moments_of(M);
  static constexpr int NB = (N + 15) / 16;        // 16-wide MFMA tiles per side
  static constexpr int RC = ((N + LABFM_NUM_OPS) + 1) & ~1;  // row length, even
  // order 10: n = 65 rows, one more than the lanes (see step 3)
  static constexpr bool kExtra = N > 64;
  static_assert(N <= 65, "one row beyond the wavefront at most");
  static constexpr int TW = M + 1;                 // one basis table's length
  static constexpr int TABLE = 4 * TW + 1;         // four tables and a zero
  static constexpr int ZERO = 4 * TW;
  static constexpr int SS = 17;                    // strip row stride (doubles)
  static constexpr int kTable = kChunk * TABLE;
  static constexpr int kStrip = NB * 16 * SS;
  static constexpr int kPsi = N * LABFM_NUM_OPS;
  static constexpr int kShared = (kTable > kStrip ? (kTable > kPsi ? kTable : kPsi)
                                                  : (kStrip > kPsi ? kStrip : kPsi));
};

// LDS of the rows kernel: the basis tables during the assembly, then the
// strips that carry M~ into the lanes' registers, then the solution Psi (read
// by every lane in the weights phase).
template <int M>
struct alignas(16) RowSmem {
  double buf[RowShape<M>::kShared];
  // order 10: the pivot row of column 0 of [M~ | C~]
  double extra[RowShape<M>::kExtra ? RowShape<M>::RC : 2];
};

// Register fence: an empty asm statement that reads and writes v. Such
// statements keep their program order, so a value pinned after its update
// is computed there, not sunk to its next use (the compiler otherwise defers
// the trailing updates and the weight sums and keeps all their operands live
// in registers). It emits no instruction.
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)); }

// Largest 32-bit key of the wavefront, in every lane (all 64 lanes active):
// the max of each row of 16 lanes by DPP, then of row pairs and of the two
// halves by gfx950's permlane swaps (each lane sees its own and its
// partner's value in the swap's two results).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xF,
                                                               0xF, false)));  // quad [1,0,3,2]
  v = max(v, static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xF,
                                                               0xF, false)));  // quad [2,3,0,1]
  v = max(v, static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x141, 0xF,
                                                               0xF, false)));  // half-row mirror
  v = max(v, static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x140, 0xF,
                                                               0xF, false)));  // row mirror
  const auto rows = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = max(static_cast<unsigned>(rows[0]), static_cast<unsigned>(rows[1]));
  const auto halves = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return max(static_cast<unsigned>(halves[0]), static_cast<unsigned>(halves[1]));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) |
                                                     lo));
}

// Row r of C~ (the six right-hand sides C^d h^-(a+b)) for the monomial of
// exponents (a, b) of an order-m system.
__device__ __forceinline__ void rhs_row(int a, int b, int m, double h, double* c) {
  const double h1 = 1.0 / h, h2 = 1.0 / (h * h);
  c[LABFM_OP_X] = (a == 1 && b == 0) ? h1 : 0.0;
  c[LABFM_OP_Y] = (a == 0 && b == 1) ? h1 : 0.0;
  c[LABFM_OP_L] = (m >= 2 && ((a == 2 && b == 0) || (a == 0 && b == 2))) ? h2 : 0.0;
  c[LABFM_OP_XX] = (m >= 2 && a == 2 && b == 0) ? h2 : 0.0;
  c[LABFM_OP_XY] = (m >= 2 && a == 1 && b == 1) ? h2 : 0.0;
  const int mp = (m % 2 == 0) ? m : m - 1;
  double hyp = 0.0;
  if (mp >= 2 && a + b == mp && a % 2 == 0) {
    double hp = 1.0;
    for (int k = 0; k < mp; ++k) hp *= h;
    const int half = mp / 2;
    double binom = 1.0;  // binom(half, p) for p = a/2, built as the other kernels do
    for (int p = 0; p < a / 2; ++p)
      binom = binom * static_cast<double>(half - p) / static_cast<double>(p + 1);
    hyp = binom / hp;
  }
  c[LABFM_OP_HYP] = hyp;
}

// Wavefronts per SIMD the rows kernel is compiled for (its registers: the
// row, n + 6 doubles, and the assembly's accumulators). Measured on 262,144
// nodes: at m = 8 four waves (now 123 registers, no spills) took 6.89 ms
// against 7.06 ms at three when the choice was made; at m = 9 three waves
// (168 registers, 17 of them spilled) take 10.72 ms against 11.19 ms at two
// (200 registers, none spilled); five at m <= 6 gain nothing.
template <int M>
constexpr int rows_waves() {
  return M <= 8 ? 4 : (M == 9 ? 3 : 2);
}

// Order 10's first pivot row among its 65 rows: lane l holds row l's
// column-0 value c0 and every lane row 64's (v64). The largest |value|,
// compared exactly (high words, then low words on a tie), the lowest row on
// equal magnitudes.
__device__ __forceinline__ int first_pivot_of_65(double c0, double v64) {
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(fabs(c0)));
  const unsigned hi = static_cast<unsigned>(bits >> 32);
  const unsigned khi = wave_max_u32(hi);
  unsigned long long cand = __builtin_amdgcn_ballot_w64(hi == khi);
  if (__builtin_popcountll(cand) > 1) {
    const unsigned lo = hi == khi ? static_cast<unsigned>(bits) : 0u;
    const unsigned klo = wave_max_u32(lo);
    cand = __builtin_amdgcn_ballot_w64(hi == khi && lo == klo);
  }
  const int pl = static_cast<int>(__builtin_ctzll(cand));
  const double vl = readlane_f64(c0, pl);
  const double v = readlane_f64(v64, 0);
  // row 64 only when strictly larger
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v))) >
                 static_cast<unsigned long long>(__double_as_longlong(fabs(vl)))
             ? 64
             : pl;
}

// The build kernel's arguments read again from the kernel-argument segment
// (a BuildArgs passed as the kernel's first argument sits at its offset 0).
// The empty asm statement makes the pointer a new value, so the loads through
// it are issued where they are used rather than at the kernel's entry: values
// that the assembly reads need not then be kept (or spilled) across the LU,
// the kernel's register peak, for the weights.
typedef const __attribute__((address_space(4))) BuildArgs KernargBuildArgs;
__device__ __forceinline__ KernargBuildArgs* build_args_again() {
  KernargBuildArgs* p = (KernargBuildArgs*)(__builtin_amdgcn_kernarg_segment_ptr());
  asm volatile("" : "+s"(p));
  return p;
}

// Systems given to the rows kernel's LU and back substitution directly (its
// solve variant): row r of system k at sys + (k n + r)(n + 6), its n values
// of M~, then its six of C~.
struct SolveArgs {
  const double* sys = nullptr;
  int count = 0;
  double* psi = nullptr;     // [k][q][d]: the solution Psi
  int* pivot_row = nullptr;  // [k][c]: the row whose pivot column c took
  int8_t* status = nullptr;  // [k]: LABFM_NODE_OK or LABFM_NODE_SINGULAR
};

// One wavefront's work of the rows kernel: node list[blockIdx.x]'s build or,
// with kSolve, system blockIdx.x of sv through the same LU and back
// substitution (steps 3 and 4) in place of the assembly and the weights.
template <int M, bool kSolve>
__device__ __forceinline__ void rows_node(BuildArgs g, const int* __restrict__ list, int count,
                                          SolveArgs sv) {
  using S = RowShape<M>;
  constexpr int N = S::N, NB = S::NB, RC = S::RC, TW = S::TW;
  __shared__ RowSmem<M> sm;
  const int k_ = blockIdx.x;
  if (k_ >= count) return;
  const int lane = threadIdx.x;
  const int i = kSolve ? k_ : uniform(list ? list[k_] : k_);
  if (!kSolve && g.active && uniform(g.active[i]) == 0) return;
  const int e0 = kSolve ? 0 : uniform(g.row_ptr[i]);
  const int K = kSolve ? N : uniform(g.row_ptr[i + 1]) - e0;
  const double xi = kSolve ? 0.0 : g.x[i], yi = kSolve ? 0.0 : g.y[i];
  const double h = kSolve ? 1.0 : g.h[i], s = kSolve ? 1.0 : g.s[i];
  const int px = g.box.periodic_x, py = g.box.periodic_y;
  const double hinv = 1.0 / h;
  double* T = sm.buf;

  // lane l's row of [M~ | C~] (row myrow: l, or l + 1 from p0 on at order 10)
  double a[RC];
  int p0 = 64, myrow = lane;
  if constexpr (kSolve) {
    // the given system's rows where the assembly leaves a node's (order 10:
    // the first pivot row chosen as from the first strip, kept in LDS)
    constexpr int W = N + LABFM_NUM_OPS;
    const double* A = sv.sys + static_cast<long long>(k_) * N * W;
    if constexpr (S::kExtra) {
      p0 = first_pivot_of_65(A[static_cast<long long>(lane) * W], A[64LL * W]);
      myrow = lane + (lane >= p0 ? 1 : 0);
      for (int j = lane; j < RC; j += 64)
        sm.extra[j] = j < W ? A[static_cast<long long>(p0) * W + j] : 0.0;
    }
    const long long r = lane < N ? myrow : 0;
#pragma unroll
    for (int j = 0; j < RC; ++j) a[j] = (lane < N && j < W) ? A[r * W + j] : 0.0;
    lds_barrier();
  } else {
    // ---- 1, 2: basis tables, MFMA assembly, rows of M~ into registers ---------
    // exponents of this lane's moment index in each tile (row p or column q)
    int ea[NB], eb[NB];
#pragma unroll
    for (int P = 0; P < NB; ++P) {
      const int p = P * 16 + (lane & 15);
      if (p < N) {
        exponents_of(p, ea[P], eb[P]);
      } else {
        ea[P] = -1;
        eb[P] = -1;
      }
    }
    // Column tiles per pass over the neighbours: all of them up to order 9;
    // at order 10 (5 x 5 tiles, 200 registers of accumulators) three, then
    // two, each group moved into the rows before the next pass, so the
    // accumulators of all 25 tiles are never live at once.
    constexpr int QG = S::kExtra ? 3 : NB;
    const int kk = lane >> 2, t = lane & 3;  // table lanes: neighbour kk, table t
    double* strip = sm.buf;  // the strips reuse the tables' LDS
    // Order 10: p0, the pivot row of column 0 (the largest |M~_r0| of the 65
    // rows, compared exactly, the lowest row on ties), is found in the first
    // strip; it goes to LDS (sm.extra) and lane l takes row l, or l + 1 from p0
    // on, so the other 64 rows fill the 64 lanes in order.
#pragma unroll
    for (int Q0 = 0; Q0 < NB; Q0 += QG) {
      const int QN = (NB - Q0 < QG) ? NB - Q0 : QG;
      double4_t acc[NB][QG];
#pragma unroll
      for (int P = 0; P < NB; ++P)
#pragma unroll
        for (int Q = 0; Q < QG; ++Q) acc[P][Q] = double4_t{0.0, 0.0, 0.0, 0.0};
      // coordinates of the lane's neighbour one chunk ahead
      double xn = 0.0, yn = 0.0;
      if (kk < K) {
        const int j = g.col[e0 + kk];
        xn = g.x[j];
        yn = g.y[j];
      }
      if (lane < kChunk) T[lane * S::TABLE + S::ZERO] = 0.0;
      for (int k0 = 0; k0 < K; k0 += kChunk) {
        const bool have = k0 + kk < K;
        const double xj = xn, yj = yn;
        if (k0 + kChunk + kk < K) {  // the next chunk's coordinates, in flight meanwhile
          const int j = g.col[e0 + k0 + kChunk + kk];
          xn = g.x[j];
          yn = g.y[j];
        }
        double* tab = &T[kk * S::TABLE + t * TW];
        if (have) {
          const double dx = wrap_axis(xj - xi, g.box.Lx, px);
          const double dy = wrap_axis(yj - yi, g.box.Ly, py);
          const double xs = dx * hinv, ys = dy * hinv;
          const double z = (t == 0 || t == 2) ? xs : ys;
          if (t < 2) {
            double v = 1.0;
            tab[0] = 1.0;
#pragma unroll
            for (int a2 = 1; a2 <= M; ++a2) {
              v = v * z * (1.0 / static_cast<double>(a2));  // z^a / a!
              tab[a2] = v;
            }
          } else {
            const double psi = (t == 2) ? wendland_c2(sqrt(xs * xs + ys * ys)) : 1.0;
            double h0 = 1.0, h1 = z;
            tab[0] = psi;
            if (M >= 1) tab[1] = psi * z;
#pragma unroll
            for (int a2 = 1; a2 < M; ++a2) {
              const double h2 = z * h1 - static_cast<double>(a2) * h0;
              h0 = h1;
              h1 = h2;
              tab[a2 + 1] = psi * h2;
            }
          }
        } else {
#pragma unroll
          for (int a2 = 0; a2 <= M; ++a2) tab[a2] = 0.0;
        }
        lds_barrier();
#pragma unroll
        for (int ks = 0; ks < kChunk / 4; ++ks) {
          // steps of the last chunk past the K neighbours add only zeros
          if (k0 + ks * 4 >= K) break;
          const double* tk = &T[(ks * 4 + (lane >> 4)) * S::TABLE];
          double av[NB], bv[QG];
#pragma unroll
          for (int P = 0; P < NB; ++P) {
            const int oa = ea[P] >= 0 ? ea[P] : S::ZERO, ob = ea[P] >= 0 ? TW + eb[P] : S::ZERO;
            av[P] = tk[oa] * tk[ob];
          }
#pragma unroll
          for (int Q = 0; Q < QG; ++Q) {
            if (Q < QN) {
              const int P = Q0 + Q;
              const int oc = ea[P] >= 0 ? 2 * TW + ea[P] : S::ZERO;
              const int od = ea[P] >= 0 ? 3 * TW + eb[P] : S::ZERO;
              bv[Q] = tk[oc] * tk[od];
            }
          }
#pragma unroll
          for (int P = 0; P < NB; ++P)
#pragma unroll
            for (int Q = 0; Q < QG; ++Q)
              if (Q < QN)
                acc[P][Q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[P], bv[Q], acc[P][Q], 0, 0, 0);
        }
        lds_barrier();
      }

      // rows of this group's columns into registers, one 16-column strip at a
      // time; element v of lane l holds D[l/16 + 4v][l%16] of its 16x16 tile
#pragma unroll
      for (int Q = 0; Q < QG; ++Q) {
        if (Q < QN) {
          const int QC = Q0 + Q;
#pragma unroll
          for (int P = 0; P < NB; ++P)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              strip[(P * 16 + (lane >> 4) + 4 * v) * S::SS + (lane & 15)] = acc[P][Q][v];
          lds_barrier();
          if constexpr (S::kExtra) {
            if (QC == 0) {
              p0 = first_pivot_of_65(strip[lane * S::SS], strip[64 * S::SS]);
              myrow = lane + (lane >= p0 ? 1 : 0);
            }
          }
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (QC * 16 + j < N) a[QC * 16 + j] = (lane < N) ? strip[myrow * S::SS + j] : 0.0;
          if constexpr (S::kExtra) {
            if (lane < 16 && QC * 16 + lane < N) sm.extra[QC * 16 + lane] = strip[p0 * S::SS + lane];
          }
          lds_barrier();
        }
      }
    }
    int ra = 0, rb = 0;
    if (lane < N) exponents_of(myrow, ra, rb);
    {
      double c[LABFM_NUM_OPS];
      rhs_row(ra, rb, M, h, c);
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) a[N + d] = (lane < N) ? c[d] : 0.0;
      if (RC > N + LABFM_NUM_OPS) a[RC - 1] = 0.0;
      if constexpr (S::kExtra) {
        if (lane == 0) {
          int a64, b64;
          exponents_of(p0, a64, b64);
          rhs_row(a64, b64, M, h, c);
#pragma unroll
          for (int d = 0; d < LABFM_NUM_OPS; ++d) sm.extra[N + d] = c[d];
          if (RC > N + LABFM_NUM_OPS) sm.extra[RC - 1] = 0.0;
        }
        lds_barrier();
      }
    }
  }

  // ---- 3: LU with partial pivoting, rows in place ---------------------------
  // (no early exit: a zero pivot sets `singular`, a wave-uniform flag, and
  // the remaining columns are skipped, so the loop unrolls fully and the rows
  // stay in registers)
  bool used = lane >= N;  // rows beyond n never pivot and are never updated
  // the same as a wave-uniform mask
  unsigned long long usedm = N >= 64 ? 0ull : (~0ull << (N < 64 ? N : 0));
  int mycol = used ? N : -1;
  double myinv = 0.0;
  bool singular = false;
  // order 10: column 0 is eliminated with its pivot row p0 from LDS (pr);
  // the lanes then hold the 64 rows that columns 1..64 factor
  const double* pr = nullptr;
  double inv0 = 0.0;
  if constexpr (S::kExtra) {
    // the offset passes through an empty asm statement, so the reads of the
    // row count as per lane (vector registers), not as wave-uniform values
    // the compiler would hold in scalar registers
    int xo = 0;
    asm volatile("" : "+v"(xo));
    pr = sm.extra + xo;
    const double ucc = readlane_f64(pr[0], 0);
    singular = (ucc == 0.0 || !isfinite(ucc));  // wave-uniform
    if (!singular) {
      double inv = __builtin_amdgcn_rcp(ucc);
      inv = fma(inv, fma(-ucc, inv, 1.0), inv);
      inv0 = inv;
      const double l = a[0] * inv;
#pragma unroll
      for (int j = 1; j < RC; ++j) {
        a[j] = fma(-l, pr[j], a[j]);
        pin(a[j]);
        // eight reads of the pivot row in flight at a time, not all of them
        if (j % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
#pragma unroll
  for (int c = S::kExtra ? 1 : 0; c < N; ++c) {
    if (!singular) {
      // |a| of a finite double orders as its bit pattern
      const unsigned long long bits =
          static_cast<unsigned long long>(__double_as_longlong(fabs(a[c])));
      const unsigned hi = used ? 0u : static_cast<unsigned>(bits >> 32);
      const unsigned khi = wave_max_u32(hi);
      unsigned long long cand = __builtin_amdgcn_ballot_w64(hi == khi) & ~usedm;  // never empty
      if (__builtin_popcountll(cand) > 1) {  // equal high words: compare the low words
        const bool top = !used && hi == khi;
        const unsigned lo = top ? static_cast<unsigned>(bits) : 0u;
        const unsigned klo = wave_max_u32(lo);
        cand = __builtin_amdgcn_ballot_w64(top && lo == klo);
      }
      const int p = static_cast<int>(__builtin_ctzll(cand));
      // the pivot row is broadcast lane to scalar registers (v_readlane):
      // through LDS every lane would pull the whole row (64 lanes x 8 bytes
      // per value), more than the CU's shared LDS data path feeds (measured:
      // 8.7 ms against 7.3 ms at m = 8, 262,144 nodes; splitting each row
      // between the two ways was slower than read lanes alone)
      const double ucc = readlane_f64(a[c], p);
      singular = (ucc == 0.0 || !isfinite(ucc));  // wave-uniform
      if (!singular) {
        // 1 / u_cc: hardware reciprocal and one Newton step
        double inv = __builtin_amdgcn_rcp(ucc);
        inv = fma(inv, fma(-ucc, inv, 1.0), inv);
        usedm |= 1ull << p;
        if (lane == p) {
          used = true;
          mycol = c;
          myinv = inv;
        }
        // minus the multiplier (zero for used rows, +0.0)
        const double ln = used ? 0.0 : a[c] * -inv;
        // 8 values of the pivot row read out first, then their updates (a
        // read lane's result is used a few instructions later, not at once)
#pragma unroll
        for (int j0 = c + 1; j0 < RC; j0 += 8) {
          double u[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) u[t] = (j0 + t < RC) ? readlane_f64(a[j0 + t], p) : 0.0;
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (j0 + t < RC) {
              a[j0 + t] = fma(ln, u[t], a[j0 + t]);
              pin(a[j0 + t]);
            }
        }
      }
    }
  }

  int st = (K < N) ? LABFM_NODE_FEW_NEIGHBOURS : LABFM_NODE_OK;
  if (!singular) {
    // ---- 4: back substitution ------------------------------------------------
    // each lane keeps its right-hand sides divided by its own pivot u_qq
    // (q = mycol), so column c's pivot lane holds x_c = y_c / u_cc once the
    // later columns have been subtracted; every lane reads x_c from that
    // lane and subtracts (u_rc / u_qq) x_c, then writes its x into Psi (LDS)
    // at its column.
    double* psi_t = sm.buf;  // Psi[q][d], q < n (the strips are done)
    // order 10: the right-hand sides of column 0's pivot row (in LDS), kept
    // in every lane and updated as the lanes' own
    double ypr[LABFM_NUM_OPS];
    if constexpr (S::kExtra) {
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) ypr[d] = pr[N + d] * inv0;
    }
#pragma unroll
    for (int d = 0; d < LABFM_NUM_OPS; ++d) a[N + d] *= myinv;
#pragma unroll
    for (int c = N - 1; c >= (S::kExtra ? 1 : 0); --c) {
      const unsigned long long b = __builtin_amdgcn_ballot_w64(mycol == c);
      const int pc = static_cast<int>(__builtin_ctzll(b));
      const double coef = (mycol < c) ? a[c] * myinv : 0.0;
      double cpr = 0.0;
      if constexpr (S::kExtra) cpr = pr[c] * inv0;
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const double yc = readlane_f64(a[N + d], pc);
        a[N + d] = fma(-coef, yc, a[N + d]);
        if constexpr (S::kExtra) {
          ypr[d] = fma(-cpr, yc, ypr[d]);
          pin(ypr[d]);  // formed here, not deferred with every y_c held
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (mycol < N) {
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; d += 2)
        *reinterpret_cast<double2*>(&psi_t[mycol * LABFM_NUM_OPS + d]) =
            make_double2(a[N + d], a[N + d + 1]);
    }
    if constexpr (S::kExtra) {
      if (lane == 0) {
#pragma unroll
        for (int d = 0; d < LABFM_NUM_OPS; d += 2)
          *reinterpret_cast<double2*>(&psi_t[d]) = make_double2(ypr[d], ypr[d + 1]);
      }
    }
    lds_barrier();
    if constexpr (kSolve) {
      const long long k = k_;
      for (int j = lane; j < N * LABFM_NUM_OPS; j += 64) sv.psi[k * N * LABFM_NUM_OPS + j] = psi_t[j];
      if (mycol >= 0 && mycol < N) sv.pivot_row[k * N + mycol] = myrow;
      if (S::kExtra && lane == 0) sv.pivot_row[k * N] = p0;
      if (lane == 0) sv.status[k] = LABFM_NODE_OK;
      return;
    }

    // ---- 5: weights, filter calibration, row sums, first moments -------------
    // one lane per neighbour; Psi read from LDS a row at a time (the lanes'
    // reads of one row are a broadcast). The arguments and the node's
    // position, scale and spacing are read again here (see build_args_again).
    KernargBuildArgs* ga = build_args_again();
    const double xw = ga->x[i], yw = ga->y[i], hinvw = 1.0 / ga->h[i];
    const int pxw = ga->box.periodic_x, pyw = ga->box.periodic_y;
    const double kf = 2.0 * M_PI / (3.0 * ga->s[i]);
    double f0 = 0.0;
    double rs[LABFM_NUM_OPS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mo[kMoments] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const long long s32 = w32_stride(ga->nnz);
    // offsets of neighbour k and its Hermite ABF factors: hx[a] = psi He_a(x),
    // hy[b] = He_b(y) (scaled offsets)
    auto basis_of = [&](int k, double& dx, double& dy, double* hx, double* hy) {
      const int j = ga->col[e0 + k];
      dx = wrap_axis(ga->x[j] - xw, ga->box.Lx, pxw);
      dy = wrap_axis(ga->y[j] - yw, ga->box.Ly, pyw);
      const double xs = dx * hinvw, ys = dy * hinvw;
      const double psi = wendland_c2(sqrt(xs * xs + ys * ys));
      hx[0] = psi;
      hy[0] = 1.0;
      hx[1] = psi * xs;
      hy[1] = ys;
      double a0 = 1.0, a1 = xs, b0 = 1.0, b1 = ys;
#pragma unroll
      for (int q = 1; q < M; ++q) {
        const double a2 = xs * a1 - static_cast<double>(q) * a0;
        const double b2 = ys * b1 - static_cast<double>(q) * b0;
        a0 = a1;
        a1 = a2;
        b0 = b1;
        b1 = b2;
        hx[q + 1] = psi * a2;
        hy[q + 1] = b2;
      }
    };
    // full passes of 64 neighbours, then a last pass over at most 32
    // neighbours in which lanes l and l + 32 share neighbour k0 + l, the
    // first forming operators x, y, L, the second xx, xy, hyp (og = 0, 1)
    int k0 = 0;
    for (; K - k0 > 32; k0 += 64) {
      const int k = k0 + lane;
      // Psi's offset passes through an empty asm statement every pass, so the
      // compiler does not hoist all of its reads out of the loop (n * 6
      // values held in registers)
      int pbase = 0;
      asm volatile("" : "+v"(pbase));
      if (k < K) {
        double dx, dy, hx[M + 1], hy[M + 1];
        basis_of(k, dx, dy, hx, hy);
        const long long e = e0 + k;
          double wd[LABFM_NUM_OPS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // Psi row q in registers, row q+1 read from LDS while q is used
        double r0[LABFM_NUM_OPS], r1[LABFM_NUM_OPS];
#pragma unroll
        for (int d = 0; d < LABFM_NUM_OPS; ++d) r0[d] = psi_t[pbase + d];
#pragma unroll
        for (int deg = 1, q = 0; deg <= M; ++deg) {
#pragma unroll
          for (int bb = 0; bb <= deg; ++bb, ++q) {
            if (q + 1 < N) {
#pragma unroll
              for (int d = 0; d < LABFM_NUM_OPS; ++d)
                r1[d] = psi_t[pbase + (q + 1) * LABFM_NUM_OPS + d];
            }
            const double Wq = hx[deg - bb] * hy[bb];
#pragma unroll
            for (int d = 0; d < LABFM_NUM_OPS; ++d) {
              wd[d] = fma(Wq, r0[d], wd[d]);
              pin(wd[d]);
            }
#pragma unroll
            for (int d = 0; d < LABFM_NUM_OPS; ++d) r0[d] = r1[d];
          }
        }
#pragma unroll
        for (int d = 0; d < LABFM_NUM_OPS; ++d) {
          const int r = op_row(ga->rows, d);
          if (r != kNoRow) {
            ga->w[r * ga->nnz + e] = wd[d];
            if (ga->w32) ga->w32[r * s32 + e] = static_cast<float>(wd[d]);
          }
          rs[d] += wd[d];
        }
#pragma unroll
        for (int d = LABFM_OP_L; d <= LABFM_OP_XY; ++d) {
          const double v32 = static_cast<double>(static_cast<float>(wd[d]));
          mo[2 * (d - LABFM_OP_L)] += v32 * dx;
          mo[2 * (d - LABFM_OP_L) + 1] += v32 * dy;
        }
        f0 += (1.0 - cos(kf * dx) * cos(kf * dy)) * wd[LABFM_OP_HYP];
      }
    }
    if (k0 < K) {
      const int k = k0 + (lane & 31);
      const int og = lane >> 5;
      int pbase = 0;
      asm volatile("" : "+v"(pbase));
      if (k < K) {
        double dx, dy, hx[M + 1], hy[M + 1];
        basis_of(k, dx, dy, hx, hy);
        const long long e = e0 + k;
        constexpr int H3 = LABFM_NUM_OPS / 2;
        static_assert(LABFM_OP_L == 2 && LABFM_OP_XX == 3 && LABFM_OP_XY == 4 &&
                          LABFM_OP_HYP == 5,
                      "operator groups of a half pass: (x, y, L), (xx, xy, hyp)");
        const int ob = pbase + og * H3;  // this lane's operators in a Psi row
        double wd[H3] = {0.0, 0.0, 0.0};
        double r0[H3], r1[H3];
#pragma unroll
        for (int d = 0; d < H3; ++d) r0[d] = psi_t[ob + d];
#pragma unroll
        for (int deg = 1, q = 0; deg <= M; ++deg) {
#pragma unroll
          for (int bb = 0; bb <= deg; ++bb, ++q) {
            if (q + 1 < N) {
#pragma unroll
              for (int d = 0; d < H3; ++d) r1[d] = psi_t[ob + (q + 1) * LABFM_NUM_OPS + d];
            }
            const double Wq = hx[deg - bb] * hy[bb];
#pragma unroll
            for (int d = 0; d < H3; ++d) {
              wd[d] = fma(Wq, r0[d], wd[d]);
              pin(wd[d]);
            }
#pragma unroll
            for (int d = 0; d < H3; ++d) r0[d] = r1[d];
          }
        }
#pragma unroll
        for (int d = 0; d < H3; ++d) {
          const int r = op_row(ga->rows, og * H3 + d);
          if (r != kNoRow) {
            ga->w[r * ga->nnz + e] = wd[d];
            if (ga->w32) ga->w32[r * s32 + e] = static_cast<float>(wd[d]);
          }
          // each sum takes this lane's value for its own operators only
          rs[d] += og ? 0.0 : wd[d];
          rs[H3 + d] += og ? wd[d] : 0.0;
        }
        // L is the first group's third operator, xx and xy the second's
        // first two, hyp its third
        const double vl = og ? 0.0 : static_cast<double>(static_cast<float>(wd[2]));
        const double vxx = og ? static_cast<double>(static_cast<float>(wd[0])) : 0.0;
        const double vxy = og ? static_cast<double>(static_cast<float>(wd[1])) : 0.0;
        mo[0] += vl * dx;
        mo[1] += vl * dy;
        mo[2] += vxx * dx;
        mo[3] += vxx * dy;
        mo[4] += vxy * dx;
        mo[5] += vxy * dy;
        // one cosine per lane: the first half takes x, the second y and
        // the x factor from its partner (lanes l and l + 32 share neighbour
        // k and are active together); the second half holds hyp
        const double cf = cos(kf * (og ? dy : dx));
        const double cx = __shfl_xor(cf, 32);
        f0 += og ? (1.0 - cx * cf) * wd[2] : 0.0;
      }
    }
    f0 = group_sum<64>(f0);
    // the row sums and first moments are reduced only when they are asked for
    if (ga->rowsum) {
#pragma unroll
      for (int d = 0; d < LABFM_NUM_OPS; ++d) rs[d] = group_sum<64>(rs[d]);
    }
    if (ga->mom32) {
#pragma unroll
      for (int q = 0; q < kMoments; ++q) mo[q] = group_sum<64>(mo[q]);
    }
    if (lane == 0) {
      if (ga->mom32)
#pragma unroll
        for (int q = 0; q < kMoments; ++q) ga->mom32[q * (long long)ga->n + i] = static_cast<float>(mo[q]);
      const bool bad = !isfinite(f0) || f0 == 0.0;
      ga->kappa[i] = bad ? 0.0 : 2.0 / (3.0 * f0);
      if (st == LABFM_NODE_OK && bad) st = LABFM_NODE_BAD_FILTER;
      ga->status[i] = static_cast<int8_t>(st);
      if (ga->rowsum)
#pragma unroll
        for (int d = 0; d < LABFM_NUM_OPS; ++d)
          if (op_row(ga->rows, d) != kNoRow) ga->rowsum[op_row(ga->rows, d) * (long long)ga->n + i] = rs[d];
    }
  } else {
    if constexpr (kSolve) {
      if (lane == 0) sv.status[k_] = LABFM_NODE_SINGULAR;
      return;
    }
    KernargBuildArgs* ga = build_args_again();
    const long long s32 = w32_stride(ga->nnz);
    for (int k = lane; k < K; k += 64)
      for (int d = 0; d < LABFM_NUM_OPS; ++d) {
        const int r = op_row(ga->rows, d);
        if (r == kNoRow) continue;
        ga->w[r * ga->nnz + e0 + k] = 0.0;
        if (ga->w32) ga->w32[r * s32 + e0 + k] = 0.0f;
      }
    if (lane == 0) {
      ga->kappa[i] = 0.0;
      ga->status[i] = LABFM_NODE_SINGULAR;
      if (ga->rowsum)
        for (int d = 0; d < LABFM_NUM_OPS; ++d)
          if (op_row(ga->rows, d) != kNoRow) ga->rowsum[op_row(ga->rows, d) * (long long)ga->n + i] = 0.0;
      if (ga->mom32)
        for (int q = 0; q < kMoments; ++q) ga->mom32[q * (long long)ga->n + i] = 0.0f;
    }
  }
}

template <int M>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(rows_waves<M>())))
build_rows_kernel(BuildArgs g, const int* __restrict__ list, int count) {
  rows_node<M, false>(g, list, count, SolveArgs{});
}

template <int M>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(rows_waves<M>())))
rows_solve_kernel(SolveArgs sv) {
  rows_node<M, true>(BuildArgs{}, nullptr, sv.count, sv);
}

template <int M>
hipError_t launch_rows(const BuildArgs& g, const int* list, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(build_rows_kernel<M>, dim3(count), dim3(64), 0, st, g, list, count);
  return hipGetLastError();
}

// Calls fn(integral_constant<M>) for an order 1..10 of the rows kernel.
template <class Fn>
hipError_t with_rows_order(int m, Fn&& fn) {
  using std::integral_constant;
  switch (m) {
    case 1: return fn(integral_constant<int, 1>{});
    case 2: return fn(integral_constant<int, 2>{});
    case 3: return fn(integral_constant<int, 3>{});
    case 4: return fn(integral_constant<int, 4>{});
    case 5: return fn(integral_constant<int, 5>{});
    case 6: return fn(integral_constant<int, 6>{});
    case 7: return fn(integral_constant<int, 7>{});
    case 8: return fn(integral_constant<int, 8>{});
    case 9: return fn(integral_constant<int, 9>{});
    case 10: return fn(integral_constant<int, 10>{});
  }
  return hipErrorInvalidValue;
}

// ---- stencil optimisation (section "Stencil optimisation") -------------------
//
// The shrinking loop runs in passes over the nodes: each pass builds the x, y
// and L weights of every node still shrinking at its current scale h (the
// rows-in-registers build on the h0 stencils, so neighbours beyond 2h have
// psi = 0 and drop out of the system and the weights), then one wavefront per
// node tests them. A node whose test fails, whose system is singular, or that
// has taken max_iter + 1 shrinks keeps its last accepted scale and leaves the
// loop; the host runs passes until no node is left.

constexpr int kNk = 16;  // wavenumbers of the amplitude test

// Nodes, this pass's weights and the loop's state.
struct OptArgs {
  const double* x;
  const double* y;
  const double* s;
  const int8_t* order;
  labfm_box box;
  const int* row_ptr;  // CSR of the h0 stencils
  const int* col;
  long long nnz;
  const double* w;        // this pass's weights, rows x, y, L ([3][nnz])
  const int8_t* status;   // this pass's build status
  double* h;              // current scale
  int* k;                 // shrinks taken to reach it
  int8_t* active;         // 1 while the node shrinks
  int* remaining;         // nodes still shrinking
  double* h_out;          // last accepted scale (h0 until one is)
  int* iters;             // its shrink count
  double shrink, gain_max, res_coef;
  int max_iter;
};

// LDS of the test (one wavefront per node) for a chunk of neighbours: the
// scaled monomial factors x^a/a! and y^b/b!, the sequences sin(k_q x),
// sin(k_q y), cos(k_q x), cos(k_q y) for q = 1..16 (wavenumber innermost,
// so the amplitude lanes of one operator read consecutive words; padded to
// 17 against conflicts of the lanes writing them), and the weights.
template <int MMAX>
struct AcceptSmem {
  double tab[kChunk][2][MMAX + 1];
  double trig[kChunk][4][kNk + 1];
  double wv[3][kChunk];
};

__global__ void __launch_bounds__(256)
stencil_opt_init_kernel(const double* __restrict__ h0, const int8_t* __restrict__ order, int n,
                        double* __restrict__ h, int* __restrict__ k, int8_t* __restrict__ active,
                        double* __restrict__ h_out, int* __restrict__ iters,
                        int* __restrict__ remaining, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *remaining = count;
  if (i >= n) return;
  h[i] = h0[i];
  k[i] = 0;
  h_out[i] = h0[i];
  iters[i] = 0;
  active[i] = (order[i] >= 1 && order[i] <= kMaxOrder) ? 1 : 0;
}

// The test of node i at its current scale h:
//   1. the residual of the unscaled Laplacian system,
//        alpha_L = || sum_j X_j w^L_j - C^L ||_2  (X_j the monomials
//        x^a y^b/(a!b!)), at most res_coef eps n^4 / (h m);
//   2. the amplitude responses A^x(k) = L^x(sin k x)/k,
//      A^y(k) = L^y(sin k y)/k, A^L(k) = L^L(1/2 - cos k x cos k y / 2)/k^2
//      at k = q k_Ny / 16, q = 1..16, k_Ny = pi/s: none above gain_max and
//      none NaN.
// Passed, h becomes the node's accepted scale and is shrunk for the next
// pass; failed (or singular, or past max_iter), the node leaves the loop.
template <int MMAX>
__global__ void __launch_bounds__(64)
stencil_accept_kernel(OptArgs a, const int* __restrict__ list, int count) {
  __shared__ AcceptSmem<MMAX> sm;
  const int kn = blockIdx.x;
  if (kn >= count) return;
  const int i = uniform(list[kn]);
  if (uniform(a.active[i]) == 0) return;
  const int lane = threadIdx.x;
  const int m = uniform(a.order[i]);
  const int n = moments_of(m);
  const int e0 = uniform(a.row_ptr[i]);
  const int K = uniform(a.row_ptr[i + 1]) - e0;
  const int kcur = uniform(a.k[i]);
  const double h = a.h[i], s = a.s[i], xi = a.x[i], yi = a.y[i];
  const int px = a.box.periodic_x, py = a.box.periodic_y;
  const double hinv = 1.0 / h;
  const double k1 = M_PI / (s * kNk);
  // residual lanes: moments p = lane and lane + 64 (order 10 has 65)
  int pa0 = 0, pb0 = 0, pa1 = 0, pb1 = 0;
  if (lane < n) exponents_of(lane, pa0, pb0);
  if (lane + 64 < n) exponents_of(lane + 64, pa1, pb1);
  double res0 = 0.0, res1 = 0.0;  // sum_j X~^p_j w^L_j (scaled monomials)
  // amplitude lanes 0..47: operator aop (x, y, L), wavenumber aq
  const int aop = lane >> 4, aq = lane & 15;
  double amp = 0.0;
  // chunk lanes: neighbour kk of the chunk, sequence t
  const int kk = lane >> 2, t = lane & 3;
  // the lane's neighbour one chunk ahead: coordinates and weight (t < 3)
  double xn = 0.0, yn = 0.0, wn = 0.0;
  if (kk < K) {
    const int j = a.col[e0 + kk];
    xn = a.x[j];
    yn = a.y[j];
    if (t < 3) wn = a.w[t * a.nnz + e0 + kk];
  }
  for (int k0 = 0; k0 < K; k0 += kChunk) {
    const bool have = k0 + kk < K;
    const double xj = xn, yj = yn, wj = wn;
    if (k0 + kChunk + kk < K) {  // in flight while this chunk is tested
      const int j = a.col[e0 + k0 + kChunk + kk];
      xn = a.x[j];
      yn = a.y[j];
      if (t < 3) wn = a.w[t * a.nnz + e0 + k0 + kChunk + kk];
    }
    double dx = 0.0, dy = 0.0;
    if (have) {
      dx = wrap_axis(xj - xi, a.box.Lx, px);
      dy = wrap_axis(yj - yi, a.box.Ly, py);
    }
    if (t < 2) {
      const double z = (t == 0 ? dx : dy) * hinv;
      double v = 1.0;
      sm.tab[kk][t][0] = have ? 1.0 : 0.0;
#pragma unroll
      for (int q = 1; q <= MMAX; ++q) {
        v = v * z * (1.0 / static_cast<double>(q));  // z^q / q!
        sm.tab[kk][t][q] = have ? v : 0.0;
      }
    }
    if (t < 3) sm.wv[t][kk] = have ? wj : 0.0;
    {
      // f(q+1) = 2 cos(theta) f(q) - f(q-1), from sin or cos of theta; the
      // sine lanes (t = 0: x, 1: y) form sin and cos of their angle once and
      // pass them to the cosine lanes (t = 2, 3) of the same neighbour
      double sn = 0.0, cs = 0.0;
      if (t < 2) sincos(k1 * (t == 0 ? dx : dy), &sn, &cs);
      const int from = (lane & ~3) | (t & 1);
      sn = __shfl(sn, from, 64);
      cs = __shfl(cs, from, 64);
      double f0 = (t < 2) ? 0.0 : 1.0, f1 = (t < 2) ? sn : cs;
      sm.trig[kk][t][0] = f1;
#pragma unroll
      for (int q = 1; q < kNk; ++q) {
        const double f2 = 2.0 * cs * f1 - f0;
        f0 = f1;
        f1 = f2;
        sm.trig[kk][t][q] = f1;
      }
    }
    lds_barrier();
    for (int c = 0; c < kChunk; ++c) {
      const double wl = sm.wv[2][c];
      if (lane < n) res0 += (sm.tab[c][0][pa0] * sm.tab[c][1][pb0]) * wl;
      if (lane + 64 < n) res1 += (sm.tab[c][0][pa1] * sm.tab[c][1][pb1]) * wl;
      if (lane < 3 * kNk) {
        const double f = (aop == 2) ? 0.5 - 0.5 * sm.trig[c][2][aq] * sm.trig[c][3][aq]
                                    : sm.trig[c][aop][aq];
        amp += sm.wv[aop][c] * f;
      }
    }
    lds_barrier();
  }
  // r_p = h^(a+b) res_p - C^L_p of the unscaled system
  auto rsq = [&](int pa, int pb, double res) {
    double hp = 1.0;
    for (int d = 0; d < pa + pb; ++d) hp *= h;
    const double target = ((pa == 2 && pb == 0) || (pa == 0 && pb == 2)) ? 1.0 : 0.0;
    const double r = hp * res - target;
    return r * r;
  };
  double sq = 0.0;
  if (lane < n) sq += rsq(pa0, pb0, res0);
  if (lane + 64 < n) sq += rsq(pa1, pb1, res1);
  const double ss = group_sum<64>(sq);
  double av = -1.0;
  bool bad = false;
  if (lane < 3 * kNk) {
    const double kq = k1 * static_cast<double>(aq + 1);
    av = (aop == 2) ? amp / (kq * kq) : amp / kq;
    bad = !(av == av);
  }
  const bool nan_amp = __builtin_amdgcn_ballot_w64(bad) != 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) av = fmax(av, __shfl_xor(av, off, 64));
  double n4 = static_cast<double>(n);
  n4 = n4 * n4 * n4 * n4;
  const double alpha0 = a.res_coef * 2.220446049250313e-16 * n4 / (h * static_cast<double>(m));
  const bool ok = a.status[i] != LABFM_NODE_SINGULAR && sqrt(ss) <= alpha0 && !nan_amp &&
                  av <= a.gain_max;
  if (lane == 0) {
    if (!ok || kcur > a.max_iter) {
      a.active[i] = 0;
      atomicSub(a.remaining, 1);
    } else {
      a.h_out[i] = h;
      a.iters[i] = kcur;
      a.h[i] = h * a.shrink;
      a.k[i] = kcur + 1;
    }
  }
}

// Work list: node indices grouped by order, highest order first (counting
// sort; the order inside a group is immaterial, every node's result is its
// own).
// Histogram and scatter count in LDS and issue one global atomic per order
// per workgroup.
__device__ __forceinline__ int order_bucket(const int8_t* m, int i) {
  int o = m[i];
  o = o < 0 ? 0 : (o > 15 ? 15 : o);
  return 15 - o;
}

__global__ void __launch_bounds__(256)
order_histogram_kernel(const int8_t* __restrict__ m, int n, int* __restrict__ hist) {
  __shared__ int local[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < 16) local[threadIdx.x] = 0;
  __syncthreads();
  if (i < n) atomicAdd(&local[order_bucket(m, i)], 1);
  __syncthreads();
  if (threadIdx.x < 16 && local[threadIdx.x] > 0) atomicAdd(&hist[threadIdx.x], local[threadIdx.x]);
}

__global__ void order_offsets_kernel(int* __restrict__ hist) {
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < 16; ++b) {
      const int c = hist[b];
      hist[16 + b] = acc;  // start of bucket b
      hist[b] = acc;       // cursor
      acc += c;
    }
    hist[32] = acc;
  }
}

__global__ void __launch_bounds__(256)
order_scatter_kernel(const int8_t* __restrict__ m, int n, int* __restrict__ hist,
                     int* __restrict__ list) {
  __shared__ int local[16];
  __shared__ int base[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < 16) local[threadIdx.x] = 0;
  __syncthreads();
  const int b = (i < n) ? order_bucket(m, i) : 0;
  const int rank = (i < n) ? atomicAdd(&local[b], 1) : 0;
  __syncthreads();
  if (threadIdx.x < 16 && local[threadIdx.x] > 0)
    base[threadIdx.x] = atomicAdd(&hist[threadIdx.x], local[threadIdx.x]);
  __syncthreads();
  if (i < n) list[base[b] + rank] = i;
}

// Zeroes count ints: the clears of the build's work area are kernels, not
// memset nodes.
__global__ void zero_ints_kernel(int* __restrict__ p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void max_order_kernel(const int8_t* __restrict__ m, int n, int* out) {
  __shared__ int sh[256];
  int v = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int o = m[i];
    v = o > v ? o : v;
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

template <int MMAX>
hipError_t launch_build(const double* x, const double* y, const double* h, const double* s,
                        const int8_t* m, int n, labfm_box box, const int* row_ptr,
                        const int* col, long long nnz, double* w, float* w32, float* mom32,
                        double* kappa, double* rowsum, int8_t* status, unsigned rows,
                        hipStream_t st) {
  hipLaunchKernelGGL(build_weights_kernel<MMAX>, dim3(n), dim3(64), 0, st, x, y, h, s, m, n, box,
                     row_ptr, col, nnz, w, w32, mom32, kappa, rowsum, status, rows);
  return hipGetLastError();
}

template <int MMAX>
hipError_t launch_block(const BuildArgs& g, const int* list, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(build_block_kernel<MMAX>, dim3(count), dim3(kBlock), 0, st, g, list, count);
  return hipGetLastError();
}

template <int MMAX>
hipError_t launch_persistent(const BuildArgs& g, const int* list, int count, int* counter,
                             int per_cu, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int dev = 0, cus = 0, blocks = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, build_persistent_kernel<MMAX>,
                                                     kBlock, 0);
  if (e != hipSuccess) return e;
  blocks = std::max(1, blocks);
  if (per_cu > 0) blocks = std::min(blocks, per_cu);
  const int grid = std::max(1, std::min(count, cus * blocks));
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, counter, 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(build_persistent_kernel<MMAX>, dim3(grid), dim3(kBlock), 0, st, g, list,
                     count, counter);
  return hipGetLastError();
}

template <class Fn>
hipError_t with_mmax(int mmax, Fn&& fn) {
  if (mmax <= 4) return fn(std::integral_constant<int, 4>{});
  if (mmax <= 6) return fn(std::integral_constant<int, 6>{});
  if (mmax <= 8) return fn(std::integral_constant<int, 8>{});
  return fn(std::integral_constant<int, 10>{});  // orders above 10: LABFM_NODE_BAD_ORDER
}

std::mutex g_build_mutex;
labfm_build_config g_build_cfg = {LABFM_BUILD_ROWS, 0};

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" int labfm_set_build_config(const labfm_build_config* cfg) {
  clear_error();
  labfm_build_config c{LABFM_BUILD_ROWS, 0};
  if (cfg) {
    LABFM_REQUIRE(cfg->mode >= LABFM_BUILD_WAVE && cfg->mode <= LABFM_BUILD_ROWS,
                  "set_build_config: unknown mode %d", cfg->mode);
    LABFM_REQUIRE(cfg->workgroups_per_cu >= 0, "set_build_config: negative workgroups_per_cu");
    c = *cfg;
  }
  std::lock_guard<std::mutex> lock(g_build_mutex);
  g_build_cfg = c;
  return LABFM_OK;
}

extern "C" int labfm_get_build_config(labfm_build_config* cfg) {
  clear_error();
  LABFM_REQUIRE(cfg, "get_build_config: null argument");
  std::lock_guard<std::mutex> lock(g_build_mutex);
  *cfg = g_build_cfg;
  return LABFM_OK;
}

namespace labfm {
namespace {

// Body of labfm_build_weights over a work area of kBuildWorkInts + n ints:
// [0, 16) bucket cursors, [16, 33) bucket starts and their total, [40] the
// persistent distribution's work counter, [64, 64 + n) the node list ordered
// by decreasing order. The area is cleared here; nothing else is kept.
constexpr int kBuildWorkInts = 64;

// The node list of a build, grouped by order (bucket b holds order 15 - b,
// orders outside 0..15 share the buckets of their nearest end), in `work`;
// starts[b] (host) is bucket b's first position, starts[16] = n.
// Synchronises the stream.
int order_buckets(const int8_t* order_m, int32_t n, int* work, int starts[17], hipStream_t st) {
  int* hist = work;  // [0,16) cursors, [16,32) starts, [32] total
  int* list = hist + kBuildWorkInts;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, hist, kBuildWorkInts);
  hipLaunchKernelGGL(order_histogram_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, order_m,
                     n, hist);
  hipLaunchKernelGGL(order_offsets_kernel, dim3(1), dim3(64), 0, st, hist);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, order_m,
                     n, hist, list);
  LABFM_LAUNCHED();
  LABFM_HIP(hipMemcpyAsync(starts, hist + 16, sizeof(int) * 17, hipMemcpyDeviceToHost, st));
  LABFM_HIP(hipStreamSynchronize(st));
  return LABFM_OK;
}

int build_weights_with(const double* x, const double* y, const double* h, const double* s,
                       const int8_t* order_m, int32_t n, labfm_box box, const int32_t* row_ptr,
                       const int32_t* col, int64_t nnz, uint32_t op_mask, double* w, float* w32,
                       float* mom32, double* kappa, double* rowsum, int8_t* status, int* work,
                       hipStream_t st) {
  labfm_build_config cfg;
  {
    std::lock_guard<std::mutex> lock(g_build_mutex);
    cfg = g_build_cfg;
  }
  int* counter = work + 40;
  int* list = work + kBuildWorkInts;
  int starts[17] = {0};
  if (int r = order_buckets(order_m, n, work, starts, st)) return r;
  const unsigned rows = rows_of_mask(op_mask);
  // bucket b holds order 15 - b; the highest order present sets the template
  int mmax = 0;
  for (int b = 0; b < 16; ++b)
    if (starts[b + 1] > starts[b]) {
      mmax = 15 - b;
      break;
    }
  const BuildArgs g{x, y, h, s, order_m, n, box, row_ptr, col, nnz, w, w32, mom32, kappa,
                    rowsum, status, rows};
  hipError_t e = hipSuccess;
  switch (cfg.mode) {
    case LABFM_BUILD_WAVE:
      e = with_mmax(mmax, [&](auto M) {
        return launch_build<decltype(M)::value>(x, y, h, s, order_m, n, box, row_ptr, col, nnz,
                                                w, w32, mom32, kappa, rowsum, status, rows, st);
      });
      break;
    case LABFM_BUILD_BLOCK:
      e = with_mmax(mmax, [&](auto M) { return launch_block<decltype(M)::value>(g, list, n, st); });
      break;
    case LABFM_BUILD_PERSISTENT:
      e = with_mmax(mmax, [&](auto M) {
        return launch_persistent<decltype(M)::value>(g, list, n, counter, cfg.workgroups_per_cu,
                                                     st);
      });
      break;
    case LABFM_BUILD_ROWS: {
      // orders 1..10: one wavefront per node with the rows in registers, one
      // launch per order present; out-of-range orders (buckets of orders
      // 15..11, and the bucket of orders <= 0) go to the workgroup kernel,
      // which marks them unsupported
      for (int m = 1; m <= 10 && e == hipSuccess; ++m) {
        const int b = 15 - m;
        const int first = starts[b], count = starts[b + 1] - first;
        if (count <= 0) continue;
        e = with_rows_order(m, [&](auto M) {
          return launch_rows<decltype(M)::value>(g, list + first, count, st);
        });
      }
      if (e == hipSuccess && starts[5] > starts[0])
        e = launch_block<10>(g, list + starts[0], starts[5] - starts[0], st);
      if (e == hipSuccess && starts[16] > starts[15])
        e = launch_block<10>(g, list + starts[15], starts[16] - starts[15], st);
      break;
    }
    case LABFM_BUILD_BUCKETED: {
      // one launch per order class, each with the template of the highest
      // order present in it
      // classes by template: orders 9..15 (MMAX 10), 7..8, 5..6, 0..4
      const int hi[4] = {15, 8, 6, 4};
      const int lo[4] = {9, 7, 5, 0};
      for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        const int b0 = 15 - hi[c], b1 = 15 - lo[c];  // buckets b0..b1
        const int first = starts[b0], count = starts[b1 + 1] - first;
        if (count <= 0) continue;
        int top = lo[c];
        for (int b = b0; b <= b1; ++b)
          if (starts[b + 1] > starts[b]) {
            top = 15 - b;
            break;
          }
        e = with_mmax(std::min(top, 10), [&](auto M) {
          return launch_block<decltype(M)::value>(g, list + first, count, st);
        });
      }
      break;
    }
    default:
      e = hipErrorInvalidValue;
  }
  LABFM_HIP(e);
  return LABFM_OK;
}

int check_build_args(const double* x, const double* y, const double* h, const double* s,
                     const int8_t* order_m, int32_t n, const int32_t* row_ptr, const int32_t* col,
                     int64_t nnz, uint32_t op_mask, const double* w, const float* mom32,
                     const double* kappa, const int8_t* status, const char* who) {
  LABFM_REQUIRE(n > 0, "%s: n must be positive (got %d)", who, n);
  LABFM_REQUIRE(x && y && h && s && order_m && row_ptr && w && kappa && status,
                "%s: null pointer argument", who);
  LABFM_REQUIRE(nnz >= 0 && (nnz == 0 || col), "%s: bad CSR arguments", who);
  LABFM_REQUIRE(op_mask != 0 && (op_mask & ~0x3Fu) == 0,
                "%s: op_mask 0x%x must select operators among the six (bits 0..5)", who, op_mask);
  constexpr uint32_t kSecond = (1u << LABFM_OP_L) | (1u << LABFM_OP_XX) | (1u << LABFM_OP_XY);
  LABFM_REQUIRE(!mom32 || (op_mask & kSecond) == kSecond,
                "%s: mom32 needs the L, xx and xy operators in op_mask (got 0x%x)", who, op_mask);
  return LABFM_OK;
}

size_t build_work_bytes(int32_t n) {
  return align256(sizeof(int) * (kBuildWorkInts + static_cast<size_t>(n)));
}

// Scratch of labfm_build_weights_noalloc: the work area of the largest node
// set it accepts. Each GPU the library runs on holds its own copy until the
// process ends. Host code never uses this name as an address: it takes the
// device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) int scratch[kBuildWorkInts + LABFM_NOALLOC_MAX_NODES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
int* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// device's first use).
int scratch_of_current_device(int** out) {
  int dev = 0;
  LABFM_HIP(hipGetDevice(&dev));
  LABFM_REQUIRE(dev >= 0 && dev < kMaxDevices, "build_weights_noalloc: device %d out of range",
                dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("build_weights_noalloc: hipGetSymbolAddress(scratch) failed: %s",
                hipGetErrorString(e));
      return LABFM_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<int*>(p);
  }
  *out = g_scratch_ptr[dev];
  return LABFM_OK;
}

}  // namespace
}  // namespace labfm

extern "C" size_t labfm_build_workspace_bytes(int32_t n) {
  return n > 0 ? build_work_bytes(n) : 0;
}

extern "C" int labfm_build_weights(const double* x, const double* y, const double* h,
                                   const double* s, const int8_t* order_m, int32_t n,
                                   labfm_box box, const int32_t* row_ptr, const int32_t* col,
                                   int64_t nnz, uint32_t op_mask, double* w, float* w32,
                                   float* mom32, double* kappa, double* rowsum, int8_t* status,
                                   void* workspace, size_t workspace_bytes, void* stream_) {
  clear_error();
  if (int r = check_build_args(x, y, h, s, order_m, n, row_ptr, col, nnz, op_mask, w, mom32,
                               kappa, status, "build_weights"))
    return r;
  LABFM_WORKSPACE(workspace, workspace_bytes, build_work_bytes(n), "build_weights");
  return build_weights_with(x, y, h, s, order_m, n, box, row_ptr, col, nnz, op_mask, w, w32,
                            mom32, kappa, rowsum, status, static_cast<int*>(workspace),
                            as_stream(stream_));
}

extern "C" int labfm_build_weights_noalloc(const double* x, const double* y, const double* h,
                                           const double* s, const int8_t* order_m, int32_t n,
                                           labfm_box box, const int32_t* row_ptr,
                                           const int32_t* col, int64_t nnz, uint32_t op_mask,
                                           double* w, float* w32, float* mom32, double* kappa,
                                           double* rowsum, int8_t* status, void* stream_) {
  clear_error();
  if (int r = check_build_args(x, y, h, s, order_m, n, row_ptr, col, nnz, op_mask, w, mom32,
                               kappa, status, "build_weights_noalloc"))
    return r;
  LABFM_REQUIRE(n <= LABFM_NOALLOC_MAX_NODES,
                "build_weights_noalloc: %d nodes exceed the scratch's maximum of %d nodes "
                "(use labfm_build_weights)",
                n, LABFM_NOALLOC_MAX_NODES);
  int* work = nullptr;
  if (int r = scratch_of_current_device(&work)) return r;
  return build_weights_with(x, y, h, s, order_m, n, box, row_ptr, col, nnz, op_mask, w, w32,
                            mom32, kappa, rowsum, status, work, as_stream(stream_));
}

extern "C" int labfm_solve_systems(int32_t m, const double* systems, int32_t count,
                                   double* psi, int32_t* pivot_row, int8_t* status,
                                   void* stream_) {
  clear_error();
  LABFM_REQUIRE(m >= 1 && m <= 10, "solve_systems: order %d outside 1..10", m);
  LABFM_REQUIRE(count >= 0, "solve_systems: count %d < 0", count);
  if (count == 0) return LABFM_OK;
  LABFM_REQUIRE(systems && psi && pivot_row && status, "solve_systems: null pointer");
  SolveArgs sv;
  sv.sys = systems;
  sv.count = count;
  sv.psi = psi;
  sv.pivot_row = pivot_row;
  sv.status = status;
  const hipStream_t st = as_stream(stream_);
  LABFM_HIP(with_rows_order(m, [&](auto mc) -> hipError_t {
    hipLaunchKernelGGL(rows_solve_kernel<decltype(mc)::value>, dim3(count), dim3(64), 0, st, sv);
    return hipGetLastError();
  }));
  return LABFM_OK;
}

extern "C" int labfm_tune_build(const double* x, const double* y, const double* h,
                                const double* s, const int8_t* order_m, int32_t n, labfm_box box,
                                const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                                uint32_t op_mask, double* w, float* w32, float* mom32,
                                double* kappa, double* rowsum, int8_t* status, void* workspace,
                                size_t workspace_bytes, const char* cache_path,
                                labfm_build_config* best, double* best_ms, int32_t* from_cache,
                                void* stream_) {
  clear_error();
  LABFM_REQUIRE(best && best_ms, "tune_build: null output");
  if (int r = check_build_args(x, y, h, s, order_m, n, row_ptr, col, nnz, op_mask, w, mom32,
                               kappa, status, "tune_build"))
    return r;
  LABFM_WORKSPACE(workspace, workspace_bytes, build_work_bytes(n), "tune_build");
  hipStream_t st = as_stream(stream_);
  if (from_cache) *from_cache = 0;

  // the cache key: device, node set (size, stencil entries, nodes per
  // order) and the outputs requested
  const std::string path = tune_cache_path(cache_path);
  std::vector<TuneEntry> entry(1);
  if (!path.empty()) {
    int starts[17] = {0};
    if (int r = order_buckets(order_m, n, static_cast<int*>(workspace), starts, st)) return r;
    std::string key = "build/" + tune_device_key() + "/n" + std::to_string(n) + "/nnz" +
                      std::to_string(static_cast<long long>(nnz)) + "/orders";
    for (int b = 0; b < 16; ++b)
      if (starts[b + 1] > starts[b])
        key += ":" + std::to_string(15 - b) + "x" + std::to_string(starts[b + 1] - starts[b]);
    char tail[64];
    std::snprintf(tail, sizeof tail, "/ops%x/w32%d/rowsum%d", op_mask, w32 ? 1 : 0,
                  rowsum ? 1 : 0);
    entry[0].key = key + tail;
    if (tune_cache_lookup(path, entry)) {
      const labfm_build_config c{entry[0].a, entry[0].b};
      if (labfm_set_build_config(&c) == LABFM_OK) {
        *best = c;
        *best_ms = entry[0].ms;
        if (from_cache) *from_cache = 1;
        return labfm_build_weights(x, y, h, s, order_m, n, box, row_ptr, col, nnz, op_mask, w,
                                   w32, mom32, kappa, rowsum, status, workspace,
                                   workspace_bytes, stream_);
      }
      clear_error();  // an entry the library no longer accepts: tune again
    }
  }

  const labfm_build_config cands[6] = {{LABFM_BUILD_WAVE, 0},
                                       {LABFM_BUILD_BLOCK, 0},
                                       {LABFM_BUILD_PERSISTENT, 0},
                                       {LABFM_BUILD_PERSISTENT, 2},
                                       {LABFM_BUILD_BUCKETED, 0},
                                       {LABFM_BUILD_ROWS, 0}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LABFM_HIP(hipEventCreate(&e0));
  LABFM_HIP(hipEventCreate(&e1));
  double bms = 1e300;
  labfm_build_config bc = cands[5];
  int rc = LABFM_OK;
  for (int k = 0; k < 6 && rc == LABFM_OK; ++k) {
    labfm_set_build_config(&cands[k]);
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess)
      rc = labfm_build_weights(x, y, h, s, order_m, n, box, row_ptr, col, nnz, op_mask, w, w32,
                               mom32, kappa, rowsum, status, workspace, workspace_bytes, stream_);
    if (rc == LABFM_OK && e == hipSuccess) e = hipEventRecord(e1, st);
    if (rc == LABFM_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (rc == LABFM_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      set_error("tune_build: %s", hipGetErrorString(e));
      rc = LABFM_ERR_HIP;
    }
    if (rc == LABFM_OK && ms < bms) {
      bms = ms;
      bc = cands[k];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LABFM_OK) return rc;
  labfm_set_build_config(&bc);
  *best = bc;
  *best_ms = bms;
  // leave the outputs of the chosen distribution in place
  rc = labfm_build_weights(x, y, h, s, order_m, n, box, row_ptr, col, nnz, op_mask, w, w32, mom32,
                           kappa, rowsum, status, workspace, workspace_bytes, stream_);
  if (rc != LABFM_OK || path.empty()) return rc;
  entry[0].a = bc.mode;
  entry[0].b = bc.workgroups_per_cu;
  entry[0].ms = bms;
  std::string err;
  if (!tune_cache_store(path, entry, err)) {
    set_error("tune_build: tune cache: %s", err.c_str());
    return LABFM_ERR_ARG;
  }
  return LABFM_OK;
}

// Workspace of labfm_optimise_stencils: the node list, the x, y and L
// weights of a pass, and the per-node state.
struct OptLayout {
  size_t list, w, h, kappa, k, iters, active, status, remaining, total;
  OptLayout(int32_t n, int64_t nnz) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
      const size_t at = o;
      o += align256(bytes);
      return at;
    };
    list = take(build_work_bytes(n));
    w = take(sizeof(double) * 3 * static_cast<size_t>(nnz));
    h = take(sizeof(double) * static_cast<size_t>(n));
    kappa = take(sizeof(double) * static_cast<size_t>(n));
    k = take(sizeof(int) * static_cast<size_t>(n));
    iters = take(sizeof(int) * static_cast<size_t>(n));
    active = take(static_cast<size_t>(n));
    status = take(static_cast<size_t>(n));
    remaining = take(sizeof(int));
    total = o;
  }
};

extern "C" size_t labfm_optimise_workspace_bytes(int32_t n, int64_t nnz) {
  return (n > 0 && nnz >= 0) ? OptLayout(n, nnz).total : 0;
}

extern "C" int labfm_optimise_stencils(const double* x, const double* y, const double* h0,
                                       const double* s, const int8_t* order_m, int32_t n,
                                       labfm_box box, const int32_t* row_ptr, const int32_t* col,
                                       int64_t nnz, const labfm_stencil_opt_params* prm,
                                       double* h_out, int32_t* iters, void* workspace,
                                       size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0, "optimise_stencils: n must be positive (got %d)", n);
  LABFM_REQUIRE(x && y && h0 && s && order_m && row_ptr && h_out,
                "optimise_stencils: null pointer argument");
  LABFM_REQUIRE(nnz >= 0 && (nnz == 0 || col), "optimise_stencils: bad CSR arguments");
  labfm_stencil_opt_params p{0.99, 1.01, 1e4, 200};
  if (prm) p = *prm;
  LABFM_REQUIRE(p.shrink > 0.0 && p.shrink < 1.0 && p.gain_max > 0.0 && p.res_coef > 0.0 &&
                    p.max_iter >= 0 && p.max_iter <= 10000,
                "optimise_stencils: bad parameters");
  const OptLayout L(n, nnz);
  LABFM_WORKSPACE(workspace, workspace_bytes, L.total, "optimise_stencils");
  hipStream_t st = as_stream(stream_);
  char* base = static_cast<char*>(workspace);
  int* work = reinterpret_cast<int*>(base + L.list);
  int* list = work + kBuildWorkInts;
  int starts[17] = {0};
  if (int r = order_buckets(order_m, n, work, starts, st)) return r;
  // bucket b holds order 15 - b: orders 10..1 are buckets 5..14
  int mmax = 0;
  for (int b = 5; b <= 14; ++b)
    if (starts[b + 1] > starts[b]) {
      mmax = 15 - b;
      break;
    }
  const int first = starts[5], count = starts[15] - starts[5];
  OptArgs a{};
  a.x = x;
  a.y = y;
  a.s = s;
  a.order = order_m;
  a.box = box;
  a.row_ptr = row_ptr;
  a.col = col;
  a.nnz = nnz;
  a.w = reinterpret_cast<double*>(base + L.w);
  a.status = reinterpret_cast<int8_t*>(base + L.status);
  a.h = reinterpret_cast<double*>(base + L.h);
  a.k = reinterpret_cast<int*>(base + L.k);
  a.active = reinterpret_cast<int8_t*>(base + L.active);
  a.remaining = reinterpret_cast<int*>(base + L.remaining);
  a.h_out = h_out;
  a.iters = iters ? iters : reinterpret_cast<int*>(base + L.iters);
  a.shrink = p.shrink;
  a.gain_max = p.gain_max;
  a.res_coef = p.res_coef;
  a.max_iter = p.max_iter;
  hipLaunchKernelGGL(stencil_opt_init_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, h0,
                     order_m, n, a.h, a.k, a.active, a.h_out, a.iters, a.remaining, count);
  LABFM_HIP(hipGetLastError());
  if (count == 0) return LABFM_OK;
  // x, y and L weights of the nodes still shrinking, at their current scales
  BuildArgs g{x, y, a.h, s, order_m, n, box, row_ptr, col, nnz,
              reinterpret_cast<double*>(base + L.w), nullptr, nullptr,
              reinterpret_cast<double*>(base + L.kappa), nullptr,
              reinterpret_cast<int8_t*>(base + L.status),
              rows_of_mask((1u << LABFM_OP_X) | (1u << LABFM_OP_Y) | (1u << LABFM_OP_L))};
  g.active = a.active;
  // a node takes at most max_iter + 2 tests (the last one rejected)
  for (int pass = 0; pass <= p.max_iter + 1; ++pass) {
    for (int m = 1; m <= kMaxOrder; ++m) {
      const int b = 15 - m;
      const int cnt = starts[b + 1] - starts[b];
      if (cnt <= 0) continue;
      const hipError_t e = with_rows_order(m, [&](auto M) {
        return launch_rows<decltype(M)::value>(g, list + starts[b], cnt, st);
      });
      LABFM_HIP(e);
    }
    const hipError_t e = with_mmax(mmax, [&](auto M) {
      hipLaunchKernelGGL(stencil_accept_kernel<decltype(M)::value>, dim3(count), dim3(64), 0, st,
                         a, list + first, count);
      return hipGetLastError();
    });
    LABFM_HIP(e);
    int left = 0;
    LABFM_HIP(hipMemcpyAsync(&left, a.remaining, sizeof(int), hipMemcpyDeviceToHost, st));
    LABFM_HIP(hipStreamSynchronize(st));
    if (left == 0) return LABFM_OK;
  }
  set_error("optimise_stencils: %s", "nodes still shrinking after max_iter + 2 passes");
  return LABFM_ERR_HIP;
}
