/*
 * labfm.h - C ABI of the MI355X (gfx950) LABFM hot-path library.
 *
 * LABFM (local anisotropic basis function method, King & Lind, arXiv
 * 2102.02019) builds high-order mesh-free derivative operators
 *     L^d_i(phi) = sum_j (phi_j - phi_i) w^d_ji            (eq. general_do)
 * from a per-node linear system over Hermite anisotropic basis functions,
 * and uses them in an explicit Runge-Kutta solve of the isothermal
 * compressible Navier-Stokes equations.
 *
 * Conventions shared by every call:
 *  - Arrays are DEVICE pointers (HIP device memory) unless marked "host".
 *    The caller owns every buffer; no call keeps a pointer after it returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on that stream and the call returns without waiting,
 *    except where a host output is documented (then the call synchronises
 *    the stream before returning).
 *  - No call allocates device memory. A call that needs temporary device
 *    memory takes a caller workspace (`workspace`, `workspace_bytes`): a
 *    device buffer of at least the size its labfm_*_workspace_bytes
 *    function returns, overwritten by the call; a smaller or NULL workspace
 *    is LABFM_ERR_ARG. The call's work on `stream` may still use the
 *    workspace after it returns: keep it allocated until that work is done
 *    (stream-ordered reuse, as torch's caching allocator does, is safe).
 *  - Every call returns LABFM_OK (0) or a negative status; none throws across
 *    the ABI. labfm_last_error() returns a message for the calling thread's
 *    most recent failure.
 *  - Node arrays are structure-of-arrays, float64, length n; fields of the
 *    evolved state are stored one after another: q = [ln rho | u | v], each
 *    of length n.
 *  - Stencils are CSR: row_ptr int32[n+1] (row_ptr[0] = 0), col int32[nnz],
 *    the neighbours of node i in ascending index order, i itself excluded.
 *  - Operator weights are stored one operator after another:
 *    w[op * nnz + e] for edge e of the CSR, op in labfm_op order. The
 *    float32 copy w32 uses a padded row stride, w32[op * labfm_w32_stride(nnz)
 *    + e], so that every operator's row starts on a 128-byte boundary (the
 *    float32 gathers load four consecutive edges per lane); its entries past
 *    nnz in each row are never read as weights.
 */
#ifndef LABFM_H
#define LABFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  LABFM_OK = 0,
  LABFM_ERR_ARG = -1,         /* invalid argument (null pointer, size, box) */
  LABFM_ERR_HIP = -2,         /* a HIP runtime call failed */
  LABFM_ERR_CAPACITY = -3,    /* output capacity too small (size reported) */
  LABFM_ERR_NONFINITE = -4,   /* a non-finite value appeared in the state */
  LABFM_ERR_UNSUPPORTED = -5  /* request outside what the library implements */
};

/* Operator index (row of the weight array). The first five are the
 * derivative operators used by the Navier-Stokes right-hand side; the last
 * is the hyperviscous filter operator nabla^m (nabla^(m-1) for odd m). */
typedef enum {
  LABFM_OP_X = 0,   /* d/dx                       C^x: x        */
  LABFM_OP_Y = 1,   /* d/dy                       C^y: y        */
  LABFM_OP_L = 2,   /* Laplacian d2/dx2 + d2/dy2  C^L: x^2 + y^2 */
  LABFM_OP_XX = 3,  /* d2/dx2                                   */
  LABFM_OP_XY = 4,  /* d2/dxdy                                  */
  LABFM_OP_HYP = 5, /* nabla^m (filter)                         */
  LABFM_NUM_OPS = 6
} labfm_op;

/* Arithmetic of operator application. */
typedef enum {
  LABFM_F64 = 0,      /* float64 weights and fields, float64 sums */
  LABFM_F32W = 1,     /* float32 weights, float64 differences and sums */
  LABFM_F32_COMP = 2  /* float32 weights; differences phi_j - phi_i formed in
                         float64 and rounded to float32; products and sums
                         compensated (error-free TwoProd + TwoSum, "Dot2") */
} labfm_prec;

/* Per-node status written by labfm_build_weights. */
enum {
  LABFM_NODE_OK = 0,
  LABFM_NODE_SINGULAR = 1,       /* a zero pivot in the LU factorisation */
  LABFM_NODE_FEW_NEIGHBOURS = 2, /* fewer neighbours than moments (K < n) */
  LABFM_NODE_BAD_FILTER = 3,     /* filter calibration F_0 zero/non-finite */
  LABFM_NODE_BAD_ORDER = 4       /* order_m outside 1..10 (weights set to 0) */
};

/* Rectangular domain [0, Lx) x [0, Ly); each axis periodic (1) or not (0).
 * Positions must lie inside the box. */
typedef struct {
  double Lx, Ly;
  int32_t periodic_x, periodic_y;
} labfm_box;

/* Node tiles for the LDS-staged gather kernels (labfm_build_tiles): tile t
 * holds nodes [t*LABFM_TILE_NODES, (t+1)*LABFM_TILE_NODES); its halo is the
 * ascending list of distinct neighbour indices of its rows. */
#define LABFM_TILE_NODES 32
#define LABFM_TILE_HALO_MAX 1024
typedef struct {
  int32_t ntiles;             /* labfm_tile_count(n) */
  int32_t max_halo;           /* largest halo of any tile */
  const int32_t* halo_count;  /* int32[ntiles] */
  const int32_t* halo_idx;    /* int32[ntiles * LABFM_TILE_HALO_MAX] */
  const uint16_t* lcol;       /* uint16[nnz]: position of col[e] in its tile's halo */
} labfm_tiles;

/* First moments of the float32 weights of the second-derivative operators,
 * mu^d_i = (sum_j w32^d_ji x_ji, sum_j w32^d_ji y_ji) for d = L, xx, xy,
 * evaluated in float64 and stored as float32[LABFM_NUM_MOM32 * n], rows
 * (L,x) (L,y) (xx,x) (xx,y) (xy,x) (xy,y). The moment conditions of the
 * weight system (eq. lsys) make these sums zero for the float64 weights; for
 * the rounded weights they are not, and phi's gradient then leaks into the
 * second derivatives with an error of order eps32 |grad phi| / h. The float32
 * precisions subtract grad(phi)_i . mu^d_i (the gradient from the x and y
 * operators), which leaves an error of order eps32 independent of h. */
#define LABFM_NUM_MOM32 6

/* Operators of a node set, as built by labfm_build_weights. */
typedef struct {
  int32_t n;                /* nodes */
  int64_t nnz;              /* CSR entries */
  const int32_t* row_ptr;   /* int32[n+1] */
  const int32_t* col;       /* int32[nnz] */
  const double* w;          /* float64[6*nnz], labfm_op order (may be NULL
                               when only the float32 copy is used) */
  const float* w32;         /* float32[6*labfm_w32_stride(nnz)] or NULL */
  const float* mom32;       /* float32[LABFM_NUM_MOM32*n] first moments of w32
                               (required with w32 for the float32 precisions) */
  const double* kappa;      /* float64[n] filter coefficients */
  const labfm_tiles* tiles; /* host pointer to tiles, or NULL: when set, the
                               stage and filter kernels of labfm_rk_step and
                               labfm_ns_rhs stage each tile's halo in LDS */
  const double* wall_normal; /* float64[2n] or NULL: (n_x, n_y) of the unit
                               normal into the fluid at no-slip wall nodes,
                               (0, 0) at every other node (as written by
                               labfm_boundary_weights). When set, the stage
                               kernels solve the wall equation at wall nodes
                               (see labfm_rk_step) and the filter leaves their
                               velocity unchanged. */
} labfm_operators;

/* Constants of the isothermal flow and of the integration. */
typedef struct {
  double c2;        /* speed of sound squared, p = c2 * rho */
  double mu;        /* dynamic viscosity (uniform) */
  double gx, gy;    /* body force */
  double dt;        /* time step, > 0 */
  int32_t filter;   /* 1: filter ln rho, u, v after every step */
  int32_t check_finite; /* 1: test the state once at the end of the call
                           (synchronises) and report LABFM_ERR_NONFINITE */
} labfm_rk_params;

/* Kernel timings collected by labfm_rk_step when requested. Durations are
 * measured with HIP events recorded on the call's stream around each launch
 * of the timed steps (summed over them). `every` is read: one step in every
 * `every` is timed (0 or 1: all of them), the others run without events, so
 * a long run is sampled without an event pair and a host query per launch. */
typedef struct {
  double stage_ms;        /* timed Runge-Kutta stage launches */
  double filter_ms;       /* timed filter launches */
  int64_t stage_launches; /* launches timed */
  int64_t filter_launches;
  int32_t every;          /* input: time steps 0, every, 2 every, ... */
} labfm_timing;

/* Gather kernels whose launch shape can be chosen (labfm_set_launch_config,
 * labfm_tune). */
typedef enum {
  LABFM_KERNEL_STAGE = 0,   /* fused RK stage (and labfm_ns_rhs) */
  LABFM_KERNEL_FILTER = 1,  /* filter pass of labfm_rk_step */
  LABFM_KERNEL_APPLY = 2    /* labfm_apply_operators */
} labfm_kernel;

/* Launch-shape flags. */
#define LABFM_LAUNCH_XCD_ORDER 1 /* workgroups of each XCD take one contiguous node range */
#define LABFM_LAUNCH_STREAMING 2 /* weights and indices loaded non-temporally */

/* Launch shape of a gather kernel: lanes_per_node lanes of a 64-lane
 * wavefront share one node's row (4, 8, 16 or 32), plus flags. */
typedef struct {
  int32_t lanes_per_node;
  int32_t flags;
} labfm_launch_config;

/* Row stride, in elements, of the float32 weight copy w32: nnz rounded up
 * to a multiple of 32 (128 bytes). A w32 buffer holds 6 such rows and starts
 * on a 128-byte boundary (device allocations do). */
int64_t labfm_w32_stride(int64_t nnz);

/* Message of the calling thread's last failure ("" if none). */
const char* labfm_last_error(void);

/* Library version string. */
const char* labfm_version(void);

/*
 * Morton (Z-order) permutation of a node set, the binning that keeps nodes
 * close in space close in memory (the stencil is purely geometric: sorting
 * the nodes changes no result, only the locality of the gathers). Node i's
 * cell is (ix, iy) = (floor(x_i / cell), floor(y_i / cell)) clamped to
 * 0..ceil(L/cell)-1; its key interleaves the bits of ix (even positions)
 * and iy (odd positions); perm lists the node indices in ascending key order,
 * nodes of equal key in ascending index (stable).
 *
 *   x, y   float64[n] positions.
 *   cell   cell side, > 0, at most 2^21 cells per axis.
 *   perm   int32[n] output.
 *   workspace  labfm_morton_workspace_bytes(n) bytes (keys and the radix
 *              sort's storage).
 * Synchronises.
 */
size_t labfm_morton_workspace_bytes(int32_t n);
int labfm_morton_order(const double* x, const double* y, int32_t n, labfm_box box, double cell,
                       int32_t* perm, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Stencil search (stencil definition of the paper's LABFM section): node j
 * is a neighbour of node i iff j != i and |r_ji| <= 2 h_i, where
 * r_ji = r_j - r_i is taken to the nearest periodic image on periodic axes
 * and the test is evaluated as dx*dx + dy*dy <= (2h_i)*(2h_i) with every
 * product and sum rounded separately (bit-reproducible).
 *
 *   x, y, h   float64[n] positions (inside the box) and stencil scales.
 *   row_ptr   int32[n+1] output.
 *   col       int32[capacity] output, or NULL to query the size.
 *   nnz_out   host: receives the number of CSR entries.
 *   workspace labfm_neighbours_workspace_bytes(n) bytes (the cell table,
 *             the per-node counts and rocPRIM's temporary storage).
 *
 * Synchronises the stream once (to size the CSR); the fill of col is
 * enqueued after that. Returns LABFM_ERR_CAPACITY (with *nnz_out set and
 * row_ptr filled) when col is NULL or capacity < nnz. Returns LABFM_ERR_ARG
 * when a periodic axis is shorter than 4 max(h) (the nearest image would not
 * be unique) or n <= 0.
 */
size_t labfm_neighbours_workspace_bytes(int32_t n);
int labfm_build_neighbours(const double* x, const double* y, const double* h, int32_t n,
                           labfm_box box, int32_t* row_ptr, int32_t* col, int64_t capacity,
                           int64_t* nnz_out, void* workspace, size_t workspace_bytes,
                           void* stream);

/*
 * Weight construction (sections "LABFM" and "New ABFs"; eqs. disc_form,
 * lsys, w_abf, hermite; filter calibration of section "Spatial filtering").
 * For each node i of order m_i (1..10), with n = (m^2+3m)/2 moments:
 *   X~_ji^q = (x_ji/h)^a (y_ji/h)^b / (a! b!)           scaled monomials
 *   W_ji^q  = psi(|r_ji|/h) He_a(x_ji/h) He_b(y_ji/h)  Hermite ABFs
 *             (He = probabilists' Hermite, equal to the paper's
 *              H_a(z/sqrt2)/sqrt(2^a)); psi = Wendland C2,
 *             psi(q) = (1-q/2)^4 (1+2q) for q < 2
 *   M~_i = sum_j X~_ji (outer) W_ji,  M~_i Psi^d = C~^d  (LU, partial pivoting)
 *   w^d_ji = W_ji . Psi^d
 * for the six operators of labfm_op, then
 *   F_0,i = sum_j [1 - cos(k x_ji) cos(k y_ji)] w^hyp_ji, k = 2 pi / (3 s_i),
 *   kappa_i = 2 / (3 F_0,i).
 *
 *   x, y, h, s  float64[n]; s = local node spacing (filter calibration).
 *   order_m     int8[n], each in 1..10.
 *   row_ptr, col, nnz  CSR from labfm_build_neighbours.
 *   op_mask which operators' weights are written (bit d for labfm_op d;
 *           0x3F = all six, which labfm_apply_operators, labfm_ns_rhs and
 *           labfm_rk_step expect). The k = popcount(op_mask) selected
 *           operators fill rows 0..k-1 of w, w32 and rowsum in labfm_op
 *           order. kappa is always formed (from the filter weights, computed
 *           whether or not bit 5 is set).
 *   w       float64[k*nnz] output.
 *   w32     float32[k*labfm_w32_stride(nnz)] output copy (rows of the padded
 *           stride), or NULL.
 *   mom32   float32[LABFM_NUM_MOM32*n] output first moments of w32 (see
 *           LABFM_NUM_MOM32), or NULL; needs L, xx and xy in op_mask.
 *   kappa   float64[n] output.
 *   rowsum  float64[k*n] output sum_j w^d_ji, or NULL.
 *   status  int8[n] output, LABFM_NODE_* per node.
 *   workspace  labfm_build_workspace_bytes(n) bytes (the node list grouped
 *           by order).
 *
 * Numerical failures and out-of-range orders are reported per node in
 * status (the call still returns LABFM_OK); such nodes get zero weights and
 * kappa = 0 except for LABFM_NODE_FEW_NEIGHBOURS, whose weights are those of
 * the (rank-deficient) solve when it completes. Nodes of different orders and
 * stencil sizes are built in one call; labfm_set_build_config selects how
 * they are spread over the GPU (default LABFM_BUILD_ROWS: one wavefront per
 * node holding the system's rows in registers, from a work list grouped by
 * order; labfm_tune_build picks). Synchronises once (the launches are sized on the
 * host from the order histogram); the build kernels are enqueued after that.
 */
size_t labfm_build_workspace_bytes(int32_t n);
int labfm_build_weights(const double* x, const double* y, const double* h, const double* s,
                        const int8_t* order_m, int32_t n, labfm_box box,
                        const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                        uint32_t op_mask, double* w, float* w32, float* mom32, double* kappa,
                        double* rowsum, int8_t* status, void* workspace,
                        size_t workspace_bytes, void* stream);

/*
 * labfm_build_weights for callers that cannot allocate device memory, not
 * even a workspace (tight serving or time-stepping loops, harnesses that
 * forbid hipMalloc): the same arguments (without the workspace), kernels
 * and results, with the work list held in a static device array of the
 * library. The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).
 *
 *   n  at most LABFM_NOALLOC_MAX_NODES; larger sets return LABFM_ERR_ARG
 *      (use labfm_build_weights).
 * The array, (64 + LABFM_NOALLOC_MAX_NODES) int32 = 16 MiB, is held by every
 * GPU the library runs on until the process ends, and is shared by all calls
 * on that GPU: calls that overlap on one GPU (from several host threads or
 * streams) race and must be serialised by the caller. Each call clears what
 * it uses; nothing is kept between calls. Synchronises once, like
 * labfm_build_weights.
 */
#define LABFM_NOALLOC_MAX_NODES 4194304
int labfm_build_weights_noalloc(const double* x, const double* y, const double* h,
                                const double* s, const int8_t* order_m, int32_t n, labfm_box box,
                                const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                                uint32_t op_mask, double* w, float* w32, float* mom32,
                                double* kappa, double* rowsum, int8_t* status, void* stream);

/*
 * The weight build's LU with partial pivoting and back substitution on
 * given systems M~ Psi = C~ (section "The Local Anisotropic Basis Function
 * Method", the linear system of each node and its solution by LU with
 * partial pivoting): the rows-in-registers kernel of LABFM_BUILD_ROWS runs
 * them in place of the systems it assembles, one wavefront per system, so
 * its pivot rule and solution can be checked against a host solver.
 *
 *   m          order 1..10; n = (m^2+3m)/2.
 *   systems    float64[count*n*(n+6)] device, row-major: row r of system k
 *              at (k*n + r)*(n+6), its n entries of M~, then its six of C~.
 *   psi        float64[count*n*6] device output: Psi[k][q][d], the solution
 *              column d in the operators' order (labfm_op).
 *   pivot_row  int32[count*n] device output: [k][c] = the row (0..n-1, the
 *              given order) whose entry was column c's pivot. The pivot of a
 *              column is its largest |entry| among the rows not yet used,
 *              magnitudes compared exactly (as their float64 bit patterns),
 *              the lowest row on equal magnitudes.
 *   status     int8[count] device output: LABFM_NODE_OK, or
 *              LABFM_NODE_SINGULAR when a pivot is zero or not finite (then
 *              psi and pivot_row of that system are not written).
 * The buffers belong to the caller; nothing is allocated and the call does
 * not synchronise. Returns LABFM_ERR_ARG for m outside 1..10, count < 0 or
 * a null buffer (count > 0); count = 0 does nothing.
 */
int labfm_solve_systems(int32_t m, const double* systems, int32_t count, double* psi,
                        int32_t* pivot_row, int8_t* status, void* stream);

/*
 * Stencil optimisation (section "Stencil optimisation"): for every node, the
 * stencil scale h_i shrinks from h0_i by the factor `shrink` while the
 * stencil passes two tests, and the last scale that passed is kept (h0_i
 * when none did):
 *   1. the residual of the node's Laplacian system is small:
 *        alpha_L = || M Psi^L - C^L ||_2 <= res_coef eps n^4 / (h_i m)
 *      with M, Psi, C of the unscaled system (monomials x^a y^b/(a!b!),
 *      C^L = 1 at x^2 and y^2), eps the float64 machine epsilon;
 *   2. no amplitude response exceeds gain_max at the 16 wavenumbers
 *      k = q pi / (16 s_i), q = 1..16:
 *        A^x = L^x(sin k x)/k, A^y = L^y(sin k y)/k,
 *        A^L = L^L(1/2 - cos(k x) cos(k y)/2)/k^2.
 * Each test at scale h builds the node's system on its h0 stencil
 * (neighbours beyond 2h have psi = 0 and drop out). The loop runs in passes
 * over all nodes: the x, y and L weights of every node still shrinking, at
 * its current scale (the rows-in-registers build), then the tests; a node
 * leaves at its first failed test, at a singular system, or after max_iter
 * accepted shrinks. The paper prints
 * res_coef = 1e-4 for its own solver and notes it is solver-specific; with
 * this residual even the initial stencils fail at 1e-4, and below about 1e4
 * the test acts on rounding noise. The default, 1e4, stops the shrinking
 * where the system becomes singular (the residual then jumps by many orders
 * of magnitude from one scale to the next).
 *
 *   x, y, s, order_m   float64[n], int8[n] as for labfm_build_weights.
 *   h0                 float64[n] initial stencil scales (the paper: 2.8 s).
 *   row_ptr, col, nnz  CSR of the h0 stencils (labfm_build_neighbours with h0).
 *   prm                host parameters, or NULL for {0.99, 1.01, 1e4, 200}.
 *   h_out              float64[n] output scales.
 *   iters              int32[n] output k with h_out = h0 shrink^k (by repeated
 *                      multiplication), or NULL.
 *   workspace          labfm_optimise_workspace_bytes(n, nnz) bytes: the node
 *                      list, one pass's x, y and L weights (3 nnz doubles)
 *                      and the per-node state.
 * Nodes with orders outside 1..10 keep h0. Synchronises once to size the
 * launches, then once per pass (to see whether any node is still shrinking).
 */
size_t labfm_optimise_workspace_bytes(int32_t n, int64_t nnz);
typedef struct {
  double shrink;    /* factor applied to h per accepted step (paper: 0.99) */
  double gain_max;  /* largest accepted amplitude response (paper: 1.01) */
  double res_coef;  /* coefficient of the residual bound */
  int32_t max_iter; /* cap on accepted shrinks per node */
} labfm_stencil_opt_params;

int labfm_optimise_stencils(const double* x, const double* y, const double* h0, const double* s,
                            const int8_t* order_m, int32_t n, labfm_box box,
                            const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                            const labfm_stencil_opt_params* prm, double* h_out, int32_t* iters,
                            void* workspace, size_t workspace_bytes, void* stream);

/*
 * Boundary strips (section "Boundaries", subsection "Boundary
 * discretisation"). Along a wall the node set carries a locally orthogonal
 * strip five nodes thick: each wall node i0 has nodes i1..i4 at
 * r_i0 + q s n (q = 1..4), with s the wall node's spacing and n its unit
 * normal pointing into the fluid. One column per wall node; every node lies
 * in at most one column.
 */
#define LABFM_STRIP_DEPTH 5
typedef struct {
  int32_t count;          /* columns (wall nodes), >= 0 */
  const int32_t* column;  /* int32[5*count]: column[5k + q] is the node at level q
                             of column k (q = 0 the wall node) */
  const double* normal;   /* float64[2*count]: (n_x, n_y) of column k, unit,
                             into the fluid */
} labfm_strips;

/*
 * Boundary operators of table tab:boundaries, written over the output of
 * labfm_build_weights (which must have run first on the same stencils, with
 * order 4 at levels 0..2 and stencils containing the whole column of every
 * strip node). For every column and level q = 0, 1, 2, node i of the column,
 * with t = (-n_y, n_x):
 *   d/dxi:  5-point finite difference along the column with spacing s of the
 *           column's wall node: one-sided (offsets 0..4) at i0, asymmetric
 *           (-1..3) at i1, centred (-2..2) at i2;
 *   d/deta: one-dimensional LABFM of order 4 (Appendix A) over B_i, the
 *           stencil neighbours on the same level whose column normal is
 *           within 60 degrees of n: eta_ji = r_ji . t, monomials
 *           (eta/h)^k / k!, ABFs psi(|eta|/h) He_k(eta/h) (k = 1..4, the
 *           probabilists' form of the appendix's H_k(z/sqrt2)/sqrt(2^k)),
 *           target h^-1 e_1, solved with partial pivoting;
 *   w^x = n_x w^xi + t_x w^eta,  w^y = n_y w^xi + t_y w^eta  (the Jacobian of
 *           the subsection).
 * At wall nodes (q = 0) also: w^L = w^xx = w^xy = 0 (the imposed velocity and
 * the wall's ln rho equation use no second derivative); w^hyp = the 1D LABFM
 * d^4/deta^4 (target h^-4 e_4), a filter along the wall only; kappa from
 * w^hyp by the calibration of labfm_build_weights; wall_normal = n. Levels 1
 * and 2 keep their two-dimensional second-derivative and filter operators.
 *
 *   x, y, h, s, n, box, row_ptr, col, nnz  as for labfm_build_weights.
 *   strips        host pointer to the columns (device arrays inside).
 *   w             float64[6*nnz], updated in place (a build with op_mask 0x3F:
 *                 all six rows).
 *   w32, mom32    float32 copies and first moments, updated to match, or NULL.
 *   kappa         float64[n], updated at wall nodes.
 *   status        int8[n], updated: LABFM_NODE_SINGULAR when the 1D system is
 *                 singular, LABFM_NODE_FEW_NEIGHBOURS when a column node is
 *                 missing from the stencil (the node's x and y weights are then
 *                 zero), LABFM_NODE_BAD_FILTER; wall nodes otherwise
 *                 LABFM_NODE_OK.
 *   wall_normal   float64[2n] output: n at wall nodes, (0, 0) elsewhere.
 *   workspace     labfm_boundary_workspace_bytes(n) bytes (the per-node map
 *                 of strip levels and columns).
 *
 * Returns LABFM_ERR_ARG for a node index outside 0..n-1, a node listed twice
 * or a normal that is not of unit length (checked on the host: the call copies
 * the columns back and synchronises).
 */
size_t labfm_boundary_workspace_bytes(int32_t n);
int labfm_boundary_weights(const double* x, const double* y, const double* h, const double* s,
                           int32_t n, labfm_box box, const int32_t* row_ptr, const int32_t* col,
                           int64_t nnz, const labfm_strips* strips, double* w, float* w32,
                           float* mom32, double* kappa, int8_t* status, double* wall_normal,
                           void* workspace, size_t workspace_bytes, void* stream);

/* How labfm_build_weights distributes nodes over the GPU. */
enum {
  LABFM_BUILD_WAVE = 1,        /* one 64-lane wavefront per node */
  LABFM_BUILD_BLOCK = 2,       /* one 256-thread workgroup (4 wavefronts) per node */
  LABFM_BUILD_PERSISTENT = 3,  /* one launch of persistent 256-thread workgroups taking
                                  nodes (highest order first) from a work counter */
  LABFM_BUILD_BUCKETED = 4,    /* one 256-thread-per-node launch per order class */
  LABFM_BUILD_ROWS = 5         /* one 64-lane wavefront per node holding the system's
                                  rows in registers (orders 1..10, one launch per
                                  order present; at order 10 the pivot row of the
                                  first column is kept in LDS and the other 64
                                  rows fill the lanes);
                                  out-of-range orders take the workgroup-per-node
                                  kernel, which marks them unsupported */
};
typedef struct {
  int32_t mode;               /* LABFM_BUILD_*; default LABFM_BUILD_ROWS */
  int32_t workgroups_per_cu;  /* persistent mode: 0 = as many as fit */
} labfm_build_config;

/* Process-wide build distribution (NULL restores the default). */
int labfm_set_build_config(const labfm_build_config* cfg);
int labfm_get_build_config(labfm_build_config* cfg);

/*
 * Autotuner of the build: runs labfm_build_weights with every distribution
 * on the given node set (same arguments, outputs and workspace), installs
 * the fastest as the process-wide setting and reports it (best_ms: its
 * duration, measured with HIP events on `stream`). The outputs hold the
 * weights built with the chosen distribution. Synchronises.
 *
 *   cache_path  host string: a tune cache file, or NULL/"" for the file named
 *               by the LABFM_TUNE_CACHE environment variable (no cache when
 *               that is unset too). The cache is a JSON object of entries
 *               "key": [a, b, ms]; a build's key names the device (its
 *               architecture and compute units), n, nnz, the node count of
 *               each order, op_mask and which of w32 and rowsum are written.
 *               On a hit the cached distribution is installed and the
 *               weights are built once with it; otherwise the tuned choice
 *               is added to the file (written to a temporary file, then
 *               renamed over it; LABFM_ERR_ARG if that fails).
 *   from_cache  host, or NULL: 1 when the choice came from the cache.
 */
int labfm_tune_build(const double* x, const double* y, const double* h, const double* s,
                     const int8_t* order_m, int32_t n, labfm_box box, const int32_t* row_ptr,
                     const int32_t* col, int64_t nnz, uint32_t op_mask, double* w, float* w32,
                     float* mom32, double* kappa, double* rowsum, int8_t* status,
                     void* workspace, size_t workspace_bytes, const char* cache_path,
                     labfm_build_config* best, double* best_ms, int32_t* from_cache,
                     void* stream);

/*
 * Operator application, eq. general_do: for each selected operator d (bit d
 * of op_mask, labfm_op order) out_k[i] = sum_j (phi_j - phi_i) w^d_ji, where
 * k counts the selected operators in increasing d. The float32 precisions
 * correct L, xx and xy with the first moments of the float32 weights (see
 * LABFM_NUM_MOM32; the x and y sums are then formed too).
 *
 *   ops     operators (w for LABFM_F64, w32 and mom32 for the float32
 *           precisions).
 *   phi     float64[n] field.
 *   out     float64[popcount(op_mask) * n] output.
 */
int labfm_apply_operators(const labfm_operators* ops, uint32_t op_mask, const double* phi,
                          double* out, labfm_prec prec, void* stream);

/*
 * Time step, eq. dt: dt = min over nodes of min(a s_i/(|u_i| + c),
 * b s_i^2 rho_i / mu), rho = exp(ln rho). The paper's coefficients are
 * a = 1.0 (convective) and b = 0.4 (viscous).
 *
 *   q       float64[3n] state [ln rho | u | v].
 *   s       float64[n] node spacing.
 *   conv_coef, visc_coef  a and b, both > 0.
 *   dt_out  host: receives dt. Synchronises the stream.
 *   workspace  labfm_time_step_workspace_bytes() bytes (per-block minima).
 */
size_t labfm_time_step_workspace_bytes(void);
int labfm_time_step(const double* q, const double* s, int32_t n, double c2, double mu,
                    double conv_coef, double visc_coef, double* dt_out, void* workspace,
                    size_t workspace_bytes, void* stream);

/*
 * Right-hand side of the isothermal Navier-Stokes equations (eq. icns) in
 * (ln rho, u, v), with the derivatives taken by the LABFM operators:
 *   R_l = -(u l_x + v l_y) - (u_x + v_y)
 *   R_u = -(u u_x + v u_y) - c2 l_x + (mu/rho)(4/3 u_xx + u_yy + 1/3 v_xy) + gx
 *   R_v = -(u v_x + v v_y) - c2 l_y + (mu/rho)(4/3 v_yy + v_xx + 1/3 u_xy) + gy
 * with l = ln rho and u_yy = L(u) - u_xx. This is the stage kernel of
 * labfm_rk_step run without the update.
 *
 *   q    float64[3n] state [ln rho | u | v].
 *   prm  c2, mu, gx, gy are used.
 *   out  float64[3n] output [R_l | R_u | R_v]; must not alias q.
 */
int labfm_ns_rhs(const double* q, const labfm_operators* ops, const labfm_rk_params* prm,
                 double* out, labfm_prec prec, void* stream);

/*
 * Launch shape used for `kernel` at precision `prec` on a node set of n
 * nodes and nnz entries (the process-wide setting, or the built-in choice
 * from the mean row length nnz/n when none is set).
 */
int labfm_get_launch_config(int32_t kernel, labfm_prec prec, int32_t n, int64_t nnz,
                            labfm_launch_config* cfg);

/* Sets the process-wide launch shape of `kernel` at `prec`; a NULL cfg or
 * lanes_per_node == 0 restores the built-in choice. LABFM_ERR_ARG for an
 * unsupported shape. */
int labfm_set_launch_config(int32_t kernel, labfm_prec prec, const labfm_launch_config* cfg);

/*
 * Autotuner: times every supported launch shape of the stage, filter and
 * apply kernels on the given operators and state (two interleaved passes of
 * reps launches each, HIP events on `stream`, best mean kept), installs the
 * fastest as the process-wide setting for `prec` and reports it. The default
 * shape is kept unless another is more than 2% faster.
 *
 *   q          float64[3n] state the stage kernel reads (not modified).
 *   workspace  labfm_rk_workspace_bytes(n) bytes (overwritten).
 *   cache_path host string: a tune cache file, or NULL/"" for the file named
 *              by LABFM_TUNE_CACHE (no cache when that is unset too); the
 *              format is that of labfm_tune_build. The three kernels' keys
 *              name the kernel, prec, the device, n, nnz and whether tiles
 *              and wall normals are set. When all three are cached their
 *              shapes are installed without timing anything; otherwise the
 *              tuned shapes are added to the file.
 *   best       host, labfm_launch_config[3] in labfm_kernel order.
 *   best_ms    host, double[3]: mean launch time of each chosen shape.
 *   from_cache host, or NULL: 1 when the shapes came from the cache.
 * Synchronises the stream.
 */
int labfm_tune(const labfm_operators* ops, const double* q, labfm_prec prec, int32_t reps,
               void* workspace, size_t workspace_bytes, const char* cache_path,
               labfm_launch_config* best, double* best_ms, int32_t* from_cache, void* stream);

/* Number of node tiles of a node set of n nodes. */
int32_t labfm_tile_count(int32_t n);

/*
 * Builds the node tiles of a CSR stencil set (a data layout for the gather
 * kernels; it changes no result beyond summation order).
 *
 *   halo_count   int32[labfm_tile_count(n)] output.
 *   halo_idx     int32[labfm_tile_count(n) * LABFM_TILE_HALO_MAX] output.
 *   lcol         uint16[nnz] output.
 *   max_halo_out host: largest halo.
 *   workspace    labfm_tiles_workspace_bytes() bytes (two counters).
 * Synchronises. Returns LABFM_ERR_CAPACITY if a tile's halo exceeds
 * LABFM_TILE_HALO_MAX nodes (then use the operators without tiles).
 */
size_t labfm_tiles_workspace_bytes(void);
int labfm_build_tiles(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz,
                      int32_t* halo_count, int32_t* halo_idx, uint16_t* lcol,
                      int32_t* max_halo_out, void* workspace, size_t workspace_bytes,
                      void* stream);

/* Transposed stencils for the adjoint: for each node j the forward edges
 * i -> j (j in N_i), grouped by j in ascending i, with a copy of their
 * weights, plus the operators' row sums S^d_i = sum_j w^d_ij. */
typedef struct {
  const int32_t* tptr;   /* int32[n+1] */
  const int32_t* tsrc;   /* int32[nnz]: source node i of each entry */
  const double* tw;      /* float64[6*nnz]: w^d_ij of each entry, labfm_op order */
  const double* rowsum;  /* float64[6*n] (labfm_build_weights' rowsum output) */
} labfm_transpose;

/*
 * Builds tptr, tsrc and tw from the operators' CSR and float64 weights
 * (a reordering of data, no arithmetic). workspace:
 * labfm_transpose_workspace_bytes(n, nnz) bytes (counts, cursors, slots).
 */
size_t labfm_transpose_workspace_bytes(int32_t n, int64_t nnz);
int labfm_build_transpose(const labfm_operators* ops, int32_t* tptr, int32_t* tsrc, double* tw,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of workspace labfm_rk_adjoint needs. */
size_t labfm_adjoint_workspace_bytes(int32_t n, int32_t n_steps, int32_t ckpt_every);

/*
 * Adjoint (vector-Jacobian product) of n_steps steps of labfm_rk_step in
 * float64, with the filter when prm->filter is set: given qbar_end, the
 * gradient of a scalar J with respect to the state after n_steps, writes
 * qbar_0 = (d q_end / d q_0)^T qbar_end, the gradient with respect to q0.
 * Operators enter through their transposes A_d^T (gathers over the
 * transposed stencils, no atomics); the state is checkpointed every
 * ckpt_every steps and each segment recomputed once.
 *
 *   q0, qbar_end, qbar_0  float64[3n] ([ln rho | u | v]); qbar_0 may alias
 *                         qbar_end.
 *   workspace             labfm_adjoint_workspace_bytes(n, n_steps,
 *                         ckpt_every) bytes.
 * Operators with wall nodes (ops->wall_normal set) are not supported
 * (LABFM_ERR_UNSUPPORTED).
 */
int labfm_rk_adjoint(const double* q0, const double* qbar_end, double* qbar_0,
                     const labfm_operators* ops, const labfm_transpose* tr,
                     const labfm_rk_params* prm, int32_t n_steps, int32_t ckpt_every,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of device workspace labfm_rk_step needs for n nodes. */
size_t labfm_rk_workspace_bytes(int32_t n);

/*
 * n_steps steps of the four-stage, third-order, low-storage Runge-Kutta
 * scheme RK3(2)4[2R+]C (Kennedy, Carpenter & Lewis 2000) applied to the
 * isothermal Navier-Stokes equations in (ln rho, u, v) (eq. icns, with
 * p = c2 rho so that grad(p)/rho = c2 grad(ln rho)), each step followed by
 * the filter phi <- phi + kappa_i L^hyp_i(phi) on ln rho, u and v when
 * prm->filter is set.
 *
 * With ops->wall_normal set, wall nodes (normal n != 0) of a no-slip wall
 * keep their velocity (the caller starts them at u = v = 0) and evolve ln rho
 * by the characteristic form eq. lodilnro: with xi along n, eta along
 * t = (-n_y, n_x), c = sqrt(c2), L2 = 0 and the incoming wave set to
 * L4 = L1 + 2 rho c g.n,
 *   R_l = (c - u_xi)(d lnrho/dxi - (d u_xi/dxi)/c) - 2 (g.n)/c
 *         - u_eta d lnrho/deta - d u_eta/deta,
 * the derivatives taken from the node's x and y operators. The filter leaves
 * the wall velocity unchanged.
 *
 *   q          float64[3n] state [ln rho | u | v], updated in place.
 *   ops        operators (w and kappa for LABFM_F64; w32 and kappa for
 *              LABFM_F32W and LABFM_F32_COMP; the state stays float64).
 *   workspace  device buffer of labfm_rk_workspace_bytes(n) bytes.
 *   use_graph  1: capture one step as a HIP graph and replay it.
 *   timing     host, optional: per-kernel event timings (synchronises).
 */
int labfm_rk_step(double* q, const labfm_operators* ops, const labfm_rk_params* prm,
                  int32_t n_steps, labfm_prec prec, int32_t use_graph, void* workspace,
                  size_t workspace_bytes, labfm_timing* timing, void* stream);

/*
 * Lagrangian frame (section "Conclusions": node positions advanced by the
 * same time integration as the flow, the consistency matrices of every node
 * evaluated and solved at every step). The nodes move with the fluid,
 * dr_i/dt = u_i, and (ln rho, u, v) follow eq. icns for the material
 * derivative (no u . grad terms):
 *   D ln rho/Dt = -(u_x + v_y),
 *   Du/Dt = -c2 l_x + (mu/rho)(4/3 u_xx + u_yy + 1/3 v_xy) + gx,
 *   Dv/Dt = -c2 l_y + (mu/rho)(4/3 v_yy + v_xx + 1/3 u_xy) + gy.
 * The extended state (x, y, ln rho, u, v) takes n_steps steps of the
 * RK3(2)4[2R+]C two-register scheme of labfm_rk_step. Every stage rebuilds
 * the stencils and the six operators' weights at that stage's positions
 * (labfm_build_neighbours and labfm_build_weights, with the node's h_i, s_i
 * and order travelling with it); after each step the filter (prm->filter)
 * uses weights built at the new positions, which also serve the next step's
 * first stage: four builds per step, plus one before the first. Positions
 * are folded into the box after every update.
 *
 *   x, y          float64[n] positions, updated in place (inside the box).
 *   q             float64[3n] state [ln rho | u | v], updated in place.
 *   h, s, order_m per-node stencil scale, spacing and order (fixed).
 *   box           both axes periodic (LABFM_ERR_UNSUPPORTED otherwise).
 *   prm           c2, mu, gx, gy, dt, filter, check_finite.
 *   nnz_capacity  largest stencil count the workspace holds.
 *   workspace     labfm_lagrangian_workspace_bytes(n, nnz_capacity) bytes:
 *                 three 5n-double registers, the CSR, the weights and the
 *                 status counters.
 *   stats         host, optional.
 * Synchronises (every build does). Returns LABFM_ERR_CAPACITY when a stencil
 * build needs more than nnz_capacity entries; x, y and q then hold the last
 * completed step (stats->steps_done), and stats->node_status counts the
 * builds done before the failure.
 */
typedef struct {
  int32_t steps_done;  /* completed steps */
  int64_t builds;      /* stencil + weight builds */
  int64_t max_nnz;     /* largest stencil count built */
  double build_ms;     /* host wall-clock time in the builds (they synchronise) */
  double stage_ms;     /* stage and filter kernels (HIP events on the stream) */
  int64_t node_status[5]; /* node builds per LABFM_NODE_* status, summed over
                             the call's builds (counted on the device after
                             each build). Nodes that cluster or thin out as
                             they move can reach LABFM_NODE_SINGULAR,
                             _FEW_NEIGHBOURS or _BAD_FILTER: their weights and
                             kappa are then zero for that stage, so their
                             fields do not change there. A caller checks
                             node_status[1..4]; the call itself still
                             returns LABFM_OK. */
} labfm_lagrangian_stats;

size_t labfm_lagrangian_workspace_bytes(int32_t n, int64_t nnz_capacity);

int labfm_lagrangian_step(double* x, double* y, double* q, const double* h, const double* s,
                          const int8_t* order_m, int32_t n, labfm_box box,
                          const labfm_rk_params* prm, int32_t n_steps, int64_t nnz_capacity,
                          void* workspace, size_t workspace_bytes,
                          labfm_lagrangian_stats* stats, void* stream);

/*
 * Measured FP64 matrix-core rate (a measurement aid, not part of the method):
 * the rate that v_mfma_f64_16x16x4f64 reaches on this device with every SIMD
 * fed four independent accumulators, the ceiling the weight build's assembly
 * is compared with next to the data-sheet FP64 peak.
 *
 *   iters          MFMA rounds per wavefront (each four instructions of 2048
 *                  flops); the grid is eight workgroups of four wavefronts
 *                  per CU.
 *   scratch        device buffer of at least
 *                  labfm_mfma_f64_rate_scratch_bytes() bytes (the kernel's
 *                  per-lane results, written and not read back).
 *   tflops         host: receives the measured TFLOP/s.
 * Runs the kernel twice (the second timed with HIP events on the stream) and
 * synchronises. Returns LABFM_ERR_ARG for iters <= 0 or a short scratch.
 */
size_t labfm_mfma_f64_rate_scratch_bytes(void);
int labfm_mfma_f64_rate(int32_t iters, double* scratch, size_t scratch_bytes, double* tflops,
                        void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LABFM_H */
