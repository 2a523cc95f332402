// Device code of the pipelined BiCGStab library (gfx950, wave64).
//
// Every solver iteration is a short chain of fused kernels.  A fused kernel
// streams over the rows once: one SpMV row, the AXPY recurrences of that row
// and the row's products for the dot products of the next reduction phase.
// The kernel boundary is the only grid-wide synchronisation, and the last
// workgroup to finish a kernel completes that kernel's reduction and computes
// the scalars of the method on the device, so the host is never in the loop.
//
//   p-BiCGStab (paper Algorithms 9 and 11, Sections 3.3 and 3.6):
//     k_pa  t := A w^ ; lines 5-11 and 13 of Algorithm 11 ; partial (q,y), (y,y)
//           last workgroup: omega_i                                (reduction 1)
//     k_pb  v := A z^ ; lines 17-20 and 22 ; partial (r0,r), (r0,w), (r0,s),
//           (r0,z), (r,r); last workgroup: beta_i, alpha_{i+1}, stop (reduction 2)
//   two kernel boundaries per iteration, against five for BiCGStab (Algorithm 7:
//   SpMV | reduction | AXPY | SpMV + reduction | AXPY + reduction | AXPY).
//
// Determinism: rows map to threads one to one inside tiles of 256 rows; a
// workgroup owns a contiguous, aligned run of tpw tiles (tpw a power of two),
// and the workgroups' partial sums are combined in workgroup order.  Wave
// butterflies (xor 1, 2, ..., 32), the (w0 + w1) + (w2 + w3) combination of
// the four waves, the tree over the tiles of a workgroup and the tree over the
// workgroups all follow the balanced binary tree over the row index.  The sum
// is therefore the pairwise sum of the products, whatever the grid shape, and
// equals a sequential pairwise evaluation bit for bit.  (Padding subtrees of
// zeros only add +0, which changes no value; the final + 0.0 fixes the sign
// of a zero result.)  Compiled with -ffp-contract=off: no fused multiply-add.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbcgs {

constexpr int kWG = 256;                      // threads per workgroup: 4 x wave64
constexpr int kTile = 256;                    // rows per tile: one row per thread
constexpr int kMaxTpw = 256;                  // tiles per workgroup (power of two)
constexpr int kFinalChunk = 4;                // partials per thread in the final tree
constexpr int kMaxG = kWG * kFinalChunk;      // workgroups per reduction kernel
constexpr int kMaxD = 5;                      // dot products per reduction phase

enum : int32_t { DS_RUNNING = 0, DS_SUCCESS = 1, DS_BREAKDOWN = 2, DS_NONFINITE = 3 };

// Device-resident solver state: scalars of the method and the status word.
struct alignas(64) DevState {
  double alpha;   // alpha_i
  double beta;    // beta_{i-1}
  double omega;   // omega_{i-1} (omega_i once reduction 1 of iteration i is done)
  double gamma;   // (r0, r_i)
  double rho0;    // ||r_0||
  double relres;  // last ||r_i|| / ||r_0||
  double tol;
  double result;  // output of utility reductions
  int32_t status;
  int32_t iters;  // completed x updates
  int32_t yzero;  // (y, y) == 0 seen in reduction 1: the next x update finishes
  int32_t n_rr;
  uint32_t counter;  // arrivals for the last-workgroup election
  int32_t errflag;   // utility kernels: structural error seen
  int32_t pad[2];
};

// ---------------------------------------------------------------------------
// Operators: apply one row of y = A x, summing in ascending column order.
// ---------------------------------------------------------------------------
struct CsrOp {
  const int32_t* __restrict__ rp;
  const int32_t* __restrict__ ci;
  const double* __restrict__ va;
  __device__ __forceinline__ double apply(int32_t row, const double* __restrict__ x) const {
    const int32_t e = rp[row + 1];
    double acc = 0.0;
    for (int32_t k = rp[row]; k < e; ++k) acc = acc + va[k] * x[ci[k]];
    return acc;
  }
};

// Constant-coefficient 5-point (nz == 1) or 7-point stencil, Dirichlet
// boundaries; c[] in ascending column order, so the result equals the CSR
// product of the assembled matrix bit for bit.
template <int NPTS>
struct StencilOp {
  int32_t nx, ny, nz, pad;
  double c[NPTS];
  __device__ __forceinline__ double apply(int32_t row, const double* __restrict__ x) const {
    const int32_t i = row % nx;
    const int32_t jk = row / nx;
    double acc = 0.0;
    if (NPTS == 7) {
      const int32_t j = jk % ny, k = jk / ny;
      const int32_t nxy = nx * ny;
      if (k > 0) acc = acc + c[0] * x[row - nxy];
      if (j > 0) acc = acc + c[1] * x[row - nx];
      if (i > 0) acc = acc + c[2] * x[row - 1];
      acc = acc + c[3] * x[row];
      if (i < nx - 1) acc = acc + c[4] * x[row + 1];
      if (j < ny - 1) acc = acc + c[5] * x[row + nx];
      if (k < nz - 1) acc = acc + c[6] * x[row + nxy];
    } else {
      const int32_t j = jk;
      if (j > 0) acc = acc + c[0] * x[row - nx];
      if (i > 0) acc = acc + c[1] * x[row - 1];
      acc = acc + c[2] * x[row];
      if (i < nx - 1) acc = acc + c[3] * x[row + 1];
      if (j < ny - 1) acc = acc + c[4] * x[row + nx];
    }
    return acc;
  }
};

// Preconditioner modes: none (Algorithms 7 and 9), Jacobi with a vector of
// 1/a_ii, Jacobi with one constant 1/a_ii (constant diagonal).
enum { PC_NONE = 0, PC_VEC = 1, PC_SCALAR = 2 };

// Kernel arguments: sizes, launch shape and every vector of the solvers.
// Without a preconditioner the hatted pointers alias the unhatted ones.
struct Args {
  int32_t n, ntiles, tpw, G;
  DevState* st;
  double* part;       // [kMaxD][kMaxG] workgroup partial sums
  double* hist;       // nullable history of ||r_i|| / ||r_0||
  const double* b;
  double* x;
  double *r0, *r, *rh, *w, *wh, *t, *ph, *s, *sh, *z, *zh, *v;  // p-BiCGStab
  double *p, *q, *qh, *y;                                       // BiCGStab
  const double* dinv;
  double dinv_s;
};

template <int PC>
__device__ __forceinline__ double apply_pc(const Args& a, int32_t row, double val) {
  if (PC == PC_VEC) return a.dinv[row] * val;
  if (PC == PC_SCALAR) return a.dinv_s * val;
  return val;
}

// ---------------------------------------------------------------------------
// Pairwise reduction machinery.
// ---------------------------------------------------------------------------
template <int ND>
__device__ __forceinline__ void wave_tree(double (&v)[ND]) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
    for (int k = 0; k < ND; ++k) v[k] = v[k] + __shfl_xor(v[k], m, 64);
  }
}

template <int ND>
struct TileRed {
  double lw[2][4][ND];        // per-wave sums, double-buffered by tile parity
  double tp[ND][kMaxTpw];     // the workgroup's tile sums, in tile order
};

// Sum of the 256 rows of one tile into sm.tp[.][tl] (thread 0 writes).
template <int ND>
__device__ __forceinline__ void tile_reduce(TileRed<ND>& sm, double (&v)[ND], int tl) {
  wave_tree<ND>(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k) sm.lw[tl & 1][wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k)
      sm.tp[k][tl] = (sm.lw[tl & 1][0][k] + sm.lw[tl & 1][1][k]) +
                     (sm.lw[tl & 1][2][k] + sm.lw[tl & 1][3][k]);
  }
}

// Tree over the workgroup's ntl tile sums (wave w holds tiles 64w..64w+63);
// thread 0 writes part[k][bid].
template <int ND>
__device__ __forceinline__ void wg_partial(TileRed<ND>& sm, int ntl, double* part, int bid) {
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = ((int)threadIdx.x < ntl) ? sm.tp[k][threadIdx.x] : 0.0;
  wave_tree<ND>(v);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k) sm.lw[0][wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k)
      part[k * kMaxG + bid] = (sm.lw[0][0][k] + sm.lw[0][1][k]) + (sm.lw[0][2][k] + sm.lw[0][3][k]);
  }
}

// Arrival at the end of a kernel; true in the workgroup that arrives last,
// which then sees every other workgroup's writes.
__device__ __forceinline__ bool elect_last(DevState* st, int G) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&st->counter, 1u);
    s_last = (prev == (unsigned)(G - 1));
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Tree over the G workgroup partials of each of the ND sums (G <= kMaxG);
// result valid in thread 0, already "+ 0.0".
template <int ND>
__device__ __forceinline__ void final_reduce(const double* part, int G, double (&out)[ND]) {
  __shared__ double lw[4][kMaxD];
  double v[ND];
  const int base = threadIdx.x * kFinalChunk;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    double c[kFinalChunk];
#pragma unroll
    for (int j = 0; j < kFinalChunk; ++j)
      c[j] = (base + j < G) ? part[k * kMaxG + base + j] : 0.0;
#pragma unroll
    for (int w = 1; w < kFinalChunk; w <<= 1) {
#pragma unroll
      for (int j = 0; j < kFinalChunk; j += 2 * w) c[j] = c[j] + c[j + w];
    }
    v[k] = c[0];
  }
  wave_tree<ND>(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k) lw[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k) out[k] = ((lw[0][k] + lw[1][k]) + (lw[2][k] + lw[3][k])) + 0.0;
  }
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// ---------------------------------------------------------------------------
// Scalar steps of the method, run by thread 0 of the last workgroup.
// ---------------------------------------------------------------------------

// gamma = (r0, r0), rho0 = ||r0|| (Algorithms 7-11, line 2).
__device__ __forceinline__ void fin_setup_gamma(DevState* st, double* hist, double g) {
  st->gamma = g;
  const double rho0 = sqrt(g);
  st->rho0 = rho0;
  st->relres = 1.0;
  if (hist) hist[0] = 1.0;
  if (!finite(rho0)) st->status = DS_NONFINITE;
  else if (rho0 == 0.0) { st->status = DS_SUCCESS; st->relres = 0.0; }
}

// alpha_0 = (r0, r0) / (r0, w0), beta_{-1} = omega_{-1} = 0 (Algorithm 9/11, lines 2-3).
__device__ __forceinline__ void fin_setup_alpha(DevState* st, double delta) {
  if (!finite(delta)) { st->status = DS_NONFINITE; return; }
  if (delta == 0.0) { st->status = DS_BREAKDOWN; return; }
  const double alpha = st->gamma / delta;
  if (!finite(alpha)) { st->status = DS_NONFINITE; return; }
  st->alpha = alpha;
  st->beta = 0.0;
  st->omega = 0.0;
}

// omega_i = (q, y) / (y, y)  (reduction 1; Algorithm 9 line 12, Algorithm 11 line 16).
__device__ __forceinline__ void fin_omega(DevState* st, double qy, double yy) {
  if (!finite(qy) || !finite(yy)) { st->status = DS_NONFINITE; return; }
  if (yy == 0.0) { st->yzero = 1; return; }  // y = A q^ = 0: q = 0, exact convergence
  const double omega = qy / yy;
  if (!finite(omega)) { st->status = DS_NONFINITE; return; }
  st->omega = omega;
}

// The x update of (y, y) == 0 finished the solve.
__device__ __forceinline__ void fin_yzero(DevState* st, double* hist) {
  st->iters += 1;
  st->relres = 0.0;
  if (hist) hist[st->iters] = 0.0;
  st->status = DS_SUCCESS;
}

// Reduction 2 of p-BiCGStab: stopping test, beta_i and alpha_{i+1} by eq. (3)
// (Algorithm 9 lines 17-20, Algorithm 11 lines 24-26).
__device__ __forceinline__ void fin_pipe_b(DevState* st, double* hist, const double (&d)[5]) {
  const double g1 = d[0], eta = d[1], sig_s = d[2], sig_z = d[3], nu = d[4];
  st->iters += 1;
  if (!finite(g1) || !finite(eta) || !finite(sig_s) || !finite(sig_z) || !finite(nu)) {
    st->status = DS_NONFINITE;
    return;
  }
  const double relres = sqrt(nu) / st->rho0;
  st->relres = relres;
  if (hist) hist[st->iters] = relres;
  if (relres <= st->tol) { st->status = DS_SUCCESS; return; }
  const double alpha = st->alpha, omega = st->omega, gamma = st->gamma;
  if (omega == 0.0 || gamma == 0.0) { st->status = DS_BREAKDOWN; return; }
  const double beta = (alpha / omega) * (g1 / gamma);
  if (!finite(beta)) { st->status = DS_NONFINITE; return; }
  st->beta = beta;
  const double den = eta + beta * sig_s - beta * omega * sig_z;
  if (den == 0.0 || g1 == 0.0) { st->status = DS_BREAKDOWN; return; }
  const double an = g1 / den;
  if (!finite(an)) { st->status = DS_NONFINITE; return; }
  st->alpha = an;
  st->gamma = g1;
}

// alpha_i = (r0, r_i) / (r0, s_i)  (Algorithm 7 lines 5-6).
__device__ __forceinline__ void fin_bicg_alpha(DevState* st, double delta) {
  if (!finite(delta)) { st->status = DS_NONFINITE; return; }
  if (delta == 0.0) { st->status = DS_BREAKDOWN; return; }
  const double alpha = st->gamma / delta;
  if (!finite(alpha)) { st->status = DS_NONFINITE; return; }
  st->alpha = alpha;
}

// Stopping test and beta_i = (alpha/omega) (r0, r_{i+1}) / (r0, r_i)  (Algorithm 7 lines 13-14).
__device__ __forceinline__ void fin_bicg_beta(DevState* st, double* hist, double g1, double nu) {
  st->iters += 1;
  if (!finite(g1) || !finite(nu)) { st->status = DS_NONFINITE; return; }
  const double relres = sqrt(nu) / st->rho0;
  st->relres = relres;
  if (hist) hist[st->iters] = relres;
  if (relres <= st->tol) { st->status = DS_SUCCESS; return; }
  const double alpha = st->alpha, omega = st->omega, gamma = st->gamma;
  if (omega == 0.0 || gamma == 0.0) { st->status = DS_BREAKDOWN; return; }
  const double beta = (alpha / omega) * (g1 / gamma);
  if (!finite(beta)) { st->status = DS_NONFINITE; return; }
  st->beta = beta;
  st->gamma = g1;
}

// ---------------------------------------------------------------------------
// Kernel skeleton: loop over the workgroup's tiles, one row per thread.
// Body(row, d) computes the row and its ND products; rows past n give zeros.
// ---------------------------------------------------------------------------
template <int ND, class Body>
__device__ __forceinline__ void tile_loop(TileRed<ND>& sm, const Args& a, Body body) {
  const int bid = blockIdx.x;
  int ntl = 0;
  for (int tl = 0; tl < a.tpw; ++tl) {
    const int tile = bid * a.tpw + tl;
    if (tile >= a.ntiles) break;
    ++ntl;
    const int32_t row = tile * kTile + (int32_t)threadIdx.x;
    double d[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = 0.0;
    if (row < a.n) body(row, d);
    tile_reduce<ND>(sm, d, tl);
  }
  wg_partial<ND>(sm, ntl, a.part, bid);
}

template <class Body>
__device__ __forceinline__ void row_loop(const Args& a, Body body) {
  const int bid = blockIdx.x;
  for (int tl = 0; tl < a.tpw; ++tl) {
    const int tile = bid * a.tpw + tl;
    if (tile >= a.ntiles) break;
    const int32_t row = tile * kTile + (int32_t)threadIdx.x;
    if (row < a.n) body(row);
  }
}

__device__ __forceinline__ bool running(const DevState* st) { return st->status == DS_RUNNING; }

// ===========================================================================
// p-BiCGStab kernels (Algorithm 9, PC == PC_NONE; Algorithm 11 otherwise).
// ===========================================================================

// Setup 1: r0 = b - A x0 ; r = r0 ; r^ = M^{-1} r0 ; p^ = s = s^ = z = z^ = v = 0 ;
// reduction (r0, r0).  PIPE = false: BiCGStab setup, p = r0 ; p^ = M^{-1} p.
template <class Op, int PC, bool PIPE>
__global__ __launch_bounds__(kWG) void k_setup_r0(Op op, Args a) {
  __shared__ TileRed<1> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  tile_loop<1>(sm, a, [&](int32_t row, double (&d)[1]) {
    const double r0 = a.b[row] - op.apply(row, a.x);
    a.r0[row] = r0;
    a.r[row] = r0;
    if (PIPE) {
      if (PC != PC_NONE) {
        a.rh[row] = apply_pc<PC>(a, row, r0);
        a.sh[row] = 0.0;
        a.zh[row] = 0.0;
      }
      a.ph[row] = 0.0;
      a.s[row] = 0.0;
      a.z[row] = 0.0;
      a.v[row] = 0.0;
    } else {
      a.p[row] = r0;
      if (PC != PC_NONE) a.ph[row] = apply_pc<PC>(a, row, r0);
    }
    d[0] = r0 * r0;
  });
  if (!elect_last(st, a.G)) return;
  double g[1];
  final_reduce<1>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_setup_gamma(st, a.hist, g[0]);
    st->counter = 0;
  }
}

// Setup 2: w0 = A r^0 ; w^0 = M^{-1} w0 ; reduction (r0, w0) -> alpha_0.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_setup_w0(Op op, Args a) {
  __shared__ TileRed<1> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  tile_loop<1>(sm, a, [&](int32_t row, double (&d)[1]) {
    const double w = op.apply(row, a.rh);
    a.w[row] = w;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, w);
    d[0] = a.r0[row] * w;
  });
  if (!elect_last(st, a.G)) return;
  double g[1];
  final_reduce<1>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_setup_alpha(st, g[0]);
    st->counter = 0;
  }
}

// Phase A of iteration i.  RR2 = false: t = A w^ and the recurrences of lines
// 5-11 (13).  RR2 = true (the iteration after a residual replacement): p^, s,
// s^ were already recomputed, so t = A w^ and z = A s^ (both gathers), then
// lines 9-11 and 13.  Reduction 1: (q, y), (y, y) -> omega_i.
template <class Op, int PC, bool RR2>
__global__ __launch_bounds__(kWG) void k_pa(Op op, Args a) {
  __shared__ TileRed<2> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  const double alpha = st->alpha, beta = st->beta, omega = st->omega;
  tile_loop<2>(sm, a, [&](int32_t row, double (&d)[2]) {
    const double t = op.apply(row, a.wh);  // line 23 of the previous iteration
    const double r = a.r[row], w = a.w[row];
    double s, z;
    if (RR2) {
      s = a.s[row];
      z = op.apply(row, a.sh);
    } else {
      const double v = a.v[row];
      const double s_old = a.s[row], z_old = a.z[row];
      if (PC != PC_NONE) {
        const double rh = a.rh[row], wh = a.wh[row];
        const double sh_old = a.sh[row], zh_old = a.zh[row];
        a.ph[row] = rh + beta * (a.ph[row] - omega * sh_old);          // line 5
        a.sh[row] = wh + beta * (sh_old - omega * zh_old);             // line 7
      } else {
        a.ph[row] = r + beta * (a.ph[row] - omega * s_old);            // Alg. 9 line 4
      }
      s = w + beta * (s_old - omega * z_old);                          // line 6
      z = t + beta * (z_old - omega * v);                              // line 8
      a.s[row] = s;
    }
    const double q = r - alpha * s;                                    // line 9
    const double y = w - alpha * z;                                    // line 11
    a.t[row] = t;
    a.z[row] = z;
    if (PC != PC_NONE) a.zh[row] = apply_pc<PC>(a, row, z);            // line 13
    d[0] = q * y;
    d[1] = y * y;
  });
  if (!elect_last(st, a.G)) return;
  double g[2];
  final_reduce<2>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_omega(st, g[0], g[1]);
    st->counter = 0;
  }
}

// Phase B of iteration i: v = A z^ ; lines 9-11 recomputed ; lines 17-20 ;
// line 22 ; reduction 2 (r0,r), (r0,w), (r0,s), (r0,z), (r,r) -> beta, alpha.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_pb(Op op, Args a) {
  __shared__ TileRed<5> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  const double alpha = st->alpha, omega = st->omega;
  const bool yz = st->yzero != 0;
  if (yz) {
    row_loop(a, [&](int32_t row) { a.x[row] = a.x[row] + alpha * a.ph[row]; });
    if (elect_last(st, a.G) && threadIdx.x == 0) {
      fin_yzero(st, a.hist);
      st->counter = 0;
    }
    return;
  }
  tile_loop<5>(sm, a, [&](int32_t row, double (&d)[5]) {
    const double v = op.apply(row, a.zh);                              // line 14
    const double r = a.r[row], s = a.s[row], w = a.w[row], z = a.z[row];
    const double q = r - alpha * s;
    const double y = w - alpha * z;
    const double t = a.t[row];
    double rn;
    if (PC != PC_NONE) {
      const double rh = a.rh[row], sh = a.sh[row], wh = a.wh[row], zh = a.zh[row];
      const double qh = rh - alpha * sh;                               // line 10
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * qh;            // line 17
      rn = q - omega * y;                                              // line 18
      a.rh[row] = qh - omega * (wh - alpha * zh);                      // line 19
    } else {
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * q;
      rn = q - omega * y;
    }
    const double wn = y - omega * (t - alpha * v);                     // line 20
    a.v[row] = v;
    a.r[row] = rn;
    a.w[row] = wn;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, wn);           // line 22
    const double r0 = a.r0[row];
    d[0] = r0 * rn;
    d[1] = r0 * wn;
    d[2] = r0 * s;
    d[3] = r0 * z;
    d[4] = rn * rn;
  });
  if (!elect_last(st, a.G)) return;
  double g[5];
  final_reduce<5>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_pipe_b(st, a.hist, g);
    st->counter = 0;
  }
}

// Residual-replacement iteration, phase B': only the x update of line 17
// (r, r^, w are replaced next, so lines 18-20 and v are not needed).
template <int PC>
__global__ __launch_bounds__(kWG) void k_rr_x(Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  const double alpha = st->alpha, omega = st->omega;
  const bool yz = st->yzero != 0;
  row_loop(a, [&](int32_t row) {
    if (yz) {
      a.x[row] = a.x[row] + alpha * a.ph[row];
    } else {
      const double qh = (PC != PC_NONE) ? a.rh[row] - alpha * a.sh[row] : a.r[row] - alpha * a.s[row];
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * qh;
    }
  });
  if (yz && elect_last(st, a.G) && threadIdx.x == 0) {
    fin_yzero(st, a.hist);
    st->counter = 0;
  }
}

// Residual replacement, first half (Section 4.2): r = b - A x ; r^ = M^{-1} r.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_r(Op op, Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  row_loop(a, [&](int32_t row) {
    const double r = a.b[row] - op.apply(row, a.x);
    a.r[row] = r;
    if (PC != PC_NONE) a.rh[row] = apply_pc<PC>(a, row, r);
  });
}

// Residual replacement, first half continued: w = A r^ ; w^ = M^{-1} w ;
// reduction 2 on the true r, w.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_w(Op op, Args a) {
  __shared__ TileRed<5> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  tile_loop<5>(sm, a, [&](int32_t row, double (&d)[5]) {
    const double w = op.apply(row, a.rh);
    a.w[row] = w;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, w);
    const double r0 = a.r0[row], r = a.r[row];
    d[0] = r0 * r;
    d[1] = r0 * w;
    d[2] = r0 * a.s[row];
    d[3] = r0 * a.z[row];
    d[4] = r * r;
  });
  if (!elect_last(st, a.G)) return;
  double g[5];
  final_reduce<5>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    st->n_rr += 1;
    fin_pipe_b(st, a.hist, g);
    st->counter = 0;
  }
}

// Second half, iteration after a replacement: line 5 (p^ update) alone.
template <int PC>
__global__ __launch_bounds__(kWG) void k_rr_p(Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  const double beta = st->beta, omega = st->omega;
  row_loop(a, [&](int32_t row) {
    if (PC != PC_NONE) a.ph[row] = a.rh[row] + beta * (a.ph[row] - omega * a.sh[row]);
    else a.ph[row] = a.r[row] + beta * (a.ph[row] - omega * a.s[row]);
  });
}

// Second half continued: s = A p^ ; s^ = M^{-1} s.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_s(Op op, Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  row_loop(a, [&](int32_t row) {
    const double s = op.apply(row, a.ph);
    a.s[row] = s;
    if (PC != PC_NONE) a.sh[row] = apply_pc<PC>(a, row, s);
  });
}

// ===========================================================================
// BiCGStab kernels (Algorithm 7, PC == PC_NONE; Algorithm 10 otherwise).
// ===========================================================================

// s = A p^ ; reduction (r0, s) -> alpha_i.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_b1(Op op, Args a) {
  __shared__ TileRed<1> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  tile_loop<1>(sm, a, [&](int32_t row, double (&d)[1]) {
    const double s = op.apply(row, a.ph);
    a.s[row] = s;
    d[0] = a.r0[row] * s;
  });
  if (!elect_last(st, a.G)) return;
  double g[1];
  final_reduce<1>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_bicg_alpha(st, g[0]);
    st->counter = 0;
  }
}

// q = r - alpha s ; q^ = M^{-1} q.
template <int PC>
__global__ __launch_bounds__(kWG) void k_b2(Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  const double alpha = st->alpha;
  row_loop(a, [&](int32_t row) {
    const double q = a.r[row] - alpha * a.s[row];
    a.q[row] = q;
    if (PC != PC_NONE) a.qh[row] = apply_pc<PC>(a, row, q);
  });
}

// y = A q^ ; reduction (q, y), (y, y) -> omega_i.
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_b3(Op op, Args a) {
  __shared__ TileRed<2> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  tile_loop<2>(sm, a, [&](int32_t row, double (&d)[2]) {
    const double y = op.apply(row, a.qh);
    a.y[row] = y;
    d[0] = a.q[row] * y;
    d[1] = y * y;
  });
  if (!elect_last(st, a.G)) return;
  double g[2];
  final_reduce<2>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_omega(st, g[0], g[1]);
    st->counter = 0;
  }
}

// x = x + alpha p^ + omega q^ ; r = q - omega y ; reduction (r0, r), (r, r).
template <int PC>
__global__ __launch_bounds__(kWG) void k_b4(Args a) {
  __shared__ TileRed<2> sm;
  DevState* st = a.st;
  if (!running(st)) return;
  const double alpha = st->alpha, omega = st->omega;
  if (st->yzero != 0) {
    row_loop(a, [&](int32_t row) { a.x[row] = a.x[row] + alpha * a.ph[row]; });
    if (elect_last(st, a.G) && threadIdx.x == 0) {
      fin_yzero(st, a.hist);
      st->counter = 0;
    }
    return;
  }
  tile_loop<2>(sm, a, [&](int32_t row, double (&d)[2]) {
    const double q = a.q[row];
    a.x[row] = a.x[row] + alpha * a.ph[row] + omega * a.qh[row];
    const double r = q - omega * a.y[row];
    a.r[row] = r;
    d[0] = a.r0[row] * r;
    d[1] = r * r;
  });
  if (!elect_last(st, a.G)) return;
  double g[2];
  final_reduce<2>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    fin_bicg_beta(st, a.hist, g[0], g[1]);
    st->counter = 0;
  }
}

// p = r + beta (p - omega s) ; p^ = M^{-1} p.
template <int PC>
__global__ __launch_bounds__(kWG) void k_b5(Args a) {
  DevState* st = a.st;
  if (!running(st)) return;
  const double beta = st->beta, omega = st->omega;
  row_loop(a, [&](int32_t row) {
    const double p = a.r[row] + beta * (a.p[row] - omega * a.s[row]);
    a.p[row] = p;
    if (PC != PC_NONE) a.ph[row] = apply_pc<PC>(a, row, p);
  });
}

// ===========================================================================
// Utility kernels.
// ===========================================================================

__global__ void k_init_state(DevState* st, double tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->alpha = 0.0; st->beta = 0.0; st->omega = 0.0; st->gamma = 0.0;
    st->rho0 = 0.0; st->relres = 1.0; st->tol = tol; st->result = 0.0;
    st->status = DS_RUNNING; st->iters = 0; st->yzero = 0; st->n_rr = 0;
    st->counter = 0; st->errflag = 0;
  }
}

template <class Op>
__global__ __launch_bounds__(kWG) void k_spmv(Op op, Args a, const double* __restrict__ xin,
                                              double* __restrict__ yout) {
  row_loop(a, [&](int32_t row) { yout[row] = op.apply(row, xin); });
}

// result = (x, y) in pairwise order.
__global__ __launch_bounds__(kWG) void k_dot(Args a, const double* __restrict__ xv,
                                             const double* __restrict__ yv) {
  __shared__ TileRed<1> sm;
  DevState* st = a.st;
  tile_loop<1>(sm, a, [&](int32_t row, double (&d)[1]) { d[0] = xv[row] * yv[row]; });
  if (!elect_last(st, a.G)) return;
  double g[1];
  final_reduce<1>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    st->result = g[0];
    st->counter = 0;
  }
}

// result = ||b - A x||^2 in pairwise order (true residual of the returned x).
template <class Op>
__global__ __launch_bounds__(kWG) void k_true_res(Op op, Args a) {
  __shared__ TileRed<1> sm;
  DevState* st = a.st;
  tile_loop<1>(sm, a, [&](int32_t row, double (&d)[1]) {
    const double r = a.b[row] - op.apply(row, a.x);
    d[0] = r * r;
  });
  if (!elect_last(st, a.G)) return;
  double g[1];
  final_reduce<1>(a.part, a.G, g);
  if (threadIdx.x == 0) {
    st->result = g[0];
    st->counter = 0;
  }
}

// dinv_i = 1 / a_ii ; errflag if a diagonal entry is zero, non-finite or absent.
__global__ __launch_bounds__(kWG) void k_dinv_csr(CsrOp op, int32_t n, double* dinv, DevState* st) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  double d = 0.0;
  for (int32_t k = op.rp[row]; k < op.rp[row + 1]; ++k)
    if (op.ci[k] == row) d = op.va[k];
  if (d == 0.0 || !finite(d)) atomicOr(&st->errflag, 1);
  dinv[row] = 1.0 / d;
}

// errflag bit 1 unless every dinv_i equals dinv_0 (then Jacobi is one scalar).
__global__ __launch_bounds__(kWG) void k_dinv_const(int32_t n, const double* dinv, DevState* st) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  if (!(dinv[row] == dinv[0]) || !finite(dinv[row]) || dinv[row] == 0.0) atomicOr(&st->errflag, 2);
}

// CSR structure check: errflag bit 0 on a malformed row pointer or column.
__global__ __launch_bounds__(kWG) void k_csr_check(CsrOp op, int32_t n, int64_t nnz, DevState* st) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const int32_t b = op.rp[row], e = op.rp[row + 1];
  bool bad = (b > e) || (b < 0) || ((int64_t)e > nnz);
  if (row == 0 && b != 0) bad = true;
  if (row == n - 1 && (int64_t)e != nnz) bad = true;
  if (!bad) {
    for (int32_t k = b; k < e; ++k) {
      const int32_t c = op.ci[k];
      if (c < 0 || c >= n) { bad = true; break; }
    }
  }
  if (bad) atomicOr(&st->errflag, 1);
}

}  // namespace pbcgs
