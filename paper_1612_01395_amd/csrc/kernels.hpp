// Device code of the pipelined BiCGStab library (gfx950, wave64).
//
// Every solver iteration is a short chain of fused kernels.  A fused kernel
// streams over the rows once: one SpMV row, the AXPY recurrences of that row
// and the row's products for the dot products of the next reduction phase.
// The kernel boundary is the only grid-wide synchronisation and the scalars of
// the method are computed on the device, so the host is never in the loop.
//
//   p-BiCGStab (paper Algorithms 9 and 11, Sections 3.3 and 3.6):
//     k_pa  finishes reduction 2 of the previous iteration (stop test, beta,
//           alpha), then t := A w^ ; the p^, s, s^, z, q, y recurrences and z^ ; partials (q,y), (y,y)
//     k_pb  finishes reduction 1 (omega), then v := A z^ ; the x, r, r^, w updates and w^ ;
//           partials (r0,r), (r0,w), (r0,s), (r0,z), (r,r)
//   two kernel boundaries per iteration, against five for BiCGStab (Algorithm 7:
//   SpMV | reduction | AXPY | SpMV + reduction | AXPY + reduction | AXPY).
//
// Reductions complete on read: a kernel writes one partial sum per workgroup,
// and every workgroup of the next kernel adds those partials itself (a few KB
// from L2, the same pairwise tree, so every workgroup obtains the same bits)
// before computing the method's scalars.  No workgroup waits for another and
// no device-scope fence or atomic is needed; the kernel boundary is the only
// synchronisation.  The scalars travel in a two-slot state: launch q reads
// slot q mod 2 and workgroup 0 writes slot (q+1) mod 2.
//
// Row layout and determinism: wave w of workgroup b handles R consecutive
// blocks of 64 rows starting at row 64 R (4 b + w); lane l handles row l of
// each block, so vector loads are fully coalesced.  A DPP tree sums each
// block into lane 63, the workgroup adds its 4 R block sums as a balanced
// tree, and the consumer adds the workgroups' partials as a balanced tree:
// altogether the balanced binary tree over the row index, whatever R and the
// grid size are.  (Padding subtrees of zeros only add +0, which changes no
// value; the final + 0.0 fixes the sign of a zero result.)  Compiled with
// -ffp-contract=off: no fused multiply-add anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pbcgs {

constexpr int kWG = 256;                  // threads per workgroup: 4 x wave64
constexpr int kMaxD = 5;                  // dot products per reduction phase
constexpr int kMaxR = 1024;               // 64-row blocks per wave (a power of two)
constexpr int kLevels = 11;               // levels of a wave's pairwise tree: kMaxR = 2^(kLevels-1)
constexpr int kMaxG = 1024;               // workgroups of a producing kernel
constexpr int kChunk = kMaxG / kWG;       // partials per thread when consuming

// DS_CHECK (precision form only): the binary32 recursive residual passed tol;
// the host confirms with the binary64 true residual before declaring SUCCESS.
enum : int32_t { DS_RUNNING = 0, DS_SUCCESS = 1, DS_BREAKDOWN = 2, DS_NONFINITE = 3, DS_CHECK = 4 };

// Device-resident solver state: scalars of the method and the status word.
struct alignas(128) DevState {
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
  int32_t n_rr;   // residual replacements done
  int32_t pad[5];
};

// ---------------------------------------------------------------------------
// Operators: apply one row of y = A x, summing in ascending column order.
// ---------------------------------------------------------------------------
//
// Column indices (type I) take one of three forms:
//  - int32_t: the caller's columns;
//  - int16_t: a compact copy holding each column as its offset from the first
//    row of its row's 64-row block (row & ~63).  A wave always works on a
//    whole block that starts at a multiple of 64, so that row is known to
//    every lane;
//  - uint16_t: a compact copy holding, for a matrix with at most 64 distinct
//    diagonals j - i, the row's place in its block (6 bits) and the index of
//    its diagonal in a 64-entry table dg (6 bits): j = (i & ~63) + (i & 63) +
//    dg[index].  Each lane holds one table entry in a register and the
//    columns are decoded with a cross-lane read, so no shared memory is used.
template <class V, class I = int32_t>
struct CsrOpT {
  using Val = V;
  const int32_t* __restrict__ rp;
  const I* __restrict__ ci;
  const V* __restrict__ va;
  int32_t n;
  // explicit, always 0: the driver keys its cached graphs on the operator's
  // bytes, which must then hold no indeterminate padding
  int32_t pad_ = 0;
  const int32_t* __restrict__ dg = nullptr;  // diagonal table of the uint16_t form

  static constexpr int kStage = 512;  // staged non-zeros per wave and round

  static constexpr bool kDiag = std::is_same<I, uint16_t>::value;

  // column of a stored index; base = first row of the row's 64-row block,
  // dreg = this lane's entry of the diagonal table (uint16_t form).  All 64
  // lanes must call it together in the uint16_t form.
  static __device__ __forceinline__ int32_t col(I c, int32_t base, int32_t dreg) {
    if constexpr (sizeof(I) == sizeof(int32_t)) return (int32_t)c;
    else if constexpr (!kDiag) return base + (int32_t)c;
    else return base + (int32_t)(c & 63u) + __shfl(dreg, (int)(c >> 6), 64);
  }
  // a staged column inside [0, n): a round may begin one non-zero before the
  // block (the last one of the previous row), whose compact column (either
  // 16-bit form) is then decoded against this block's start.  Its product's
  // slot is never read; the clamp only keeps its gather in bounds (int32
  // columns are valid as they are).
  __device__ __forceinline__ int32_t staged_col(int32_t c) const {
    if constexpr (sizeof(I) == sizeof(int32_t)) return c;
    else return min(max(c, 0), n - 1);
  }

  // Row `row` of A x, computed by the whole wave for its 64-row block (all 64
  // lanes call it; lanes with valid == false return 0).  The block's
  // non-zeros are contiguous in CSR, so the wave loads them with coalesced
  // loads, multiplies by the gathered x and stages the products in LDS
  // (CSR-stream); each lane then adds its own row's products in stored order,
  // starting from 0.0 -- the same operations as a row-by-row loop.  V is the
  // arithmetic type of the product; x (type X) is widened to it first.
  //
  // Each lane loads two neighbouring non-zeros at once (a pair of values and
  // of columns; rounds start at an even non-zero), halving the load
  // instructions.  A pair that starts at a round's last non-zero also reads
  // the next one, which at the very end of an odd-length matrix would be past
  // nnz: that one round (a wave-uniform test) loads one non-zero per lane.
  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    __shared__ V stage[4][kStage];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t b0 = __builtin_amdgcn_readfirstlane(row);  // lane 0: first row of the block
    const int32_t rc = min(row, n - 1);  // clamped: the loads issue together
    const int32_t rlo = rp[b0];
    const int32_t rhi = rp[min(b0 + 64, n)];
    const int32_t nnz = rp[n];
    const int32_t rb0 = rp[rc], re0 = rp[rc + 1];
    const int32_t dreg = kDiag ? dg[lane] : 0;
    const int32_t rb = valid ? rb0 : rhi;
    const int32_t re = valid ? re0 : rhi;
    V acc = V(0);
    for (int32_t c0 = rlo & ~1; c0 < rhi; c0 += kStage) {
      const int32_t c1 = min(c0 + kStage, rhi);
      // branch-free: indices past the chunk are clamped into it (their
      // products land in slots that are never read), so all loads issue at once
      // The matrix is streamed once per product: its loads are non-temporal
      // so that they do not evict the Krylov vectors, which the next kernel
      // reads again, from L2 and the Infinity Cache.
      if (!(c1 == nnz && (c1 & 1))) {
        const int32_t pmax = (c1 - 1) & ~1;  // the last pair start of the round
        int32_t ca[kStage / 128], cb[kStage / 128];
        V va0[kStage / 128], va1[kStage / 128];
#pragma unroll
        for (int u = 0; u < kStage / 128; ++u) {
          const int32_t k = min(c0 + 2 * (u * 64 + lane), pmax);
          if constexpr (sizeof(I) == 2) {
            // one 32-bit word: the low half is non-zero k, the high half k + 1
            const uint32_t w = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(ci) + (k >> 1));
            ca[u] = col((I)(w & 0xffffu), b0, dreg);
            cb[u] = col((I)(w >> 16), b0, dreg);
          } else {
            ca[u] = __builtin_nontemporal_load(&ci[k]);
            cb[u] = __builtin_nontemporal_load(&ci[k + 1]);
          }
          va0[u] = __builtin_nontemporal_load(&va[k]);
          va1[u] = __builtin_nontemporal_load(&va[k + 1]);
        }
#pragma unroll
        for (int u = 0; u < kStage / 128; ++u) {
          stage[wave][2 * (u * 64 + lane)] = va0[u] * V(x[staged_col(ca[u])]);
          stage[wave][2 * (u * 64 + lane) + 1] = va1[u] * V(x[staged_col(cb[u])]);
        }
      } else {
        int32_t cc[kStage / 64];
        V vv[kStage / 64];
#pragma unroll
        for (int u = 0; u < kStage / 64; ++u) {
          const int32_t k = min(c0 + u * 64 + lane, c1 - 1);
          cc[u] = staged_col(col(__builtin_nontemporal_load(&ci[k]), b0, dreg));
          vv[u] = __builtin_nontemporal_load(&va[k]);
        }
#pragma unroll
        for (int u = 0; u < kStage / 64; ++u) stage[wave][u * 64 + lane] = vv[u] * V(x[cc[u]]);
      }
      __builtin_amdgcn_wave_barrier();
      const int32_t kb = max(rb, c0), ke = min(re, c1);
      for (int32_t k = kb; k < ke; ++k) acc = acc + stage[wave][k - c0];
      __builtin_amdgcn_wave_barrier();
    }
    return acc;
  }
};
using CsrOp = CsrOpT<double>;
using CsrOp32 = CsrOpT<float>;
using CsrOp16 = CsrOpT<double, int16_t>;
using CsrOp16f = CsrOpT<float, int16_t>;
using CsrOpDg = CsrOpT<double, uint16_t>;
using CsrOpDgf = CsrOpT<float, uint16_t>;

template <class Op> struct IsCsr : std::false_type {};
template <class V, class I> struct IsCsr<CsrOpT<V, I>> : std::true_type {};

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1): lane l receives the
// value of lane l - 1 (shr) or l + 1 (shl); the lane without a source (0 or 63)
// keeps `fill`.
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double wave_shift(double fill, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float wave_shift(float fill, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Constant-coefficient 5-point (nz == 1) or 7-point stencil, Dirichlet
// boundaries; c[] in ascending column order, so the result equals the CSR
// product of the assembled matrix bit for bit.  All 64 lanes of a row block
// call spmv / spmv2 together (lane l holds row b0 + l, or rows b0 + 2l and
// b0 + 2l + 1): each lane loads the x of its own rows once, and the x-direction
// neighbours x[row - 1], x[row + 1] come from the adjacent lanes by a wave
// shift (one shared load for each end of the block), so a row costs five x
// loads instead of seven (the 5-point stencil three instead of five).
template <int NPTS, class V = double>
struct StencilOp {
  using Val = V;
  int32_t nx, ny, nz, pad;
  V c[NPTS];
  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    const int lane = threadIdx.x & 63;
    const int32_t n = nx * ny * nz;
    const int32_t b0 = row - lane;
    const X xc = x[min(row, n - 1)];
    const X xm = wave_shift<kWaveShr1>(x[max(b0 - 1, 0)], xc);      // x[row - 1]
    const X xp = wave_shift<kWaveShl1>(x[min(b0 + 64, n - 1)], xc);  // x[row + 1]
    return valid ? apply(row, x, xm, xc, xp) : V(0);
  }
  // Rows row and row + 1 (row even) by one lane.  valid1 implies valid0.
  template <class X>
  __device__ __forceinline__ void spmv2(int32_t row, bool valid0, bool valid1, const X* __restrict__ x, V& y0,
                                        V& y1) const {
    typedef X X2 __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63;
    const int32_t n = nx * ny * nz;
    const int32_t b0 = row - 2 * lane;
    X c0, c1;
    if (valid1) {  // row + 1 < n: an aligned pair of the (at least 16-byte aligned) vector
      const X2 q = *reinterpret_cast<const X2*>(&x[row]);
      c0 = q.x;
      c1 = q.y;
    } else {
      c0 = x[min(row, n - 1)];
      c1 = x[min(row + 1, n - 1)];
    }
    const X xm = wave_shift<kWaveShr1>(x[max(b0 - 1, 0)], c1);       // x[row - 1]
    const X xp = wave_shift<kWaveShl1>(x[min(b0 + 128, n - 1)], c0);  // x[row + 2]
    if ((nx & 1) == 0) {
      // an even x extent: row and row + 1 lie on one grid line (and n is even,
      // so valid0 implies valid1), and their y / z neighbours are aligned pairs
      y0 = V(0);
      y1 = V(0);
      if (valid0) apply_pair(row, x, xm, c0, c1, xp, y0, y1);
      return;
    }
    y0 = valid0 ? apply(row, x, xm, c0, c1) : V(0);
    y1 = valid1 ? apply(row + 1, x, c0, c1, xp) : V(0);
  }
  // Rows row, row + 1 of one grid line (row even, nx even) with x[row - 1],
  // x[row], x[row + 1], x[row + 2] given: each row's terms in the order of apply.
  template <class X>
  __device__ __forceinline__ void apply_pair(int32_t row, const X* __restrict__ x, X xm, X c0, X c1, X xp, V& y0,
                                             V& y1) const {
    typedef X X2 __attribute__((ext_vector_type(2)));
    const int32_t i = row % nx;  // even, so i + 1 <= nx - 1 and row + 1 has a left neighbour
    const int32_t jk = row / nx;
    V a0 = V(0), a1 = V(0);
    if constexpr (NPTS == 7) {
      const int32_t j = jk % ny, k = jk / ny;
      const int32_t nxy = nx * ny;
      if (k > 0) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row - nxy]);
        a0 = a0 + c[0] * V(q.x);
        a1 = a1 + c[0] * V(q.y);
      }
      if (j > 0) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row - nx]);
        a0 = a0 + c[1] * V(q.x);
        a1 = a1 + c[1] * V(q.y);
      }
      if (i > 0) a0 = a0 + c[2] * V(xm);
      a1 = a1 + c[2] * V(c0);
      a0 = a0 + c[3] * V(c0);
      a1 = a1 + c[3] * V(c1);
      a0 = a0 + c[4] * V(c1);
      if (i + 1 < nx - 1) a1 = a1 + c[4] * V(xp);
      if (j < ny - 1) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row + nx]);
        a0 = a0 + c[5] * V(q.x);
        a1 = a1 + c[5] * V(q.y);
      }
      if (k < nz - 1) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row + nxy]);
        a0 = a0 + c[6] * V(q.x);
        a1 = a1 + c[6] * V(q.y);
      }
    } else {
      const int32_t j = jk;
      if (j > 0) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row - nx]);
        a0 = a0 + c[0] * V(q.x);
        a1 = a1 + c[0] * V(q.y);
      }
      if (i > 0) a0 = a0 + c[1] * V(xm);
      a1 = a1 + c[1] * V(c0);
      a0 = a0 + c[2] * V(c0);
      a1 = a1 + c[2] * V(c1);
      a0 = a0 + c[3] * V(c1);
      if (i + 1 < nx - 1) a1 = a1 + c[3] * V(xp);
      if (j < ny - 1) {
        const X2 q = *reinterpret_cast<const X2*>(&x[row + nx]);
        a0 = a0 + c[4] * V(q.x);
        a1 = a1 + c[4] * V(q.y);
      }
    }
    y0 = a0;
    y1 = a1;
  }
  // Row `row` with x[row - 1], x[row], x[row + 1] given (xm / xp are used only
  // where the row has that neighbour).
  template <class X>
  __device__ __forceinline__ V apply(int32_t row, const X* __restrict__ x, X xm, X xc, X xp) const {
    const int32_t i = row % nx;
    const int32_t jk = row / nx;
    V acc = V(0);
    if constexpr (NPTS == 7) {
      const int32_t j = jk % ny, k = jk / ny;
      const int32_t nxy = nx * ny;
      if (k > 0) acc = acc + c[0] * V(x[row - nxy]);
      if (j > 0) acc = acc + c[1] * V(x[row - nx]);
      if (i > 0) acc = acc + c[2] * V(xm);
      acc = acc + c[3] * V(xc);
      if (i < nx - 1) acc = acc + c[4] * V(xp);
      if (j < ny - 1) acc = acc + c[5] * V(x[row + nx]);
      if (k < nz - 1) acc = acc + c[6] * V(x[row + nxy]);
    } else {
      const int32_t j = jk;
      if (j > 0) acc = acc + c[0] * V(x[row - nx]);
      if (i > 0) acc = acc + c[1] * V(xm);
      acc = acc + c[2] * V(xc);
      if (i < nx - 1) acc = acc + c[3] * V(xp);
      if (j < ny - 1) acc = acc + c[4] * V(x[row + nx]);
    }
    return acc;
  }
};

// Matrix-free stencil on an nx x ny x nz grid (rows x fastest, Dirichlet
// boundaries: entries that would leave the grid are dropped) with 5 (nz = 1),
// 7 or 27 points, and either one set of constant coefficients (VAR = false:
// the 27-point stencil, c[] kernel arguments) or coefficients per row
// (VAR = true: coefficient d of row r at cf[d * n + r], so the rows of a block
// read consecutive addresses).  Term d runs over the neighbour offsets in
// ascending column order: 5-point {-y, -x, 0, +x, +y}, 7-point {-z, -y, -x, 0,
// +x, +y, +z}, 27-point (dz, dy, dx) with dz slowest and dx fastest, each in
// {-1, 0, +1}; a row's present terms are summed in that order, so the product
// equals the CSR product of the equivalent matrix bit for bit.  All 64 lanes
// of a row block call spmv together (lane l holds row b0 + l): each grid line
// a row touches is loaded once per lane, and its x-direction neighbours come
// from the adjacent lanes by a wave shift, with one load per lane for the
// ends of the block.
template <class V, bool VAR>
struct GridOp {
  using Val = V;
  // the array length keeps the struct free of padding (it is hashed as bytes)
  static constexpr int kC = VAR ? int(8 / sizeof(V)) : (sizeof(V) == 4 ? 28 : 27);
  const V* __restrict__ cf;  // VAR: npts * n per-row coefficients (borrowed)
  int32_t nx, ny, nz, npts;
  V c[kC];                   // constant coefficients (the 27-point stencil)

  // per-row coefficients are read once per product: the nontemporal hint keeps
  // them from displacing the gathered vector in the caches
  __device__ __forceinline__ V coef(int d, int32_t row, int32_t n) const {
    if constexpr (VAR) return __builtin_nontemporal_load(&cf[(int64_t)d * n + row]);
    else return c[d];
  }

  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    const int lane = threadIdx.x & 63;
    const int32_t nxy = nx * ny, n = nxy * nz;
    const int32_t rc = min(row, n - 1);  // rows past the grid compute a discarded copy of the last
    const int32_t b0 = row - lane;
    const int32_t i = rc % nx, jk = rc / nx, j = jk % ny, k = jk / ny;
    V acc = V(0);
    if (npts == 27) {
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        const int dz = l / 3 - 1, dy = l % 3 - 1;
        const bool lin = (dz < 0 ? k > 0 : (dz > 0 ? k < nz - 1 : true)) && (dy < 0 ? j > 0 : (dy > 0 ? j < ny - 1 : true));
        const int32_t off = dz * nxy + dy * nx;
        const X xc = x[lin ? rc + off : rc];
        // lanes 0..31 fetch the line's entry left of the block, 32..63 the one right of it
        const X xe = x[min(max(lane < 32 ? b0 + off - 1 : b0 + 64 + off, 0), n - 1)];
        const X xm = wave_shift<kWaveShr1>(xe, xc), xp = wave_shift<kWaveShl1>(xe, xc);
        if (lin && i > 0) acc = acc + coef(3 * l, rc, n) * V(xm);
        if (lin) acc = acc + coef(3 * l + 1, rc, n) * V(xc);
        if (lin && i < nx - 1) acc = acc + coef(3 * l + 2, rc, n) * V(xp);
      }
    } else if constexpr (VAR) {  // constant coefficients are the 27-point stencil only
      const X xc = x[rc];
      const X xe = x[min(max(lane < 32 ? b0 - 1 : b0 + 64, 0), n - 1)];
      const X xm = wave_shift<kWaveShr1>(xe, xc), xp = wave_shift<kWaveShl1>(xe, xc);
      int d = 0;
      if (npts == 7) {
        if (k > 0) acc = acc + coef(d, rc, n) * V(x[rc - nxy]);
        ++d;
      }
      if (j > 0) acc = acc + coef(d, rc, n) * V(x[rc - nx]);
      if (i > 0) acc = acc + coef(d + 1, rc, n) * V(xm);
      acc = acc + coef(d + 2, rc, n) * V(xc);
      if (i < nx - 1) acc = acc + coef(d + 3, rc, n) * V(xp);
      if (j < ny - 1) acc = acc + coef(d + 4, rc, n) * V(x[rc + nx]);
      if (npts == 7 && k < nz - 1) acc = acc + coef(d + 5, rc, n) * V(x[rc + nxy]);
    }
    return valid ? acc : V(0);
  }

  // Rows row and row + 1 (row even) by one lane; all 64 lanes of a 128-row
  // block call it together.  With an even x extent (then n is even too) the
  // two rows lie on one grid line and share every neighbour line: each line's
  // x values and each term's two per-row coefficients are aligned pairs, and
  // x[row + off - 1], x[row + off + 2] come from the adjacent lanes.  With an
  // odd extent each row is summed on its own with direct loads.
  template <class X>
  __device__ __forceinline__ void spmv2(int32_t row, bool valid0, bool valid1, const X* __restrict__ x, V& y0,
                                        V& y1) const {
    typedef X X2 __attribute__((ext_vector_type(2)));
    const int32_t nxy = nx * ny, n = nxy * nz;
    if (nx & 1) {
      y0 = valid0 ? direct(row, x, nxy, n) : V(0);
      y1 = valid1 ? direct(row + 1, x, nxy, n) : V(0);
      return;
    }
    const int lane = threadIdx.x & 63;
    const int32_t b0 = row - 2 * lane;
    const int32_t rc = min(row, n - 2);  // a pair inside the grid for the lanes past it
    const int32_t i = rc % nx, jk = rc / nx, j = jk % ny, k = jk / ny;
    V a0 = V(0), a1 = V(0);
    auto pair = [&](int d, V& c0, V& c1) {
      if constexpr (VAR) {
        typedef V V2 __attribute__((ext_vector_type(2)));
        const V2 q = __builtin_nontemporal_load(reinterpret_cast<const V2*>(&cf[(int64_t)d * n + rc]));
        c0 = q.x;
        c1 = q.y;
      } else {
        c0 = c[d];
        c1 = c[d];
      }
    };
    // one neighbour line (offset off, present for both rows or for neither)
    // with its terms d - 1, d, d + 1 in the x direction; xside: that line has
    // x-direction terms (27-point) or only the centre term (5/7-point y, z lines)
    auto line = [&](bool lin, int32_t off, int d, bool xside) {
      const X2 q = *reinterpret_cast<const X2*>(&x[lin ? rc + off : rc]);
      if (xside) {
        const X xe = x[min(max(lane < 32 ? b0 + off - 1 : b0 + 128 + off, 0), n - 1)];
        const X xm = wave_shift<kWaveShr1>(xe, q.y), xp = wave_shift<kWaveShl1>(xe, q.x);
        if (lin) {
          // row: x[row + off - 1], x[row + off], x[row + off + 1] = xm, q.x, q.y;
          // row + 1: q.x, q.y, xp (i is even, so row + 1 always has its -x term
          // and row its +x term)
          V m0, m1, c0, c1, p0, p1;
          pair(d - 1, m0, m1);
          pair(d, c0, c1);
          pair(d + 1, p0, p1);
          if (i > 0) a0 = a0 + m0 * V(xm);
          a0 = a0 + c0 * V(q.x);
          a0 = a0 + p0 * V(q.y);
          a1 = a1 + m1 * V(q.x);
          a1 = a1 + c1 * V(q.y);
          if (i + 1 < nx - 1) a1 = a1 + p1 * V(xp);
        }
      } else if (lin) {
        V c0, c1;
        pair(d, c0, c1);
        a0 = a0 + c0 * V(q.x);
        a1 = a1 + c1 * V(q.y);
      }
    };
    if (npts == 27) {
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        const int dz = l / 3 - 1, dy = l % 3 - 1;
        const bool lin = (dz < 0 ? k > 0 : (dz > 0 ? k < nz - 1 : true)) && (dy < 0 ? j > 0 : (dy > 0 ? j < ny - 1 : true));
        line(lin, dz * nxy + dy * nx, 3 * l + 1, true);
      }
    } else if constexpr (VAR) {  // constant coefficients are the 27-point stencil only
      const int base = (npts == 7) ? 1 : 0;  // index of the -y term
      if (npts == 7) line(k > 0, -nxy, 0, false);
      line(j > 0, -nx, base, false);
      line(true, 0, base + 2, true);
      line(j < ny - 1, nx, base + 4, false);
      if (npts == 7) line(k < nz - 1, nxy, 6, false);
    }
    y0 = valid0 ? a0 : V(0);
    y1 = valid1 ? a1 : V(0);
  }

  // Row `row` summed with direct loads of every neighbour (any lane mapping).
  template <class X>
  __device__ __forceinline__ V direct(int32_t row, const X* __restrict__ x, int32_t nxy, int32_t n) const {
    const int32_t i = row % nx, jk = row / nx, j = jk % ny, k = jk / ny;
    V acc = V(0);
    if (npts == 27) {
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const bool in = (dz < 0 ? k > 0 : (dz > 0 ? k < nz - 1 : true)) &&
                        (dy < 0 ? j > 0 : (dy > 0 ? j < ny - 1 : true)) &&
                        (dx < 0 ? i > 0 : (dx > 0 ? i < nx - 1 : true));
        if (in) acc = acc + coef(t, row, n) * V(x[row + dz * nxy + dy * nx + dx]);
      }
    } else if constexpr (VAR) {
      int d = 0;
      if (npts == 7) {
        if (k > 0) acc = acc + coef(d, row, n) * V(x[row - nxy]);
        ++d;
      }
      if (j > 0) acc = acc + coef(d, row, n) * V(x[row - nx]);
      if (i > 0) acc = acc + coef(d + 1, row, n) * V(x[row - 1]);
      acc = acc + coef(d + 2, row, n) * V(x[row]);
      if (i < nx - 1) acc = acc + coef(d + 3, row, n) * V(x[row + 1]);
      if (j < ny - 1) acc = acc + coef(d + 4, row, n) * V(x[row + nx]);
      if (npts == 7 && k < nz - 1) acc = acc + coef(d + 5, row, n) * V(x[row + nxy]);
    }
    return acc;
  }
};
template <class Op> struct IsGrid : std::false_type {};
template <class V, bool VAR> struct IsGrid<GridOp<V, VAR>> : std::true_type {};

// Diagonal layout of a CSR operator with at most kMaxDia distinct diagonals j - i
// (stencil discretisations): the values of diagonal d (offset off[d], the
// offsets ascending) lie contiguously, va[d * ld + i], and a 32-bit mask per
// row marks the diagonals the row holds.  A product reads per row the mask and
// one value per diagonal -- no row pointers, no column indices, every load
// coalesced -- and sums the row's present diagonals in ascending offset
// order, which is its CSR order (the layout is made only for rows stored with
// ascending columns), so the result is the CSR product bit for bit.  The
// values are a copy the context makes for each solve (binary64, the folded
// values of A M^{-1}, or their binary32 rounding); the mask is structure and
// belongs to the operator.
constexpr int kMaxDia = 32;
// OFFP: the offsets are read through a pointer (the batch's per-system table)
// instead of being held in the operator (a kernel argument, whose array the
// loops index directly).  NT: the values are loaded with the nontemporal
// hint, which keeps them from displacing the vectors in the caches (and in the
// memory-side cache); without it they compete like any other data, which is
// the better choice when the vectors and the layout fit there together.
template <class T>
__device__ __forceinline__ T load_nt(const T* p, std::true_type) { return __builtin_nontemporal_load(p); }
template <class T>
__device__ __forceinline__ T load_nt(const T* p, std::false_type) { return *p; }
template <class V, bool OFFP = false, bool NT = true>
struct DiaOpT {
  using Val = V;
  const uint32_t* __restrict__ mask;
  const V* __restrict__ va;
  int32_t n;
  int32_t nd;
  int32_t ld;     // stride between diagonals (rows rounded up to a multiple of 64)
  int32_t pad_ = 0;
  std::conditional_t<OFFP, const int32_t*, int32_t[kMaxDia]> off;

  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    const int32_t rc = min(row, n - 1);
    const uint32_t m = valid ? mask[rc] : 0u;
    V acc = V(0);
#pragma unroll 4
    for (int d = 0; d < nd; ++d) {
      const bool present = (m >> d) & 1u;
      const int32_t c = present ? rc + off[d] : rc;  // a present diagonal's column lies in [0, n)
      const V v = load_nt(&va[(int64_t)d * ld + rc], std::integral_constant<bool, NT>());
      const V t = acc + v * V(x[c]);
      acc = present ? t : acc;
    }
    return acc;
  }

  // Rows row and row + 1 (row even) by one lane, for the kernels that take two
  // rows per lane: the two values of a diagonal are one 2-element load, and
  // for an even offset so are the two x values.  valid1 implies valid0.
  template <class X>
  __device__ __forceinline__ void spmv2(int32_t row, bool valid0, bool valid1, const X* __restrict__ x, V& y0,
                                        V& y1) const {
    typedef V V2 __attribute__((ext_vector_type(2)));
    typedef X X2 __attribute__((ext_vector_type(2)));
    const int32_t r0 = min(row, n - 1);
    const int32_t r1 = min(row + 1, n - 1);
    const uint32_t m0 = valid0 ? mask[r0] : 0u, m1 = valid1 ? mask[r1] : 0u;
    // an even slot whose pair lies inside the layout (rows past n read a
    // discarded copy of the last pair)
    const int32_t rv = min(row, (n - 1) & ~1);
    V a0 = V(0), a1 = V(0);
#pragma unroll 4
    for (int d = 0; d < nd; ++d) {
      const bool p0 = (m0 >> d) & 1u, p1 = (m1 >> d) & 1u;
      const V2 v = load_nt(reinterpret_cast<const V2*>(&va[(int64_t)d * ld + rv]), std::integral_constant<bool, NT>());
      X x0, x1;
      // with an even offset and row + 1's entry present, x[row + off], x[row + off + 1]
      // both lie in [0, n) (row + 1 + off is odd, so at least 1) and form an
      // aligned pair of the (at least 16-byte aligned) vector
      if ((off[d] & 1) == 0 && p1) {
        const X2 xx = *reinterpret_cast<const X2*>(&x[row + off[d]]);
        x0 = xx.x;
        x1 = xx.y;
      } else {
        x0 = x[p0 ? r0 + off[d] : r0];
        x1 = x[p1 ? r1 + off[d] : r1];
      }
      const V t0 = a0 + v.x * V(x0), t1 = a1 + v.y * V(x1);
      a0 = p0 ? t0 : a0;
      a1 = p1 ? t1 : a1;
    }
    y0 = a0;
    y1 = a1;
  }

  // Rows row .. row + 3 (row a multiple of 4) by one lane, for the kernels
  // that take four rows per lane; nv of the four lie below n.  The four
  // values of a diagonal are one 4-element load.  The four x values are one
  // aligned 4-element load for an offset that is a multiple of 4, two aligned
  // pairs for an offset of 2 modulo 4, else four single loads.  Each row's sum
  // runs over its present diagonals in ascending order, as spmv's.
  template <class X>
  __device__ __forceinline__ void spmv4(int32_t row, int nv, const X* __restrict__ x, V (&y)[4]) const {
    typedef V V4 __attribute__((ext_vector_type(4)));
    typedef X X4 __attribute__((ext_vector_type(4)));
    typedef X X2 __attribute__((ext_vector_type(2)));
    int32_t rr[4];
    uint32_t m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rr[k] = min(row + k, n - 1);
    if (nv == 4) {
      // row .. row + 3 < n: one aligned 16-byte load of the four masks
      typedef uint32_t U4 __attribute__((ext_vector_type(4)));
      const U4 mm = *reinterpret_cast<const U4*>(&mask[row]);
      m[0] = mm.x;
      m[1] = mm.y;
      m[2] = mm.z;
      m[3] = mm.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) m[k] = (k < nv) ? mask[rr[k]] : 0u;
    }
    // a slot of four inside the layout (rows past n read a discarded copy of the last four)
    const int32_t rv = min(row, (n - 1) & ~3);
    V acc[4] = {V(0), V(0), V(0), V(0)};
#pragma unroll 2
    for (int d = 0; d < nd; ++d) {
      bool p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = (m[k] >> d) & 1u;
      const V4 v = load_nt(reinterpret_cast<const V4*>(&va[(int64_t)d * ld + rv]), std::integral_constant<bool, NT>());
      const int32_t o = off[d];
      X xs[4];
      // a present entry's column lies in [0, n).  For an offset of 0 mod 4 with
      // row + 3's entry present, row + o .. row + o + 3 lie in [0, n) (row + o is
      // a multiple of 4 and row + 3 + o >= 0), an aligned four of the (at least
      // 16-byte aligned) vector; likewise an offset of 2 mod 4 and row + 1's
      // (row + 3's) entry for the aligned pair at row + o (row + o + 2).
      if ((o & 3) == 0 && p[3]) {
        const X4 q = *reinterpret_cast<const X4*>(&x[row + o]);
        xs[0] = q.x;
        xs[1] = q.y;
        xs[2] = q.z;
        xs[3] = q.w;
      } else if ((o & 1) == 0) {
        if (p[1]) {
          const X2 q = *reinterpret_cast<const X2*>(&x[row + o]);
          xs[0] = q.x;
          xs[1] = q.y;
        } else {
          xs[0] = x[p[0] ? rr[0] + o : rr[0]];
          xs[1] = x[rr[1]];
        }
        if (p[3]) {
          const X2 q = *reinterpret_cast<const X2*>(&x[row + 2 + o]);
          xs[2] = q.x;
          xs[3] = q.y;
        } else {
          xs[2] = x[p[2] ? rr[2] + o : rr[2]];
          xs[3] = x[rr[3]];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[k] = x[p[k] ? rr[k] + o : rr[k]];
      }
      const V vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const V t = acc[k] + vv[k] * V(xs[k]);
        acc[k] = p[k] ? t : acc[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = acc[k];
  }
};
using DiaOp = DiaOpT<double>;
using DiaOpF = DiaOpT<float>;
using DiaOpB = DiaOpT<double, true>;  // batched: offsets in the system table
using DiaOpC = DiaOpT<double, false, false>;  // ordinary value loads

// The diagonal layout with its values given by value indexing (the value
// compression of CSR-VI, Kourtis, Goumas and Koziris, 2008), for at most
// kViDia diagonals: row i's word code[i] holds in byte d a code into
// diagonal d's table of at most kViTab distinct values, or kViAbsent where
// the row has no entry on d (and in the bytes past nd).  The operator is 8
// bytes per row instead of 4 + sizeof(V) nd, and one load gives a row all its
// codes, so each diagonal's table read depends on that one load only.  The
// table keeps each value's bit pattern (binary32 ones zero-extended).  A
// product reads the same value of every present entry as DiaOpT<V> does and
// sums the same terms in the same order: the same bits.
constexpr int kViTab = 16;
constexpr int kViDia = 8;
constexpr uint32_t kViAbsent = 0xffu;
template <class V>
struct DiaViOpT {
  using Val = V;
  const uint64_t* __restrict__ code;  // [ld] (rows past n: every byte kViAbsent)
  const uint64_t* __restrict__ tab;   // [nd][kViTab] bit patterns
  int32_t n;
  int32_t nd;
  int32_t ld;
  int32_t pad_ = 0;
  int32_t off[kViDia];

  __device__ __forceinline__ V val(int d, uint32_t c, bool present) const {
    const uint64_t b = tab[d * kViTab + (present ? c : 0u)];
    if constexpr (sizeof(V) == 8) return __longlong_as_double((long long)b);
    else return __uint_as_float((uint32_t)b);
  }

  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    const int32_t rc = min(row, n - 1);
    const uint64_t w = valid ? code[rc] : ~0ull;
    V acc = V(0);
#pragma unroll
    for (int d = 0; d < kViDia; ++d) {
      if (d < nd) {
        const uint32_t c = (uint32_t)(w >> (8 * d)) & 0xffu;
        const bool present = c != kViAbsent;
        const int32_t col = present ? rc + off[d] : rc;  // a present diagonal's column lies in [0, n)
        const V t = acc + val(d, c, present) * V(x[col]);
        acc = present ? t : acc;
      }
    }
    return acc;
  }

  // Rows row and row + 1 (row even) by one lane, as DiaOpT::spmv2: the two
  // rows' code words are one 16-byte load.
  template <class X>
  __device__ __forceinline__ void spmv2(int32_t row, bool valid0, bool valid1, const X* __restrict__ x, V& y0,
                                        V& y1) const {
    typedef X X2 __attribute__((ext_vector_type(2)));
    typedef uint64_t U2 __attribute__((ext_vector_type(2)));
    const int32_t r0 = min(row, n - 1);
    const int32_t r1 = min(row + 1, n - 1);
    // an even word whose pair lies inside the array (ld is a multiple of 64)
    const int32_t rv = min(row, (n - 1) & ~1);
    const U2 ww = *reinterpret_cast<const U2*>(&code[rv]);
    const uint64_t w0 = valid0 ? (rv == row ? ww.x : code[r0]) : ~0ull;
    const uint64_t w1 = valid1 ? ww.y : ~0ull;
    V a0 = V(0), a1 = V(0);
#pragma unroll
    for (int d = 0; d < kViDia; ++d) {
      if (d < nd) {
        const uint32_t c0 = (uint32_t)(w0 >> (8 * d)) & 0xffu, c1 = (uint32_t)(w1 >> (8 * d)) & 0xffu;
        const bool p0 = c0 != kViAbsent, p1 = c1 != kViAbsent;
        const V v0 = val(d, c0, p0), v1 = val(d, c1, p1);
        X x0, x1;
        // as DiaOpT::spmv2: an even offset with row + 1's entry present makes an aligned pair
        if ((off[d] & 1) == 0 && p1) {
          const X2 xx = *reinterpret_cast<const X2*>(&x[row + off[d]]);
          x0 = xx.x;
          x1 = xx.y;
        } else {
          x0 = x[p0 ? r0 + off[d] : r0];
          x1 = x[p1 ? r1 + off[d] : r1];
        }
        const V t0 = a0 + v0 * V(x0), t1 = a1 + v1 * V(x1);
        a0 = p0 ? t0 : a0;
        a1 = p1 ? t1 : a1;
      }
    }
    y0 = a0;
    y1 = a1;
  }

  // Rows row .. row + 3 (row a multiple of 4) by one lane, as DiaOpT::spmv4;
  // nv of the four lie below n.  Their code words are two 16-byte loads when
  // all four rows exist.
  template <class X>
  __device__ __forceinline__ void spmv4(int32_t row, int nv, const X* __restrict__ x, V (&y)[4]) const {
    typedef X X4 __attribute__((ext_vector_type(4)));
    typedef X X2 __attribute__((ext_vector_type(2)));
    typedef uint64_t U2 __attribute__((ext_vector_type(2)));
    int32_t rr[4];
    uint64_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rr[k] = min(row + k, n - 1);
    if (nv == 4) {
      // row .. row + 3 < n: the four words, 32-byte aligned
      const U2 a = *reinterpret_cast<const U2*>(&code[row]);
      const U2 b = *reinterpret_cast<const U2*>(&code[row + 2]);
      w[0] = a.x;
      w[1] = a.y;
      w[2] = b.x;
      w[3] = b.y;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = (k < nv) ? code[rr[k]] : ~0ull;
    }
    V acc[4] = {V(0), V(0), V(0), V(0)};
#pragma unroll
    for (int d = 0; d < kViDia; ++d) {
      if (d < nd) {
        bool p[4];
        V vv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t c = (uint32_t)(w[k] >> (8 * d)) & 0xffu;
          p[k] = c != kViAbsent;
          vv[k] = val(d, c, p[k]);
        }
        const int32_t o = off[d];
        X xs[4];
        // as DiaOpT::spmv4: aligned fours, aligned pairs or single loads by the offset
        if ((o & 3) == 0 && p[3]) {
          const X4 q = *reinterpret_cast<const X4*>(&x[row + o]);
          xs[0] = q.x;
          xs[1] = q.y;
          xs[2] = q.z;
          xs[3] = q.w;
        } else if ((o & 1) == 0) {
          if (p[1]) {
            const X2 q = *reinterpret_cast<const X2*>(&x[row + o]);
            xs[0] = q.x;
            xs[1] = q.y;
          } else {
            xs[0] = x[p[0] ? rr[0] + o : rr[0]];
            xs[1] = x[rr[1]];
          }
          if (p[3]) {
            const X2 q = *reinterpret_cast<const X2*>(&x[row + 2 + o]);
            xs[2] = q.x;
            xs[3] = q.y;
          } else {
            xs[2] = x[p[2] ? rr[2] + o : rr[2]];
            xs[3] = x[rr[3]];
          }
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) xs[k] = x[p[k] ? rr[k] + o : rr[k]];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const V t = acc[k] + vv[k] * V(xs[k]);
          acc[k] = p[k] ? t : acc[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = acc[k];
  }
};
using DiaViOp = DiaViOpT<double>;
using DiaViOpF = DiaViOpT<float>;

// Matrix-free 27-point variable-coefficient convection-diffusion operator on
// the n^3 interior nodes of the unit cube (h = 1/(n+1)), Dirichlet boundaries,
// rows x fastest.  Its entries are formed from the (n+1)^3 cell coefficients
// kappa exactly as the workload's assembly forms them: for each offset d of
// the 26 neighbours, in (dz, dy, dx) order, kbar_d is the sum of the 4, 2 or 1
// cells node p shares with p + d (in (c, b, a) order, from 0.0) times
// 1/count; the coupling is -kbar_d, minus |hb_a| on the upwind face of axis
// a; the diagonal is (sum of all 26 kbar_d + hsum) + shift.  The row is then
// summed in ascending column order from 0, so the product equals the
// assembled CSR product bit for bit.  FOLD: the entries are scaled by the
// column's dscale (A M^{-1}, each a_ij * dinv_j rounded once, as the folded
// CSR values are).  V: the arithmetic type of the product; a binary32 product
// rounds each binary64 entry once, like the binary32 copy of a CSR operator.
template <class V, bool FOLD>
struct Conv27Op {
  using Val = V;
  int32_t n;
  int32_t upneg;                          // bit a: beta_a >= 0, the upwind neighbour is p - e_a
  const double* __restrict__ kappa;       // (n+1)^3 cells, x fastest
  const double* __restrict__ dscale;      // FOLD: dinv per column
  double hab[3];                          // |hb_a| = |beta_a / (n+1)|
  double hsum;                            // (|hb_x| + |hb_y|) + |hb_z|
  double shift;

  // The cells node (i, j, k) touches: K[c][b][a] = kappa(i+a, j+b, k+c).
  __device__ __forceinline__ void cells(int32_t i, int32_t j, int32_t k, double (&K)[2][2][2]) const {
    const int64_t cn = (int64_t)n + 1;
    const double* kp = kappa + (i + cn * (j + cn * (int64_t)k));
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) K[c][b][a] = kp[a + cn * (b + cn * c)];
  }

  // kbar of offset e = (dz+1)*9 + (dy+1)*3 + (dx+1), e != 13.
  template <int E>
  static __device__ __forceinline__ double kbar(const double (&K)[2][2][2]) {
    constexpr int dx = E % 3 - 1, dy = (E / 3) % 3 - 1, dz = E / 9 - 1;
    constexpr int alo = dx > 0 ? 1 : 0, ahi = dx < 0 ? 0 : 1;
    constexpr int blo = dy > 0 ? 1 : 0, bhi = dy < 0 ? 0 : 1;
    constexpr int clo = dz > 0 ? 1 : 0, chi = dz < 0 ? 0 : 1;
    constexpr int cnt = (ahi - alo + 1) * (bhi - blo + 1) * (chi - clo + 1);
    double ks = 0.0;
#pragma unroll
    for (int c = clo; c <= chi; ++c)
#pragma unroll
      for (int b = blo; b <= bhi; ++b)
#pragma unroll
        for (int a = alo; a <= ahi; ++a) ks = ks + K[c][b][a];
    return ks * (1.0 / (double)cnt);
  }

  template <int E>
  static __device__ __forceinline__ void kbars(const double (&K)[2][2][2], double (&kb)[27], double& dsum) {
    if constexpr (E < 27) {
      if constexpr (E != 13) {
        kb[E] = kbar<E>(K);
        dsum = dsum + kb[E];
      }
      kbars<E + 1>(K, kb, dsum);
    }
  }

  // Entry E = (dz+1)*9 + (dy+1)*3 + (dx+1) of the row (before any scaling).
  template <int E>
  __device__ __forceinline__ double entry(const double (&kb)[27], double diag) const {
    if constexpr (E == 13) {
      return diag;
    } else {
      constexpr int dx = E % 3 - 1, dy = (E / 3) % 3 - 1, dz = E / 9 - 1;
      double a = -kb[E];
      if constexpr ((dx != 0) + (dy != 0) + (dz != 0) == 1) {
        constexpr int ax = dx != 0 ? 0 : (dy != 0 ? 1 : 2);
        constexpr int side = dx != 0 ? dx : (dy != 0 ? dy : dz);
        const bool upwind = ((upneg >> ax) & 1) ? (side < 0) : (side > 0);
        if (upwind) a = -kb[E] - hab[ax];
      }
      return a;
    }
  }

  // The three terms of grid line L = (dz+1)*3 + (dy+1) (dx = -1, 0, +1).  All
  // 64 lanes take part: the centre value x[row + off] is loaded by every lane
  // (its own row when the line leaves the grid, a value then never used), and
  // the dx = -1 / +1 neighbours come from the adjacent lanes by a wave shift;
  // lanes 0 and 63 receive instead the one extra value loaded per line (the
  // element before / after the block), supplied as the shift's fill value.
  // Terms whose neighbour lies outside the grid are not added (the selected
  // accumulator keeps its value), as the assembled row has no such entry.
  template <int L, class X>
  __device__ __forceinline__ void line(int32_t row, int32_t b0, int lane, int32_t i, int32_t j, int32_t k,
                                       const double (&kb)[27], double diag, const X* __restrict__ x, V& acc) const {
    if constexpr (L < 9) {
      constexpr int dy = L % 3 - 1, dz = L / 3 - 1;
      const int32_t N = n * n * n;
      const int32_t off = n * dy + n * n * dz;
      const bool lin = (dy < 0 ? j > 0 : (dy > 0 ? j < n - 1 : true)) && (dz < 0 ? k > 0 : (dz > 0 ? k < n - 1 : true));
      const int32_t c = lin ? row + off : row;
      const int32_t e = min(max(lane < 32 ? b0 + off - 1 : b0 + 64 + off, 0), N - 1);
      const X xc = x[c], xe = x[e];
      const X xs[3] = {wave_shift<kWaveShr1>(xe, xc), xc, wave_shift<kWaveShl1>(xe, xc)};
      double ss[3] = {1.0, 1.0, 1.0};
      if constexpr (FOLD) {
        const double sc = dscale[c], se = dscale[e];
        ss[0] = wave_shift<kWaveShr1>(se, sc);
        ss[1] = sc;
        ss[2] = wave_shift<kWaveShl1>(se, sc);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bool in = lin && (q == 0 ? i > 0 : (q == 2 ? i < n - 1 : true));
        double a = (q == 0) ? entry<L * 3>(kb, diag) : (q == 1 ? entry<L * 3 + 1>(kb, diag) : entry<L * 3 + 2>(kb, diag));
        if constexpr (FOLD) a = a * ss[q];
        const V t = acc + V(a) * V(xs[q]);
        acc = in ? t : acc;
      }
      line<L + 1>(row, b0, lane, i, j, k, kb, diag, x, acc);
    }
  }

  __device__ __forceinline__ double diag_of(const double (&kb)[27], double dsum) const {
    (void)kb;
    return (dsum + hsum) + shift;
  }

  // a_ii of row `row` (the unscaled operator).
  __device__ __forceinline__ double diagonal(int32_t row) const {
    const int32_t i = row % n, jk = row / n, j = jk % n, k = jk / n;
    double K[2][2][2], kb[27];
    cells(i, j, k, K);
    double dsum = 0.0;
    kbars<0>(K, kb, dsum);
    return diag_of(kb, dsum);
  }

  // Row `row` of A x (all 64 lanes of the row's 64-row block call it together;
  // lanes with valid == false return 0).
  template <class X>
  __device__ __forceinline__ V spmv(int32_t row, bool valid, const X* __restrict__ x) const {
    const int lane = threadIdx.x & 63;
    const int32_t b0 = row - lane;
    const int32_t rc = min(row, n * n * n - 1);  // rows past the grid compute a discarded copy of the last
    const int32_t i = rc % n, jk = rc / n, j = jk % n, k = jk / n;
    double K[2][2][2], kb[27];
    cells(i, j, k, K);
    double dsum = 0.0;
    kbars<0>(K, kb, dsum);
    const double diag = diag_of(kb, dsum);
    V acc = V(0);
    line<0>(rc, b0, lane, i, j, k, kb, diag, x, acc);
    return valid ? acc : V(0);
  }
};
using Conv27 = Conv27Op<double, false>;
using Conv27F = Conv27Op<double, true>;

template <class Op> struct IsConv27 : std::false_type {};
template <class V, bool F> struct IsConv27<Conv27Op<V, F>> : std::true_type {};

// Preconditioner modes: none (Algorithms 7 and 9), Jacobi with a vector of
// 1/a_ii, Jacobi with one constant 1/a_ii (constant diagonal).
enum { PC_NONE = 0, PC_VEC = 1, PC_SCALAR = 2 };

// Folded Jacobi on per-row coefficients (Section 3.6 with A M^{-1} formed):
// out[d * n + r] = coef(d, r) * dinv[column of term d], one rounding each, for
// the terms present (the others are left as they are: never read).
template <int PC>
__global__ __launch_bounds__(256) void k_fold_grid(GridOp<double, true> op, double* __restrict__ out,
                                                   const double* __restrict__ dinv, double dinv_s) {
  const int32_t nxy = op.nx * op.ny, n = nxy * op.nz;
  for (int32_t r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const int32_t i = r % op.nx, jk = r / op.nx, j = jk % op.ny, k = jk / op.ny;
    auto put = [&](int d, bool present, int32_t col) {
      if (present) out[(int64_t)d * n + r] = op.coef(d, r, n) * (PC == PC_VEC ? dinv[col] : dinv_s);
    };
    if (op.npts == 27) {
      for (int l = 0; l < 27; ++l) {
        const int dz = l / 9 - 1, dy = (l / 3) % 3 - 1, dx = l % 3 - 1;
        const bool in = (dz < 0 ? k > 0 : (dz > 0 ? k < op.nz - 1 : true)) &&
                        (dy < 0 ? j > 0 : (dy > 0 ? j < op.ny - 1 : true)) &&
                        (dx < 0 ? i > 0 : (dx > 0 ? i < op.nx - 1 : true));
        put(l, in, r + dz * nxy + dy * op.nx + dx);
      }
    } else {
      int d = 0;
      if (op.npts == 7) put(d++, k > 0, r - nxy);
      put(d, j > 0, r - op.nx);
      put(d + 1, i > 0, r - 1);
      put(d + 2, true, r);
      put(d + 3, i < op.nx - 1, r + 1);
      put(d + 4, j < op.ny - 1, r + op.nx);
      if (op.npts == 7) put(d + 5, k < op.nz - 1, r + nxy);
    }
  }
}

// dinv[r] = 1 / (the centre coefficient of row r) of per-row coefficients; bit 0
// of *flag is set for a zero or non-finite diagonal entry.
__global__ __launch_bounds__(256) void k_dinv_grid(GridOp<double, true> op, double* __restrict__ dinv,
                                                   int32_t* flag) {
  const int32_t n = op.nx * op.ny * op.nz;
  const int centre = op.npts / 2;
  for (int32_t r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double a = op.coef(centre, r, n);
    if (a == 0.0 || !isfinite(a)) atomicOr(flag, 1);
    dinv[r] = 1.0 / a;
  }
}


// Kernel arguments: sizes, launch shape, state slots, partial-sum buffers and
// every vector of the solvers.  Without a preconditioner the hatted pointers
// alias the unhatted ones.
struct Args {
  int32_t n;              // rows
  int32_t G;              // workgroups of this launch (producing kernels)
  int32_t R;              // 64-row blocks per wave (power of two <= kMaxR)
  int32_t Gin;            // partials to consume (workgroups of the producer)
  int32_t first;          // first iteration: consume the setup reduction
  int32_t mode;           // precision form: 1 = reduction after a forced replacement
  int32_t wg;             // workgroup index within the system (-1: blockIdx.x; -2: XCD-contiguous)
  int32_t pstride;        // stride between the ND partial-sum rows (kMaxG, or the batch's workgroups)
  int32_t par;            // batched launches: state slot read (written: par ^ 1)
  int32_t aform;          // alpha_{i+1} of the pipelined solvers: 5 = eq. (5), otherwise eq. (3)
  const DevState* sin;    // state read by this launch
  DevState* sout;         // state written by workgroup 0
  const double* pin;      // partials consumed: pin[k * kMaxG + wg]
  double* pout;           // partials produced: pout[k * kMaxG + wg]
  double* hist;           // nullable history of ||r_i|| / ||r_0||
  const double* b;
  double* x;
  double *r0, *r, *rh, *w, *wh, *t, *ph, *s, *sh, *z, *zh, *v;  // p-BiCGStab
  double *p, *q, *qh, *y;                                       // BiCGStab
  const double* dinv;
  double dinv_s;
  // precision form: binary32 vectors and binary64 replacement scratch
  float *r0f, *rf, *wf, *tf, *pf, *sf, *zf, *vf;
  double *r64, *s64;
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

// 64-bit DPP move: lane l receives the value of the lane selected by CTRL in
// the rows enabled by ROW_MASK; other lanes receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_t(T v) {
  if constexpr (sizeof(T) == 8) return dpp_f64<CTRL, ROW_MASK>(v);
  else return dpp_f32<CTRL, ROW_MASK>(v);
}

// Balanced-tree sum over the 64 lanes of a wave; the result is valid in lane
// 63.  Level m adds to the last lane of every aligned block of 2m lanes the
// sum held by the last lane of the block's left half (row_shr 1, 2, 4, 8,
// then row_bcast 15 and 31 across the 16-lane rows), so lane 63 ends with
// ((l0 + l1) + (l2 + l3)) + ... exactly as the pairwise order prescribes.
template <int ND, class T>
__device__ __forceinline__ void wave_sum63(T (&v)[ND]) {
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x111, 0xF>(v[k]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x112, 0xF>(v[k]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x114, 0xF>(v[k]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x118, 0xF>(v[k]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x142, 0xA>(v[k]);
#pragma unroll
  for (int k = 0; k < ND; ++k) v[k] = v[k] + dpp_t<0x143, 0xC>(v[k]);
}

// Balanced-tree sum of one value per thread over the workgroup (256 threads,
// 4 waves); every thread receives the totals.  No barrier after the last read
// of lw: a kernel gathers at most once per launch (its branches are
// exclusive), and the persistent kernel's grid barrier separates its gathers.
template <int ND, class T>
__device__ __forceinline__ void wg_sum_all(T (&v)[ND], T (&out)[ND]) {
  __shared__ T lw[4][ND];
  wave_sum63<ND, T>(v);
  if ((threadIdx.x & 63) == 63) {
#pragma unroll
    for (int k = 0; k < ND; ++k) lw[threadIdx.x >> 6][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < ND; ++k) out[k] = (lw[0][k] + lw[1][k]) + (lw[2][k] + lw[3][k]);
}

// Totals of the Gin partials of each of the ND sums in pin, in pairwise
// order, "+ 0.0"; identical in every thread of every workgroup.  T is the
// arithmetic type of the sums (binary32 partials are stored widened, exactly);
// the totals are returned widened to binary64.
template <int ND, class T = double>
__device__ __forceinline__ void gather_sums(const Args& a, double (&res)[ND]) {
  const int base = (int)threadIdx.x * kChunk;
  T v[ND], tot[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    T c[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      const T p = T(a.pin[k * a.pstride + min(base + j, a.Gin - 1)]);  // clamped: branch-free
      c[j] = (base + j < a.Gin) ? p : T(0);
    }
#pragma unroll
    for (int w = 1; w < kChunk; w <<= 1) {
#pragma unroll
      for (int j = 0; j < kChunk; j += 2 * w) c[j] = c[j] + c[j + w];
    }
    v[k] = c[0];
  }
  wg_sum_all<ND, T>(v, tot);
#pragma unroll
  for (int k = 0; k < ND; ++k) res[k] = double(tot[k] + T(0));
}

// Index of this workgroup among the workgroups of its system.  With
// wg == -2, consecutive indices share an XCD: the hardware deals the
// workgroups of a launch to the 8 XCDs in turn (workgroup b runs on XCD
// b % 8), so XCD x is given the x-th contiguous run of indices, and a row's
// neighbours a grid plane away are mostly read through the same L2.  The map
// is a bijection of [0, gridDim.x); which rows and partial slot an index owns
// is unchanged, so are the results.
__device__ __forceinline__ int wg_index(const Args& a) {
  if (a.wg >= 0) return a.wg;
  const int b = (int)blockIdx.x;
  if (a.wg == -1) return b;
  const int G = (int)gridDim.x, q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}
// first thread of the system's first workgroup (batched launches hold many systems)
__device__ __forceinline__ bool sys_leader(const Args& a) { return wg_index(a) == 0 && threadIdx.x == 0; }

// The workgroup's rows with ND products each; writes its partial sums to
// pout[k][blockIdx.x].  Body(row, valid, d) is called by all 64 lanes of a
// block (so an operator may work on the block cooperatively); lanes with
// valid == false (rows past n) must leave d at 0 and touch no vector.
//
// The partial is the pairwise sum of the workgroup's 4 R block totals in row
// order.  Each wave builds the balanced tree over its R blocks (R a power of
// two) as the blocks complete, like the digits of a binary counter: lvl[l]
// holds the sum of the last finished group of 2^l blocks, and finishing block
// j merges one level per trailing 1 bit of j (left subtree + right subtree).
// Only lane 63, which holds a block's wave sum, touches the wave's levels.
// The four wave totals then combine as (w0 + w1) + (w2 + w3).
template <int ND, class T = double, class Body>
__device__ __forceinline__ void produce(const Args& a, Body body) {
  __shared__ T lvl[4][kLevels][ND];
  __shared__ T wtot[ND][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = ((int64_t)wg_index(a) * 4 + wave) * a.R * 64;
  for (int j = 0; j < a.R; ++j) {
    const int64_t b0 = wbase + (int64_t)j * 64;
    T d[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = T(0);
    if (b0 < a.n) {
      const int32_t row = (int32_t)(b0 + lane);
      body(row, row < a.n, d);
      wave_sum63<ND, T>(d);
    }
    if (lane == 63) {
      int l = 0;
      for (int bits = j; bits & 1; bits >>= 1, ++l) {
#pragma unroll
        for (int k = 0; k < ND; ++k) d[k] = lvl[wave][l][k] + d[k];
      }
#pragma unroll
      for (int k = 0; k < ND; ++k) lvl[wave][l][k] = d[k];
    }
  }
  if (lane == 63) {
    const int top = __builtin_ctz((unsigned)a.R);  // the whole tree of R = 2^top blocks
#pragma unroll
    for (int k = 0; k < ND; ++k) wtot[k][wave] = lvl[wave][top][k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k)
      a.pout[k * a.pstride + wg_index(a)] = double((wtot[k][0] + wtot[k][1]) + (wtot[k][2] + wtot[k][3]));
  }
  // no barrier here: a kernel produces once per launch, and the persistent
  // kernel's grid barrier separates its reductions
}

// As produce(), with each lane taking two neighbouring rows: lane l of a
// 128-row block handles rows 2l and 2l + 1, and the body returns their sum.
// Those two rows are sibling leaves of the balanced tree over the row index,
// so the wave, workgroup and grid sums are the same tree and the partials are
// bit for bit those of produce(); the wave covers the same 64 R rows as R / 2
// blocks of 128.  Body(row, valid0, valid1, d) with row even; needs R >= 2.
template <int ND, class T = double, class Body>
__device__ __forceinline__ void produce2(const Args& a, Body body) {
  __shared__ T lvl[4][kLevels][ND];
  __shared__ T wtot[ND][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = ((int64_t)wg_index(a) * 4 + wave) * a.R * 64;
  const int R2 = a.R >> 1;
  for (int j = 0; j < R2; ++j) {
    const int64_t b0 = wbase + (int64_t)j * 128;
    T d[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = T(0);
    if (b0 < a.n) {
      const int32_t row = (int32_t)(b0 + 2 * lane);
      body(row, row < a.n, row + 1 < a.n, d);
      wave_sum63<ND, T>(d);
    }
    if (lane == 63) {
      int l = 0;
      for (int bits = j; bits & 1; bits >>= 1, ++l) {
#pragma unroll
        for (int k = 0; k < ND; ++k) d[k] = lvl[wave][l][k] + d[k];
      }
#pragma unroll
      for (int k = 0; k < ND; ++k) lvl[wave][l][k] = d[k];
    }
  }
  if (lane == 63) {
    const int top = __builtin_ctz((unsigned)R2);
#pragma unroll
    for (int k = 0; k < ND; ++k) wtot[k][wave] = lvl[wave][top][k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k)
      a.pout[k * a.pstride + wg_index(a)] = double((wtot[k][0] + wtot[k][1]) + (wtot[k][2] + wtot[k][3]));
  }
}

// x[row] = (x[row] + u0) + v0 and x[row + 1] = (x[row + 1] + u1) + v1 (row
// even) on the caller's x: one 16-byte load and store when x is 16-byte
// aligned, so each cache line is written whole by one instruction; else row
// by row.  The same arithmetic either way.
__device__ __forceinline__ void update_x2(double* __restrict__ x, int32_t row, bool valid1, double u0, double u1,
                                          double v0, double v1) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  if (valid1 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    D2 xx = *reinterpret_cast<const D2*>(&x[row]);
    xx.x = xx.x + u0 + v0;
    xx.y = xx.y + u1 + v1;
    *reinterpret_cast<D2*>(&x[row]) = xx;
    return;
  }
  x[row] = x[row] + u0 + v0;
  if (valid1) x[row + 1] = x[row + 1] + u1 + v1;
}

// As produce2, with each lane taking four neighbouring rows: lane l of a
// 256-row block handles rows 4l .. 4l + 3, which form one subtree of two
// levels of the balanced tree over the row index, and the body returns that
// subtree's sum ((d0 + d1) + (d2 + d3), a row past n a zero leaf).  The wave
// covers the same 64 R rows as R / 4 blocks of 256, so the partials are bit
// for bit those of produce().  Body(row, nv, d) with row a multiple of 4 and
// nv = the rows of the four below n (0 to 4); needs R >= 4.
template <int ND, class T = double, class Body>
__device__ __forceinline__ void produce4(const Args& a, Body body) {
  __shared__ T lvl[4][kLevels][ND];
  __shared__ T wtot[ND][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = ((int64_t)wg_index(a) * 4 + wave) * a.R * 64;
  const int R4 = a.R >> 2;
  for (int j = 0; j < R4; ++j) {
    const int64_t b0 = wbase + (int64_t)j * 256;
    T d[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = T(0);
    if (b0 < a.n) {
      const int32_t row = (int32_t)(b0 + 4 * lane);
      body(row, (int)max(0, min(4, a.n - row)), d);
      wave_sum63<ND, T>(d);
    }
    if (lane == 63) {
      int l = 0;
      for (int bits = j; bits & 1; bits >>= 1, ++l) {
#pragma unroll
        for (int k = 0; k < ND; ++k) d[k] = lvl[wave][l][k] + d[k];
      }
#pragma unroll
      for (int k = 0; k < ND; ++k) lvl[wave][l][k] = d[k];
    }
  }
  if (lane == 63) {
    const int top = __builtin_ctz((unsigned)R4);
#pragma unroll
    for (int k = 0; k < ND; ++k) wtot[k][wave] = lvl[wave][top][k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < ND; ++k)
      a.pout[k * a.pstride + wg_index(a)] = double((wtot[k][0] + wtot[k][1]) + (wtot[k][2] + wtot[k][3]));
  }
}

// x[row + k] = (x[row + k] + u[k]) + v[k] for the nv rows of four (row a
// multiple of 4) on the caller's x: two 16-byte loads and stores when all four
// are rows and x is 16-byte aligned, else row by row.  The same arithmetic
// either way.
__device__ __forceinline__ void update_x4(double* __restrict__ x, int32_t row, int nv, const double (&u)[4],
                                          const double (&v)[4]) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  if (nv == 4 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    D2 lo = *reinterpret_cast<const D2*>(&x[row]);
    D2 hi = *reinterpret_cast<const D2*>(&x[row + 2]);
    lo.x = lo.x + u[0] + v[0];
    lo.y = lo.y + u[1] + v[1];
    hi.x = hi.x + u[2] + v[2];
    hi.y = hi.y + u[3] + v[3];
    *reinterpret_cast<D2*>(&x[row]) = lo;
    *reinterpret_cast<D2*>(&x[row + 2]) = hi;
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < nv) x[row + k] = x[row + k] + u[k] + v[k];
}

// produce2 for a kernel written row by row: the operator's product for both
// rows of a lane comes from spmv2 (the two-row loads), and Body(row, valid,
// y, d) -- the same one-row body produce() would run with y = A x at the row --
// is called for each row; the pair's leaves are summed as produce2 requires
// (a row past n leaves its d at 0, a zero leaf).  The body's vector accesses
// stay one row at a time (8 bytes per lane, every other element), so this
// pays for kernels that touch few vectors besides the product: measured at
// 128^3, CG's s = A p and w = A u gained 14-16 %, while p-CG's one kernel
// (ten vectors read or written) lost a third that way and has a two-row form
// of its own with pair accesses (d_pcg2).
template <int ND, class Op, class X, class Body>
__device__ __forceinline__ void produce2_rows(const Args& a, const Op& op, const X* x, Body body) {
  produce2<ND>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[ND]) {
    double y0, y1;
    op.spmv2(row, valid0, valid1, x, y0, y1);
    double d0[ND], d1[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) d0[k] = d1[k] = 0.0;
    body(row, valid0, y0, d0);
    body(row + 1, valid1, y1, d1);
#pragma unroll
    for (int k = 0; k < ND; ++k) d[k] = d0[k] + d1[k];
  });
}

// The workgroup's rows without a reduction, two neighbouring rows per lane
// (as produce2); Body(row, valid0, valid1) with row even; needs R >= 2.
template <class Body>
__device__ __forceinline__ void each_row2(const Args& a, Body body) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = ((int64_t)wg_index(a) * 4 + wave) * a.R * 64;
  for (int j = 0; j < (a.R >> 1); ++j) {
    const int64_t b0 = wbase + (int64_t)j * 128;
    if (b0 < a.n) {
      const int32_t row = (int32_t)(b0 + 2 * lane);
      body(row, row < a.n, row + 1 < a.n);
    }
  }
}

// The workgroup's rows without a reduction; Body(row, valid) as above.
template <class Body>
__device__ __forceinline__ void each_row(const Args& a, Body body) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wbase = ((int64_t)wg_index(a) * 4 + wave) * a.R * 64;
  for (int j = 0; j < a.R; ++j) {
    const int64_t b0 = wbase + (int64_t)j * 64;
    if (b0 < a.n) {
      const int32_t row = (int32_t)(b0 + lane);
      body(row, row < a.n);
    }
  }
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool leader() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Register copy of the state (field by field: no aligned aggregate on the stack).
struct State {
  double alpha, beta, omega, gamma, rho0, relres, tol, result;
  int32_t status, iters, n_rr;
};

__device__ __forceinline__ State load_state(const DevState* p) {
  State s;
  s.alpha = p->alpha; s.beta = p->beta; s.omega = p->omega; s.gamma = p->gamma;
  s.rho0 = p->rho0; s.relres = p->relres; s.tol = p->tol; s.result = p->result;
  s.status = p->status; s.iters = p->iters; s.n_rr = p->n_rr;
  return s;
}

__device__ __forceinline__ void publish(const Args& a, const State& s) {
  if (sys_leader(a)) {
    DevState* p = a.sout;
    p->alpha = s.alpha; p->beta = s.beta; p->omega = s.omega; p->gamma = s.gamma;
    p->rho0 = s.rho0; p->relres = s.relres; p->tol = s.tol; p->result = s.result;
    p->status = s.status; p->iters = s.iters; p->n_rr = s.n_rr;
  }
}

// ---------------------------------------------------------------------------
// Scalar steps of the method.  Every thread evaluates them on identical
// inputs; only the leader writes the history.
// ---------------------------------------------------------------------------

// gamma = (r0, r0), rho0 = ||r0|| (the setup of Algorithms 7-11).
__device__ __forceinline__ void fin_setup_gamma(State& s, double* hist, double g) {
  s.gamma = g;
  const double rho0 = sqrt(g);
  s.rho0 = rho0;
  s.relres = 1.0;
  if (hist && leader()) hist[0] = 1.0;
  if (!finite(rho0)) s.status = DS_NONFINITE;
  else if (rho0 == 0.0) { s.status = DS_SUCCESS; s.relres = 0.0; }
}

// alpha_0 = (r0, r0) / (r0, w0), beta_{-1} = omega_{-1} = 0 (the setup of Algorithms 9 and 11).
__device__ __forceinline__ void fin_setup_alpha(State& s, double delta) {
  if (!finite(delta)) { s.status = DS_NONFINITE; return; }
  if (delta == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double alpha = s.gamma / delta;
  if (!finite(alpha)) { s.status = DS_NONFINITE; return; }
  s.alpha = alpha;
  s.beta = 0.0;
  s.omega = 0.0;
}

// omega_i = (q, y) / (y, y)  (reduction 1 of Algorithms 7, 9, 10 and 11).
// Returns true when (y, y) = 0: then q = 0
// and x_i + alpha_i p^_i is the solution; the caller applies that update.
__device__ __forceinline__ bool fin_omega(State& s, double* hist, double qy, double yy) {
  if (!finite(qy) || !finite(yy)) { s.status = DS_NONFINITE; return false; }
  if (yy == 0.0) {
    s.iters += 1;
    s.relres = 0.0;
    if (hist && leader()) hist[s.iters] = 0.0;
    s.status = DS_SUCCESS;
    return true;
  }
  const double omega = qy / yy;
  if (!finite(omega)) { s.status = DS_NONFINITE; return false; }
  s.omega = omega;
  return false;
}

// alpha_{i+1} of the pipelined solvers from gamma' = (r0, r_{i+1}), eta = (r0, w_{i+1}),
// sigma_s = (r0, s_i), sigma_z = (r0, z_i): eq. (3) is gamma' / (eta + beta sigma_s
// - beta omega sigma_z); eq. (5) is the same quantity rearranged so that sigma_s
// drops out, (1/omega + eta/gamma' - (beta omega) (sigma_z/gamma'))^{-1}.  Both
// evaluate in the order and grouping the equations write, without contraction.
__device__ __forceinline__ void next_alpha(State& s, int32_t aform, double g1, double eta, double sig_s,
                                           double sig_z, double beta, double omega) {
  double an;
  if (aform == 5) {
    if (g1 == 0.0) { s.status = DS_BREAKDOWN; return; }
    const double den = (1.0 / omega + eta / g1) - (beta * omega) * (sig_z / g1);
    if (den == 0.0) { s.status = DS_BREAKDOWN; return; }
    an = 1.0 / den;
  } else {
    const double den = eta + beta * sig_s - beta * omega * sig_z;
    if (den == 0.0 || g1 == 0.0) { s.status = DS_BREAKDOWN; return; }
    an = g1 / den;
  }
  if (!finite(an)) { s.status = DS_NONFINITE; return; }
  s.alpha = an;
  s.gamma = g1;
}

// Reduction 2 of p-BiCGStab: stopping test, beta_i and alpha_{i+1} by eq. (3)
// or eq. (5) (Algorithm 9, Algorithm 11).
__device__ __forceinline__ void fin_pipe_b(State& s, double* hist, const double (&d)[5], int32_t aform) {
  const double g1 = d[0], eta = d[1], sig_s = d[2], sig_z = d[3], nu = d[4];
  s.iters += 1;
  if (!finite(g1) || !finite(eta) || !finite(sig_s) || !finite(sig_z) || !finite(nu)) {
    s.status = DS_NONFINITE;
    return;
  }
  const double relres = sqrt(nu) / s.rho0;
  s.relres = relres;
  if (hist && leader()) hist[s.iters] = relres;
  if (relres <= s.tol) { s.status = DS_SUCCESS; return; }
  const double alpha = s.alpha, omega = s.omega, gamma = s.gamma;
  if (omega == 0.0 || gamma == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double beta = (alpha / omega) * (g1 / gamma);
  if (!finite(beta)) { s.status = DS_NONFINITE; return; }
  s.beta = beta;
  next_alpha(s, aform, g1, eta, sig_s, sig_z, beta, omega);
}

// alpha_i = (r0, r_i) / (r0, s_i)  (the first reduction of Algorithm 7).
__device__ __forceinline__ void fin_bicg_alpha(State& s, double delta) {
  if (!finite(delta)) { s.status = DS_NONFINITE; return; }
  if (delta == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double alpha = s.gamma / delta;
  if (!finite(alpha)) { s.status = DS_NONFINITE; return; }
  s.alpha = alpha;
}

// Stopping test and beta_i = (alpha/omega) (r0, r_{i+1}) / (r0, r_i)  (the last reduction of Algorithm 7).
__device__ __forceinline__ void fin_bicg_beta(State& s, double* hist, double g1, double nu) {
  s.iters += 1;
  if (!finite(g1) || !finite(nu)) { s.status = DS_NONFINITE; return; }
  const double relres = sqrt(nu) / s.rho0;
  s.relres = relres;
  if (hist && leader()) hist[s.iters] = relres;
  if (relres <= s.tol) { s.status = DS_SUCCESS; return; }
  const double alpha = s.alpha, omega = s.omega, gamma = s.gamma;
  if (omega == 0.0 || gamma == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double beta = (alpha / omega) * (g1 / gamma);
  if (!finite(beta)) { s.status = DS_NONFINITE; return; }
  s.beta = beta;
  s.gamma = g1;
}

// Reads the incoming state; a stopped solve is passed through unchanged.
#define PBCGS_PROLOGUE(st)                      \
  State st = load_state(a.sin);                 \
  if (st.status != DS_RUNNING) {                \
    publish(a, st);                             \
    return;                                     \
  }

// ===========================================================================
// p-BiCGStab kernels (Algorithm 9, PC == PC_NONE; Algorithm 11 otherwise).
// ===========================================================================

// Setup 1: r0 = b - A x0 ; r = r0 ; r^ = M^{-1} r0 ; p^ = s = s^ = z = z^ = v = 0 ;
// partials of (r0, r0).  PIPE = false: BiCGStab setup, p = r0 ; p^ = M^{-1} p.
template <class Op, int PC, bool PIPE>
__device__ __forceinline__ void d_setup_r0(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r0 = a.b[row] - ax;
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
}
template <class Op, int PC, bool PIPE>
__global__ __launch_bounds__(kWG) void k_setup_r0(Op op, Args a) { d_setup_r0<Op, PC, PIPE>(op, a); }

// Setup 2: gamma, rho0 from setup 1 ; w0 = A r^0 ; w^0 = M^{-1} w0 ;
// partials of (r0, w0).
template <class Op, int PC>
__device__ __forceinline__ void d_setup_w0(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  double g[1];
  gather_sums<1>(a, g);
  fin_setup_gamma(st, a.hist, g[0]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) {
    const double w = op.spmv(row, valid, a.rh);
    if (!valid) return;
    a.w[row] = w;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, w);
    d[0] = a.r0[row] * w;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_setup_w0(Op op, Args a) { d_setup_w0<Op, PC>(op, a); }

// Phase A of iteration i.  First it finishes the previous reduction: in the
// first iteration alpha_0 (setup 2), later reduction 2 of iteration i-1 (stop
// test, beta_{i-1}, alpha_i).  RR2 = false: t = A w^, the recurrences of p^,
// s, s^, z, q, y, and z^.  RR2 = true (the iteration after a residual replacement):
// p^, s, s^ were already recomputed and reduction 2 already finished, so
// t = A w^ and z = A s^ (both gathers), then q, q^, y and z^.
// Partials: (q, y), (y, y).
template <class Op, int PC, bool RR2>
__device__ __forceinline__ void d_pa(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  if (!RR2) {
    if (a.first) {
      double g[1];
      gather_sums<1>(a, g);
      fin_setup_alpha(st, g[0]);
    } else {
      double g[5];
      gather_sums<5>(a, g);
      fin_pipe_b(st, a.hist, g, a.aform);
    }
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha, beta = st.beta, omega = st.omega;
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    const double t = op.spmv(row, valid, a.wh);  // t = A w^, the last step of the previous iteration
    const double z_rr = RR2 ? op.spmv(row, valid, a.sh) : 0.0;
    if (!valid) return;
    const double r = a.r[row], w = a.w[row];
    double s, z;
    if (RR2) {
      s = a.s[row];
      z = z_rr;
    } else {
      const double v = a.v[row];
      const double s_old = a.s[row], z_old = a.z[row];
      if (PC != PC_NONE) {
        const double rh = a.rh[row], wh = a.wh[row];
        const double sh_old = a.sh[row], zh_old = a.zh[row];
        a.ph[row] = rh + beta * (a.ph[row] - omega * sh_old);          // p^
        a.sh[row] = wh + beta * (sh_old - omega * zh_old);             // s^
      } else {
        a.ph[row] = r + beta * (a.ph[row] - omega * s_old);            // p (Algorithm 9)
      }
      s = w + beta * (s_old - omega * z_old);                          // s
      z = t + beta * (z_old - omega * v);                              // z
      a.s[row] = s;
    }
    const double q = r - alpha * s;                                    // q
    const double y = w - alpha * z;                                    // y
    a.t[row] = t;
    a.z[row] = z;
    if (PC != PC_NONE) a.zh[row] = apply_pc<PC>(a, row, z);            // z^ = M^{-1} z
    d[0] = q * y;
    d[1] = y * y;
  });
}
template <class Op, int PC, bool RR2>
__global__ __launch_bounds__(kWG) void k_pa(Op op, Args a) { d_pa<Op, PC, RR2>(op, a); }

// Phase B of iteration i: omega_i from phase A's partials ; v = A z^ ;
// q, q^, y recomputed ; the x, r, r^, w updates ; w^ ; partials of (r0,r),
// (r0,w), (r0,s), (r0,z), (r,r) (reduction 2).
template <class Op, int PC>
__device__ __forceinline__ void d_pb(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * a.ph[row];
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  produce<5>(a, [&](int32_t row, bool valid, double (&d)[5]) {
    const double v = op.spmv(row, valid, a.zh);                        // v = A z^
    if (!valid) return;
    const double r = a.r[row], s = a.s[row], w = a.w[row], z = a.z[row];
    const double q = r - alpha * s;
    const double y = w - alpha * z;
    const double t = a.t[row];
    double rn;
    if (PC != PC_NONE) {
      const double rh = a.rh[row], sh = a.sh[row], wh = a.wh[row], zh = a.zh[row];
      const double qh = rh - alpha * sh;                               // q^
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * qh;            // x
      rn = q - omega * y;                                              // r
      a.rh[row] = qh - omega * (wh - alpha * zh);                      // r^
    } else {
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * q;
      rn = q - omega * y;
    }
    const double wn = y - omega * (t - alpha * v);                     // w
    a.v[row] = v;
    a.r[row] = rn;
    a.w[row] = wn;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, wn);           // w^ = M^{-1} w
    const double r0 = a.r0[row];
    d[0] = r0 * rn;
    d[1] = r0 * wn;
    d[2] = r0 * s;
    d[3] = r0 * z;
    d[4] = rn * rn;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_pb(Op op, Args a) { d_pb<Op, PC>(op, a); }

// Residual-replacement iteration, phase B': omega_i, then only the x update
// of x (r, r^, w are replaced next, so their recurrences and v are not needed).
template <int PC>
__device__ __forceinline__ void d_rr_x(Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (!yz && st.status != DS_RUNNING) return;
  const double omega = st.omega;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    if (yz) {
      a.x[row] = a.x[row] + alpha * a.ph[row];
    } else {
      const double qh = (PC != PC_NONE) ? a.rh[row] - alpha * a.sh[row] : a.r[row] - alpha * a.s[row];
      a.x[row] = a.x[row] + alpha * a.ph[row] + omega * qh;
    }
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_rr_x(Args a) { d_rr_x<PC>(a); }

// Residual replacement, first half (Section 4.2): r = b - A x ; r^ = M^{-1} r.
template <class Op, int PC>
__device__ __forceinline__ void d_rr_r(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  each_row(a, [&](int32_t row, bool valid) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r = a.b[row] - ax;
    a.r[row] = r;
    if (PC != PC_NONE) a.rh[row] = apply_pc<PC>(a, row, r);
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_r(Op op, Args a) { d_rr_r<Op, PC>(op, a); }

// Residual replacement, first half continued: w = A r^ ; w^ = M^{-1} w ;
// partials of reduction 2 on the true r, w.
template <class Op, int PC>
__device__ __forceinline__ void d_rr_w(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  st.n_rr += 1;
  publish(a, st);
  produce<5>(a, [&](int32_t row, bool valid, double (&d)[5]) {
    const double w = op.spmv(row, valid, a.rh);
    if (!valid) return;
    a.w[row] = w;
    if (PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, w);
    const double r0 = a.r0[row], r = a.r[row];
    d[0] = r0 * r;
    d[1] = r0 * w;
    d[2] = r0 * a.s[row];
    d[3] = r0 * a.z[row];
    d[4] = r * r;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_w(Op op, Args a) { d_rr_w<Op, PC>(op, a); }

// Second half, in the iteration after a replacement: reduction 2 (stop test,
// beta, alpha), then the p^ update alone.
template <int PC>
__device__ __forceinline__ void d_rr_p(Args a) {
  PBCGS_PROLOGUE(st)
  double g[5];
  gather_sums<5>(a, g);
  fin_pipe_b(st, a.hist, g, a.aform);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double beta = st.beta, omega = st.omega;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    if (PC != PC_NONE) a.ph[row] = a.rh[row] + beta * (a.ph[row] - omega * a.sh[row]);
    else a.ph[row] = a.r[row] + beta * (a.ph[row] - omega * a.s[row]);
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_rr_p(Args a) { d_rr_p<PC>(a); }

// Second half continued: s = A p^ ; s^ = M^{-1} s.
template <class Op, int PC>
__device__ __forceinline__ void d_rr_s(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  each_row(a, [&](int32_t row, bool valid) {
    const double s = op.spmv(row, valid, a.ph);
    if (!valid) return;
    a.s[row] = s;
    if (PC != PC_NONE) a.sh[row] = apply_pc<PC>(a, row, s);
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_rr_s(Op op, Args a) { d_rr_s<Op, PC>(op, a); }

// ===========================================================================
// CA-BiCGStab kernels (Algorithm 8, no preconditioner; Jacobi reaches it
// folded into the operator).  s and y follow their recurrences (eqs. (1) and
// (4)); the two reductions are those of p-BiCGStab, so the scalar steps are
// shared.  Each SpMV reads a vector that the preceding kernel finished, which
// gives four kernel boundaries per iteration.  p is stored in the p^ slot.
// The setup is that of p-BiCGStab (r0, r, w = A r0, alpha_0); its t is not
// used.
// ===========================================================================

// First finishes the previous reduction (alpha_0 in the first iteration, else
// the stop test, beta_{i-1} and alpha_i), then
// p_i = r_i + beta (p_{i-1} - omega s_{i-1}) ; s_i = w_i + beta (s_{i-1} - omega z_{i-1}).
__device__ __forceinline__ void d_ca_ps(Args a) {
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1>(a, g);
    fin_setup_alpha(st, g[0]);
  } else {
    double g[5];
    gather_sums<5>(a, g);
    fin_pipe_b(st, a.hist, g, a.aform);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double beta = st.beta, omega = st.omega;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    const double s_old = a.s[row];
    a.ph[row] = a.r[row] + beta * (a.ph[row] - omega * s_old);
    a.s[row] = a.w[row] + beta * (s_old - omega * a.z[row]);
  });
}
__global__ __launch_bounds__(kWG) void k_ca_ps(Args a) { d_ca_ps(a); }

// z_i = A s_i ; q_i = r_i - alpha_i s_i ; y_i = w_i - alpha_i z_i ;
// partials of (q, y), (y, y).  q and y are recomputed by the next kernel.
template <class Op>
__device__ __forceinline__ void d_ca_z(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  const double alpha = st.alpha;
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    const double z = op.spmv(row, valid, a.s);
    if (!valid) return;
    const double q = a.r[row] - alpha * a.s[row];
    const double y = a.w[row] - alpha * z;
    a.z[row] = z;
    d[0] = q * y;
    d[1] = y * y;
  });
}
template <class Op>
__global__ __launch_bounds__(kWG) void k_ca_z(Op op, Args a) { d_ca_z<Op>(op, a); }

// omega_i ; x_{i+1} = x_i + alpha_i p_i + omega_i q_i ; r_{i+1} = q_i - omega_i y_i.
__device__ __forceinline__ void d_ca_x(Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (!yz && st.status != DS_RUNNING) return;
  const double omega = st.omega;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    if (yz) {
      a.x[row] = a.x[row] + alpha * a.ph[row];
      return;
    }
    const double q = a.r[row] - alpha * a.s[row];
    const double y = a.w[row] - alpha * a.z[row];
    a.x[row] = a.x[row] + alpha * a.ph[row] + omega * q;
    a.r[row] = q - omega * y;
  });
}
__global__ __launch_bounds__(kWG) void k_ca_x(Args a) { d_ca_x(a); }

// w_{i+1} = A r_{i+1} ; partials of (r0, r), (r0, w), (r0, s), (r0, z), (r, r).
template <class Op>
__device__ __forceinline__ void d_ca_w(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce<5>(a, [&](int32_t row, bool valid, double (&d)[5]) {
    const double w = op.spmv(row, valid, a.r);
    if (!valid) return;
    a.w[row] = w;
    const double r0 = a.r0[row], r = a.r[row];
    d[0] = r0 * r;
    d[1] = r0 * w;
    d[2] = r0 * a.s[row];
    d[3] = r0 * a.z[row];
    d[4] = r * r;
  });
}
template <class Op>
__global__ __launch_bounds__(kWG) void k_ca_w(Op op, Args a) { d_ca_w<Op>(op, a); }

// ===========================================================================
// CG family (Section 2), for symmetric positive definite A with Jacobi
// M = diag(A) or none.  u = M^{-1} r lives in the r^ slot (aliasing r without a
// preconditioner).  Reductions of the two one-phase forms carry, in order,
// gamma = (r, u), delta = (w, u), nu = (r, r).
//   Algorithm 2 (CG): s = A p | alpha ; x, r, u | stop, beta ; p  -- three kernels.
//   Algorithm 4 (Chronopoulos & Gear): alpha, beta ; p, s, x, r, u | w = A u  -- two.
//   Algorithm 6 (p-CG): alpha, beta ; n = A M^{-1} w and every recurrence -- one.
// ===========================================================================

// First reduction of Algorithms 4 and 6: rho0 = sqrt(nu_0), alpha_0 = gamma_0 / delta_0, beta_0 = 0.
__device__ __forceinline__ void fin_cgs_first(State& s, double* hist, const double (&d)[3]) {
  const double gamma = d[0], delta = d[1], nu = d[2];
  s.relres = 1.0;
  if (hist && leader()) hist[0] = 1.0;
  if (!finite(gamma) || !finite(delta) || !finite(nu)) { s.status = DS_NONFINITE; return; }
  const double rho0 = sqrt(nu);
  s.rho0 = rho0;
  if (rho0 == 0.0) { s.status = DS_SUCCESS; s.relres = 0.0; return; }
  if (delta == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double alpha = gamma / delta;
  if (!finite(alpha)) { s.status = DS_NONFINITE; return; }
  s.alpha = alpha;
  s.beta = 0.0;
  s.gamma = gamma;
}

// Later reductions of Algorithms 4 and 6: stopping test on ||r_i|| (i = s.iters),
// beta_i = gamma_i / gamma_{i-1}, alpha_i = (delta / gamma_i - beta_i / alpha_{i-1})^{-1}.
__device__ __forceinline__ void fin_cgs_next(State& s, double* hist, const double (&d)[3]) {
  const double g1 = d[0], delta = d[1], nu = d[2];
  if (!finite(g1) || !finite(delta) || !finite(nu)) { s.status = DS_NONFINITE; return; }
  const double relres = sqrt(nu) / s.rho0;
  s.relres = relres;
  if (hist && leader()) hist[s.iters] = relres;
  if (relres <= s.tol) { s.status = DS_SUCCESS; return; }
  if (s.gamma == 0.0 || g1 == 0.0 || s.alpha == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double beta = g1 / s.gamma;
  if (!finite(beta)) { s.status = DS_NONFINITE; return; }
  const double den = delta / g1 - beta / s.alpha;
  if (den == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double alpha = 1.0 / den;
  if (!finite(alpha)) { s.status = DS_NONFINITE; return; }
  s.beta = beta;
  s.alpha = alpha;
  s.gamma = g1;
}

// Setup of Algorithm 2: r = b - A x ; u = M^{-1} r ; p = u ; partials (r, r), (r, u).
// ONEPHASE (Algorithms 4 and 6): no p; p = s = z = q = 0 instead.
template <class Op, int PC, bool ONEPHASE>
__device__ __forceinline__ void d_cg_setup(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r = a.b[row] - ax;
    a.r[row] = r;
    const double u = (PC != PC_NONE) ? apply_pc<PC>(a, row, r) : r;
    if (PC != PC_NONE) a.rh[row] = u;
    if (ONEPHASE) {
      a.p[row] = 0.0;
      a.s[row] = 0.0;
      a.z[row] = 0.0;
      if (PC != PC_NONE) a.sh[row] = 0.0;
    } else {
      a.p[row] = u;
    }
    d[0] = r * r;
    d[1] = r * u;
  });
}
template <class Op, int PC, bool ONEPHASE>
__global__ __launch_bounds__(kWG) void k_cg_setup(Op op, Args a) { d_cg_setup<Op, PC, ONEPHASE>(op, a); }

// Setup of Algorithms 4 and 6, continued: w = A u ; with PIPE (Algorithm 6)
// and a preconditioner also m = M^{-1} w into w^ ; partials (r, u), (w, u),
// (r, r).
// TWO: two rows per lane for the product (produce2_rows), the same bits.
template <class Op, int PC, bool PIPE, bool TWO>
__device__ __forceinline__ void d_cg_setup_w(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  auto body = [&](int32_t row, bool valid, double w, double (&d)[3]) {
    if (!valid) return;
    a.w[row] = w;
    if (PIPE && PC != PC_NONE) a.wh[row] = apply_pc<PC>(a, row, w);
    const double r = a.r[row], u = a.rh[row];
    d[0] = r * u;
    d[1] = w * u;
    d[2] = r * r;
  };
  if constexpr (TWO) {
    produce2_rows<3>(a, op, a.rh, body);
  } else {
    produce<3>(a, [&](int32_t row, bool valid, double (&d)[3]) { body(row, valid, op.spmv(row, valid, a.rh), d); });
  }
}
template <class Op, int PC, bool PIPE, bool TWO = false>
__global__ __launch_bounds__(kWG) void k_cg_setup_w(Op op, Args a) { d_cg_setup_w<Op, PC, PIPE, TWO>(op, a); }

// Algorithm 2, kernel 1: (first iteration: rho0, gamma_0 from the setup) ;
// s = A p ; partials of (s, p).
template <class Op, bool TWO>
__device__ __forceinline__ void d_cg_a(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[2];
    gather_sums<2>(a, g);
    st.relres = 1.0;
    if (a.hist && leader()) a.hist[0] = 1.0;
    const double rho0 = sqrt(g[0]);
    st.rho0 = rho0;
    st.gamma = g[1];
    if (!finite(rho0) || !finite(g[1])) st.status = DS_NONFINITE;
    else if (rho0 == 0.0) { st.status = DS_SUCCESS; st.relres = 0.0; }
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  auto body = [&](int32_t row, bool valid, double s, double (&d)[1]) {
    if (!valid) return;
    a.s[row] = s;
    d[0] = s * a.p[row];
  };
  if constexpr (TWO) {
    produce2_rows<1>(a, op, a.p, body);
  } else {
    produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) { body(row, valid, op.spmv(row, valid, a.p), d); });
  }
}
template <class Op, bool TWO = false>
__global__ __launch_bounds__(kWG) void k_cg_a(Op op, Args a) { d_cg_a<Op, TWO>(op, a); }

// Algorithm 2, kernel 2: alpha = gamma / (s, p) ; x += alpha p ; r -= alpha s ;
// u = M^{-1} r ; partials (r, u), (r, r).
template <int PC>
__device__ __forceinline__ void d_cg_b(Args a) {
  PBCGS_PROLOGUE(st)
  double g[1];
  gather_sums<1>(a, g);
  const double delta = g[0];
  if (!finite(delta)) st.status = DS_NONFINITE;
  else if (delta == 0.0) st.status = DS_BREAKDOWN;
  else {
    const double alpha = st.gamma / delta;
    if (!finite(alpha)) st.status = DS_NONFINITE;
    else st.alpha = alpha;
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha;
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    if (!valid) return;
    const double p = a.p[row];
    a.x[row] = a.x[row] + alpha * p;
    const double r = a.r[row] - alpha * a.s[row];
    a.r[row] = r;
    const double u = (PC != PC_NONE) ? apply_pc<PC>(a, row, r) : r;
    if (PC != PC_NONE) a.rh[row] = u;
    d[0] = r * u;
    d[1] = r * r;
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_cg_b(Args a) { d_cg_b<PC>(a); }

// Algorithm 2, kernel 3: stopping test, beta = (r', u') / (r, u) ; p = u + beta p.
__device__ __forceinline__ void fin_cg_beta(State& s, double* hist, const double (&d)[2]) {
  const double g1 = d[0], nu = d[1];
  s.iters += 1;
  if (!finite(g1) || !finite(nu)) { s.status = DS_NONFINITE; return; }
  const double relres = sqrt(nu) / s.rho0;
  s.relres = relres;
  if (hist && leader()) hist[s.iters] = relres;
  if (relres <= s.tol) { s.status = DS_SUCCESS; return; }
  if (s.gamma == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double beta = g1 / s.gamma;
  if (!finite(beta)) { s.status = DS_NONFINITE; return; }
  s.beta = beta;
  s.gamma = g1;
}

template <int PC>
__device__ __forceinline__ void d_cg_c(Args a) {
  PBCGS_PROLOGUE(st)
  double g[2];
  gather_sums<2>(a, g);
  fin_cg_beta(st, a.hist, g);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double beta = st.beta;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    a.p[row] = a.rh[row] + beta * a.p[row];
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_cg_c(Args a) { d_cg_c<PC>(a); }

// Algorithm 4, kernel 1: finish the reduction (alpha_0 in the first
// iteration, else stop test, beta, alpha) ; p = u + beta p ; s = w + beta s ;
// x += alpha p ; r -= alpha s ; u = M^{-1} r.
template <int PC>
__device__ __forceinline__ void d_cc_a(Args a) {
  PBCGS_PROLOGUE(st)
  double g[3];
  gather_sums<3>(a, g);
  if (a.first) fin_cgs_first(st, a.hist, g);
  else fin_cgs_next(st, a.hist, g);
  if (st.status == DS_RUNNING) st.iters += 1;  // the x update below
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha, beta = st.beta;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    const double p = a.rh[row] + beta * a.p[row];
    const double s = a.w[row] + beta * a.s[row];
    a.p[row] = p;
    a.s[row] = s;
    a.x[row] = a.x[row] + alpha * p;
    const double r = a.r[row] - alpha * s;
    a.r[row] = r;
    if (PC != PC_NONE) a.rh[row] = apply_pc<PC>(a, row, r);
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_cc_a(Args a) { d_cc_a<PC>(a); }

// Algorithm 6, the whole iteration: finish the reduction (alpha_0, or stop
// test, beta_i, alpha_i) ; n = A m with m = M^{-1} w (gathered from w^, which
// the previous launch finished) ; z, q, s, p, x, r, u, w by their recurrences ;
// m' = M^{-1} w' into the other buffer t (without a preconditioner m = w, so
// w itself alternates between w^ and t) ; partials (r, u), (w, u), (r, r).
template <class Op, int PC>
__device__ __forceinline__ void d_pcg(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  double g[3];
  gather_sums<3>(a, g);
  if (a.first) fin_cgs_first(st, a.hist, g);
  else fin_cgs_next(st, a.hist, g);
  if (st.status == DS_RUNNING) st.iters += 1;  // the x update below
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha, beta = st.beta;
  produce<3>(a, [&](int32_t row, bool valid, double (&d)[3]) {
    const double nv = op.spmv(row, valid, a.wh);
    if (!valid) return;
    const double m = a.wh[row];
    const double w = (PC != PC_NONE) ? a.w[row] : m;
    const double z = nv + beta * a.z[row];
    const double sv = w + beta * a.s[row];
    a.z[row] = z;
    a.s[row] = sv;
    double p, r, u, wn;
    if (PC != PC_NONE) {
      const double q = m + beta * a.sh[row];
      a.sh[row] = q;
      p = a.rh[row] + beta * a.p[row];
      a.x[row] = a.x[row] + alpha * p;
      r = a.r[row] - alpha * sv;
      u = a.rh[row] - alpha * q;
      wn = w - alpha * z;
      a.rh[row] = u;
      a.w[row] = wn;
      a.t[row] = apply_pc<PC>(a, row, wn);
    } else {
      p = a.r[row] + beta * a.p[row];
      a.x[row] = a.x[row] + alpha * p;
      r = a.r[row] - alpha * sv;
      u = r;
      wn = w - alpha * z;
      a.t[row] = wn;
    }
    a.p[row] = p;
    a.r[row] = r;
    d[0] = r * u;
    d[1] = wn * u;
    d[2] = r * r;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_pcg(Op op, Args a) { d_pcg<Op, PC>(op, a); }

// d_pcg with two neighbouring rows per lane (see produce2): every workspace
// vector is read and written as a 16-byte pair, the caller's x as a pair when
// it is 16-byte aligned (else row by row), and the operator provides spmv2.
// The arithmetic of each row and the reduction trees are d_pcg's, so the
// results are the same bits.
template <class Op, int PC>
__device__ __forceinline__ void d_pcg2(Op op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  double g[3];
  gather_sums<3>(a, g);
  if (a.first) fin_cgs_first(st, a.hist, g);
  else fin_cgs_next(st, a.hist, g);
  if (st.status == DS_RUNNING) st.iters += 1;  // the x update below
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha, beta = st.beta;
  produce2<3>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[3]) {
    double nv[2];
    op.spmv2(row, valid0, valid1, a.wh, nv[0], nv[1]);
    if (!valid0) return;
    auto ld = [&](const double* v, double (&o)[2]) {
      const D2 q = *reinterpret_cast<const D2*>(&v[row]);
      o[0] = q.x;
      o[1] = q.y;
    };
    auto stv = [&](double* v, const double (&o)[2]) { *reinterpret_cast<D2*>(&v[row]) = D2{o[0], o[1]}; };
    double m[2], zo[2], so[2], po[2], ro[2], w[2];
    ld(a.wh, m);
    ld(a.z, zo);
    ld(a.s, so);
    ld(a.p, po);
    ld(a.r, ro);
    if (PC != PC_NONE) ld(a.w, w);
    else w[0] = m[0], w[1] = m[1];
    double z[2], sv[2], p[2], r[2], u[2], wn[2], tt[2];
    if (PC != PC_NONE) {
      double sho[2], rho[2], q[2];
      ld(a.sh, sho);
      ld(a.rh, rho);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        z[k] = nv[k] + beta * zo[k];
        sv[k] = w[k] + beta * so[k];
        q[k] = m[k] + beta * sho[k];
        p[k] = rho[k] + beta * po[k];
        r[k] = ro[k] - alpha * sv[k];
        u[k] = rho[k] - alpha * q[k];
        wn[k] = w[k] - alpha * z[k];
      }
      tt[0] = apply_pc<PC>(a, row, wn[0]);
      tt[1] = valid1 ? apply_pc<PC>(a, row + 1, wn[1]) : 0.0;  // dinv holds n entries
      stv(a.sh, q);
      stv(a.rh, u);
      stv(a.w, wn);
    } else {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        z[k] = nv[k] + beta * zo[k];
        sv[k] = w[k] + beta * so[k];
        p[k] = ro[k] + beta * po[k];
        r[k] = ro[k] - alpha * sv[k];
        u[k] = r[k];
        wn[k] = w[k] - alpha * z[k];
        tt[k] = wn[k];
      }
    }
    stv(a.z, z);
    stv(a.s, sv);
    stv(a.t, tt);
    stv(a.p, p);
    stv(a.r, r);
    if (valid1 && (reinterpret_cast<uintptr_t>(a.x) & 15) == 0) {
      D2 xx = *reinterpret_cast<const D2*>(&a.x[row]);
      xx.x = xx.x + alpha * p[0];
      xx.y = xx.y + alpha * p[1];
      *reinterpret_cast<D2*>(&a.x[row]) = xx;
    } else {
      a.x[row] = a.x[row] + alpha * p[0];
      if (valid1) a.x[row + 1] = a.x[row + 1] + alpha * p[1];
    }
    d[0] = r[0] * u[0] + (valid1 ? r[1] * u[1] : 0.0);
    d[1] = wn[0] * u[0] + (valid1 ? wn[1] * u[1] : 0.0);
    d[2] = r[0] * r[0] + (valid1 ? r[1] * r[1] : 0.0);
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_pcg2(Op op, Args a) { d_pcg2<Op, PC>(op, a); }

// Final reduction of the CG family.  MODE 0: Algorithm 2's setup (rho0,
// gamma_0); 1: first reduction of Algorithms 4 and 6; 2: a later one.
template <int MODE>
__device__ __forceinline__ void d_cg_finish(Args a) {
  State st = load_state(a.sin);
  if (st.status != DS_RUNNING) {
    publish(a, st);
    return;
  }
  if (MODE == 0) {
    double g[2];
    gather_sums<2>(a, g);
    st.relres = 1.0;
    if (a.hist && leader()) a.hist[0] = 1.0;
    const double rho0 = sqrt(g[0]);
    st.rho0 = rho0;
    st.gamma = g[1];
    if (!finite(rho0) || !finite(g[1])) st.status = DS_NONFINITE;
    else if (rho0 == 0.0) { st.status = DS_SUCCESS; st.relres = 0.0; }
  } else {
    double g[3];
    gather_sums<3>(a, g);
    if (MODE == 1) fin_cgs_first(st, a.hist, g);
    else fin_cgs_next(st, a.hist, g);
  }
  publish(a, st);
}
template <int MODE>
__global__ __launch_bounds__(kWG) void k_cg_finish(Args a) { d_cg_finish<MODE>(a); }

// ===========================================================================
// BiCGStab kernels (Algorithm 7, PC == PC_NONE; Algorithm 10 otherwise).
// ===========================================================================

// (first iteration: gamma, rho0 from the setup) ; s = A p^ ; partials of (r0, s).
template <class Op, int PC>
__device__ __forceinline__ void d_b1(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1>(a, g);
    fin_setup_gamma(st, a.hist, g[0]);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) {
    const double s = op.spmv(row, valid, a.ph);
    if (!valid) return;
    a.s[row] = s;
    d[0] = a.r0[row] * s;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_b1(Op op, Args a) { d_b1<Op, PC>(op, a); }

// alpha_i ; q = r - alpha s ; q^ = M^{-1} q.
template <int PC>
__device__ __forceinline__ void d_b2(Args a) {
  PBCGS_PROLOGUE(st)
  double g[1];
  gather_sums<1>(a, g);
  fin_bicg_alpha(st, g[0]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    const double q = a.r[row] - alpha * a.s[row];
    a.q[row] = q;
    if (PC != PC_NONE) a.qh[row] = apply_pc<PC>(a, row, q);
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_b2(Args a) { d_b2<PC>(a); }

// y = A q^ ; partials of (q, y), (y, y).
template <class Op, int PC>
__device__ __forceinline__ void d_b3(Op op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    const double y = op.spmv(row, valid, a.qh);
    if (!valid) return;
    a.y[row] = y;
    d[0] = a.q[row] * y;
    d[1] = y * y;
  });
}
template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_b3(Op op, Args a) { d_b3<Op, PC>(op, a); }

// omega_i ; x = x + alpha p^ + omega q^ ; r = q - omega y ; partials of (r0, r), (r, r).
template <int PC>
__device__ __forceinline__ void d_b4(Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * a.ph[row];
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  produce<2>(a, [&](int32_t row, bool valid, double (&d)[2]) {
    if (!valid) return;
    const double q = a.q[row];
    a.x[row] = a.x[row] + alpha * a.ph[row] + omega * a.qh[row];
    const double r = q - omega * a.y[row];
    a.r[row] = r;
    d[0] = a.r0[row] * r;
    d[1] = r * r;
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_b4(Args a) { d_b4<PC>(a); }

// stop test and beta_i ; p = r + beta (p - omega s) ; p^ = M^{-1} p.
template <int PC>
__device__ __forceinline__ void d_b5(Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  fin_bicg_beta(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double beta = st.beta, omega = st.omega;
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    const double p = a.r[row] + beta * (a.p[row] - omega * a.s[row]);
    a.p[row] = p;
    if (PC != PC_NONE) a.ph[row] = apply_pc<PC>(a, row, p);
  });
}
template <int PC>
__global__ __launch_bounds__(kWG) void k_b5(Args a) { d_b5<PC>(a); }

// Finishes a pending reduction in one workgroup: MODE 0 reduction 2 of
// p-BiCGStab, 1 the setup alpha, 2 the setup gamma, 3 a plain sum into result.
template <int MODE>
__device__ __forceinline__ void d_finish(Args a) {
  State st = load_state(a.sin);
  if (MODE == 3) {
    double g[1];
    gather_sums<1>(a, g);
    st.result = g[0];
    publish(a, st);
    return;
  }
  if (st.status != DS_RUNNING) {
    publish(a, st);
    return;
  }
  if (MODE == 0) {
    double g[5];
    gather_sums<5>(a, g);
    fin_pipe_b(st, a.hist, g, a.aform);
  } else {
    double g[1];
    gather_sums<1>(a, g);
    if (MODE == 1) fin_setup_alpha(st, g[0]);
    else fin_setup_gamma(st, a.hist, g[0]);
  }
  publish(a, st);
}
template <int MODE>
__global__ __launch_bounds__(kWG) void k_finish(Args a) { d_finish<MODE>(a); }

// ===========================================================================
// Precision form of Algorithm 9 with residual replacement: binary32 vectors,
// SpMV (on the operator rounded to binary32), recurrences and dot products
// (binary32 pairwise sums); binary64 replacement steps on the binary64
// operator, x update and scalars alpha, beta, omega.  Vector updates use the
// scalars rounded to binary32.  The setup is a replacement: r_0 = f(b - A x_0),
// w_0 = f(A (b - A x_0)) with f the rounding to binary32.  When the recursive
// residual passes tol the status becomes DS_CHECK and the host confirms with
// the binary64 true residual (Section 4.2 supplies the replacement that
// continues the iteration when it is not yet below tol).
// ===========================================================================

// Reduction 2 of the precision form.  recheck: the reduction that follows a
// forced replacement -- it neither counts an iteration nor tests convergence.
__device__ __forceinline__ void fin_pipe_b_mp(State& s, double* hist, const double (&d)[5], bool recheck,
                                              int32_t aform) {
  const double g1 = d[0], eta = d[1], sig_s = d[2], sig_z = d[3], nu = d[4];
  if (!recheck) s.iters += 1;
  if (!finite(g1) || !finite(eta) || !finite(sig_s) || !finite(sig_z) || !finite(nu)) {
    s.status = DS_NONFINITE;
    return;
  }
  const double relres = sqrt(nu) / s.rho0;
  s.relres = relres;
  if (hist && leader()) hist[s.iters] = relres;
  if (!recheck && relres <= s.tol) { s.status = DS_CHECK; return; }
  const double alpha = s.alpha, omega = s.omega, gamma = s.gamma;
  if (omega == 0.0 || gamma == 0.0) { s.status = DS_BREAKDOWN; return; }
  const double beta = (alpha / omega) * (g1 / gamma);
  if (!finite(beta)) { s.status = DS_NONFINITE; return; }
  s.beta = beta;
  next_alpha(s, aform, g1, eta, sig_s, sig_z, beta, omega);
}

// Setup 1: r64 = b - A x0 (binary64) ; r0 = r = f(r64) ; p = s = z = v = 0 ;
// partials of (r0, r0) in binary32.
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_setup_r0(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce<1, float>(a, [&](int32_t row, bool valid, float (&d)[1]) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r = a.b[row] - ax;
    a.r64[row] = r;
    const float rf = float(r);
    a.r0f[row] = rf;
    a.rf[row] = rf;
    a.pf[row] = 0.0f;
    a.sf[row] = 0.0f;
    a.zf[row] = 0.0f;
    a.vf[row] = 0.0f;
    d[0] = rf * rf;
  });
}

// Setup 2: gamma, rho0 ; w = f(A r64) ; partials of (r0, w).
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_setup_w0(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  double g[1];
  gather_sums<1, float>(a, g);
  fin_setup_gamma(st, a.hist, g[0]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  produce<1, float>(a, [&](int32_t row, bool valid, float (&d)[1]) {
    const double w = op.spmv(row, valid, a.r64);
    if (!valid) return;
    const float wf = float(w);
    a.wf[row] = wf;
    d[0] = a.r0f[row] * wf;
  });
}

// Phase A: finishes the previous reduction (setup alpha or reduction 2), then
// t = A w (binary32) and the p, s, z, q, y recurrences of Algorithm 9.  RR2: s was replaced by
// f(A p) already; z = f(A s64) in binary64 instead of the recurrence.
template <class Op32, class Op64, bool RR2>
__global__ __launch_bounds__(kWG) void k_mp_pa(Op32 op, Op64 op64, Args a) {
  PBCGS_PROLOGUE(st)
  if (!RR2) {
    if (a.first) {
      double g[1];
      gather_sums<1, float>(a, g);
      fin_setup_alpha(st, g[0]);
    } else {
      double g[5];
      gather_sums<5, float>(a, g);
      fin_pipe_b_mp(st, a.hist, g, false, a.aform);
    }
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const float af = float(st.alpha), bf = float(st.beta), wf_ = float(st.omega);
  produce<2, float>(a, [&](int32_t row, bool valid, float (&d)[2]) {
    const float t = op.spmv(row, valid, a.wf);
    const double z64 = RR2 ? op64.spmv(row, valid, a.s64) : 0.0;
    if (!valid) return;
    const float r = a.rf[row], w = a.wf[row];
    float s, z;
    if (RR2) {
      s = a.sf[row];
      z = float(z64);
    } else {
      const float v = a.vf[row];
      const float s_old = a.sf[row], z_old = a.zf[row];
      a.pf[row] = r + bf * (a.pf[row] - wf_ * s_old);
      s = w + bf * (s_old - wf_ * z_old);
      z = t + bf * (z_old - wf_ * v);
      a.sf[row] = s;
    }
    const float q = r - af * s;
    const float y = w - af * z;
    a.tf[row] = t;
    a.zf[row] = z;
    d[0] = q * y;
    d[1] = y * y;
  });
}

// Phase B: omega (binary64) ; v = A z (binary32) ; x += alpha p + omega q in
// binary64 ; r, w in binary32 ; partials (r0,r), (r0,w), (r0,s), (r0,z), (r,r).
template <class Op32>
__global__ __launch_bounds__(kWG) void k_mp_pb(Op32 op, Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2, float>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * double(a.pf[row]);
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  const float af = float(alpha), wn = float(omega);
  produce<5, float>(a, [&](int32_t row, bool valid, float (&d)[5]) {
    const float v = op.spmv(row, valid, a.zf);
    if (!valid) return;
    const float r = a.rf[row], s = a.sf[row], w = a.wf[row], z = a.zf[row];
    const float q = r - af * s;
    const float y = w - af * z;
    const float t = a.tf[row];
    a.x[row] = a.x[row] + alpha * double(a.pf[row]) + omega * double(q);
    const float rn = q - wn * y;
    const float wnew = y - wn * (t - af * v);
    a.vf[row] = v;
    a.rf[row] = rn;
    a.wf[row] = wnew;
    const float r0 = a.r0f[row];
    d[0] = r0 * rn;
    d[1] = r0 * wnew;
    d[2] = r0 * s;
    d[3] = r0 * z;
    d[4] = rn * rn;
  });
}

// k_mp_pa (without a pending replacement) and k_mp_pb with two neighbouring
// rows per lane (see produce2): each binary32 vector access is one 8-byte
// load or store of the pair, so a wave moves 512 instead of 256 bytes per
// access; the operator provides spmv2.  The arithmetic of each row and the
// reduction trees are those of k_mp_pa / k_mp_pb, so the results are the same
// bits.  The workspace vectors are padded to 64 rows, so a pair starting at
// the last row stays inside them (the element past n receives an unused
// value); x, the caller's n doubles, is accessed row by row.
template <class Op32>
__global__ __launch_bounds__(kWG) void k_mp_pa2(Op32 op, Args a) {
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1, float>(a, g);
    fin_setup_alpha(st, g[0]);
  } else {
    double g[5];
    gather_sums<5, float>(a, g);
    fin_pipe_b_mp(st, a.hist, g, false, a.aform);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const float af = float(st.alpha), bf = float(st.beta), wf_ = float(st.omega);
  produce2<2, float>(a, [&](int32_t row, bool valid0, bool valid1, float (&d)[2]) {
    float t0, t1;
    op.spmv2(row, valid0, valid1, a.wf, t0, t1);
    if (!valid0) return;
    const float2 r = *reinterpret_cast<const float2*>(&a.rf[row]);
    const float2 w = *reinterpret_cast<const float2*>(&a.wf[row]);
    const float2 v = *reinterpret_cast<const float2*>(&a.vf[row]);
    const float2 so = *reinterpret_cast<const float2*>(&a.sf[row]);
    const float2 zo = *reinterpret_cast<const float2*>(&a.zf[row]);
    const float2 po = *reinterpret_cast<const float2*>(&a.pf[row]);
    float2 p, s, z, t;
    p.x = r.x + bf * (po.x - wf_ * so.x);
    p.y = r.y + bf * (po.y - wf_ * so.y);
    s.x = w.x + bf * (so.x - wf_ * zo.x);
    s.y = w.y + bf * (so.y - wf_ * zo.y);
    z.x = t0 + bf * (zo.x - wf_ * v.x);
    z.y = t1 + bf * (zo.y - wf_ * v.y);
    t.x = t0;
    t.y = t1;
    *reinterpret_cast<float2*>(&a.pf[row]) = p;
    *reinterpret_cast<float2*>(&a.sf[row]) = s;
    *reinterpret_cast<float2*>(&a.tf[row]) = t;
    *reinterpret_cast<float2*>(&a.zf[row]) = z;
    const float q0 = r.x - af * s.x, y0 = w.x - af * z.x;
    const float q1 = r.y - af * s.y, y1 = w.y - af * z.y;
    // the pair's two leaves of the reduction tree (a row past n is a zero leaf)
    d[0] = q0 * y0 + (valid1 ? q1 * y1 : 0.0f);
    d[1] = y0 * y0 + (valid1 ? y1 * y1 : 0.0f);
  });
}

template <class Op32>
__global__ __launch_bounds__(kWG) void k_mp_pb2(Op32 op, Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2, float>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * double(a.pf[row]);
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  const float af = float(alpha), wn = float(omega);
  produce2<5, float>(a, [&](int32_t row, bool valid0, bool valid1, float (&d)[5]) {
    float v0, v1;
    op.spmv2(row, valid0, valid1, a.zf, v0, v1);
    if (!valid0) return;
    const float2 r = *reinterpret_cast<const float2*>(&a.rf[row]);
    const float2 s = *reinterpret_cast<const float2*>(&a.sf[row]);
    const float2 w = *reinterpret_cast<const float2*>(&a.wf[row]);
    const float2 z = *reinterpret_cast<const float2*>(&a.zf[row]);
    const float2 t = *reinterpret_cast<const float2*>(&a.tf[row]);
    const float2 p = *reinterpret_cast<const float2*>(&a.pf[row]);
    const float2 r0 = *reinterpret_cast<const float2*>(&a.r0f[row]);
    const float q0 = r.x - af * s.x, y0 = w.x - af * z.x;
    const float q1 = r.y - af * s.y, y1 = w.y - af * z.y;
    float2 rn, wnew, vv;
    rn.x = q0 - wn * y0;
    rn.y = q1 - wn * y1;
    wnew.x = y0 - wn * (t.x - af * v0);
    wnew.y = y1 - wn * (t.y - af * v1);
    vv.x = v0;
    vv.y = v1;
    update_x2(a.x, row, valid1, alpha * double(p.x), alpha * double(p.y), omega * double(q0), omega * double(q1));
    *reinterpret_cast<float2*>(&a.vf[row]) = vv;
    *reinterpret_cast<float2*>(&a.rf[row]) = rn;
    *reinterpret_cast<float2*>(&a.wf[row]) = wnew;
    d[0] = r0.x * rn.x + (valid1 ? r0.y * rn.y : 0.0f);
    d[1] = r0.x * wnew.x + (valid1 ? r0.y * wnew.y : 0.0f);
    d[2] = r0.x * s.x + (valid1 ? r0.y * s.y : 0.0f);
    d[3] = r0.x * z.x + (valid1 ? r0.y * z.y : 0.0f);
    d[4] = rn.x * rn.x + (valid1 ? rn.y * rn.y : 0.0f);
  });
}

// k_mp_pa2 / k_mp_pb2 with four neighbouring rows per lane (see produce4):
// each binary32 vector access is one 16-byte load or store, as wide as the
// binary64 kernels' pairs, so a wave moves 1 KB per access; the operator
// provides spmv4.  The arithmetic of each row and the reduction trees are
// those of k_mp_pa / k_mp_pb, so the results are the same bits.  A four
// starting below n stays inside the workspace vectors (padded to 64 rows);
// x, the caller's n doubles, is updated for the rows below n only.
template <class Op32>
__global__ __launch_bounds__(kWG) void k_mp_pa4(Op32 op, Args a) {
  typedef float F4 __attribute__((ext_vector_type(4)));
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1, float>(a, g);
    fin_setup_alpha(st, g[0]);
  } else {
    double g[5];
    gather_sums<5, float>(a, g);
    fin_pipe_b_mp(st, a.hist, g, false, a.aform);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const float af = float(st.alpha), bf = float(st.beta), wf_ = float(st.omega);
  produce4<2, float>(a, [&](int32_t row, int nv, float (&d)[2]) {
    float t[4];
    op.spmv4(row, nv, a.wf, t);
    if (nv <= 0) return;
    const F4 r4 = *reinterpret_cast<const F4*>(&a.rf[row]);
    const F4 w4 = *reinterpret_cast<const F4*>(&a.wf[row]);
    const F4 v4 = *reinterpret_cast<const F4*>(&a.vf[row]);
    const F4 so4 = *reinterpret_cast<const F4*>(&a.sf[row]);
    const F4 zo4 = *reinterpret_cast<const F4*>(&a.zf[row]);
    const F4 po4 = *reinterpret_cast<const F4*>(&a.pf[row]);
    const float r[4] = {r4.x, r4.y, r4.z, r4.w}, w[4] = {w4.x, w4.y, w4.z, w4.w};
    const float v[4] = {v4.x, v4.y, v4.z, v4.w}, so[4] = {so4.x, so4.y, so4.z, so4.w};
    const float zo[4] = {zo4.x, zo4.y, zo4.z, zo4.w}, po[4] = {po4.x, po4.y, po4.z, po4.w};
    float p[4], s[4], z[4], l0[4], l1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      p[k] = r[k] + bf * (po[k] - wf_ * so[k]);
      s[k] = w[k] + bf * (so[k] - wf_ * zo[k]);
      z[k] = t[k] + bf * (zo[k] - wf_ * v[k]);
      const float q = r[k] - af * s[k], y = w[k] - af * z[k];
      // the four leaves of the reduction tree (a row past n is a zero leaf)
      l0[k] = k < nv ? q * y : 0.0f;
      l1[k] = k < nv ? y * y : 0.0f;
    }
    *reinterpret_cast<F4*>(&a.pf[row]) = F4{p[0], p[1], p[2], p[3]};
    *reinterpret_cast<F4*>(&a.sf[row]) = F4{s[0], s[1], s[2], s[3]};
    *reinterpret_cast<F4*>(&a.tf[row]) = F4{t[0], t[1], t[2], t[3]};
    *reinterpret_cast<F4*>(&a.zf[row]) = F4{z[0], z[1], z[2], z[3]};
    d[0] = (l0[0] + l0[1]) + (l0[2] + l0[3]);
    d[1] = (l1[0] + l1[1]) + (l1[2] + l1[3]);
  });
}

template <class Op32>
__global__ __launch_bounds__(kWG) void k_mp_pb4(Op32 op, Args a) {
  typedef float F4 __attribute__((ext_vector_type(4)));
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2, float>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * double(a.pf[row]);
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  const float af = float(alpha), wn = float(omega);
  produce4<5, float>(a, [&](int32_t row, int nv, float (&d)[5]) {
    float vv[4];
    op.spmv4(row, nv, a.zf, vv);
    if (nv <= 0) return;
    const F4 r4 = *reinterpret_cast<const F4*>(&a.rf[row]);
    const F4 s4 = *reinterpret_cast<const F4*>(&a.sf[row]);
    const F4 w4 = *reinterpret_cast<const F4*>(&a.wf[row]);
    const F4 z4 = *reinterpret_cast<const F4*>(&a.zf[row]);
    const F4 t4 = *reinterpret_cast<const F4*>(&a.tf[row]);
    const F4 p4 = *reinterpret_cast<const F4*>(&a.pf[row]);
    const F4 r04 = *reinterpret_cast<const F4*>(&a.r0f[row]);
    const float r[4] = {r4.x, r4.y, r4.z, r4.w}, s[4] = {s4.x, s4.y, s4.z, s4.w};
    const float w[4] = {w4.x, w4.y, w4.z, w4.w}, z[4] = {z4.x, z4.y, z4.z, z4.w};
    const float t[4] = {t4.x, t4.y, t4.z, t4.w}, p[4] = {p4.x, p4.y, p4.z, p4.w};
    const float r0[4] = {r04.x, r04.y, r04.z, r04.w};
    float rn[4], wnew[4], l[5][4];
    double u[4], ux[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float q = r[k] - af * s[k], y = w[k] - af * z[k];
      rn[k] = q - wn * y;
      wnew[k] = y - wn * (t[k] - af * vv[k]);
      u[k] = alpha * double(p[k]);
      ux[k] = omega * double(q);
      const bool in = k < nv;
      l[0][k] = in ? r0[k] * rn[k] : 0.0f;
      l[1][k] = in ? r0[k] * wnew[k] : 0.0f;
      l[2][k] = in ? r0[k] * s[k] : 0.0f;
      l[3][k] = in ? r0[k] * z[k] : 0.0f;
      l[4][k] = in ? rn[k] * rn[k] : 0.0f;
    }
    update_x4(a.x, row, nv, u, ux);
    *reinterpret_cast<F4*>(&a.vf[row]) = F4{vv[0], vv[1], vv[2], vv[3]};
    *reinterpret_cast<F4*>(&a.rf[row]) = F4{rn[0], rn[1], rn[2], rn[3]};
    *reinterpret_cast<F4*>(&a.wf[row]) = F4{wnew[0], wnew[1], wnew[2], wnew[3]};
#pragma unroll
    for (int j = 0; j < 5; ++j) d[j] = (l[j][0] + l[j][1]) + (l[j][2] + l[j][3]);
  });
}

// k_pa / k_pb of the unpreconditioned p-BiCGStab (Algorithm 9, also on A M^{-1})
// with two neighbouring rows per lane, as k_mp_pa2 / k_mp_pb2: 16-byte vector
// accesses, the same arithmetic per row and the same reduction trees, so the
// same bits as k_pa / k_pb.  Not used after a residual replacement (k_pa with
// RR2 then).
template <class Op>
__device__ __forceinline__ void d_pa2(Op op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1>(a, g);
    fin_setup_alpha(st, g[0]);
  } else {
    double g[5];
    gather_sums<5>(a, g);
    fin_pipe_b(st, a.hist, g, a.aform);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha, beta = st.beta, omega = st.omega;
  produce2<2>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[2]) {
    double t0, t1;
    op.spmv2(row, valid0, valid1, a.w, t0, t1);
    if (!valid0) return;
    const D2 r = *reinterpret_cast<const D2*>(&a.r[row]);
    const D2 w = *reinterpret_cast<const D2*>(&a.w[row]);
    const D2 v = *reinterpret_cast<const D2*>(&a.v[row]);
    const D2 so = *reinterpret_cast<const D2*>(&a.s[row]);
    const D2 zo = *reinterpret_cast<const D2*>(&a.z[row]);
    const D2 po = *reinterpret_cast<const D2*>(&a.ph[row]);
    D2 p, sn, zn, t;
    p.x = r.x + beta * (po.x - omega * so.x);
    p.y = r.y + beta * (po.y - omega * so.y);
    sn.x = w.x + beta * (so.x - omega * zo.x);
    sn.y = w.y + beta * (so.y - omega * zo.y);
    zn.x = t0 + beta * (zo.x - omega * v.x);
    zn.y = t1 + beta * (zo.y - omega * v.y);
    t.x = t0;
    t.y = t1;
    *reinterpret_cast<D2*>(&a.ph[row]) = p;
    *reinterpret_cast<D2*>(&a.s[row]) = sn;
    *reinterpret_cast<D2*>(&a.t[row]) = t;
    *reinterpret_cast<D2*>(&a.z[row]) = zn;
    const double q0 = r.x - alpha * sn.x, y0 = w.x - alpha * zn.x;
    const double q1 = r.y - alpha * sn.y, y1 = w.y - alpha * zn.y;
    d[0] = q0 * y0 + (valid1 ? q1 * y1 : 0.0);
    d[1] = y0 * y0 + (valid1 ? y1 * y1 : 0.0);
  });
}

template <class Op>
__device__ __forceinline__ void d_pb2(Op op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * a.ph[row];
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  produce2<5>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[5]) {
    double v0, v1;
    op.spmv2(row, valid0, valid1, a.z, v0, v1);
    if (!valid0) return;
    const D2 r = *reinterpret_cast<const D2*>(&a.r[row]);
    const D2 s = *reinterpret_cast<const D2*>(&a.s[row]);
    const D2 w = *reinterpret_cast<const D2*>(&a.w[row]);
    const D2 z = *reinterpret_cast<const D2*>(&a.z[row]);
    const D2 t = *reinterpret_cast<const D2*>(&a.t[row]);
    const D2 p = *reinterpret_cast<const D2*>(&a.ph[row]);
    const D2 r0 = *reinterpret_cast<const D2*>(&a.r0[row]);
    const double q0 = r.x - alpha * s.x, y0 = w.x - alpha * z.x;
    const double q1 = r.y - alpha * s.y, y1 = w.y - alpha * z.y;
    update_x2(a.x, row, valid1, alpha * p.x, alpha * p.y, omega * q0, omega * q1);
    D2 rn, wn, vv;
    rn.x = q0 - omega * y0;
    rn.y = q1 - omega * y1;
    wn.x = y0 - omega * (t.x - alpha * v0);
    wn.y = y1 - omega * (t.y - alpha * v1);
    vv.x = v0;
    vv.y = v1;
    *reinterpret_cast<D2*>(&a.v[row]) = vv;
    *reinterpret_cast<D2*>(&a.r[row]) = rn;
    *reinterpret_cast<D2*>(&a.w[row]) = wn;
    d[0] = r0.x * rn.x + (valid1 ? r0.y * rn.y : 0.0);
    d[1] = r0.x * wn.x + (valid1 ? r0.y * wn.y : 0.0);
    d[2] = r0.x * s.x + (valid1 ? r0.y * s.y : 0.0);
    d[3] = r0.x * z.x + (valid1 ? r0.y * z.y : 0.0);
    d[4] = rn.x * rn.x + (valid1 ? rn.y * rn.y : 0.0);
  });
}

// The five BiCGStab kernels (Algorithm 7, also on A M^{-1}) with two
// neighbouring rows per lane, as k_pa2 / k_pb2: the same arithmetic per row
// and the same reduction trees as k_b1 ... k_b5, so the same bits.
template <class Op>
__device__ __forceinline__ void d_b1_2(Op op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  if (a.first) {
    double g[1];
    gather_sums<1>(a, g);
    fin_setup_gamma(st, a.hist, g[0]);
  }
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  produce2<1>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[1]) {
    double s0, s1;
    op.spmv2(row, valid0, valid1, a.ph, s0, s1);
    if (!valid0) return;
    D2 sv;
    sv.x = s0;
    sv.y = s1;
    *reinterpret_cast<D2*>(&a.s[row]) = sv;
    const D2 r0 = *reinterpret_cast<const D2*>(&a.r0[row]);
    d[0] = r0.x * s0 + (valid1 ? r0.y * s1 : 0.0);
  });
}

__device__ __forceinline__ void d_b2_2(Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  double g[1];
  gather_sums<1>(a, g);
  fin_bicg_alpha(st, g[0]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double alpha = st.alpha;
  each_row2(a, [&](int32_t row, bool valid0, bool) {
    if (!valid0) return;
    const D2 r = *reinterpret_cast<const D2*>(&a.r[row]);
    const D2 sv = *reinterpret_cast<const D2*>(&a.s[row]);
    D2 q;
    q.x = r.x - alpha * sv.x;
    q.y = r.y - alpha * sv.y;
    *reinterpret_cast<D2*>(&a.q[row]) = q;
  });
}

template <class Op>
__device__ __forceinline__ void d_b3_2(Op op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  publish(a, st);
  produce2<2>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[2]) {
    double y0, y1;
    op.spmv2(row, valid0, valid1, a.qh, y0, y1);
    if (!valid0) return;
    D2 yv;
    yv.x = y0;
    yv.y = y1;
    *reinterpret_cast<D2*>(&a.y[row]) = yv;
    const D2 q = *reinterpret_cast<const D2*>(&a.q[row]);
    d[0] = q.x * y0 + (valid1 ? q.y * y1 : 0.0);
    d[1] = y0 * y0 + (valid1 ? y1 * y1 : 0.0);
  });
}

__device__ __forceinline__ void d_b4_2(Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * a.ph[row];
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  produce2<2>(a, [&](int32_t row, bool valid0, bool valid1, double (&d)[2]) {
    if (!valid0) return;
    const D2 q = *reinterpret_cast<const D2*>(&a.q[row]);
    const D2 p = *reinterpret_cast<const D2*>(&a.ph[row]);
    const D2 y = *reinterpret_cast<const D2*>(&a.y[row]);
    const D2 r0 = *reinterpret_cast<const D2*>(&a.r0[row]);
    update_x2(a.x, row, valid1, alpha * p.x, alpha * p.y, omega * q.x, omega * q.y);
    D2 r;
    r.x = q.x - omega * y.x;
    r.y = q.y - omega * y.y;
    *reinterpret_cast<D2*>(&a.r[row]) = r;
    d[0] = r0.x * r.x + (valid1 ? r0.y * r.y : 0.0);
    d[1] = r.x * r.x + (valid1 ? r.y * r.y : 0.0);
  });
}

__device__ __forceinline__ void d_b5_2(Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2>(a, g2);
  fin_bicg_beta(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const double beta = st.beta, omega = st.omega;
  each_row2(a, [&](int32_t row, bool valid0, bool) {
    if (!valid0) return;
    const D2 r = *reinterpret_cast<const D2*>(&a.r[row]);
    const D2 po = *reinterpret_cast<const D2*>(&a.p[row]);
    const D2 sv = *reinterpret_cast<const D2*>(&a.s[row]);
    D2 p;
    p.x = r.x + beta * (po.x - omega * sv.x);
    p.y = r.y + beta * (po.y - omega * sv.y);
    *reinterpret_cast<D2*>(&a.p[row]) = p;
  });
}

template <class Op>
__global__ __launch_bounds__(kWG) void k_pa2(Op op, Args a) { d_pa2<Op>(op, a); }
template <class Op>
__global__ __launch_bounds__(kWG) void k_pb2(Op op, Args a) { d_pb2<Op>(op, a); }
template <class Op>
__global__ __launch_bounds__(kWG) void k_b1_2(Op op, Args a) { d_b1_2<Op>(op, a); }
__global__ __launch_bounds__(kWG) void k_b2_2(Args a) { d_b2_2(a); }
template <class Op>
__global__ __launch_bounds__(kWG) void k_b3_2(Op op, Args a) { d_b3_2<Op>(op, a); }
__global__ __launch_bounds__(kWG) void k_b4_2(Args a) { d_b4_2(a); }
__global__ __launch_bounds__(kWG) void k_b5_2(Args a) { d_b5_2(a); }

template <class Op> struct HasSpmv2 : std::false_type {};
template <class V, bool P, bool N> struct HasSpmv2<DiaOpT<V, P, N>> : std::true_type {};
template <int NPTS, class V> struct HasSpmv2<StencilOp<NPTS, V>> : std::true_type {};
template <class V, bool VAR> struct HasSpmv2<GridOp<V, VAR>> : std::true_type {};
template <class Op> struct IsStencil : std::false_type {};
template <int NPTS, class V> struct IsStencil<StencilOp<NPTS, V>> : std::true_type {};
template <class Op> struct HasSpmv4 : std::false_type {};
template <class V, bool P, bool N> struct HasSpmv4<DiaOpT<V, P, N>> : std::true_type {};
template <class Op> struct IsDia : std::false_type {};
template <class V, bool P, bool N> struct IsDia<DiaOpT<V, P, N>> : std::true_type {};
template <class V> struct HasSpmv2<DiaViOpT<V>> : std::true_type {};
template <class V> struct HasSpmv4<DiaViOpT<V>> : std::true_type {};
template <class V> struct IsDia<DiaViOpT<V>> : std::true_type {};

// Replacement iteration, phase B': omega, then only the binary64 x update.
__global__ __launch_bounds__(kWG) void k_mp_rr_x(Args a) {
  PBCGS_PROLOGUE(st)
  double g2[2];
  gather_sums<2, float>(a, g2);
  const double alpha = st.alpha;
  const bool yz = fin_omega(st, a.hist, g2[0], g2[1]);
  publish(a, st);
  if (yz) {
    each_row(a, [&](int32_t row, bool valid) {
      if (valid) a.x[row] = a.x[row] + alpha * double(a.pf[row]);
    });
    return;
  }
  if (st.status != DS_RUNNING) return;
  const double omega = st.omega;
  const float af = float(alpha);
  each_row(a, [&](int32_t row, bool valid) {
    if (!valid) return;
    const float q = a.rf[row] - af * a.sf[row];
    a.x[row] = a.x[row] + alpha * double(a.pf[row]) + omega * double(q);
  });
}

// Replacement, first half: r64 = b - A x (binary64) ; r = f(r64).
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_rr_r(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  each_row(a, [&](int32_t row, bool valid) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r = a.b[row] - ax;
    a.r64[row] = r;
    a.rf[row] = float(r);
  });
}

// w = f(A r64) ; one more replacement ; partials of reduction 2.
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_rr_w(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  st.n_rr += 1;
  publish(a, st);
  produce<5, float>(a, [&](int32_t row, bool valid, float (&d)[5]) {
    const double w = op.spmv(row, valid, a.r64);
    if (!valid) return;
    const float wf = float(w);
    a.wf[row] = wf;
    const float r0 = a.r0f[row], r = a.rf[row];
    d[0] = r0 * r;
    d[1] = r0 * wf;
    d[2] = r0 * a.sf[row];
    d[3] = r0 * a.zf[row];
    d[4] = r * r;
  });
}

// Iteration after a replacement, first kernel: reduction 2 (a.mode = 1 after
// a forced replacement), then p = r + beta (p - omega s) in binary32.
__global__ __launch_bounds__(kWG) void k_mp_rr_p(Args a) {
  PBCGS_PROLOGUE(st)
  double g[5];
  gather_sums<5, float>(a, g);
  fin_pipe_b_mp(st, a.hist, g, a.mode == 1, a.aform);
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const float bf = float(st.beta), wf_ = float(st.omega);
  each_row(a, [&](int32_t row, bool valid) {
    if (valid) a.pf[row] = a.rf[row] + bf * (a.pf[row] - wf_ * a.sf[row]);
  });
}

// Replacement, second half: s64 = A p (binary64, p widened) ; s = f(s64).
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_rr_s(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  each_row(a, [&](int32_t row, bool valid) {
    const double s = op.spmv(row, valid, a.pf);
    if (!valid) return;
    a.s64[row] = s;
    a.sf[row] = float(s);
  });
}

// The binary64 replacement steps with two neighbouring rows per lane (as
// k_mp_pa2): the same arithmetic per row and the same reduction trees as
// k_mp_rr_w, k_mp_rr_s and k_mp_pa<..., true>, so the same bits.  Their
// product inputs are workspace vectors (r64, p, s64, w), whose pairs are
// aligned; r = b - A x reads the caller's x and keeps one row per lane.
template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_rr_w2(Op64 op, Args a) {
  PBCGS_PROLOGUE(st)
  st.n_rr += 1;
  publish(a, st);
  produce2<5, float>(a, [&](int32_t row, bool valid0, bool valid1, float (&d)[5]) {
    double w0, w1;
    op.spmv2(row, valid0, valid1, a.r64, w0, w1);
    if (!valid0) return;
    float2 wf;
    wf.x = float(w0);
    wf.y = float(w1);
    *reinterpret_cast<float2*>(&a.wf[row]) = wf;
    const float2 r0 = *reinterpret_cast<const float2*>(&a.r0f[row]);
    const float2 r = *reinterpret_cast<const float2*>(&a.rf[row]);
    const float2 sv = *reinterpret_cast<const float2*>(&a.sf[row]);
    const float2 zv = *reinterpret_cast<const float2*>(&a.zf[row]);
    d[0] = r0.x * r.x + (valid1 ? r0.y * r.y : 0.0f);
    d[1] = r0.x * wf.x + (valid1 ? r0.y * wf.y : 0.0f);
    d[2] = r0.x * sv.x + (valid1 ? r0.y * sv.y : 0.0f);
    d[3] = r0.x * zv.x + (valid1 ? r0.y * zv.y : 0.0f);
    d[4] = r.x * r.x + (valid1 ? r.y * r.y : 0.0f);
  });
}

template <class Op64>
__global__ __launch_bounds__(kWG) void k_mp_rr_s2(Op64 op, Args a) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  PBCGS_PROLOGUE(st)
  publish(a, st);
  each_row2(a, [&](int32_t row, bool valid0, bool valid1) {
    double s0, s1;
    op.spmv2(row, valid0, valid1, a.pf, s0, s1);
    if (!valid0) return;
    D2 sv;
    sv.x = s0;
    sv.y = s1;
    *reinterpret_cast<D2*>(&a.s64[row]) = sv;
    float2 sf;
    sf.x = float(s0);
    sf.y = float(s1);
    *reinterpret_cast<float2*>(&a.sf[row]) = sf;
  });
}

// K_a of the iteration after a replacement (k_mp_pa<..., true>): t = A w in
// binary32, z = f(A s64) in binary64, q and y from the replaced s.
template <class Op32, class Op64>
__global__ __launch_bounds__(kWG) void k_mp_pa2_rr(Op32 op, Op64 op64, Args a) {
  PBCGS_PROLOGUE(st)
  publish(a, st);
  if (st.status != DS_RUNNING) return;
  const float af = float(st.alpha);
  produce2<2, float>(a, [&](int32_t row, bool valid0, bool valid1, float (&d)[2]) {
    float t0, t1;
    op.spmv2(row, valid0, valid1, a.wf, t0, t1);
    double z0, z1;
    op64.spmv2(row, valid0, valid1, a.s64, z0, z1);
    if (!valid0) return;
    const float2 r = *reinterpret_cast<const float2*>(&a.rf[row]);
    const float2 w = *reinterpret_cast<const float2*>(&a.wf[row]);
    const float2 sv = *reinterpret_cast<const float2*>(&a.sf[row]);
    float2 z, t;
    z.x = float(z0);
    z.y = float(z1);
    t.x = t0;
    t.y = t1;
    const float q0 = r.x - af * sv.x, y0 = w.x - af * z.x;
    const float q1 = r.y - af * sv.y, y1 = w.y - af * z.y;
    *reinterpret_cast<float2*>(&a.tf[row]) = t;
    *reinterpret_cast<float2*>(&a.zf[row]) = z;
    d[0] = q0 * y0 + (valid1 ? q1 * y1 : 0.0f);
    d[1] = y0 * y0 + (valid1 ? y1 * y1 : 0.0f);
  });
}

// Pending reduction finished by one workgroup: MODE 0 reduction 2 (a.mode as
// in k_mp_rr_p), 1 the setup alpha.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_mp_finish(Args a) {
  PBCGS_PROLOGUE(st)
  if (MODE == 0) {
    double g[5];
    gather_sums<5, float>(a, g);
    fin_pipe_b_mp(st, a.hist, g, a.mode == 1, a.aform);
  } else {
    double g[1];
    gather_sums<1, float>(a, g);
    fin_setup_alpha(st, g[0]);
  }
  publish(a, st);
}

// A solve waiting in DS_CHECK goes on (the host found the true residual above tol).
__global__ void k_resume(DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && st->status == DS_CHECK) st->status = DS_RUNNING;
}

// Binary32 copy of an operator's values.
__global__ __launch_bounds__(kWG) void k_round_vals(int64_t nnz, const double* __restrict__ v64,
                                                    float* __restrict__ v32) {
  for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kWG)
    v32[k] = float(v64[k]);
}

// ===========================================================================
// Utility kernels.
// ===========================================================================

__global__ void k_init_state(DevState* st, double tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->alpha = 0.0; st->beta = 0.0; st->omega = 0.0; st->gamma = 0.0;
    st->rho0 = 0.0; st->relres = 1.0; st->tol = tol; st->result = 0.0;
    st->status = DS_RUNNING; st->iters = 0; st->n_rr = 0;
    for (int k = 0; k < 5; ++k) st->pad[k] = 0;
  }
}

// Clears a structural-error flag word.
__global__ void k_clear_flag(int32_t* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

template <class Op>
__global__ __launch_bounds__(kWG) void k_spmv(Op op, Args a, const double* __restrict__ xin,
                                              double* __restrict__ yout) {
  each_row(a, [&](int32_t row, bool valid) {
    const double y = op.spmv(row, valid, xin);
    if (valid) yout[row] = y;
  });
}

// partials of (x, y).
__global__ __launch_bounds__(kWG) void k_dot(Args a, const double* __restrict__ xv,
                                             const double* __restrict__ yv) {
  produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) {
    if (valid) d[0] = xv[row] * yv[row];
  });
}

// partials of ||b - A x||^2 (true residual of the returned x).
template <class Op>
__device__ __forceinline__ void d_true_res(Op op, Args a) {
  produce<1>(a, [&](int32_t row, bool valid, double (&d)[1]) {
    const double ax = op.spmv(row, valid, a.x);
    if (!valid) return;
    const double r = a.b[row] - ax;
    d[0] = r * r;
  });
}
template <class Op>
__global__ __launch_bounds__(kWG) void k_true_res(Op op, Args a) { d_true_res<Op>(op, a); }

// Right preconditioning with the operator formed explicitly (Section 3.6
// solves A M^{-1} y = b and returns x = M^{-1} y): the entries of A M^{-1} are
// a_ij * dinv_j, one rounding each.  The unpreconditioned Algorithms 7 and 9
// then run on it.  Grid-stride over the non-zeros.
template <int PC>
__global__ __launch_bounds__(kWG) void k_fold_csr(CsrOp op, int64_t nnz, double* __restrict__ ahat,
                                                  const double* __restrict__ dinv, double dinv_s) {
  for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kWG) {
    const double d = (PC == PC_VEC) ? dinv[op.ci[k]] : dinv_s;
    ahat[k] = op.va[k] * d;
  }
}

// TO_Y: y_0 = M x_0 = x_0 / dinv before the iteration; otherwise x = M^{-1} y
// = dinv * y after it.  In place.
template <int PC, bool TO_Y>
__global__ __launch_bounds__(kWG) void k_fold_x(int32_t n, double* __restrict__ x,
                                                const double* __restrict__ dinv, double dinv_s) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const double d = (PC == PC_VEC) ? dinv[row] : dinv_s;
  x[row] = TO_Y ? x[row] / d : d * x[row];
}

// dinv_i = 1 / a_ii ; flag bit 0 if a diagonal entry is zero, non-finite or absent.
// One wave per 64 rows: the rows' entries are scanned in storage order
// (coalesced); a row's diagonal entry is its last entry in column i (the last
// of duplicates), found as the largest such index.
__global__ __launch_bounds__(64) void k_dinv_csr(CsrOp op, int32_t n, double* dinv, int32_t* flag) {
  __shared__ int32_t srp[65];
  __shared__ int32_t sdk[64];
  const int lane = threadIdx.x;
  const int32_t r0 = (int32_t)blockIdx.x * 64;
  srp[lane] = op.rp[min(r0 + lane, n)];
  if (lane == 0) srp[64] = op.rp[min(r0 + 64, n)];
  sdk[lane] = -1;
  __syncthreads();
  const int32_t k1 = srp[64];
  for (int32_t k = srp[0] + lane; k < k1; k += 64) {
    int lo = 0, hi = 64;  // srp[lo] <= k < srp[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (srp[mid] <= k) lo = mid;
      else hi = mid;
    }
    if (op.ci[k] == r0 + lo) atomicMax(&sdk[lo], k);
  }
  __syncthreads();
  const int32_t row = r0 + lane;
  bool bad = false;
  if (row < n) {
    const int32_t k = sdk[lane];
    const double d = k >= 0 ? op.va[k] : 0.0;
    bad = d == 0.0 || !finite(d);
    dinv[row] = 1.0 / d;
  }
  if (__any(bad) && lane == 0) atomicOr(flag, 1);
}

// flag bit 1 unless every dinv_i equals dinv_0 (then Jacobi is one scalar).
// Jacobi of the matrix-free 27-point operator: dinv = 1 / a_ii from its formed diagonal.
__global__ __launch_bounds__(kWG) void k_dinv_conv27(Conv27 op, int32_t n, double* dinv, int32_t* flag) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const double d = op.diagonal(row);
  if (d == 0.0 || !finite(d)) atomicOr(flag, 1);
  dinv[row] = 1.0 / d;
}
__global__ __launch_bounds__(kWG) void k_dinv_const(int32_t n, const double* dinv, int32_t* flag) {
  // once a wave has set the bit the rest have nothing to add: they read the
  // flag (from the device-coherent cache) and return
  if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) return;
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  bool bad = false;
  if (row < n) bad = !(dinv[row] == dinv[0]) || !finite(dinv[row]) || dinv[row] == 0.0;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 2);  // one atomic per wave
}

// ---------------------------------------------------------------------------
// Transpose of a CSR matrix (for the adjoint solve A^T lambda = g).  Row j of
// A^T lists the entries of column j of A in ascending row order (ties, which
// only duplicate entries can produce, in stored order), so that the SpMV with
// A^T sums in ascending column order as every other product does.
// ---------------------------------------------------------------------------
constexpr int kScanChunk = 4096;  // entries per workgroup in the scans below

__global__ __launch_bounds__(kWG) void k_count_cols(CsrOp op, int64_t nnz, int32_t* __restrict__ cnt) {
  for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kWG)
    atomicAdd(&cnt[op.ci[k]], 1);
}

// Exclusive prefix sum of the kScanChunk values of each workgroup (in place
// into out) and the chunk's total into bsum.
__global__ __launch_bounds__(kWG) void k_scan_chunks(const int32_t* __restrict__ in, int32_t n,
                                                     int32_t* __restrict__ out, int32_t* __restrict__ bsum) {
  __shared__ int32_t tsum[kWG];
  constexpr int per = kScanChunk / kWG;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * per;
  int32_t v[per];
  int32_t acc = 0;
  for (int j = 0; j < per; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    acc += v[j];
  }
  tsum[threadIdx.x] = acc;
  __syncthreads();
  // inclusive scan of the thread totals (Hillis-Steele)
  for (int d = 1; d < kWG; d <<= 1) {
    const int32_t t = (threadIdx.x >= (unsigned)d) ? tsum[threadIdx.x - d] : 0;
    __syncthreads();
    tsum[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = tsum[threadIdx.x] - acc;
  for (int j = 0; j < per; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == kWG - 1) bsum[blockIdx.x] = tsum[kWG - 1];
}

// Adds the exclusive prefix of the chunk totals (boff) to every chunk.
__global__ __launch_bounds__(kWG) void k_scan_add(int32_t* __restrict__ out, int32_t n, const int32_t* __restrict__ boff) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) out[i] += boff[i / kScanChunk];
}

// Scatter entry k = (i, j, a_ij) to row j of A^T; orig keeps k for the sort.
__global__ __launch_bounds__(kWG) void k_fill_t(CsrOp op, int32_t* __restrict__ cursor, int32_t* __restrict__ ci_t,
                                                double* __restrict__ va_t, int32_t* __restrict__ orig) {
  const int32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= op.n) return;
  for (int32_t k = op.rp[i]; k < op.rp[i + 1]; ++k) {
    const int32_t pos = atomicAdd(&cursor[op.ci[k]], 1);
    ci_t[pos] = i;
    va_t[pos] = op.va[k];
    orig[pos] = k;
  }
}

// Rows of A^T longer than this are ordered by a workgroup each (k_sort_t_long).
constexpr int32_t kShortRowT = 64;

// Orders each short row of A^T by (row of A, stored position): insertion sort
// by one thread.
__global__ __launch_bounds__(kWG) void k_sort_t(int32_t n, const int32_t* __restrict__ rp_t, int32_t* __restrict__ ci_t,
                                                double* __restrict__ va_t, int32_t* __restrict__ orig) {
  const int32_t j = blockIdx.x * kWG + threadIdx.x;
  if (j >= n) return;
  const int32_t b = rp_t[j], e = rp_t[j + 1];
  if (e - b > kShortRowT) return;
  for (int32_t k = b + 1; k < e; ++k) {
    const int32_t c = ci_t[k], o = orig[k];
    const double v = va_t[k];
    int32_t m = k - 1;
    while (m >= b && (ci_t[m] > c || (ci_t[m] == c && orig[m] > o))) {
      ci_t[m + 1] = ci_t[m];
      va_t[m + 1] = va_t[m];
      orig[m + 1] = orig[m];
      --m;
    }
    ci_t[m + 1] = c;
    va_t[m + 1] = v;
    orig[m + 1] = o;
  }
}

// Orders each long row of A^T (more than kShortRowT entries) by the stored
// position of its entries in A -- the same order as (row of A, stored
// position), since CSR stores rows in order; the positions are distinct.  One
// workgroup per row (grid-strided), a bitonic network in the form whose every
// compare-exchange puts the smaller key at the lower index: each merge of two
// sorted halves compares element t with its mirror in the block, then
// half-cleaners at distances size/4, ..., 1.  Indices past the row's length
// then behave as +infinity and are never read or written, so the row needs no
// padding.  O(L log^2 L) work per row of length L.
__global__ __launch_bounds__(kWG) void k_sort_t_long(int32_t n, const int32_t* __restrict__ rp_t,
                                                     int32_t* __restrict__ ci_t, double* __restrict__ va_t,
                                                     int32_t* __restrict__ orig) {
  for (int32_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int32_t b = rp_t[j], len = rp_t[j + 1] - b;
    if (len <= kShortRowT) continue;  // the same for every thread of the workgroup
    int32_t P = 1;
    while (P < len) P <<= 1;
    auto cmp_swap = [&](int32_t lo, int32_t hi) {  // lo < hi
      if (hi >= len) return;
      const int32_t ol = orig[b + lo], oh = orig[b + hi];
      if (ol > oh) {
        orig[b + lo] = oh;
        orig[b + hi] = ol;
        const int32_t c = ci_t[b + lo];
        ci_t[b + lo] = ci_t[b + hi];
        ci_t[b + hi] = c;
        const double v = va_t[b + lo];
        va_t[b + lo] = va_t[b + hi];
        va_t[b + hi] = v;
      }
    };
    for (int32_t size = 2; size <= P; size <<= 1) {
      const int32_t half = size >> 1;
      for (int32_t t = threadIdx.x; t < P / 2; t += kWG) {
        const int32_t blk = t / half, off = t % half;
        cmp_swap(blk * size + off, blk * size + size - 1 - off);
      }
      __syncthreads();
      for (int32_t d = size >> 2; d >= 1; d >>= 1) {
        for (int32_t t = threadIdx.x; t < P / 2; t += kWG) {
          const int32_t lo = (t / d) * 2 * d + t % d;
          cmp_swap(lo, lo + d);
        }
        __syncthreads();
      }
    }
  }
}

// Gradient of a loss L(x) through A x = b with respect to the stored entries:
// dL/da_ij = -lambda_i x_j, lambda = A^{-T} dL/dx.
__global__ __launch_bounds__(kWG) void k_outer_grad(CsrOp op, const double* __restrict__ lam,
                                                    const double* __restrict__ x, double* __restrict__ g) {
  const int32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= op.n) return;
  const double li = lam[i];
  for (int32_t k = op.rp[i]; k < op.rp[i + 1]; ++k) g[k] = -(li * x[op.ci[k]]);
}

// CSR structure check: flag bit 0 on a malformed row pointer or column.
__global__ __launch_bounds__(kWG) void k_csr_check(CsrOp op, int32_t n, int64_t nnz, int32_t* flag) {
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
  if (bad) atomicOr(flag, 1);
}

// flag := 1 if some stored column lies outside int16 range of its row's 64-row
// block start (the compact index copy cannot hold it).
__global__ __launch_bounds__(kWG) void k_c16_check(CsrOp op, int32_t n, int32_t* flag) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const int32_t base = row & ~63, e = op.rp[row + 1];
  bool bad = false;
  for (int32_t k = op.rp[row]; k < e; ++k) {
    const int32_t d = op.ci[k] - base;
    if (d < -32768 || d > 32767) bad = true;
  }
  if (bad) atomicOr(flag, 1);
}

// c16[k] := col_k - (row_k & ~63), one row per thread.
__global__ __launch_bounds__(kWG) void k_c16_fill(CsrOp op, int32_t n, int16_t* __restrict__ c16) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const int32_t base = row & ~63, e = op.rp[row + 1];
  for (int32_t k = op.rp[row]; k < e; ++k) c16[k] = (int16_t)(op.ci[k] - base);
}

// Diagonal table of the uint16_t column form: a 64-slot open-addressing set of
// the distinct diagonals j - i (kEmptyDiag marks a free slot; no diagonal of an
// int32-indexed matrix equals it).  Which slot a diagonal lands in depends on
// the order of the atomic operations; decoding is exact whatever the slots.
constexpr int32_t kEmptyDiag = INT32_MIN;
__device__ __forceinline__ int diag_hash(int32_t d) { return (int)(((uint32_t)d * 2654435761u) >> 26); }

// Inserts d into the 64-slot set; false when the set is full.
__device__ __forceinline__ bool diag_insert(int32_t* set, int32_t d) {
  const int h = diag_hash(d);
  for (int p = 0; p < 64; ++p) {
    const int32_t prev = atomicCAS(&set[(h + p) & 63], kEmptyDiag, d);
    if (prev == kEmptyDiag || prev == d) return true;
  }
  return false;
}

// Gathers the distinct diagonals of the operator into tab[64] (filled with
// kEmptyDiag beforehand): each workgroup collects its rows' diagonals in an LDS
// set, then merges them into tab.  flag := 1 if there are more than 64.
__global__ __launch_bounds__(kWG) void k_diag_collect(CsrOp op, int32_t n, int32_t* tab, int32_t* flag) {
  __shared__ int32_t set[64];
  __shared__ int32_t full;
  if (threadIdx.x < 64) set[threadIdx.x] = kEmptyDiag;
  if (threadIdx.x == 0) full = 0;
  __syncthreads();
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row < n) {
    const int32_t e = op.rp[row + 1];
    for (int32_t k = op.rp[row]; k < e; ++k)
      if (!diag_insert(set, op.ci[k] - row)) { full = 1; break; }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int32_t d = set[threadIdx.x];
    if (d != kEmptyDiag && !diag_insert(tab, d)) full = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && full) atomicOr(flag, 1);
}

// cd[k] := (row_k & 63) | (slot of diagonal col_k - row_k in tab) << 6, one row per thread.
__global__ __launch_bounds__(kWG) void k_diag_code(CsrOp op, int32_t n, const int32_t* __restrict__ tab,
                                                   uint16_t* __restrict__ cd) {
  __shared__ int32_t t[64];
  if (threadIdx.x < 64) t[threadIdx.x] = tab[threadIdx.x];
  __syncthreads();
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  const int32_t e = op.rp[row + 1];
  for (int32_t k = op.rp[row]; k < e; ++k) {
    const int32_t d = op.ci[k] - row;
    const int h = diag_hash(d);
    int slot = 0;
    for (int p = 0; p < 64; ++p) {
      if (t[(h + p) & 63] == d) { slot = (h + p) & 63; break; }
    }
    cd[k] = (uint16_t)((row & 63) | (slot << 6));
  }
}

// Mask of the diagonal layout: bit d of mask[i] is set when row i holds
// diagonal off[d] (off: nd sorted offsets).  flag := 1 when a row's columns do
// not strictly ascend or a diagonal is missing from off (no layout then).
__global__ __launch_bounds__(kWG) void k_dia_mask(CsrOp op, int32_t n, const int32_t* __restrict__ off, int32_t nd,
                                                  uint32_t* __restrict__ mask, int32_t* flag) {
  const int32_t row = blockIdx.x * kWG + threadIdx.x;
  if (row >= n) return;
  uint32_t m = 0;
  int32_t prev = INT32_MIN;
  bool bad = false;
  const int32_t e = op.rp[row + 1];
  for (int32_t k = op.rp[row]; k < e; ++k) {
    const int32_t d = op.ci[k] - row;
    int s = -1;
    for (int t = 0; t < nd; ++t)
      if (off[t] == d) s = t;
    if (s < 0 || d <= prev) { bad = true; break; }
    m |= 1u << s;
    prev = d;
  }
  mask[row] = m;
  if (bad) atomicOr(flag, 1);
}

// Values of the diagonal layout for one solve: each stored value goes to the
// slot of its diagonal (absent slots 0), scaled by dinv of the column when
// folded (PC_VEC: the vector, PC_SCALAR: the constant; one rounding, as the
// folded CSR values) and rounded once to V.  One wave per 64 rows: the rows'
// entries are read in storage order (coalesced), each placed in an LDS tile
// at (its diagonal, its row) -- the row by a search of the row pointers, the
// diagonal by a search of the ascending offsets -- and the tile is written
// out diagonal by diagonal.  A row holds at most one entry per diagonal (the
// layout is made only for rows with strictly ascending columns).
template <int PC, class V>
__global__ __launch_bounds__(64) void k_dia_fill(CsrOp op, int32_t n, const int32_t* __restrict__ doff, int32_t nd,
                                                 int32_t ld, V* __restrict__ dia, const double* __restrict__ dinv,
                                                 double dinv_s) {
  __shared__ V tile[kMaxDia][64];
  __shared__ int32_t srp[65];
  __shared__ int32_t soff[kMaxDia];
  const int lane = threadIdx.x;
  const int32_t r0 = (int32_t)blockIdx.x * 64;
  for (int d = 0; d < nd; ++d) tile[d][lane] = V(0);
  if (lane < nd) soff[lane] = doff[lane];
  srp[lane] = op.rp[min(r0 + lane, n)];
  if (lane == 0) srp[64] = op.rp[min(r0 + 64, n)];
  __syncthreads();
  const int32_t k1 = srp[64];
  for (int32_t k = srp[0] + lane; k < k1; k += 64) {
    int lo = 0, hi = 64;  // srp[lo] <= k < srp[hi]: k is an entry of row r0 + lo
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (srp[mid] <= k) lo = mid;
      else hi = mid;
    }
    const int32_t c = op.ci[k];
    const int32_t off = c - (r0 + lo);
    int a = 0, b = nd - 1;  // the slot whose offset is off
    while (a < b) {
      const int m = (a + b) >> 1;
      if (soff[m] < off) a = m + 1;
      else b = m;
    }
    double v = op.va[k];
    if (PC == PC_VEC) v = v * dinv[c];
    if (PC == PC_SCALAR) v = v * dinv_s;
    tile[a][lo] = V(v);
  }
  __syncthreads();
  if (r0 + lane < n)
    for (int d = 0; d < nd; ++d) dia[(int64_t)d * ld + r0 + lane] = tile[d][lane];
}

// Value indexing of the binary64 layout (see DiaViOp).  Each diagonal's table
// is a kViTab-slot open-addressing set of the bit patterns of the values its
// present entries hold; kViEmpty (a NaN pattern) marks a free slot.  Which
// slot a value lands in depends on the order of the atomic operations; the
// codes are exact whatever the slots.  tab[nd * kViTab] is the overflow word:
// nonzero when some diagonal holds more than kViTab distinct values (or the
// marker pattern itself), and then the codes are not made.
constexpr uint64_t kViEmpty = 0x7ff4a5a5a5a5a5a5ull;
__device__ __forceinline__ int vi_hash(uint64_t b) {
  return (int)(((b ^ (b >> 29) ^ (b >> 47)) * 0x9e3779b97f4a7c15ull) >> 60);
}

__global__ __launch_bounds__(kWG) void k_vi_reset(uint64_t* __restrict__ tab, int32_t nd) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < nd * kViTab) tab[i] = kViEmpty;
  if (i == nd * kViTab) tab[i] = 0;
}

// Inserts b into diagonal k's set; false when the set is full.
__device__ __forceinline__ bool vi_insert(uint64_t* __restrict__ tab, int k, uint64_t b) {
  if (b == kViEmpty) return false;
  const int h = vi_hash(b);
  for (int p = 0; p < kViTab; ++p) {
    uint64_t* slot = &tab[k * kViTab + ((h + p) & (kViTab - 1))];
    uint64_t cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kViEmpty) {
      const uint64_t old = atomicCAS((unsigned long long*)slot, (unsigned long long)kViEmpty, (unsigned long long)b);
      cur = old == kViEmpty ? b : old;
    }
    if (cur == b) return true;
  }
  return false;
}

__device__ __forceinline__ uint64_t vi_bits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ uint64_t vi_bits(float v) { return (uint64_t)__float_as_uint(v); }

// Each wave walks its rows 64 at a time (a grid-stride loop).  The lanes
// that hold the same value on a diagonal are served by one insert (their
// lowest lane's), and a value the wave inserted last on that diagonal needs
// none, so a diagonal of few values costs each wave a few inserts in all.  A
// wave stops at the first full set, and at the start of each step once any
// set is full.  At most kViDia diagonals (the host checks).
template <class D>
__global__ __launch_bounds__(kWG) void k_vi_collect(D d, uint64_t* __restrict__ tab) {
  uint64_t* over = &tab[d.nd * kViTab];
  const int lane = (int)(threadIdx.x & 63);
  uint64_t last[kViDia];  // wave-uniform
#pragma unroll
  for (int k = 0; k < kViDia; ++k) last[k] = kViEmpty;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < d.n; base += stride) {
    if (__hip_atomic_load(over, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;  // wave-uniform
    const int64_t row = base + lane;
    const uint32_t m = row < d.n ? d.mask[row] : 0u;
#pragma unroll
    for (int k = 0; k < kViDia; ++k) {
      if (k < d.nd) {
        bool pend = (m >> k) & 1u;
        const uint64_t b = pend ? vi_bits(d.va[(int64_t)k * d.ld + row]) : 0ull;
        if (pend && b == last[k]) pend = false;
        for (;;) {
          const uint64_t act = __ballot(pend);
          if (act == 0) break;
          const int leader = __ffsll((unsigned long long)act) - 1;
          const uint64_t lb = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(b >> 32), leader) << 32) |
                              (uint64_t)(uint32_t)__shfl((int)(uint32_t)b, leader);
          if (pend && b == lb) pend = false;
          int ok = 1;
          if (lane == leader) ok = vi_insert(tab, k, lb) ? 1 : 0;
          if (__shfl(ok, leader) == 0) {
            if (lane == leader) __hip_atomic_store(over, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;  // wave-uniform
          }
          last[k] = lb;
        }
      }
    }
  }
}

template <class D>
__global__ __launch_bounds__(kWG) void k_vi_encode(D d, const uint64_t* __restrict__ tab,
                                                   uint64_t* __restrict__ code) {
  const int32_t row = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (row >= d.ld) return;
  const uint32_t m = row < d.n ? d.mask[row] : 0u;
  uint64_t w = ~0ull;  // every byte kViAbsent
  for (int k = 0; k < d.nd; ++k) {
    if (!((m >> k) & 1u)) continue;
    const uint64_t b = vi_bits(d.va[(int64_t)k * d.ld + row]);
    const int h = vi_hash(b);
    for (int p = 0; p < kViTab; ++p) {
      const int s = (h + p) & (kViTab - 1);
      if (tab[k * kViTab + s] == b) {
        w = (w & ~(0xffull << (8 * k))) | ((uint64_t)s << (8 * k));
        break;
      }
    }
  }
  code[row] = w;
}

// ===========================================================================
// Batched launches: many independent CSR systems (no preconditioner) in one
// grid.  Workgroup g belongs to system map[g]; a system's workgroups are
// consecutive, so its rows, its partial sums and its scalar state are its
// own, and each reduction is the same pairwise tree as in a solve of that
// system alone (so the results are the same bits).  A system that has
// stopped passes its state on and its workgroups return at once.
// ===========================================================================
struct SysDesc {
  const int32_t* rp;
  const int32_t* ci;
  const int16_t* c16;  // the operator's compact columns (read by CsrOp16 launches only)
  const double* va;
  double* ws;        // 8 vectors of np doubles
  double* x;
  const double* b;
  DevState* st;      // 4 state slots: 0, 1 the iteration ring, 2, 3 utility sums
  int64_t np;
  int32_t n, G, R, wg0;  // rows, workgroups, blocks per wave, first workgroup of the grid
  // diagonal layout (read by DiaOpB launches only): the operator's row masks,
  // this solve's copy of the values (nd slots of np), the offsets
  const uint32_t* dmask;
  double* dva;
  int32_t nd, pad_;
  int32_t doff[kMaxDia];
};

// Per-system arguments from the launch template: rows, shape, state slots
// (template field par), partial-sum rows (offset to the system's workgroups)
// and the vector layout of p-BiCGStab (PIPE) or BiCGStab.
template <bool PIPE, class Op>
__device__ __forceinline__ void bind_sys(const SysDesc& d, const SysDesc* dp, Args& a, Op& op) {
  if constexpr (std::is_same<Op, CsrOp16>::value) {
    op = Op{d.rp, d.c16, d.va, d.n};
  } else if constexpr (std::is_same<Op, DiaOpB>::value) {
    op.off = dp->doff;  // read in place: the loops index the offsets
    op.mask = d.dmask;
    op.va = d.dva;
    op.n = d.n;
    op.nd = d.nd;
    op.ld = (int32_t)d.np;
  } else {
    op = Op{d.rp, d.ci, d.va, d.n};
  }
  a.n = d.n;
  a.G = d.G;
  a.R = d.R;
  a.Gin = d.G;
  a.sin = d.st + a.par;
  a.sout = d.st + (a.par ^ 1);
  if (a.pin) a.pin += d.wg0;
  if (a.pout) a.pout += d.wg0;
  a.x = d.x;
  a.b = d.b;
  a.hist = nullptr;
  a.dinv = nullptr;
  double* v = d.ws;
  const int64_t np = d.np;
  if (PIPE) {
    a.r0 = v; a.r = v + np; a.w = v + 2 * np; a.t = v + 3 * np;
    a.ph = v + 4 * np; a.s = v + 5 * np; a.z = v + 6 * np; a.v = v + 7 * np;
    a.rh = a.r; a.wh = a.w; a.sh = a.s; a.zh = a.z;
  } else {
    a.r0 = v; a.r = v + np; a.p = v + 2 * np; a.s = v + 3 * np; a.q = v + 4 * np; a.y = v + 5 * np;
    a.ph = a.p; a.qh = a.q;
  }
}

// Op: CsrOp (int32 columns), CsrOp16 (every system's compact columns) or
// DiaOpB (every system's diagonal layout)
#define PBCGS_BIND_WG(PIPE)                        \
  const SysDesc* dp_ = sys + map[blockIdx.x];      \
  const SysDesc d_ = *dp_;                         \
  a.wg = (int32_t)blockIdx.x - d_.wg0;             \
  Op op;                                           \
  bind_sys<PIPE>(d_, dp_, a, op);

template <class Op, bool PIPE>
__global__ __launch_bounds__(kWG) void kb_setup_r0(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(PIPE) d_setup_r0<Op, PC_NONE, PIPE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_setup_w0(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_setup_w0<Op, PC_NONE>(op, a);
}
template <class Op, bool RR2>
__global__ __launch_bounds__(kWG) void kb_pa(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_pa<Op, PC_NONE, RR2>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_pb(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_pb<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_rr_x(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) (void)op; d_rr_x<PC_NONE>(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_rr_r(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_rr_r<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_rr_w(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_rr_w<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_rr_p(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) (void)op; d_rr_p<PC_NONE>(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_rr_s(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_rr_s<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b1(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) d_b1<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b2<PC_NONE>(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b3(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) d_b3<Op, PC_NONE>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b4(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b4<PC_NONE>(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b5(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b5<PC_NONE>(a);
}
// Two rows per lane (every system's waves own at least two blocks): the
// diagonal-layout batch, as k_pa2 / k_pb2 and k_b1_2 ... k_b5_2.
template <class Op>
__global__ __launch_bounds__(kWG) void kb_pa2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_pa2<Op>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_pb2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_pb2<Op>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b1_2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) d_b1_2<Op>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b2_2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b2_2(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b3_2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) d_b3_2<Op>(op, a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b4_2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b4_2(a);
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_b5_2(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(false) (void)op; d_b5_2(a);
}
// Every system's diagonal-layout values from its CSR values (as k_dia_fill),
// over the batch's workgroups: workgroup g of a system fills the rows of its
// 256 R row range.
__global__ __launch_bounds__(kWG) void kb_dia_fill(const SysDesc* sys, const int32_t* map) {
  const SysDesc& d = sys[map[blockIdx.x]];
  const int64_t base = ((int64_t)blockIdx.x - d.wg0) * kWG * d.R;
  for (int j = 0; j < d.R; ++j) {
    const int64_t r = base + (int64_t)j * kWG + threadIdx.x;
    if (r >= d.n) return;
    const int32_t row = (int32_t)r;
    const uint32_t m = d.dmask[row];
    int32_t k = d.rp[row];
    for (int q = 0; q < d.nd; ++q) {
      double v = 0.0;
      if ((m >> q) & 1u) v = d.va[k++];
      d.dva[(int64_t)q * d.np + row] = v;
    }
  }
}
template <class Op>
__global__ __launch_bounds__(kWG) void kb_true_res(const SysDesc* sys, const int32_t* map, Args a) {
  PBCGS_BIND_WG(true) d_true_res<Op>(op, a);
}
// One workgroup per system: a pending reduction (modes of k_finish).
template <int MODE, bool PIPE>
__global__ __launch_bounds__(kWG) void kb_finish(const SysDesc* sys, Args a) {
  const SysDesc d = sys[blockIdx.x];
  a.wg = 0;
  CsrOp op;
  bind_sys<PIPE>(d, sys + blockIdx.x, a, op);
  d_finish<MODE>(a);
}
// Slot `slot` of every system's state: running, no scalars yet.
__global__ void kb_init_state(const SysDesc* sys, int32_t nsys, int32_t slot, double tol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsys) return;
  DevState* st = sys[k].st + slot;
  st->alpha = 0.0; st->beta = 0.0; st->omega = 0.0; st->gamma = 0.0;
  st->rho0 = 0.0; st->relres = 1.0; st->tol = tol; st->result = 0.0;
  st->status = DS_RUNNING; st->iters = 0; st->n_rr = 0;
  for (int j = 0; j < 5; ++j) st->pad[j] = 0;
}
#undef PBCGS_BIND_WG

// ===========================================================================
// Persistent form for small systems: the whole solve in one cooperative
// launch.  The phases are those of the graph schedule (the same device
// bodies, state ring and partial-sum buffers); a grid barrier replaces each
// kernel boundary.  Every wait is bounded: a barrier that does not complete
// in about a quarter of a second sets an error flag and the kernel ends.
// ===========================================================================
struct GridBar {
  unsigned cnt;   // arrivals at the current barrier
  unsigned gen;   // completed barriers
  int err;        // set when a wait timed out
  int pad;
};

// Partial-sum buffers by role (the same roles as the launches of the driver).
enum : int { PBR_SETUP1 = 0, PBR_SETUP2, PBR_A, PBR_B, PBR_B1, PBR_B3, PBR_B4 };

struct PersistCfg {
  DevState* st;      // the two-slot state ring
  double* parts;     // partial-sum buffers, kMaxD * kMaxG doubles per role
  GridBar* bar;
  int64_t* qout;     // phases run (the state is in slot qout & 1 at the end)
  int32_t variant;   // 0 BiCGStab, 1 p-BiCGStab, 2 p-BiCGStab with replacement
  int32_t rr_period, rr_max, maxit;
};

// Grid-wide barrier with release/acquire at agent scope; false after a timeout.
__device__ __forceinline__ bool grid_sync(GridBar* b, unsigned nwg) {
  __shared__ int ok_;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(&b->cnt, 1u);
    if (prev == nwg - 1) {
      atomicExch(&b->cnt, 0u);
      __threadfence();
      atomicAdd(&b->gen, 1u);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 22)) {
          atomicOr(&b->err, 1);
          ok = 0;
          break;
        }
      }
    }
    if (__hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    __threadfence();
    ok_ = ok;
  }
  __syncthreads();
  return ok_ != 0;
}

__device__ __forceinline__ bool rr_due_dev(const PersistCfg& c, int64_t i) {
  if (c.variant != 2 || c.rr_period <= 0 || i < 0) return false;
  if ((i + 1) % c.rr_period != 0) return false;
  const int64_t before = (i + 1) / c.rr_period - 1;
  return c.rr_max < 0 || before < c.rr_max;
}

template <class Op, int PC>
__global__ __launch_bounds__(kWG) void k_persist(Op op, Args base, PersistCfg c) {
  int64_t q = 0;
  const unsigned nwg = gridDim.x;
  bool ok = true;
  auto L = [&](int pin, int pout, bool first) {
    Args a = base;
    a.wg = -1;
    a.sin = c.st + (q & 1);
    a.sout = c.st + ((q + 1) & 1);
    a.pin = pin >= 0 ? c.parts + (size_t)pin * kMaxD * kMaxG : nullptr;
    a.pout = pout >= 0 ? c.parts + (size_t)pout * kMaxD * kMaxG : nullptr;
    a.Gin = base.G;
    a.first = first ? 1 : 0;
    ++q;
    return a;
  };
  auto sync = [&]() {
    if (ok) ok = grid_sync(c.bar, nwg);
    return ok;
  };
  const bool pipe = c.variant != 0;
  if (pipe) {
    d_setup_r0<Op, PC, true>(op, L(-1, PBR_SETUP1, false));
    if (sync()) d_setup_w0<Op, PC>(op, L(PBR_SETUP1, PBR_SETUP2, false));
  } else {
    d_setup_r0<Op, PC, false>(op, L(-1, PBR_SETUP1, false));
  }
  sync();
  int64_t i = 0;
  for (; ok && i < c.maxit; ++i) {
    if (!pipe) {
      d_b1<Op, PC>(op, L(PBR_SETUP1, PBR_B1, i == 0));
      if (sync()) d_b2<PC>(L(PBR_B1, -1, false));
      if (sync()) d_b3<Op, PC>(op, L(-1, PBR_B3, false));
      if (sync()) d_b4<PC>(L(PBR_B3, PBR_B4, false));
      if (sync()) d_b5<PC>(L(PBR_B4, -1, false));
      sync();
    } else {
      if (rr_due_dev(c, i - 1)) {
        d_rr_p<PC>(L(PBR_B, -1, false));
        if (sync()) d_rr_s<Op, PC>(op, L(-1, -1, false));
        if (sync()) d_pa<Op, PC, true>(op, L(-1, PBR_A, false));
      } else {
        d_pa<Op, PC, false>(op, L(i == 0 ? PBR_SETUP2 : PBR_B, PBR_A, i == 0));
      }
      sync();
      if (ok && rr_due_dev(c, i)) {
        d_rr_x<PC>(L(PBR_A, -1, false));
        if (sync()) d_rr_r<Op, PC>(op, L(-1, -1, false));
        if (sync()) d_rr_w<Op, PC>(op, L(-1, PBR_B, false));
      } else if (ok) {
        d_pb<Op, PC>(op, L(PBR_A, PBR_B, false));
      }
      sync();
    }
    if (!ok) break;
    // the state after this iteration, published before the barrier
    const int32_t status = __hip_atomic_load(&c.st[q & 1].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (status != DS_RUNNING) break;
  }
  // maxit reached: the reduction left pending by the last phase, in workgroup 0
  if (ok && i == c.maxit) {
    if (pipe) {
      const Args a = (c.maxit == 0) ? L(PBR_SETUP2, -1, false) : L(PBR_B, -1, false);
      if (blockIdx.x == 0) {
        Args a0 = a;
        a0.wg = 0;
        if (c.maxit == 0) d_finish<1>(a0);
        else d_finish<0>(a0);
      }
    } else if (c.maxit == 0) {
      const Args a = L(PBR_SETUP1, -1, false);
      if (blockIdx.x == 0) {
        Args a0 = a;
        a0.wg = 0;
        d_finish<2>(a0);
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *c.qout = q;
}

}  // namespace pbcgs
