// Workload builder: assembles on the device the h^2-scaled first-order upwind
// convection-diffusion operators of the test and benchmark workloads (not part
// of the solver).  One thread per row; row pointers come from a three-pass
// prefix sum of the row lengths.
//
//   hb_a = beta_a / (n + 1)   (computed on the host, one IEEE division)
//   5/7-point: coupling -1 to each in-grid neighbour, -1 - |hb_a| on the
//              upwind neighbour of axis a (p - e_a if beta_a >= 0, else
//              p + e_a); diagonal (4 + |hbx|) + |hby| or ((6 + |hbx|) + |hby|) + |hbz|.
//   27-point:  kbar_d = (sum of the 4/2/1 cell coefficients shared by p and
//              p + d, in (c, b, a) order) * (1 / count); coupling -kbar_d, and
//              -kbar_d - |hb_a| on the upwind face of axis a; diagonal
//              (sum over all 26 d of kbar_d + ((|hbx| + |hby|) + |hbz|)) + shift.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/pbcgs.h"
#include "internal.hpp"

namespace {

constexpr int kB = 256;
constexpr int kPer = 16;  // entries per thread in the scan

struct CD {
  int32_t dim, n, npts;
  double hb[3];
  int32_t up_neg[3];  // 1: beta_a >= 0 (upwind neighbour is p - e_a)
  const double* kappa;
  double shift;
};

__device__ __forceinline__ void decode(const CD& c, int32_t row, int32_t& i, int32_t& j, int32_t& k) {
  i = row % c.n;
  const int32_t jk = row / c.n;
  if (c.dim == 3) {
    j = jk % c.n;
    k = jk / c.n;
  } else {
    j = jk;
    k = 0;
  }
}

__device__ __forceinline__ bool inside(const CD& c, int32_t i, int32_t j, int32_t k) {
  const int32_t nz = (c.dim == 3) ? c.n : 1;
  return i >= 0 && i < c.n && j >= 0 && j < c.n && k >= 0 && k < nz;
}

__global__ void k_rowlen(CD c, int32_t N, int32_t* len) {
  const int32_t row = blockIdx.x * kB + threadIdx.x;
  if (row >= N) return;
  int32_t i, j, k;
  decode(c, row, i, j, k);
  int32_t cnt = 0;
  if (c.npts == 27) {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) cnt += inside(c, i + dx, j + dy, k + dz) ? 1 : 0;
  } else {
    cnt = 1 + (i > 0) + (i < c.n - 1) + (j > 0) + (j < c.n - 1);
    if (c.dim == 3) cnt += (k > 0) + (k < c.n - 1);
  }
  len[row] = cnt;
}

// Inclusive prefix sum of v[0..N) in place: per-block pass, block-sum pass, add pass.
__global__ void k_scan_local(int32_t* v, int32_t N, int64_t* bsum) {
  __shared__ int64_t sh[kB];
  const int64_t base = (int64_t)blockIdx.x * kB * kPer + (int64_t)threadIdx.x * kPer;
  int64_t loc[kPer];
  int64_t acc = 0;
  for (int e = 0; e < kPer; ++e) {
    const int64_t idx = base + e;
    acc += (idx < N) ? v[idx] : 0;
    loc[e] = acc;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < kB; off <<= 1) {
    const int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  const int64_t before = (threadIdx.x > 0) ? sh[threadIdx.x - 1] : 0;
  for (int e = 0; e < kPer; ++e) {
    const int64_t idx = base + e;
    if (idx < N) v[idx] = (int32_t)(loc[e] + before);
  }
  if (threadIdx.x == kB - 1) bsum[blockIdx.x] = sh[kB - 1];
}

__global__ void k_scan_blocks(int64_t* bsum, int32_t nb, int32_t* overflow) {
  if (threadIdx.x != 0) return;
  int64_t acc = 0;
  for (int32_t b = 0; b < nb; ++b) {
    const int64_t t = bsum[b];
    bsum[b] = acc;  // exclusive
    acc += t;
  }
  if (acc > INT32_MAX) *overflow = 1;
}

__global__ void k_scan_add(int32_t* v, int32_t N, const int64_t* bsum) {
  const int64_t base = (int64_t)blockIdx.x * kB * kPer;
  const int64_t off = bsum[blockIdx.x];
  for (int e = threadIdx.x; e < kB * kPer; e += kB) {
    const int64_t idx = base + e;
    if (idx < N) v[idx] = (int32_t)(v[idx] + off);
  }
}

__global__ void k_fill(CD c, int32_t N, const int32_t* __restrict__ rp, int32_t* __restrict__ col,
                       double* __restrict__ val) {
  const int32_t row = blockIdx.x * kB + threadIdx.x;
  if (row >= N) return;
  int32_t i, j, k;
  decode(c, row, i, j, k);
  const int32_t n = c.n;
  const int64_t nn = (int64_t)n * n;
  int64_t pos = rp[row];
  if (c.npts != 27) {
    // (-z), -y, -x, diagonal, +x, +y, (+z)
    const int nax = (c.dim == 3) ? 3 : 2;
    for (int e = 0; e < 2 * nax + 1; ++e) {
      int a, side;
      if (e < nax) { a = nax - 1 - e; side = -1; }
      else if (e == nax) { a = -1; side = 0; }
      else { a = e - nax - 1; side = 1; }
      if (side == 0) {
        double d;
        if (c.dim == 2) d = (4.0 + fabs(c.hb[0])) + fabs(c.hb[1]);
        else d = ((6.0 + fabs(c.hb[0])) + fabs(c.hb[1])) + fabs(c.hb[2]);
        col[pos] = row;
        val[pos] = d;
        ++pos;
        continue;
      }
      const int32_t ii = i + (a == 0 ? side : 0), jj = j + (a == 1 ? side : 0), kk = k + (a == 2 ? side : 0);
      if (!inside(c, ii, jj, kk)) continue;
      const bool upwind = c.up_neg[a] ? (side < 0) : (side > 0);
      col[pos] = (int32_t)(ii + (int64_t)n * jj + nn * kk);
      val[pos] = upwind ? (-1.0 - fabs(c.hb[a])) : -1.0;
      ++pos;
    }
    return;
  }
  const int64_t cn = n + 1;
  double diag_sum = 0.0;
  int64_t diag_pos = -1;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) {
          diag_pos = pos;
          col[pos] = row;
          ++pos;
          continue;
        }
        const int alo = dx > 0 ? 1 : 0, ahi = dx < 0 ? 0 : 1;
        const int blo = dy > 0 ? 1 : 0, bhi = dy < 0 ? 0 : 1;
        const int clo = dz > 0 ? 1 : 0, chi = dz < 0 ? 0 : 1;
        double ksum = 0.0;
        int cnt = 0;
        for (int cc = clo; cc <= chi; ++cc)
          for (int bb = blo; bb <= bhi; ++bb)
            for (int aa = alo; aa <= ahi; ++aa) {
              ksum = ksum + c.kappa[(i + aa) + cn * ((j + bb) + cn * (k + cc))];
              ++cnt;
            }
        const double kbar = ksum * (1.0 / (double)cnt);
        diag_sum = diag_sum + kbar;
        if (!inside(c, i + dx, j + dy, k + dz)) continue;
        double v = -kbar;
        if ((dx != 0) + (dy != 0) + (dz != 0) == 1) {
          const int a = dx != 0 ? 0 : (dy != 0 ? 1 : 2);
          const int side = dx != 0 ? dx : (dy != 0 ? dy : dz);
          const bool upwind = c.up_neg[a] ? (side < 0) : (side > 0);
          if (upwind) v = -kbar - fabs(c.hb[a]);
        }
        col[pos] = (int32_t)((i + dx) + (int64_t)n * (j + dy) + nn * (k + dz));
        val[pos] = v;
        ++pos;
      }
  val[diag_pos] = (diag_sum + ((fabs(c.hb[0]) + fabs(c.hb[1])) + fabs(c.hb[2]))) + c.shift;
}

}  // namespace

extern "C" {

int64_t pbcgs_convdiff_nnz(int32_t dim, int32_t n, int32_t npts) {
  const int64_t m = n;
  if (n <= 0) return PBCGS_ERR_INVALID_ARG;
  if (dim == 2 && npts == 5) return 5 * m * m - 4 * m;
  if (dim == 3 && npts == 7) return 7 * m * m * m - 6 * m * m;
  if (dim == 3 && npts == 27) return (3 * m - 2) * (3 * m - 2) * (3 * m - 2);
  return PBCGS_ERR_INVALID_ARG;
}

int pbcgs_assemble_convdiff(pbcgs_ctx_t ctx, int32_t dim, int32_t n, int32_t npts, const double* beta,
                            const double* kappa, double shift, int32_t* row_ptr, int32_t* col_idx, double* val) {
  if (!ctx || !beta || !row_ptr || !col_idx || !val)
    return pbcgs_internal_fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  const int64_t nnz = pbcgs_convdiff_nnz(dim, n, npts);
  if (nnz < 0) return pbcgs_internal_fail(ctx, PBCGS_ERR_INVALID_ARG, "unsupported dim/npts/n");
  if (npts == 27 && !kappa) return pbcgs_internal_fail(ctx, PBCGS_ERR_INVALID_ARG, "27-point needs kappa");
  const int64_t N64 = (dim == 3) ? (int64_t)n * n * n : (int64_t)n * n;
  if (N64 > INT32_MAX || nnz > INT32_MAX) return pbcgs_internal_fail(ctx, PBCGS_ERR_UNSUPPORTED, "too large");
  const int32_t N = (int32_t)N64;
  hipStream_t s = static_cast<hipStream_t>(pbcgs_internal_stream(ctx));
  CD c;
  c.dim = dim;
  c.n = n;
  c.npts = npts;
  for (int a = 0; a < 3; ++a) {
    c.hb[a] = (a < dim) ? beta[a] / (double)(n + 1) : 0.0;
    c.up_neg[a] = (a < dim) ? (beta[a] >= 0.0 ? 1 : 0) : 1;
  }
  c.kappa = kappa;
  c.shift = shift;
  const int nb_rows = (N + kB - 1) / kB;
  const int32_t nb_scan = (int32_t)((N + (int64_t)kB * kPer - 1) / ((int64_t)kB * kPer));
  int64_t* bsum = nullptr;
  int32_t* ovf = nullptr;
  if (hipMalloc(&bsum, sizeof(int64_t) * nb_scan + 64) != hipSuccess)
    return pbcgs_internal_fail(ctx, PBCGS_ERR_ALLOC, "scan scratch allocation failed");
  ovf = reinterpret_cast<int32_t*>(bsum + nb_scan);
  int32_t hovf = 0;
  hipError_t e = hipMemsetAsync(ovf, 0, sizeof(int32_t), s);
  if (e == hipSuccess) e = hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s);
  if (e == hipSuccess) {
    k_rowlen<<<nb_rows, kB, 0, s>>>(c, N, row_ptr + 1);
    k_scan_local<<<nb_scan, kB, 0, s>>>(row_ptr + 1, N, bsum);
    k_scan_blocks<<<1, 64, 0, s>>>(bsum, nb_scan, ovf);
    k_scan_add<<<nb_scan, kB, 0, s>>>(row_ptr + 1, N, bsum);
    k_fill<<<nb_rows, kB, 0, s>>>(c, N, row_ptr, col_idx, val);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hovf, ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bsum);
  if (e != hipSuccess) return pbcgs_internal_fail(ctx, PBCGS_ERR_HIP, hipGetErrorString(e));
  if (hovf) return pbcgs_internal_fail(ctx, PBCGS_ERR_UNSUPPORTED, "nnz overflows int32");
  return PBCGS_SUCCESS;
}

}  // extern "C"
