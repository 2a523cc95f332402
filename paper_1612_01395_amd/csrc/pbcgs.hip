// Host side of the pipelined BiCGStab library: contexts, operators, the
// iteration driver (launch schedule, HIP-graph capture, status polling) and
// the C ABI declared in include/pbcgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pbcgs.h"
#include "internal.hpp"
#include "kernels.hpp"
#include "debug.hpp"

using namespace pbcgs;

namespace {

thread_local std::string g_last_error;

// OP_ST27: the constant 27-point stencil; OP_GRID: a stencil with coefficients per row
enum OpKind { OP_CSR = 0, OP_ST5 = 1, OP_ST7 = 2, OP_CV27 = 3, OP_ST27 = 4, OP_GRID = 5 };

// Partial-sum buffers, one per producing kernel role.
enum PartBuf { PB_SETUP1 = 0, PB_SETUP2, PB_A, PB_B, PB_B1, PB_B3, PB_B4, PB_UTIL, PB_COUNT };

// Device memory of pbcgs_solve_noalloc: four state slots, the partial-sum
// buffers and a pool of doubles for the solver vectors (and A M^{-1} of a
// folded CSR solve).  One copy per device, shared by every call on it.
constexpr size_t kScratchStates = 4;
constexpr size_t kScratchPartDoubles = (size_t)PB_COUNT * kMaxD * kMaxG;
constexpr size_t kScratchPoolDoubles = (size_t)1 << 23;  // 64 MiB
constexpr size_t kScratchPartOffset = kScratchStates * sizeof(DevState);
constexpr size_t kScratchPoolOffset = kScratchPartOffset + kScratchPartDoubles * sizeof(double);
constexpr size_t kScratchBytes = kScratchPoolOffset + kScratchPoolDoubles * sizeof(double);
static_assert(kScratchPartOffset % 256 == 0 && kScratchPoolOffset % 256 == 0, "scratch regions stay 256-byte aligned");

}  // namespace

// The array itself.  Its name is a host-side stand-in in host code: kernels
// receive the device address that hipGetSymbolAddress returns (scratch_address).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on each device, looked up once per device with
// that device current (every device holds its own copy at its own address).
struct ScratchTable {
  std::mutex mu;
  std::map<int, void*> addr;
  std::map<int, std::string> err;
};
ScratchTable& scratch_table() {
  static ScratchTable t;
  return t;
}

// Called with `device` current.  Returns the address, or nullptr with *why set.
void* scratch_address(int device, std::string* why) {
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> lock(t.mu);
  auto it = t.addr.find(device);
  if (it != t.addr.end()) return it->second;
  auto e = t.err.find(device);
  if (e != t.err.end()) {
    *why = e->second;
    return nullptr;
  }
  void* ptr = nullptr;
  const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (rc != hipSuccess || !ptr) {
    *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc);
    t.err[device] = *why;
    return nullptr;
  }
  t.addr[device] = ptr;
  return ptr;
}

}  // namespace

struct pbcgs_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevState* st = nullptr;   // state slots (device): 0, 1 solver ring; 2, 3 utility reductions
  DevState* hst = nullptr;  // pinned host copies: slots 0, 1 for polling, 2 for reads of a state or a scalar
  int32_t* flag = nullptr;  // structural error flags of utility kernels
  GridBar* bar = nullptr;   // grid barrier of the persistent form
  int64_t* qout = nullptr;  // phases run by the persistent form
  int coop = -1;            // device supports cooperative launches (-1: not asked yet)
  int32_t* hflag = nullptr; // pinned host copy
  double* part = nullptr;   // PB_COUNT buffers of kMaxD * kMaxG partial sums
  double* ws = nullptr;     // solver vectors
  size_t ws_cap = 0;        // doubles
  double* ahat = nullptr;   // values of A M^{-1} (folded Jacobi, CSR)
  size_t ahat_cap = 0;      // doubles
  float* a32 = nullptr;     // binary32 operator values (precision form, CSR)
  size_t a32_cap = 0;       // floats
  void* dia[2] = {nullptr, nullptr};  // values of an operator's diagonal layout for the current solve
  size_t dia_cap[2] = {0, 0};         // bytes (slot 1: the binary64 layout beside a binary32 one)
  void* vi[2] = {nullptr, nullptr};   // value codes and tables of the layouts in dia[] (see DiaViOpT)
  size_t vi_cap[2] = {0, 0};          // bytes
  // batched solves: system table, workgroup map, vectors, states, partials, host poll copies
  SysDesc* bsys = nullptr;
  size_t bsys_cap = 0;
  int32_t* bmap = nullptr;
  size_t bmap_cap = 0;
  double* bws = nullptr;
  size_t bws_cap = 0;
  double* bdia = nullptr;    // every system's diagonal-layout values for the current batch
  size_t bdia_cap = 0;
  DevState* bst = nullptr;
  size_t bst_cap = 0;
  double* bpart = nullptr;
  size_t bpart_cap = 0;
  DevState* bhst = nullptr;  // pinned, two poll slots of bst_cap states
  size_t bhst_cap = 0;
  int32_t batch_gcap = 0;    // per-system workgroup cap chosen by pbcgs_tune_batched (0: 64)
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  hipEvent_t ev_poll[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> kev;  // pool for per-kernel timing
  std::map<std::string, hipGraphExec_t> graphs;
  std::string err;
  unsigned char* scratch = nullptr;  // device address of this device's `scratch` (nullptr: unavailable)
  std::string scratch_err;
  bool noalloc = false;              // inside pbcgs_solve_noalloc: nothing may be allocated
  // test hooks: NaN-fill the workspace before a solve writes it (opts.flags
  // bit 5, for the duration of one call); scale the recursive residual after
  // one iteration (pbcgs_debug_perturb; -1 = off)
  bool poison = false;
  int32_t perturb_iter = -1;
  double perturb_scale = 1.0;
  std::string devkey;  // "<architecture> <compute units>cu": the device part of launch-shape cache keys
};

struct pbcgs_op_s {
  pbcgs_ctx_t ctx = nullptr;
  int kind = OP_CSR;
  int32_t n = 0;
  int64_t nnz = 0;
  const int32_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* va = nullptr;
  int32_t nx = 0, ny = 0, nz = 0;
  int32_t npts = 0;                 // stencil points (5, 7 or 27)
  double coef[27] = {};             // constant stencil coefficients
  const double* vcoef = nullptr;    // OP_GRID: npts * n per-row coefficients (borrowed, device)
  // matrix-free 27-point operator: cell coefficients (borrowed) and the convection terms
  const double* kappa = nullptr;
  double hb[3] = {0, 0, 0};
  double shift = 0.0;
  // rows-per-wave blocks chosen by pbcgs_tune per variant, precision and read
  // path (read_path(); 0: default shape)
  int32_t tuned_R[PBCGS_PIPE_CG + 1][2][3] = {};
  // arrays the library allocated for this operator (a transpose), freed with it
  int32_t* own_rp = nullptr;
  int32_t* own_ci = nullptr;
  double* own_va = nullptr;
  // compact int16 column indices (offsets from the row's 64-row block start),
  // made at creation when every offset fits; owned by the operator
  int16_t* c16 = nullptr;
  // otherwise, with at most 64 distinct diagonals: 16-bit diagonal codes and
  // the 64-entry diagonal table; owned by the operator
  uint16_t* cd = nullptr;
  int32_t* dg = nullptr;
  // diagonal layout (at most kMaxDia diagonals, rows with ascending columns):
  // the per-row masks and the ascending diagonal offsets; owned by the operator
  uint32_t* dmask = nullptr;
  int32_t* ddoff = nullptr;     // the diagonal offsets, on the device
  int32_t ndia = 0;
  int32_t dia_off[kMaxDia] = {};
};

namespace {

int fail(pbcgs_ctx_t ctx, int code, const std::string& msg) {
  g_last_error = msg;
  if (ctx) ctx->err = msg;
  return code;
}

// Keeps the caller's current device; switches to the context's device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define HIP_TRY(ctx, call)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), PBCGS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

// Launch shape: a wave handles R blocks of 64 rows (R a power of two), a
// workgroup 4 R blocks; R is the smallest power of two with at most `gtarget`
// workgroups (default 1024: four workgroups per CU, 8 rows per thread for the
// 128^3 workload).
struct Shape {
  int32_t n, R, G;
};

bool make_shape(int32_t n, Shape* sh, int prefer_R = 0) {
  if (n <= 0) return false;
  int gt = env_int("PBCGS_GTARGET", 1024);
  if (gt < 1 || gt > kMaxG) gt = 1024;
  int forced = env_int("PBCGS_R", 0);
  if (forced <= 0 && !std::getenv("PBCGS_GTARGET")) forced = prefer_R;  // an autotuned shape
  for (int R = 1; R <= kMaxR; R *= 2) {
    const int64_t G = ((int64_t)n + 256 * (int64_t)R - 1) / (256 * (int64_t)R);
    if (forced > 0 && R != forced) continue;
    if (G <= gt || (R == kMaxR && G <= kMaxG) || (forced > 0 && G <= kMaxG)) {
      *sh = {n, R, (int32_t)G};
      return true;
    }
  }
  return false;
}

// ---------------------------------------------------------------------------
// Process-wide launch-shape cache (pbcgs_tune_entry in include/pbcgs.h).
// ---------------------------------------------------------------------------
// The build that measured an entry: a rebuilt library may prefer other shapes.
const char kBuildId[] = __DATE__ " " __TIME__;

struct TuneCache {
  std::mutex mu;
  std::vector<pbcgs_tune_entry> entries;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

bool same_key(const pbcgs_tune_entry& a, const pbcgs_tune_entry& b) {
  return std::strncmp(a.device, b.device, sizeof a.device) == 0 &&
         std::strncmp(a.build, b.build, sizeof a.build) == 0 && a.n == b.n && a.nnz == b.nnz &&
         a.op_kind == b.op_kind && a.variant == b.variant && a.precision == b.precision &&
         a.read_path == b.read_path;
}

// The read path of a solve, part of a tuned shape's key: 0 the operator's
// default (its diagonal layout or compact columns where it has them), 1 the
// CSR arrays (opts.flags bit 4), 2 the caller's int32 columns (bit 3).
int32_t read_path(int32_t flags) { return (flags & 8) ? 2 : (flags & 16) ? 1 : 0; }

// The shape a cache entry holds fits its row count: a power of two R whose
// grid has at most kMaxG workgroups.
bool shape_fits(int32_t n, int32_t R) {
  if (n <= 0 || R < 1 || R > kMaxR || (R & (R - 1)) != 0) return false;
  return ((int64_t)n + 256 * (int64_t)R - 1) / (256 * (int64_t)R) <= kMaxG;
}

// The cached shape for a key (best ignored), or 0.
int32_t cache_find(const pbcgs_tune_entry& key) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  for (const auto& e : c.entries)
    if (same_key(e, key)) return e.best;
  return 0;
}

void cache_store(const pbcgs_tune_entry& e) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto& x : c.entries)
    if (same_key(x, e)) {
      x.best = e.best;
      return;
    }
  c.entries.push_back(e);
}

// The cache key of (device, build, operator, variant, precision, read path); best = 0.
pbcgs_tune_entry make_key(pbcgs_ctx_t ctx, const pbcgs_op_s* A, int32_t variant, int32_t precision, int32_t path) {
  pbcgs_tune_entry e;
  std::memset(&e, 0, sizeof e);
  std::snprintf(e.device, sizeof e.device, "%s", ctx->devkey.c_str());
  std::snprintf(e.build, sizeof e.build, "%s", kBuildId);
  e.n = A->n;
  e.nnz = (A->kind == OP_CSR) ? A->nnz : 0;
  e.op_kind = A->kind;
  e.variant = variant;
  e.precision = precision;
  e.read_path = path;
  return e;
}

// Kernel boundaries of one regular iteration of each variant.
int32_t syncs_per_iteration(int32_t variant) {
  switch (variant) {
    case PBCGS_BICGSTAB: return 5;
    case PBCGS_CA_BICGSTAB: return 4;
    case PBCGS_CG: return 3;
    case PBCGS_PIPE_CG: return 1;
    default: return 2;  // p-BiCGStab, Chronopoulos & Gear CG
  }
}

bool cg_family(int32_t variant) {
  return variant == PBCGS_CG || variant == PBCGS_CGCG || variant == PBCGS_PIPE_CG;
}

// opts.flags bit 2 selects eq. (5) for alpha_{i+1}; eq. (3) otherwise.
int32_t alpha_form(const pbcgs_opts& o) { return (o.flags & 4) ? 5 : 3; }
// opts.flags bit 3 keeps a solve on the caller's int32 column indices.
bool compact_ok(const pbcgs_opts& o) { return (o.flags & 8) == 0; }
// opts.flags bit 4 (or bit 3) keeps a solve on the CSR stream where the operator has a diagonal layout.
bool dia_ok(const pbcgs_opts& o) { return (o.flags & 24) == 0; }

Args base_args(pbcgs_ctx_t ctx, const Shape& sh) {
  Args a;
  std::memset(&a, 0, sizeof a);
  a.n = sh.n;
  a.G = sh.G;
  a.R = sh.R;
  a.Gin = sh.G;
  a.sin = ctx->st;
  a.sout = ctx->st + 1;
  a.wg = -1;           // one system: the workgroup index is blockIdx.x
  a.pstride = kMaxG;
  return a;
}

double* part_buf(pbcgs_ctx_t ctx, int which) { return ctx->part + (size_t)which * kMaxD * kMaxG; }

// With the poisoning hook on, fills `bytes` of a workspace buffer with NaN
// bits (the stream orders it before the kernels that write the buffer).
void poison(pbcgs_ctx_t ctx, void* p, size_t bytes) {
  if (!ctx->poison || !p || bytes < 4) return;
  const int64_t words = (int64_t)(bytes / 4);
  k_poison<<<debug_blocks(words), kDebugWG, 0, ctx->stream>>>(static_cast<uint32_t*>(p), words);
}

// Switches the poisoning hook on for one call (off again on every return).
struct PoisonScope {
  pbcgs_ctx_t c;
  PoisonScope(pbcgs_ctx_t c_, bool on) : c(c_) { c->poison = on; }
  ~PoisonScope() { c->poison = false; }
};

int ensure_ws(pbcgs_ctx_t ctx, size_t doubles) {
  if (ctx->ws_cap >= doubles) return PBCGS_SUCCESS;
  if (ctx->noalloc) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the call may not allocate and its scratch is too small");
  if (ctx->ws) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
  }
  if (hipMalloc(&ctx->ws, doubles * sizeof(double)) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, PBCGS_ERR_ALLOC, "workspace allocation of " + std::to_string(doubles * 8) + " bytes failed");
  }
  ctx->ws_cap = doubles;
  return PBCGS_SUCCESS;
}

int ensure_ahat(pbcgs_ctx_t ctx, size_t doubles) {
  if (ctx->ahat_cap >= doubles) return PBCGS_SUCCESS;
  if (ctx->noalloc) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the call may not allocate and its scratch is too small");
  if (ctx->ahat) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->ahat);
    ctx->ahat = nullptr;
    ctx->ahat_cap = 0;
  }
  if (hipMalloc(&ctx->ahat, std::max<size_t>(doubles, 1) * sizeof(double)) != hipSuccess) {
    ctx->ahat = nullptr;
    return fail(ctx, PBCGS_ERR_ALLOC, "allocation of " + std::to_string(doubles * 8) + " bytes for A M^-1 failed");
  }
  ctx->ahat_cap = doubles;
  return PBCGS_SUCCESS;
}

int ensure_a32(pbcgs_ctx_t ctx, size_t floats) {
  if (ctx->a32_cap >= floats) return PBCGS_SUCCESS;
  if (ctx->noalloc) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the call may not allocate and its scratch is too small");
  if (ctx->a32) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->a32);
    ctx->a32 = nullptr;
    ctx->a32_cap = 0;
  }
  if (hipMalloc(&ctx->a32, std::max<size_t>(floats, 1) * sizeof(float)) != hipSuccess) {
    ctx->a32 = nullptr;
    return fail(ctx, PBCGS_ERR_ALLOC, "allocation of " + std::to_string(floats * 4) + " bytes of binary32 values failed");
  }
  ctx->a32_cap = floats;
  return PBCGS_SUCCESS;
}

int ensure_dia(pbcgs_ctx_t ctx, size_t bytes, int slot) {
  if (ctx->dia_cap[slot] >= bytes) return PBCGS_SUCCESS;
  if (ctx->noalloc) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the call may not allocate and its scratch is too small");
  if (ctx->dia[slot]) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->dia[slot]);
    ctx->dia[slot] = nullptr;
    ctx->dia_cap[slot] = 0;
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
  }
  if (hipMalloc(&ctx->dia[slot], std::max<size_t>(bytes, 8)) != hipSuccess) {
    ctx->dia[slot] = nullptr;
    return fail(ctx, PBCGS_ERR_ALLOC, "allocation of " + std::to_string(bytes) + " bytes of diagonal-layout values failed");
  }
  ctx->dia_cap[slot] = bytes;
  return PBCGS_SUCCESS;
}

// The binary32 twin of an operator: values rounded once.
template <class I>
CsrOpT<float, I> to_binary32(pbcgs_ctx_t ctx, const CsrOpT<double, I>& op, int64_t nnz) {
  if (nnz > 0) {
    const int g = (int)std::min<int64_t>((nnz + kWG - 1) / kWG, 8192);
    k_round_vals<<<g, kWG, 0, ctx->stream>>>(nnz, op.va, ctx->a32);
  }
  return CsrOpT<float, I>{op.rp, op.ci, ctx->a32, op.n, 0, op.dg};
}
template <int NPTS>
StencilOp<NPTS, float> to_binary32(pbcgs_ctx_t, const StencilOp<NPTS, double>& op, int64_t) {
  StencilOp<NPTS, float> f;
  std::memset(&f, 0, sizeof f);
  f.nx = op.nx; f.ny = op.ny; f.nz = op.nz;
  for (int k = 0; k < NPTS; ++k) f.c[k] = float(op.c[k]);
  return f;
}

template <bool F>
Conv27Op<float, F> to_binary32(pbcgs_ctx_t, const Conv27Op<double, F>& op, int64_t) {
  return Conv27Op<float, F>{op.n, op.upneg, op.kappa, op.dscale, {op.hab[0], op.hab[1], op.hab[2]}, op.hsum, op.shift};
}
inline GridOp<float, false> to_binary32(pbcgs_ctx_t, const GridOp<double, false>& op, int64_t) {
  GridOp<float, false> f;
  std::memset(&f, 0, sizeof f);
  f.nx = op.nx; f.ny = op.ny; f.nz = op.nz; f.npts = op.npts;
  for (int k = 0; k < 27; ++k) f.c[k] = float(op.c[k]);
  return f;
}
// per-row coefficients rounded once into the context's binary32 values (room
// for npts * n made by the caller)
inline GridOp<float, true> to_binary32(pbcgs_ctx_t ctx, const GridOp<double, true>& op, int64_t) {
  const int64_t cnt = (int64_t)op.npts * op.nx * op.ny * op.nz;
  const int g = (int)std::min<int64_t>((cnt + kWG - 1) / kWG, 8192);
  k_round_vals<<<g, kWG, 0, ctx->stream>>>(cnt, op.cf, ctx->a32);
  GridOp<float, true> f;
  std::memset(&f, 0, sizeof f);
  f.cf = ctx->a32;
  f.nx = op.nx; f.ny = op.ny; f.nz = op.nz; f.npts = op.npts;
  return f;
}

size_t padded(int32_t n) { return ((size_t)n + 63) / 64 * 64; }

// Reads go through the context's pinned slot 2 (no pageable staging).
int read_state(pbcgs_ctx_t ctx, int slot, DevState* out) {
  HIP_TRY(ctx, hipMemcpyAsync(&ctx->hst[2], ctx->st + slot, sizeof(DevState), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = ctx->hst[2];
  return PBCGS_SUCCESS;
}

int read_double(pbcgs_ctx_t ctx, const double* dev, double* out) {
  HIP_TRY(ctx, hipMemcpyAsync(&ctx->hst[2].result, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = ctx->hst[2].result;
  return PBCGS_SUCCESS;
}

// A kernel, not a memset, clears the flag word.
int reset_flag(pbcgs_ctx_t ctx) {
  k_clear_flag<<<1, 64, 0, ctx->stream>>>(ctx->flag);
  HIP_TRY(ctx, hipGetLastError());
  return PBCGS_SUCCESS;
}

int read_flag(pbcgs_ctx_t ctx, int32_t* out) {
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hflag, ctx->flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = *ctx->hflag;
  return PBCGS_SUCCESS;
}

int map_status(int32_t ds) {
  switch (ds) {
    case DS_SUCCESS: return PBCGS_SUCCESS;
    case DS_BREAKDOWN: return PBCGS_BREAKDOWN;
    case DS_NONFINITE: return PBCGS_NONFINITE;
    default: return PBCGS_MAXIT;
  }
}

// Residual replacement schedule (Section 4.2): iteration i replaces r, r^, w
// when (i+1) mod k == 0 and fewer than rr_max replacements came before.
bool rr_due(const pbcgs_opts& o, int64_t i) {
  if (o.variant != PBCGS_PBICGSTAB_RR || o.rr_period <= 0 || i < 0) return false;
  if ((i + 1) % o.rr_period != 0) return false;
  const int64_t before = (i + 1) / o.rr_period - 1;
  return o.rr_max < 0 || before < o.rr_max;
}

// Total of a utility reduction (k_dot / k_true_res partials), via state slot 1.
int finish_sum(pbcgs_ctx_t ctx, const Shape& sh, double* result) {
  Args f = base_args(ctx, sh);
  f.pin = part_buf(ctx, PB_UTIL);
  f.Gin = sh.G;
  f.sin = ctx->st + 2;  // slots 2, 3: utility reductions leave a solve's state alone
  f.sout = ctx->st + 3;
  k_init_state<<<1, 64, 0, ctx->stream>>>(ctx->st + 2, 0.0);
  k_finish<3><<<1, kWG, 0, ctx->stream>>>(f);
  HIP_TRY(ctx, hipGetLastError());
  DevState h;
  int rc = read_state(ctx, 3, &h);
  if (rc != PBCGS_SUCCESS) return rc;
  *result = h.result;
  return PBCGS_SUCCESS;
}

// ||b - A x|| / rho0 in the pairwise arithmetic of the method (0 when rho0 = 0).
template <class Op>
int true_relres(pbcgs_ctx_t ctx, const Op& op, const Args& a0, double rho0, double* out) {
  Args t = a0;
  t.pout = part_buf(ctx, PB_UTIL);
  k_true_res<Op><<<t.G, kWG, 0, ctx->stream>>>(op, t);
  HIP_TRY(ctx, hipGetLastError());
  const Shape sh = {a0.n, a0.R, a0.G};
  double nr = 0.0;
  const int rc = finish_sum(ctx, sh, &nr);
  if (rc != PBCGS_SUCCESS) return rc;
  *out = (rho0 > 0.0) ? std::sqrt(nr) / rho0 : 0.0;
  return PBCGS_SUCCESS;
}

// ---------------------------------------------------------------------------
// Per-(operator, preconditioner) driver.
// ---------------------------------------------------------------------------
// MP: precision form (Op is the binary32 operator, Op64 the binary64 one).
template <class Op, int PC, class Op64 = Op, bool MP = false>
struct Driver {
  pbcgs_ctx_t ctx;
  Op op;
  Op64 op64;
  Args a;
  const pbcgs_opts& o;
  bool timing = false;
  bool true_res = true;  // false: the caller computes relres_true itself
  double rho0 = 0.0;     // ||r_0|| of the finished solve
  int64_t q = 0;  // kernel launches of this solve that passed the state on
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[2];
  size_t ev_used = 0;
  std::vector<int64_t> forced;  // precision form: iterations ended by a forced replacement

  Driver(pbcgs_ctx_t c, Op op_, const Args& a_, const pbcgs_opts& o_) : ctx(c), op(op_), op64(), a(a_), o(o_) {
    a.aform = alpha_form(o);
  }
  Driver(pbcgs_ctx_t c, Op op_, Op64 op64_, const Args& a_, const pbcgs_opts& o_)
      : ctx(c), op(op_), op64(op64_), a(a_), o(o_) {
    a.aform = alpha_form(o);
  }

  bool was_forced(int64_t i) const { return std::find(forced.begin(), forced.end(), i) != forced.end(); }
  // iteration i starts with the second half of a replacement
  bool pending_rr(int64_t i) const { return rr_due(o, i - 1) || (MP && was_forced(i - 1)); }

  hipEvent_t next_event() {
    if (ev_used == ctx->kev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ctx->kev.push_back(e);
    }
    return ctx->kev[ev_used++];
  }

  template <class F>
  void timed(int slot, F launch) {
    if (!timing) { launch(); return; }
    hipEvent_t e0 = next_event(), e1 = next_event();
    if (e0 && e1) (void)hipEventRecord(e0, ctx->stream);
    launch();
    if (e0 && e1) {
      (void)hipEventRecord(e1, ctx->stream);
      tev[slot].push_back({e0, e1});
    }
  }

  // Arguments of the next launch: state slots by launch parity, partials.
  Args L(int pin, int pout, bool first = false, int mode = 0) {
    Args b = a;
    b.mode = mode;
    b.sin = ctx->st + (q & 1);
    b.sout = ctx->st + ((q + 1) & 1);
    b.pin = pin >= 0 ? part_buf(ctx, pin) : nullptr;
    b.pout = pout >= 0 ? part_buf(ctx, pout) : nullptr;
    b.Gin = a.G;
    b.first = first ? 1 : 0;
    ++q;
    return b;
  }

  dim3 grid() const { return dim3((unsigned)a.G); }

  // the unpreconditioned binary64 BiCGStab kernels likewise, and the p-BiCGStab
  // ones on the diagonal layout and on a stencil with an even x extent, whose
  // two rows share their y / z neighbours' lines (aligned pairs; measured at
  // 128^3: 72.9 against 74.5 us per iteration; with an odd extent they gain
  // nothing); PBCGS_TWO_ROWS64=0 turns all of them off
  bool two_rows64() const {
    if constexpr (!MP && PC == PC_NONE && HasSpmv2<Op>::value) {
      if (o.variant != PBCGS_BICGSTAB && !IsDia<Op>::value) {
        if constexpr (IsStencil<Op>::value || IsGrid<Op>::value) {
          if ((op.nx & 1) != 0) return false;
        } else {
          return false;
        }
      }
      return a.R >= 2 && env_int("PBCGS_TWO_ROWS64", 1) != 0;
    }
    return false;
  }

  // the CG family's product kernels (CG's s = A p, the w = A u of Algorithms 4
  // and 6, p-CG's iteration kernel) take two rows per lane on the layout and
  // on stencils with an even x extent (PBCGS_TWO_ROWS64=0 turns it off)
  bool cg_two_rows() const {
    if constexpr (!MP && HasSpmv2<Op>::value) {
      if constexpr (IsStencil<Op>::value || IsGrid<Op>::value) {
        if ((op.nx & 1) != 0) return false;
      } else if constexpr (!IsDia<Op>::value) {
        return false;
      }
      return a.R >= 2 && env_int("PBCGS_TWO_ROWS64", 1) != 0;
    }
    return false;
  }

  // the binary32 kernels take two rows per lane when the operator supports it
  // and every wave owns at least two 64-row blocks (PBCGS_TWO_ROWS=0 turns it off)
  bool two_rows() const {
    if constexpr (MP && HasSpmv2<Op>::value) return a.R >= 2 && env_int("PBCGS_TWO_ROWS", 1) != 0;
    return false;
  }
  // the binary32 fused kernels take four rows per lane (16-byte vector
  // accesses) when the operator supports it and every wave owns at least four
  // 64-row blocks (PBCGS_FOUR_ROWS=0 turns it off; then two rows per lane)
  bool four_rows() const {
    if constexpr (MP && HasSpmv4<Op>::value) return a.R >= 4 && env_int("PBCGS_FOUR_ROWS", 1) != 0;
    return false;
  }
  // the replacement steps of the binary32 form with two rows per lane too
  // (their binary64 operator has the two-row product)
  bool two_rows_rr() const {
    if constexpr (MP && HasSpmv2<Op>::value && HasSpmv2<Op64>::value) return two_rows();
    return false;
  }
  void launch_rr_w() {
    hipStream_t s = ctx->stream;
    if constexpr (MP && HasSpmv2<Op64>::value) {
      if (two_rows_rr()) {
        k_mp_rr_w2<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, PB_B));
        return;
      }
    }
    k_mp_rr_w<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, PB_B));
  }

  void setup() {
    hipStream_t s = ctx->stream;
    if constexpr (MP) {
      k_mp_setup_r0<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, PB_SETUP1));
      k_mp_setup_w0<Op64><<<grid(), kWG, 0, s>>>(op64, L(PB_SETUP1, PB_SETUP2));
    } else if (o.variant == PBCGS_BICGSTAB) {
      k_setup_r0<Op, PC, false><<<grid(), kWG, 0, s>>>(op, L(-1, PB_SETUP1));
    } else if (o.variant == PBCGS_CG) {
      k_cg_setup<Op, PC, false><<<grid(), kWG, 0, s>>>(op, L(-1, PB_SETUP1));
    } else if (o.variant == PBCGS_CGCG || o.variant == PBCGS_PIPE_CG) {
      k_cg_setup<Op, PC, true><<<grid(), kWG, 0, s>>>(op, L(-1, PB_SETUP1));
      launch_cg_setup_w(o.variant == PBCGS_PIPE_CG, L(-1, PB_SETUP2));
    } else {
      k_setup_r0<Op, PC, true><<<grid(), kWG, 0, s>>>(op, L(-1, PB_SETUP1));
      k_setup_w0<Op, PC><<<grid(), kWG, 0, s>>>(op, L(PB_SETUP1, PB_SETUP2));
    }
  }

  // w = A u of Algorithms 4 and 6 (PIPE: Algorithm 6), one or two rows per lane
  void launch_cg_setup_w(bool pipe, const Args& b) {
    hipStream_t s = ctx->stream;
    if constexpr (!MP && HasSpmv2<Op>::value) {
      if (cg_two_rows()) {
        if (pipe) k_cg_setup_w<Op, PC, true, true><<<grid(), kWG, 0, s>>>(op, b);
        else k_cg_setup_w<Op, PC, false, true><<<grid(), kWG, 0, s>>>(op, b);
        return;
      }
    }
    if (pipe) k_cg_setup_w<Op, PC, true><<<grid(), kWG, 0, s>>>(op, b);
    else k_cg_setup_w<Op, PC, false><<<grid(), kWG, 0, s>>>(op, b);
  }

  // Kernels of iteration i.
  void iteration(int64_t i) {
    hipStream_t s = ctx->stream;
    if constexpr (MP) {
      const bool pending = pending_rr(i), recheck = was_forced(i - 1), rr = rr_due(o, i);
      if (pending) {
        k_mp_rr_p<<<grid(), kWG, 0, s>>>(L(PB_B, -1, false, recheck ? 1 : 0));
        bool done = false;
        if constexpr (HasSpmv2<Op>::value && HasSpmv2<Op64>::value) {
          if (two_rows_rr()) {
            k_mp_rr_s2<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, -1));
            k_mp_pa2_rr<Op, Op64><<<grid(), kWG, 0, s>>>(op, op64, L(-1, PB_A));
            done = true;
          }
        }
        if (!done) {
          k_mp_rr_s<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, -1));
          k_mp_pa<Op, Op64, true><<<grid(), kWG, 0, s>>>(op, op64, L(-1, PB_A));
        }
      } else {
        timed(0, [&] {
          if (four_rows()) {
            if constexpr (HasSpmv4<Op>::value)
              k_mp_pa4<Op><<<grid(), kWG, 0, s>>>(op, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
          } else if (two_rows()) {
            if constexpr (HasSpmv2<Op>::value)
              k_mp_pa2<Op><<<grid(), kWG, 0, s>>>(op, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
          } else {
            k_mp_pa<Op, Op64, false><<<grid(), kWG, 0, s>>>(op, op64, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
          }
        });
      }
      if (rr) {
        k_mp_rr_x<<<grid(), kWG, 0, s>>>(L(PB_A, -1));
        k_mp_rr_r<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, -1));
        launch_rr_w();
      } else {
        timed(1, [&] {
          if (four_rows()) {
            if constexpr (HasSpmv4<Op>::value) k_mp_pb4<Op><<<grid(), kWG, 0, s>>>(op, L(PB_A, PB_B));
          } else if (two_rows()) {
            if constexpr (HasSpmv2<Op>::value) k_mp_pb2<Op><<<grid(), kWG, 0, s>>>(op, L(PB_A, PB_B));
          } else {
            k_mp_pb<Op><<<grid(), kWG, 0, s>>>(op, L(PB_A, PB_B));
          }
        });
      }
    } else {
      iteration64(i);
    }
  }

  // Kernels of iteration i of the binary64 solvers.
  void iteration64(int64_t i) {
    hipStream_t s = ctx->stream;
    if constexpr (PC == PC_NONE) {
      if (o.variant == PBCGS_CA_BICGSTAB) {
        k_ca_ps<<<grid(), kWG, 0, s>>>(L(i == 0 ? PB_SETUP2 : PB_B, -1, i == 0));
        timed(0, [&] { k_ca_z<Op><<<grid(), kWG, 0, s>>>(op, L(-1, PB_A)); });
        k_ca_x<<<grid(), kWG, 0, s>>>(L(PB_A, -1));
        timed(1, [&] { k_ca_w<Op><<<grid(), kWG, 0, s>>>(op, L(-1, PB_B)); });
        return;
      }
    }
    if (o.variant == PBCGS_CG) {
      timed(0, [&] {
        const Args b = L(i == 0 ? PB_SETUP1 : -1, PB_A, i == 0);
        if constexpr (!MP && HasSpmv2<Op>::value) {
          if (cg_two_rows()) {
            k_cg_a<Op, true><<<grid(), kWG, 0, s>>>(op, b);
            return;
          }
        }
        k_cg_a<Op><<<grid(), kWG, 0, s>>>(op, b);
      });
      timed(1, [&] { k_cg_b<PC><<<grid(), kWG, 0, s>>>(L(PB_A, PB_B)); });
      k_cg_c<PC><<<grid(), kWG, 0, s>>>(L(PB_B, -1));
      return;
    }
    if (o.variant == PBCGS_CGCG) {
      timed(0, [&] { k_cc_a<PC><<<grid(), kWG, 0, s>>>(L(i == 0 ? PB_SETUP2 : PB_B, -1, i == 0)); });
      timed(1, [&] { launch_cg_setup_w(false, L(-1, PB_B)); });
      return;
    }
    if (o.variant == PBCGS_PIPE_CG) {
      // iteration i gathers m_i (w_i without a preconditioner) from one buffer
      // and writes m_{i+1} to the other; the partial sums alternate likewise
      Args b = L(pcg_part(i), pcg_part(i + 1), i == 0);
      if (i & 1) std::swap(b.wh, b.t);
      timed(0, [&] {
        if constexpr (!MP && HasSpmv2<Op>::value) {
          if (cg_two_rows()) {
            k_pcg2<Op, PC><<<grid(), kWG, 0, s>>>(op, b);
            return;
          }
        }
        k_pcg<Op, PC><<<grid(), kWG, 0, s>>>(op, b);
      });
      return;
    }
    if (o.variant == PBCGS_BICGSTAB) {
      if (two_rows64()) {
        if constexpr (PC == PC_NONE && HasSpmv2<Op>::value) {
          timed(0, [&] { k_b1_2<Op><<<grid(), kWG, 0, s>>>(op, L(PB_SETUP1, PB_B1, i == 0)); });
          k_b2_2<<<grid(), kWG, 0, s>>>(L(PB_B1, -1));
          timed(1, [&] { k_b3_2<Op><<<grid(), kWG, 0, s>>>(op, L(-1, PB_B3)); });
          k_b4_2<<<grid(), kWG, 0, s>>>(L(PB_B3, PB_B4));
          k_b5_2<<<grid(), kWG, 0, s>>>(L(PB_B4, -1));
        }
        return;
      }
      timed(0, [&] { k_b1<Op, PC><<<grid(), kWG, 0, s>>>(op, L(PB_SETUP1, PB_B1, i == 0)); });
      k_b2<PC><<<grid(), kWG, 0, s>>>(L(PB_B1, -1));
      timed(1, [&] { k_b3<Op, PC><<<grid(), kWG, 0, s>>>(op, L(-1, PB_B3)); });
      k_b4<PC><<<grid(), kWG, 0, s>>>(L(PB_B3, PB_B4));
      k_b5<PC><<<grid(), kWG, 0, s>>>(L(PB_B4, -1));
      return;
    }
    const bool pending = rr_due(o, i - 1);
    const bool rr = rr_due(o, i);
    if (pending) {
      k_rr_p<PC><<<grid(), kWG, 0, s>>>(L(PB_B, -1));
      k_rr_s<Op, PC><<<grid(), kWG, 0, s>>>(op, L(-1, -1));
      k_pa<Op, PC, true><<<grid(), kWG, 0, s>>>(op, L(-1, PB_A));
    } else {
      timed(0, [&] {
        if (two_rows64()) {
          if constexpr (PC == PC_NONE && HasSpmv2<Op>::value)
            k_pa2<Op><<<grid(), kWG, 0, s>>>(op, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
        } else {
          k_pa<Op, PC, false><<<grid(), kWG, 0, s>>>(op, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
        }
      });
    }
    if (rr) {
      k_rr_x<PC><<<grid(), kWG, 0, s>>>(L(PB_A, -1));
      k_rr_r<Op, PC><<<grid(), kWG, 0, s>>>(op, L(-1, -1));
      k_rr_w<Op, PC><<<grid(), kWG, 0, s>>>(op, L(-1, PB_B));
    } else {
      timed(1, [&] {
        if (two_rows64()) {
          if constexpr (PC == PC_NONE && HasSpmv2<Op>::value) k_pb2<Op><<<grid(), kWG, 0, s>>>(op, L(PB_A, PB_B));
        } else {
          k_pb<Op, PC><<<grid(), kWG, 0, s>>>(op, L(PB_A, PB_B));
        }
      });
    }
    // test hook: r_{i+1} scaled after the iteration's reductions were taken
    // (the next kernels read the scaled r; the state is not touched)
    if (i == ctx->perturb_iter) k_scale_vec<<<debug_blocks(a.n), kDebugWG, 0, s>>>(a.r, a.n, ctx->perturb_scale);
  }

  // Launch count of iteration i (the schedule of iteration()).
  void count_iteration(int64_t i) {
    if (o.variant == PBCGS_BICGSTAB) {
      q += 5;
      return;
    }
    if (o.variant == PBCGS_CA_BICGSTAB) {
      q += 4;
      return;
    }
    if (o.variant == PBCGS_CG || o.variant == PBCGS_CGCG || o.variant == PBCGS_PIPE_CG) {
      q += (o.variant == PBCGS_CG) ? 3 : (o.variant == PBCGS_CGCG) ? 2 : 1;
      return;
    }
    q += (pending_rr(i) ? 3 : 1) + (rr_due(o, i) ? 3 : 1);
  }

  // The reduction left pending by the last kernel, finished by one workgroup.
  void finish(int64_t iters_launched) {
    hipStream_t s = ctx->stream;
    if constexpr (MP) {
      if (iters_launched == 0) k_mp_finish<1><<<1, kWG, 0, s>>>(L(PB_SETUP2, -1));
      else k_mp_finish<0><<<1, kWG, 0, s>>>(L(PB_B, -1, false, was_forced(iters_launched - 1) ? 1 : 0));
      return;
    } else {
      finish64(iters_launched);
    }
  }

  // partial-sum buffer holding the reduction that p-CG's iteration i consumes
  static int pcg_part(int64_t i) { return i == 0 ? PB_SETUP2 : ((i & 1) ? PB_A : PB_B); }

  void finish64(int64_t iters_launched) {
    hipStream_t s = ctx->stream;
    if (o.variant == PBCGS_CG) {
      if (iters_launched == 0) k_cg_finish<0><<<1, kWG, 0, s>>>(L(PB_SETUP1, -1));
      return;
    }
    if (o.variant == PBCGS_CGCG || o.variant == PBCGS_PIPE_CG) {
      const int pin = (o.variant == PBCGS_CGCG) ? (iters_launched == 0 ? PB_SETUP2 : PB_B) : pcg_part(iters_launched);
      if (iters_launched == 0) k_cg_finish<1><<<1, kWG, 0, s>>>(L(pin, -1));
      else k_cg_finish<2><<<1, kWG, 0, s>>>(L(pin, -1));
      return;
    }
    if (o.variant == PBCGS_BICGSTAB) {
      if (iters_launched == 0) k_finish<2><<<1, kWG, 0, s>>>(L(PB_SETUP1, -1));
      return;
    }
    if (iters_launched == 0) k_finish<1><<<1, kWG, 0, s>>>(L(PB_SETUP2, -1));
    else k_finish<0><<<1, kWG, 0, s>>>(L(PB_B, -1));
  }

  std::string graph_key(int64_t i0, int m) const {
    std::string k;
    char buf[96];
    k.append(reinterpret_cast<const char*>(&a), sizeof(Args));
    k.append(reinterpret_cast<const char*>(&op), sizeof(Op));
    k.append(reinterpret_cast<const char*>(&op64), sizeof(Op64));
    // the kernel forms the environment selects are part of the schedule
    std::snprintf(buf, sizeof buf, "|%d|%d|%d|%d|%lld|%d|%d|%d%d%d%d|", PC, MP ? 1 : 0, o.variant, m,
                  (long long)(q & 1), i0 == 0 ? 1 : 0, (int)(i0 & 1), four_rows() ? 1 : 0, two_rows() ? 1 : 0,
                  two_rows64() ? 1 : 0, cg_two_rows() ? 1 : 0);
    k += buf;
    for (int j = 0; j < m; ++j) {
      const int64_t i = i0 + j;
      const int code = (pending_rr(i) ? 1 : 0) | (rr_due(o, i) ? 2 : 0) | (MP && was_forced(i - 1) ? 4 : 0);
      k += char('0' + code);
    }
    return k;
  }

  int chunk(int64_t i0, int m, bool use_graph) {
    if (!use_graph) {
      for (int j = 0; j < m; ++j) iteration(i0 + j);
      HIP_TRY(ctx, hipGetLastError());
      return PBCGS_SUCCESS;
    }
    const std::string key = graph_key(i0, m);
    const int64_t q0 = q;
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      if (ctx->graphs.size() >= 32) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
        ctx->graphs.clear();
      }
      hipGraph_t g = nullptr;
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      for (int j = 0; j < m; ++j) iteration(i0 + j);
      hipError_t ce = hipStreamEndCapture(ctx->stream, &g);
      if (ce != hipSuccess) return fail(ctx, PBCGS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
      hipGraphExec_t ex = nullptr;
      hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(ctx, PBCGS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
      it = ctx->graphs.emplace(key, ex).first;
    } else {
      // replaying: advance the launch counter as the captured launches did
      q = q0;
      for (int j = 0; j < m; ++j) count_iteration(i0 + j);
    }
    HIP_TRY(ctx, hipGraphLaunch(it->second, ctx->stream));
    return PBCGS_SUCCESS;
  }

  // The persistent form (binary64, no per-kernel timing), on request only
  // (PBCGS_PERSIST=1): measured on MI355X, a grid barrier -- an agent-scope
  // release per workgroup, which writes back the per-XCD L2 caches -- costs
  // more than a kernel boundary between graph-launched kernels, and more the
  // larger the grid, so the graph schedule is the default at every size.
  bool use_persistent() {
    if constexpr (MP) return false;
    if (ctx->noalloc) return false;
    if (o.flags & 2) return false;
    if (o.variant >= PBCGS_CA_BICGSTAB) return false;
    if (o.maxit > 200000) return false;
    if (ctx->perturb_iter >= 0) return false;
    if (env_int("PBCGS_PERSIST", 0) != 1) return false;
    if (ctx->coop < 0) {
      int v = 0;
      ctx->coop = (hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, ctx->device) == hipSuccess && v) ? 1 : 0;
    }
    if (ctx->coop != 1) return false;
    // every workgroup must be resident at once
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_persist<Op, PC>), kWG,
                                                     0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
      return false;
    return (int64_t)a.G <= (int64_t)per_cu * cus;
  }

  int run_persistent(pbcgs_info* info) {
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_start, s));
    k_init_state<<<1, 64, 0, s>>>(ctx->st, o.tol);
    HIP_TRY(ctx, hipMemsetAsync(ctx->bar, 0, sizeof(GridBar), s));
    PersistCfg c;
    c.st = ctx->st;
    c.parts = ctx->part;
    c.bar = ctx->bar;
    c.qout = ctx->qout;
    c.variant = o.variant;
    c.rr_period = o.rr_period;
    c.rr_max = o.rr_max;
    c.maxit = o.maxit;
    Args base = a;
    void* args[] = {&op, &base, &c};
    HIP_TRY(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_persist<Op, PC>), dim3((unsigned)a.G),
                                            dim3(kWG), args, 0, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_stop, s));
    GridBar hb;
    int64_t hq = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hb, ctx->bar, sizeof hb, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(&hq, ctx->qout, sizeof hq, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hb.err) return fail(ctx, PBCGS_ERR_HIP, "persistent solve: a grid barrier timed out");
    q = hq;
    DevState fin;
    int rc = read_state(ctx, (int)(q & 1), &fin);
    if (rc != PBCGS_SUCCESS) return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop);
    return report(info, fin, ms);
  }

  int run(pbcgs_info* info) {
    if constexpr (!MP) {  // the precision form has no persistent kernel (and instantiates none)
      if (use_persistent()) return run_persistent(info);
    }
    // graphs are instantiated (allocated) on first use: never without allocation
    const bool use_graph = !(o.flags & 1) && !(o.flags & 2) && !ctx->noalloc && ctx->perturb_iter < 0;
    timing = (o.flags & 2) != 0 && !ctx->noalloc;
    const int check = o.check_every > 0 ? o.check_every : (a.n >= (1 << 20) ? 8 : 32);
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_start, s));
    k_init_state<<<1, 64, 0, s>>>(ctx->st, o.tol);
    q = 0;
    setup();
    HIP_TRY(ctx, hipGetLastError());
    // Chunks of at most `check` iterations; the status after chunk c is polled
    // while chunk c+1 is already queued, so the device does not wait for the
    // host.  Near the end the chunks shrink: the observed convergence rate of
    // ||r_i|| / ||r_0|| predicts how many iterations remain, so few kernels
    // are queued past the stop (those see the final status and exit at once).
    int64_t launched = 0;
    int pend[2];
    int next_slot = 0;
    double last_rel = 1.0;
    int64_t last_it = 0;
    double rate = 0.0;  // d log(relres) / d iteration, < 0 when converging
    DevState fin;
    for (;;) {  // the precision form comes back here after a forced replacement
      int npend = 0;
      bool stop = false;
      for (;;) {
        while (!stop && launched < o.maxit && npend < 2) {
          int m = (int)std::min<int64_t>(check, o.maxit - launched);
          if (rate < 0.0 && o.tol > 0.0 && last_rel > 0.0) {
            const double need = (std::log(o.tol) - std::log(last_rel)) / rate;  // from the last poll
            const int64_t ahead = launched - last_it;                           // queued since then
            const int64_t left = (int64_t)std::ceil(need) - ahead;
            if (left < m) m = (int)std::max<int64_t>(1, left);
          }
          int rc = chunk(launched, m, use_graph);
          if (rc != PBCGS_SUCCESS) return rc;
          launched += m;
          HIP_TRY(ctx, hipMemcpyAsync(&ctx->hst[next_slot], ctx->st + (q & 1), sizeof(DevState),
                                      hipMemcpyDeviceToHost, s));
          HIP_TRY(ctx, hipEventRecord(ctx->ev_poll[next_slot], s));
          pend[npend++] = next_slot;
          next_slot ^= 1;
        }
        if (npend == 0) break;
        const int slot = pend[0];
        pend[0] = pend[1];
        --npend;
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev_poll[slot]));
        const DevState& h = ctx->hst[slot];
        if (h.status != DS_RUNNING) {
          stop = true;
        } else if (h.iters > last_it && h.relres > 0.0 && last_rel > 0.0) {
          const double r = (std::log(h.relres) - std::log(last_rel)) / (double)(h.iters - last_it);
          rate = (rate < 0.0) ? 0.5 * (rate + r) : r;
          last_rel = h.relres;
          last_it = h.iters;
        }
      }
      finish(launched);
      HIP_TRY(ctx, hipGetLastError());
      int rc = read_state(ctx, (int)(q & 1), &fin);
      if (rc != PBCGS_SUCCESS) return rc;
      if constexpr (MP) {
        if (fin.status == DS_CHECK) {
          // the binary32 recursive residual passed tol: confirm in binary64
          double tr = 0.0;
          rc = true_relres(ctx, op64, a, fin.rho0, &tr);
          if (rc != PBCGS_SUCCESS) return rc;
          if (tr <= o.tol) {
            fin.status = DS_SUCCESS;
            break;
          }
          // not yet: replace r, w now and go on (s, z follow in the next iteration)
          k_resume<<<1, 64, 0, s>>>(ctx->st + (q & 1));
          k_mp_rr_r<Op64><<<grid(), kWG, 0, s>>>(op64, L(-1, -1));
          launch_rr_w();
          HIP_TRY(ctx, hipGetLastError());
          forced.push_back((int64_t)fin.iters - 1);
          launched = fin.iters;
          last_it = fin.iters;  // predict the remaining iterations from the true residual
          last_rel = tr;
          continue;
        }
      }
      break;
    }
    HIP_TRY(ctx, hipEventRecord(ctx->ev_stop, s));
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev_stop));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop);
    return report(info, fin, ms);
  }

  // Fills info from the final state (and the true residual of the returned x).
  int report(pbcgs_info* info, const DevState& fin, float ms) {
    int rc = PBCGS_SUCCESS;
    rho0 = fin.rho0;
    if (true_res) {  // true residual of the returned x, same pairwise arithmetic (binary64)
      if constexpr (MP) rc = true_relres(ctx, op64, a, fin.rho0, &info->relres_true);
      else rc = true_relres(ctx, op, a, fin.rho0, &info->relres_true);
      if (rc != PBCGS_SUCCESS) return rc;
    }
    info->iters = fin.iters;
    info->n_rr = fin.n_rr;
    info->status = map_status(fin.status);
    info->syncs_per_iter = syncs_per_iteration(o.variant);
    info->relres_rec = fin.relres;
    info->ms = ms;
    info->rows_per_wave_blocks = a.R;
    info->workgroups = a.G;
    for (int k = 0; k < 2; ++k) {
      double tot = 0.0;
      for (auto& pr : tev[k]) {
        float e = 0.f;
        if (hipEventElapsedTime(&e, pr.first, pr.second) == hipSuccess) tot += e;
      }
      info->kernel_ms[k] = tot;
      info->kernel_calls[k] = (int32_t)tev[k].size();
    }
    return info->status;
  }
};

// Graph keys hold the bytes of the operator and argument structs, so these
// structs must have no padding (whose contents would be indeterminate).
static_assert(sizeof(CsrOp) == 4 * sizeof(void*) + 2 * sizeof(int32_t), "CsrOp padding");
static_assert(sizeof(CsrOp16) == sizeof(CsrOp) && sizeof(CsrOp32) == sizeof(CsrOp) &&
              sizeof(CsrOp16f) == sizeof(CsrOp) && sizeof(CsrOpDg) == sizeof(CsrOp) &&
              sizeof(CsrOpDgf) == sizeof(CsrOp), "CsrOpT padding");
static_assert(sizeof(StencilOp<7>) == 4 * sizeof(int32_t) + 7 * sizeof(double), "StencilOp padding");
static_assert(sizeof(StencilOp<5>) == 4 * sizeof(int32_t) + 5 * sizeof(double), "StencilOp padding");
static_assert(sizeof(StencilOp<7, float>) == 4 * sizeof(int32_t) + 7 * sizeof(float), "StencilOp padding");
static_assert(sizeof(StencilOp<5, float>) == 4 * sizeof(int32_t) + 5 * sizeof(float), "StencilOp padding");
static_assert(sizeof(GridOp<double, true>) == sizeof(void*) + 4 * sizeof(int32_t) + 8 &&
              sizeof(GridOp<float, true>) == sizeof(GridOp<double, true>) &&
              sizeof(GridOp<double, false>) == sizeof(void*) + 4 * sizeof(int32_t) + 27 * sizeof(double) &&
              sizeof(GridOp<float, false>) == sizeof(void*) + 4 * sizeof(int32_t) + 28 * sizeof(float),
              "GridOp padding");
static_assert(sizeof(DiaOp) == 2 * sizeof(void*) + (4 + kMaxDia) * sizeof(int32_t) && sizeof(DiaOpF) == sizeof(DiaOp),
              "DiaOpT padding");
static_assert(sizeof(Conv27) == 2 * sizeof(int32_t) + 2 * sizeof(void*) + 5 * sizeof(double) &&
              sizeof(Conv27Op<float, true>) == sizeof(Conv27), "Conv27Op padding");

// The matrix-free 27-point operator of A (kind OP_CV27).
Conv27 conv27_of(pbcgs_op_t A) {
  Conv27 c;
  std::memset(&c, 0, sizeof c);
  c.n = A->nx;
  c.kappa = A->kappa;
  for (int ax = 0; ax < 3; ++ax) {
    c.hab[ax] = std::fabs(A->hb[ax]);
    if (A->hb[ax] >= 0.0) c.upneg |= 1 << ax;
  }
  c.hsum = (c.hab[0] + c.hab[1]) + c.hab[2];
  c.shift = A->shift;
  return c;
}

// Values an operator stores per solve in its folded or binary32 form: a CSR
// operator's non-zeros, a stencil's per-row coefficients; 0 for the others.
int64_t stored_values(const pbcgs_op_s* A) {
  if (A->kind == OP_CSR) return A->nnz;
  if (A->kind == OP_GRID) return (int64_t)A->npts * A->n;
  return 0;
}

// A stencil with one set of constant coefficients, and its centre coefficient.
bool const_stencil(const pbcgs_op_s* A) { return A->kind == OP_ST5 || A->kind == OP_ST7 || A->kind == OP_ST27; }
double stencil_centre(const pbcgs_op_s* A) { return A->coef[A->kind == OP_ST27 ? 13 : (A->kind == OP_ST7 ? 3 : 2)]; }

// f(op) with the operator's device form: for CSR the compact copy the
// operator holds (int16 block offsets or diagonal codes) when `compact`
// allows, else the int32 columns.
template <class F>
int with_op(pbcgs_op_t A, F f, bool compact = true) {
  if (A->kind == OP_CSR) {
    if (compact && A->c16) return f(CsrOp16{A->rp, A->c16, A->va, A->n});
    if (compact && A->cd) return f(CsrOpDg{A->rp, A->cd, A->va, A->n, 0, A->dg});
    return f(CsrOp{A->rp, A->ci, A->va, A->n});
  }
  if (A->kind == OP_CV27) return f(conv27_of(A));
  if (A->kind == OP_ST27) {
    GridOp<double, false> g;
    std::memset(&g, 0, sizeof g);
    g.nx = A->nx; g.ny = A->ny; g.nz = A->nz; g.npts = 27;
    for (int k = 0; k < 27; ++k) g.c[k] = A->coef[k];
    return f(g);
  }
  if (A->kind == OP_GRID) {
    GridOp<double, true> g;
    std::memset(&g, 0, sizeof g);
    g.cf = A->vcoef;
    g.nx = A->nx; g.ny = A->ny; g.nz = A->nz; g.npts = A->npts;
    return f(g);
  }
  if (A->kind == OP_ST7) {
    StencilOp<7> s;
    std::memset(&s, 0, sizeof s);
    s.nx = A->nx; s.ny = A->ny; s.nz = A->nz;
    for (int k = 0; k < 7; ++k) s.c[k] = A->coef[k];
    return f(s);
  }
  StencilOp<5> s;
  std::memset(&s, 0, sizeof s);
  s.nx = A->nx; s.ny = A->ny; s.nz = 1;
  for (int k = 0; k < 5; ++k) s.c[k] = A->coef[k];
  return f(s);
}

// A M^{-1} (Section 3.6 with the product formed), each entry a_ij * dinv_j
// rounded once: CSR values written to the context's ahat (enough room made by
// the caller), stencil coefficients scaled by the constant dinv, the
// matrix-free 27-point operator scaling its entries by dinv as it forms them.
template <class Op>
auto fold_operator(pbcgs_ctx_t ctx, pbcgs_op_t A, const Op& op, int pc, const double* dv, double ds) {
  if constexpr (IsCsr<Op>::value) {
    const int fg = (int)std::min<int64_t>((A->nnz + kWG - 1) / kWG, 8192);
    const CsrOp op32i{A->rp, A->ci, A->va, A->n};  // the fold reads each entry's int32 column
    if (A->nnz > 0) {
      if (pc == PC_VEC) k_fold_csr<PC_VEC><<<fg, kWG, 0, ctx->stream>>>(op32i, A->nnz, ctx->ahat, dv, ds);
      else k_fold_csr<PC_SCALAR><<<fg, kWG, 0, ctx->stream>>>(op32i, A->nnz, ctx->ahat, dv, ds);
    }
    Op fop = op;
    fop.va = ctx->ahat;
    return fop;
  } else if constexpr (IsConv27<Op>::value) {
    return Conv27Op<double, true>{op.n, op.upneg, op.kappa, dv, {op.hab[0], op.hab[1], op.hab[2]}, op.hsum, op.shift};
  } else if constexpr (std::is_same<Op, GridOp<double, true>>::value) {
    // per-row coefficients: every present entry times its column's dinv, into ahat
    const int g = (int)std::min<int64_t>((A->n + 255) / 256, 8192);
    if (pc == PC_VEC) k_fold_grid<PC_VEC><<<g, 256, 0, ctx->stream>>>(op, ctx->ahat, dv, ds);
    else k_fold_grid<PC_SCALAR><<<g, 256, 0, ctx->stream>>>(op, ctx->ahat, dv, ds);
    Op fop = op;
    fop.cf = ctx->ahat;
    return fop;
  } else {
    Op fop = op;
    for (double& c : fop.c) c = c * ds;  // one rounding per coefficient, as a_ij * dinv_j
    return fop;
  }
}

}  // namespace

void* pbcgs_internal_stream(pbcgs_ctx_t ctx) { return ctx ? ctx->stream : nullptr; }

int pbcgs_internal_fail(pbcgs_ctx_t ctx, int code, const char* msg) { return fail(ctx, code, msg); }

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

// Device buffer of at least `count` elements (contents not kept).
template <class T>
int grow(pbcgs_ctx_t ctx, T*& p, size_t& cap, size_t count, const char* what) {
  if (cap >= count) return PBCGS_SUCCESS;
  if (ctx->noalloc) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the call may not allocate");
  if (p) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    p = nullptr;
    return fail(ctx, PBCGS_ERR_ALLOC, std::string("allocation failed: ") + what);
  }
  cap = count;
  return PBCGS_SUCCESS;
}

// Batched solve of independent CSR systems without a preconditioner: the
// schedule of Driver, every launch covering all systems (see SysDesc).
// Op: CsrOp (int32 columns), CsrOp16 (every system holds compact columns) or
// DiaOpB (every system has a diagonal layout: its values are laid out at the
// start of the solve, and the kernels that have a two-rows-per-lane form use
// it, every system's waves owning at least two blocks).
template <class Op>
struct BatchDriver {
  static constexpr bool kTwo = IsDia<Op>::value;
  pbcgs_ctx_t ctx;
  const pbcgs_opts& o;
  int32_t nsys, totalG;
  Args tmpl;
  int64_t q = 0;
  const bool pipe;

  BatchDriver(pbcgs_ctx_t c, const pbcgs_opts& o_, int32_t ns, int32_t tg)
      : ctx(c), o(o_), nsys(ns), totalG(tg), pipe(o_.variant != PBCGS_BICGSTAB) {
    std::memset(&tmpl, 0, sizeof tmpl);
    tmpl.pstride = tg;
    tmpl.aform = alpha_form(o_);
  }

  double* part(int which) const { return ctx->bpart + (size_t)which * kMaxD * totalG; }

  Args L(int pin, int pout, bool first = false) {
    Args b = tmpl;
    b.par = (int32_t)(q & 1);
    b.pin = pin >= 0 ? part(pin) : nullptr;
    b.pout = pout >= 0 ? part(pout) : nullptr;
    b.first = first ? 1 : 0;
    ++q;
    return b;
  }

  void setup() {
    hipStream_t s = ctx->stream;
    if (!pipe) {
      kb_setup_r0<Op, false><<<totalG, kWG, 0, s>>>(ctx->bsys, ctx->bmap, L(-1, PB_SETUP1));
      return;
    }
    kb_setup_r0<Op, true><<<totalG, kWG, 0, s>>>(ctx->bsys, ctx->bmap, L(-1, PB_SETUP1));
    kb_setup_w0<Op><<<totalG, kWG, 0, s>>>(ctx->bsys, ctx->bmap, L(PB_SETUP1, PB_SETUP2));
  }

  void iteration(int64_t i) {
    hipStream_t s = ctx->stream;
    const SysDesc* S = ctx->bsys;
    const int32_t* M = ctx->bmap;
    if (!pipe) {
      if constexpr (kTwo) {
        kb_b1_2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_SETUP1, PB_B1, i == 0));
        kb_b2_2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B1, -1));
        kb_b3_2<Op><<<totalG, kWG, 0, s>>>(S, M, L(-1, PB_B3));
        kb_b4_2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B3, PB_B4));
        kb_b5_2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B4, -1));
      } else {
        kb_b1<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_SETUP1, PB_B1, i == 0));
        kb_b2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B1, -1));
        kb_b3<Op><<<totalG, kWG, 0, s>>>(S, M, L(-1, PB_B3));
        kb_b4<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B3, PB_B4));
        kb_b5<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B4, -1));
      }
      return;
    }
    if (rr_due(o, i - 1)) {
      kb_rr_p<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_B, -1));
      kb_rr_s<Op><<<totalG, kWG, 0, s>>>(S, M, L(-1, -1));
      kb_pa<Op, true><<<totalG, kWG, 0, s>>>(S, M, L(-1, PB_A));
    } else if constexpr (kTwo) {
      kb_pa2<Op><<<totalG, kWG, 0, s>>>(S, M, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
    } else {
      kb_pa<Op, false><<<totalG, kWG, 0, s>>>(S, M, L(i == 0 ? PB_SETUP2 : PB_B, PB_A, i == 0));
    }
    if (rr_due(o, i)) {
      kb_rr_x<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_A, -1));
      kb_rr_r<Op><<<totalG, kWG, 0, s>>>(S, M, L(-1, -1));
      kb_rr_w<Op><<<totalG, kWG, 0, s>>>(S, M, L(-1, PB_B));
    } else if constexpr (kTwo) {
      kb_pb2<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_A, PB_B));
    } else {
      kb_pb<Op><<<totalG, kWG, 0, s>>>(S, M, L(PB_A, PB_B));
    }
  }

  void count_iteration(int64_t i) {
    if (!pipe) { q += 5; return; }
    q += (rr_due(o, i - 1) ? 3 : 1) + (rr_due(o, i) ? 3 : 1);
  }

  void finish(int64_t launched) {
    hipStream_t s = ctx->stream;
    if (!pipe) {
      if (launched == 0) kb_finish<2, false><<<nsys, kWG, 0, s>>>(ctx->bsys, L(PB_SETUP1, -1));
      return;
    }
    if (launched == 0) kb_finish<1, true><<<nsys, kWG, 0, s>>>(ctx->bsys, L(PB_SETUP2, -1));
    else kb_finish<0, true><<<nsys, kWG, 0, s>>>(ctx->bsys, L(PB_B, -1));
  }

  std::string key(int64_t i0, int m) const {
    std::string k = "batch|";
    char buf[160];
    std::snprintf(buf, sizeof buf, "%p|%p|%p|%d|%d|%d|%d|%lld|%d|%d|", (void*)ctx->bsys, (void*)ctx->bmap,
                  (void*)ctx->bpart, nsys, totalG, o.variant, m, (long long)(q & 1), i0 == 0 ? 1 : 0,
                  kTwo ? 1 : std::is_same<Op, CsrOp16>::value ? 2 : 4);
    k += buf;
    for (int j = 0; j < m; ++j) {
      const int64_t i = i0 + j;
      k += char('0' + ((rr_due(o, i - 1) ? 1 : 0) | (rr_due(o, i) ? 2 : 0)));
    }
    return k;
  }

  int chunk(int64_t i0, int m, bool use_graph) {
    if (!use_graph) {
      for (int j = 0; j < m; ++j) iteration(i0 + j);
      HIP_TRY(ctx, hipGetLastError());
      return PBCGS_SUCCESS;
    }
    const std::string k = key(i0, m);
    const int64_t q0 = q;
    auto it = ctx->graphs.find(k);
    if (it == ctx->graphs.end()) {
      if (ctx->graphs.size() >= 32) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
        ctx->graphs.clear();
      }
      hipGraph_t g = nullptr;
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      for (int j = 0; j < m; ++j) iteration(i0 + j);
      hipError_t ce = hipStreamEndCapture(ctx->stream, &g);
      if (ce != hipSuccess) return fail(ctx, PBCGS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
      hipGraphExec_t ex = nullptr;
      hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(ctx, PBCGS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
      it = ctx->graphs.emplace(k, ex).first;
    } else {
      q = q0;
      for (int j = 0; j < m; ++j) count_iteration(i0 + j);
    }
    HIP_TRY(ctx, hipGraphLaunch(it->second, ctx->stream));
    return PBCGS_SUCCESS;
  }

  int run(pbcgs_info* infos) {
    hipStream_t s = ctx->stream;
    const bool use_graph = !(o.flags & 1);
    const int check = o.check_every > 0 ? o.check_every : 8;
    const size_t nst = (size_t)nsys * 4;
    HIP_TRY(ctx, hipEventRecord(ctx->ev_start, s));
    if constexpr (kTwo) kb_dia_fill<<<totalG, kWG, 0, s>>>(ctx->bsys, ctx->bmap);
    kb_init_state<<<(nsys + 63) / 64, 64, 0, s>>>(ctx->bsys, nsys, 0, o.tol);
    q = 0;
    setup();
    HIP_TRY(ctx, hipGetLastError());
    int64_t launched = 0;
    int pend[2], npend = 0, next = 0;
    int64_t qpoll[2] = {0, 0};
    bool stop = false;
    for (;;) {
      while (!stop && launched < o.maxit && npend < 2) {
        const int m = (int)std::min<int64_t>(check, o.maxit - launched);
        int rc = chunk(launched, m, use_graph);
        if (rc != PBCGS_SUCCESS) return rc;
        launched += m;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->bhst + (size_t)next * nst, ctx->bst, nst * sizeof(DevState),
                                    hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipEventRecord(ctx->ev_poll[next], s));
        qpoll[next] = q;
        pend[npend++] = next;
        next ^= 1;
      }
      if (npend == 0) break;
      const int slot = pend[0];
      pend[0] = pend[1];
      --npend;
      HIP_TRY(ctx, hipEventSynchronize(ctx->ev_poll[slot]));
      const DevState* h = ctx->bhst + (size_t)slot * nst;
      const int cur = (int)(qpoll[slot] & 1);
      bool any = false;
      for (int32_t k = 0; k < nsys && !any; ++k) any = (h[(size_t)k * 4 + cur].status == DS_RUNNING);
      if (!any) stop = true;
    }
    finish(launched);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipEventRecord(ctx->ev_stop, s));
    std::vector<DevState> fin(nst);
    HIP_TRY(ctx, hipMemcpyAsync(fin.data(), ctx->bst, nst * sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop);
    // true residuals ||b - A x|| of every system, pairwise, via utility slots 2 -> 3
    Args t = tmpl;
    t.pout = part(PB_UTIL);
    kb_true_res<Op><<<totalG, kWG, 0, s>>>(ctx->bsys, ctx->bmap, t);
    kb_init_state<<<(nsys + 63) / 64, 64, 0, s>>>(ctx->bsys, nsys, 2, 0.0);
    Args f = tmpl;
    f.par = 2;
    f.pin = part(PB_UTIL);
    kb_finish<3, true><<<nsys, kWG, 0, s>>>(ctx->bsys, f);
    HIP_TRY(ctx, hipGetLastError());
    std::vector<DevState> util(nst);
    HIP_TRY(ctx, hipMemcpyAsync(util.data(), ctx->bst, nst * sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int cur = (int)(q & 1);
    int worst = PBCGS_SUCCESS;
    for (int32_t k = 0; k < nsys; ++k) {
      const DevState& d = fin[(size_t)k * 4 + cur];
      pbcgs_info& in = infos[k];
      std::memset(&in, 0, sizeof in);
      in.iters = d.iters;
      in.n_rr = d.n_rr;
      in.status = map_status(d.status);
      in.syncs_per_iter = pipe ? 2 : 5;
      in.relres_rec = d.relres;
      const double nr = util[(size_t)k * 4 + 3].result;
      in.relres_true = (d.rho0 > 0.0) ? std::sqrt(nr) / d.rho0 : 0.0;
      in.ms = ms;
      worst = std::max(worst, in.status);
    }
    return worst;
  }
};

}  // namespace

extern "C" {

const char* pbcgs_status_str(int status) {
  switch (status) {
    case PBCGS_SUCCESS: return "success";
    case PBCGS_MAXIT: return "maxit";
    case PBCGS_BREAKDOWN: return "breakdown";
    case PBCGS_NONFINITE: return "nonfinite";
    case PBCGS_ERR_INVALID_ARG: return "invalid argument";
    case PBCGS_ERR_ALLOC: return "allocation failed";
    case PBCGS_ERR_HIP: return "HIP runtime error";
    case PBCGS_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* pbcgs_last_error(pbcgs_ctx_t ctx) {
  if (ctx) return ctx->err.c_str();
  return g_last_error.c_str();
}

int pbcgs_ctx_create(int device, void* hip_stream, pbcgs_ctx_t* out) {
  if (!out) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "out is NULL");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(nullptr, PBCGS_ERR_HIP, "no HIP device available");
  if (device < 0 || device >= count) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "device index out of range");
  DeviceGuard guard(device);
  pbcgs_ctx_t c = new pbcgs_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (!c->stream) {
    // a blocking stream of our own: ordered with the null stream, and
    // unlike the null stream it can be captured into HIP graphs
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return fail(nullptr, PBCGS_ERR_HIP, "stream creation failed");
    }
    c->own_stream = true;
  }
  bool ok = hipMalloc(&c->st, 4 * sizeof(DevState)) == hipSuccess &&
            hipMalloc(&c->part, sizeof(double) * kMaxD * kMaxG * PB_COUNT) == hipSuccess &&
            hipMalloc(&c->flag, 64) == hipSuccess &&
            hipMalloc(&c->bar, sizeof(GridBar)) == hipSuccess &&
            hipMalloc(&c->qout, sizeof(int64_t)) == hipSuccess &&
            hipHostMalloc(&c->hst, 3 * sizeof(DevState), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&c->hflag, 64, hipHostMallocDefault) == hipSuccess &&
            hipEventCreate(&c->ev_start) == hipSuccess && hipEventCreate(&c->ev_stop) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_poll[0], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_poll[1], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    pbcgs_ctx_destroy(c);
    return fail(nullptr, PBCGS_ERR_ALLOC, "context allocation failed");
  }
  // the no-allocation solve's device array, once per device (the guard made it current)
  c->scratch = static_cast<unsigned char*>(scratch_address(device, &c->scratch_err));
  k_init_state<<<1, 64, 0, c->stream>>>(c->st, 0.0);
  k_init_state<<<1, 64, 0, c->stream>>>(c->st + 1, 0.0);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    pbcgs_ctx_destroy(c);
    return fail(nullptr, PBCGS_ERR_HIP, "context initialisation failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess)
    c->devkey = std::string(prop.gcnArchName) + " " + std::to_string(prop.multiProcessorCount) + "cu";
  else
    c->devkey = "device" + std::to_string(device);
  *out = c;
  return PBCGS_SUCCESS;
}

// Test hook of the residual replacement (see include/pbcgs.h).
int pbcgs_debug_perturb(pbcgs_ctx_t ctx, int32_t iter, double scale) {
  if (!ctx) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "ctx is NULL");
  if (iter < -1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "iter must be -1 (off) or an iteration index");
  if (!std::isfinite(scale)) return fail(ctx, PBCGS_ERR_INVALID_ARG, "scale must be finite");
  ctx->perturb_iter = iter;
  ctx->perturb_scale = scale;
  return PBCGS_SUCCESS;
}

int pbcgs_ctx_destroy(pbcgs_ctx_t ctx) {
  if (!ctx) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard guard(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
  for (auto e : ctx->kev) (void)hipEventDestroy(e);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
  for (auto e : ctx->ev_poll)
    if (e) (void)hipEventDestroy(e);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->ahat) (void)hipFree(ctx->ahat);
  if (ctx->a32) (void)hipFree(ctx->a32);
  for (void* d : ctx->dia)
    if (d) (void)hipFree(d);
  for (void* v : ctx->vi)
    if (v) (void)hipFree(v);
  if (ctx->bsys) (void)hipFree(ctx->bsys);
  if (ctx->bmap) (void)hipFree(ctx->bmap);
  if (ctx->bws) (void)hipFree(ctx->bws);
  if (ctx->bdia) (void)hipFree(ctx->bdia);
  if (ctx->bst) (void)hipFree(ctx->bst);
  if (ctx->bpart) (void)hipFree(ctx->bpart);
  if (ctx->bhst) (void)hipHostFree(ctx->bhst);
  if (ctx->part) (void)hipFree(ctx->part);
  if (ctx->flag) (void)hipFree(ctx->flag);
  if (ctx->bar) (void)hipFree(ctx->bar);
  if (ctx->qout) (void)hipFree(ctx->qout);
  if (ctx->st) (void)hipFree(ctx->st);
  if (ctx->hst) (void)hipHostFree(ctx->hst);
  if (ctx->hflag) (void)hipHostFree(ctx->hflag);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return PBCGS_SUCCESS;
}

namespace {
// The diagonal-coded copy (at most 64 distinct diagonals), for an operator
// whose columns do not fit the int16 block offsets.  Like the int16 copy it
// only changes how columns are read; an operator with more diagonals (or a
// failed allocation) keeps the int32 columns.
int make_diag_coded(pbcgs_ctx_t ctx, pbcgs_op_t A, const CsrOp& op, int g) {
  int32_t* dg = nullptr;
  uint16_t* cd = nullptr;
  if (hipMalloc((void**)&dg, sizeof(int32_t) * 64) != hipSuccess) {
    (void)hipGetLastError();
    return PBCGS_SUCCESS;
  }
  const std::vector<int32_t> empty(64, kEmptyDiag);
  int rc = reset_flag(ctx);
  if (rc == PBCGS_SUCCESS && hipMemcpyAsync(dg, empty.data(), sizeof(int32_t) * 64, hipMemcpyHostToDevice,
                                            ctx->stream) != hipSuccess)
    rc = fail(ctx, PBCGS_ERR_HIP, "diagonal table upload failed");
  if (rc != PBCGS_SUCCESS) {
    (void)hipFree(dg);
    return rc;
  }
  k_diag_collect<<<g, kWG, 0, ctx->stream>>>(op, A->n, dg, ctx->flag);
  int32_t flag = 0;
  rc = read_flag(ctx, &flag);  // synchronises the stream: `empty` is no longer read
  if (rc != PBCGS_SUCCESS || flag) {
    (void)hipFree(dg);
    return rc;
  }
  if (hipMalloc((void**)&cd, sizeof(uint16_t) * (size_t)A->nnz) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(dg);
    return PBCGS_SUCCESS;
  }
  k_diag_code<<<g, kWG, 0, ctx->stream>>>(op, A->n, dg, cd);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipFree(cd);
    (void)hipFree(dg);
    return fail(ctx, PBCGS_ERR_HIP, std::string("diagonal-coded column copy: ") + hipGetErrorString(e));
  }
  A->cd = cd;
  A->dg = dg;
  return PBCGS_SUCCESS;
}

// Makes the compact int16 column copy of a validated CSR operator when every
// column fits in int16 around its row's 64-row block start, else the
// diagonal-coded copy when the matrix has at most 64 distinct diagonals.  It
// only changes how the columns are read, never a result, so an operator that
// fits neither (or a failed allocation) keeps the int32 columns and no error
// is raised.
int make_compact(pbcgs_ctx_t ctx, pbcgs_op_t A) {
  if (A->nnz == 0) return PBCGS_SUCCESS;
  const CsrOp op{A->rp, A->ci, A->va, A->n};
  int rc = reset_flag(ctx);
  if (rc != PBCGS_SUCCESS) return rc;
  const int g = (A->n + kWG - 1) / kWG;
  k_c16_check<<<g, kWG, 0, ctx->stream>>>(op, A->n, ctx->flag);
  int32_t flag = 0;
  rc = read_flag(ctx, &flag);
  if (rc != PBCGS_SUCCESS) return rc;
  if (flag) return make_diag_coded(ctx, A, op, g);
  int16_t* c16 = nullptr;
  if (hipMalloc((void**)&c16, sizeof(int16_t) * (size_t)A->nnz) != hipSuccess) {
    (void)hipGetLastError();
    return PBCGS_SUCCESS;
  }
  k_c16_fill<<<g, kWG, 0, ctx->stream>>>(op, A->n, c16);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipFree(c16);
    return fail(ctx, PBCGS_ERR_HIP, std::string("compact column copy: ") + hipGetErrorString(e));
  }
  A->c16 = c16;
  return PBCGS_SUCCESS;
}
}  // namespace

// Makes the diagonal layout's structure (see DiaOpT) for a validated CSR
// operator with at most kMaxDia distinct diagonals whose rows store their
// columns in ascending order, when the layout's slots (diagonals x rows) are at
// most 5/4 of the stored entries.  Like the compact columns it changes how
// the operator is read, never a result; an operator that does not qualify (or
// a failed allocation) keeps the CSR stream and no error is raised.
int make_dia(pbcgs_ctx_t ctx, pbcgs_op_t A) {
  if (A->nnz == 0) return PBCGS_SUCCESS;
  int32_t* tab = nullptr;
  int32_t* doff = nullptr;
  uint32_t* mask = nullptr;
  auto release = [&]() {
    if (tab) (void)hipFree(tab);
    if (doff) (void)hipFree(doff);
    if (mask) (void)hipFree(mask);
  };
  if (hipMalloc((void**)&tab, sizeof(int32_t) * 64) != hipSuccess ||
      hipMalloc((void**)&doff, sizeof(int32_t) * kMaxDia) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return PBCGS_SUCCESS;
  }
  const CsrOp op{A->rp, A->ci, A->va, A->n};
  const int g = (A->n + kWG - 1) / kWG;
  std::vector<int32_t> h(64, kEmptyDiag);
  int rc = reset_flag(ctx);
  if (rc == PBCGS_SUCCESS && hipMemcpyAsync(tab, h.data(), sizeof(int32_t) * 64, hipMemcpyHostToDevice,
                                            ctx->stream) != hipSuccess)
    rc = fail(ctx, PBCGS_ERR_HIP, "diagonal table upload failed");
  if (rc != PBCGS_SUCCESS) {
    release();
    return rc;
  }
  k_diag_collect<<<g, kWG, 0, ctx->stream>>>(op, A->n, tab, ctx->flag);
  int32_t flag = 0;
  rc = read_flag(ctx, &flag);  // synchronises: `h` may be reused
  if (rc != PBCGS_SUCCESS || flag) {
    release();
    return rc;
  }
  if (hipMemcpy(h.data(), tab, sizeof(int32_t) * 64, hipMemcpyDeviceToHost) != hipSuccess) {
    release();
    return fail(ctx, PBCGS_ERR_HIP, "diagonal table download failed");
  }
  std::vector<int32_t> offs;
  for (int32_t d : h)
    if (d != kEmptyDiag) offs.push_back(d);
  std::sort(offs.begin(), offs.end());
  const int nd = (int)offs.size();
  if (nd == 0 || nd > kMaxDia || (double)nd * (double)A->n > 1.25 * (double)A->nnz) {
    release();
    return PBCGS_SUCCESS;
  }
  if (hipMalloc((void**)&mask, sizeof(uint32_t) * (size_t)A->n) != hipSuccess) {
    (void)hipGetLastError();
    mask = nullptr;
    release();
    return PBCGS_SUCCESS;
  }
  rc = reset_flag(ctx);
  if (rc == PBCGS_SUCCESS && hipMemcpyAsync(doff, offs.data(), sizeof(int32_t) * nd, hipMemcpyHostToDevice,
                                            ctx->stream) != hipSuccess)
    rc = fail(ctx, PBCGS_ERR_HIP, "diagonal offsets upload failed");
  if (rc != PBCGS_SUCCESS) {
    release();
    return rc;
  }
  k_dia_mask<<<g, kWG, 0, ctx->stream>>>(op, A->n, doff, nd, mask, ctx->flag);
  rc = read_flag(ctx, &flag);  // synchronises: `offs` may go
  if (rc != PBCGS_SUCCESS || flag) {
    release();
    return rc;
  }
  A->dmask = mask;
  A->ddoff = doff;
  A->ndia = nd;
  for (int d = 0; d < nd; ++d) A->dia_off[d] = offs[(size_t)d];
  mask = nullptr;
  doff = nullptr;
  release();
  return PBCGS_SUCCESS;
}

// The diagonal layout of A with this solve's values: the stored values, or
// those of A M^{-1} (pc_fold PC_VEC / PC_SCALAR), rounded once to V, in the
// context's values buffer `slot`.
extern "C++" {
template <class V>
int dia_operator(pbcgs_ctx_t ctx, pbcgs_op_t A, int pc_fold, const double* dv, double ds, DiaOpT<V>* out,
                 int slot = 0) {
  const int32_t ld = (int32_t)padded(A->n);
  const int rc = ensure_dia(ctx, (size_t)A->ndia * (size_t)ld * sizeof(V), slot);
  if (rc != PBCGS_SUCCESS) return rc;
  V* buf = static_cast<V*>(ctx->dia[slot]);
  poison(ctx, buf, (size_t)A->ndia * (size_t)ld * sizeof(V));
  const CsrOp op{A->rp, A->ci, A->va, A->n};
  const int g = (A->n + 63) / 64;
  if (pc_fold == PC_VEC) k_dia_fill<PC_VEC, V><<<g, 64, 0, ctx->stream>>>(op, A->n, A->ddoff, A->ndia, ld, buf, dv, ds);
  else if (pc_fold == PC_SCALAR) k_dia_fill<PC_SCALAR, V><<<g, 64, 0, ctx->stream>>>(op, A->n, A->ddoff, A->ndia, ld, buf, dv, ds);
  else k_dia_fill<PC_NONE, V><<<g, 64, 0, ctx->stream>>>(op, A->n, A->ddoff, A->ndia, ld, buf, dv, ds);
  HIP_TRY(ctx, hipGetLastError());
  DiaOpT<V> d;
  std::memset(&d, 0, sizeof d);
  d.mask = A->dmask;
  d.va = buf;
  d.n = A->n;
  d.nd = A->ndia;
  d.ld = ld;
  for (int k = 0; k < A->ndia; ++k) d.off[k] = A->dia_off[k];
  *out = d;
  return PBCGS_SUCCESS;
}

// Whether a binary64 solve reads the diagonal layout's values with ordinary
// loads (true) instead of the nontemporal hint.  Measured at 128^3 (7
// diagonals, about 264 MiB of vectors and layout per iteration), ordinary
// loads make BiCGStab 10 % and p-BiCGStab 2 % faster per iteration, as the
// layout then shares the 256 MiB memory-side cache with the vectors; with a
// working set several times larger (the 512-system batch) the hint is
// faster.  The estimate counts nine vectors (the most any solver keeps live
// per iteration) besides the layout; PBCGS_DIA_CACHED=0 or 1 overrides.
static bool dia_cached(const pbcgs_op_s* A) {
  const double n = (double)padded(A->n);
  const double ws = 9.0 * 8.0 * n + (8.0 * A->ndia + 4.0) * n;
  return env_int("PBCGS_DIA_CACHED", ws <= 320.0 * 1024 * 1024 ? 1 : 0) != 0;
}

// The same operator read with ordinary value loads (the layouts are identical).
static DiaOpC cached_loads(const DiaOp& d) {
  static_assert(sizeof(DiaOpC) == sizeof(DiaOp), "DiaOpT layouts");
  DiaOpC c;
  std::memcpy(&c, &d, sizeof c);
  return c;
}

// The value-indexed form of a layout `d` just filled (see DiaViOpT), in the
// context's codes buffer `slot`, when it has at most kViDia diagonals and
// every diagonal holds at most kViTab distinct values; false (and no error)
// otherwise or when the buffer cannot be had.  PBCGS_VALUE_CODES=0 never
// takes it, =1 wherever it fits; by default only from kViMinRows rows up:
// below that a solve is bound by latency, and the codes' extra dependent load
// per row cost more than their bytes saved (2-D 64^2: 13.1 against 12.4 us
// per iteration; 16^3 to 48^3 within 0.3-1.5 us; 96^3: 43.9 against 52.9).
// One host synchronisation reads the overflow word.
constexpr int32_t kViMinRows = 1 << 18;
template <class V>
static bool vi_operator(pbcgs_ctx_t ctx, const DiaOpT<V>& d, DiaViOpT<V>* out, int slot = 0) {
  const int mode = env_int("PBCGS_VALUE_CODES", -1);
  if (mode == 0 || (mode < 0 && d.n < kViMinRows) || d.nd <= 0 || d.nd > kViDia) return false;
  const size_t code_bytes = ((size_t)d.ld * sizeof(uint64_t) + 255) & ~(size_t)255;
  const size_t bytes = code_bytes + sizeof(uint64_t) * ((size_t)d.nd * kViTab + 1);
  if (ctx->vi_cap[slot] < bytes) {
    if (ctx->vi[slot]) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->vi[slot]);
      ctx->vi[slot] = nullptr;
      ctx->vi_cap[slot] = 0;
      for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
      ctx->graphs.clear();
    }
    if (hipMalloc(&ctx->vi[slot], bytes) != hipSuccess) {
      (void)hipGetLastError();
      ctx->vi[slot] = nullptr;
      return false;
    }
    ctx->vi_cap[slot] = bytes;
  }
  uint64_t* code = static_cast<uint64_t*>(ctx->vi[slot]);
  uint64_t* tab = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->vi[slot]) + code_bytes);
  k_vi_reset<<<(d.nd * kViTab + 1 + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(tab, d.nd);
  k_vi_collect<<<std::min((d.n + kWG - 1) / kWG, 1024), kWG, 0, ctx->stream>>>(d, tab);
  uint64_t overflow = 1;
  if (hipMemcpyAsync(&overflow, tab + (size_t)d.nd * kViTab, sizeof overflow, hipMemcpyDeviceToHost, ctx->stream) !=
          hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (overflow != 0) return false;
  k_vi_encode<<<(d.ld + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(d, tab, code);
  DiaViOpT<V> v;
  std::memset(&v, 0, sizeof v);
  v.code = code;
  v.tab = tab;
  v.n = d.n;
  v.nd = d.nd;
  v.ld = d.ld;
  for (int k = 0; k < d.nd; ++k) v.off[k] = d.off[k];
  *out = v;
  return true;
}
}  // extern "C++"

int pbcgs_op_csr(pbcgs_ctx_t ctx, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                 const double* val, pbcgs_op_t* out) {
  if (!ctx || !out) return fail(ctx, PBCGS_ERR_INVALID_ARG, "ctx or out is NULL");
  if (n <= 0 || nnz < 0 || nnz > INT32_MAX) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad n or nnz");
  if (!row_ptr || (nnz > 0 && (!col_idx || !val))) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL CSR array");
  // the product streams non-zeros in int32 index rounds of kStage past the last one
  if (nnz > (int64_t)INT32_MAX - 2 * CsrOp::kStage)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "nnz too large for int32 non-zero indexing");
  Shape sh;
  if (!make_shape(n, &sh)) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many rows for one launch");
  DeviceGuard guard(ctx->device);
  CsrOp op{row_ptr, col_idx, val, n};
  int rc = reset_flag(ctx);
  if (rc != PBCGS_SUCCESS) return rc;
  k_csr_check<<<(n + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(op, n, nnz, ctx->flag);
  int32_t flag = 0;
  rc = read_flag(ctx, &flag);
  if (rc != PBCGS_SUCCESS) return rc;
  if (flag) return fail(ctx, PBCGS_ERR_INVALID_ARG, "malformed CSR structure (row_ptr or col_idx)");
  pbcgs_op_t A = new pbcgs_op_s();
  A->ctx = ctx;
  A->kind = OP_CSR;
  A->n = n;
  A->nnz = nnz;
  A->rp = row_ptr;
  A->ci = col_idx;
  A->va = val;
  rc = make_compact(ctx, A);
  if (rc == PBCGS_SUCCESS) rc = make_dia(ctx, A);
  if (rc != PBCGS_SUCCESS) {
    (void)pbcgs_op_destroy(A);
    return rc;
  }
  *out = A;
  return PBCGS_SUCCESS;
}

int pbcgs_op_stencil(pbcgs_ctx_t ctx, int32_t nx, int32_t ny, int32_t nz, int32_t npts, const double* coef,
                     int32_t coef_per_row, pbcgs_op_t* out) {
  if (!ctx || !out || !coef) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad grid size");
  if (npts != 5 && npts != 7 && npts != 27) return fail(ctx, PBCGS_ERR_INVALID_ARG, "npts must be 5, 7 or 27");
  if (npts == 5 && nz != 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "5-point stencil needs nz == 1");
  if (coef_per_row != 0 && coef_per_row != 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "coef_per_row must be 0 or 1");
  const int64_t n = (int64_t)nx * ny * nz;
  if (n > INT32_MAX) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "grid too large");
  Shape sh;
  if (!make_shape((int32_t)n, &sh)) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many rows for one launch");
  if (coef_per_row && (int64_t)npts * n > INT32_MAX)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "npts * n per-row coefficients exceed int32 indexing");
  pbcgs_op_t A = new pbcgs_op_s();
  A->ctx = ctx;
  A->kind = coef_per_row ? OP_GRID : (npts == 27 ? OP_ST27 : (npts == 7 ? OP_ST7 : OP_ST5));
  A->n = (int32_t)n;
  A->nx = nx;
  A->ny = ny;
  A->nz = nz;
  A->npts = npts;
  if (coef_per_row) A->vcoef = coef;  // device array, borrowed
  else
    for (int k = 0; k < npts; ++k) A->coef[k] = coef[k];
  // stored entries of the equivalent CSR matrix: per neighbour offset, the
  // nodes whose neighbour lies in the grid
  const int64_t X = nx, Y = ny, Z = nz;
  auto count = [&](int dx, int dy, int dz) { return (X - std::abs(dx)) * (Y - std::abs(dy)) * (Z - std::abs(dz)); };
  int64_t nnz = 0;
  if (npts == 27) {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) nnz += count(dx, dy, dz);
  } else {
    nnz = count(0, 0, 0) + 2 * (count(1, 0, 0) + count(0, 1, 0)) + (npts == 7 ? 2 * count(0, 0, 1) : 0);
  }
  A->nnz = nnz;
  *out = A;
  return PBCGS_SUCCESS;
}

int pbcgs_op_convdiff27(pbcgs_ctx_t ctx, int32_t n, const double* kappa, const double* beta, double shift,
                        pbcgs_op_t* out) {
  if (!ctx || !out || !kappa || !beta) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad grid size");
  const int64_t N = (int64_t)n * n * n;
  if (N > INT32_MAX) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "grid too large");
  Shape sh;
  if (!make_shape((int32_t)N, &sh)) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many rows for one launch");
  pbcgs_op_t A = new pbcgs_op_s();
  A->ctx = ctx;
  A->kind = OP_CV27;
  A->n = (int32_t)N;
  A->nx = A->ny = A->nz = n;
  A->kappa = kappa;
  for (int ax = 0; ax < 3; ++ax) A->hb[ax] = beta[ax] / (double)(n + 1);  // one IEEE division, as assembled
  A->shift = shift;
  const int64_t m = 3 * (int64_t)n - 2;  // stored entries of the equivalent CSR matrix
  A->nnz = m * m * m;
  *out = A;
  return PBCGS_SUCCESS;
}

int pbcgs_op_destroy(pbcgs_op_t op) {
  if (!op) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "op is NULL");
  pbcgs_ctx_t ctx = op->ctx;
  if (ctx) {
    // cached graphs may embed this operator's arrays
    DeviceGuard guard(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
    if (op->own_rp) (void)hipFree(op->own_rp);
    if (op->own_ci) (void)hipFree(op->own_ci);
    if (op->own_va) (void)hipFree(op->own_va);
    if (op->c16) (void)hipFree(op->c16);
    if (op->cd) (void)hipFree(op->cd);
    if (op->dg) (void)hipFree(op->dg);
    if (op->dmask) (void)hipFree(op->dmask);
    if (op->ddoff) (void)hipFree(op->ddoff);
  }
  delete op;
  return PBCGS_SUCCESS;
}

int64_t pbcgs_op_rows(pbcgs_op_t op) {
  if (!op) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "op is NULL");
  return op->n;
}

int pbcgs_op_index_bytes(pbcgs_op_t op) {
  if (!op) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "op is NULL");
  if (op->kind != OP_CSR) return 0;
  return (op->c16 || op->cd) ? 2 : 4;
}

int pbcgs_op_column_form(pbcgs_op_t op) {
  if (!op) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "op is NULL");
  if (op->kind != OP_CSR) return PBCGS_COLS_NONE;
  if (op->c16) return PBCGS_COLS_BLOCK16;
  if (op->cd) return PBCGS_COLS_DIAG16;
  return PBCGS_COLS_INT32;
}

int pbcgs_op_diagonals(pbcgs_op_t op) {
  if (!op) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "op is NULL");
  return op->ndia;
}

int pbcgs_spmv(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* x, double* y) {
  if (!ctx || !A || !x || !y) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (A->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "operator belongs to another context");
  if ((const void*)x == (const void*)y) return fail(ctx, PBCGS_ERR_INVALID_ARG, "x and y must not overlap");
  DeviceGuard guard(ctx->device);
  Shape sh;
  if (!make_shape(A->n, &sh)) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many rows");
  Args a = base_args(ctx, sh);
  return with_op(A, [&](auto op) -> int {
    k_spmv<decltype(op)><<<sh.G, kWG, 0, ctx->stream>>>(op, a, x, y);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PBCGS_SUCCESS;
  });
}

int pbcgs_dot(pbcgs_ctx_t ctx, int64_t n, const double* x, const double* y, double* result) {
  if (!ctx || !x || !y || !result) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || n > INT32_MAX) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad length");
  DeviceGuard guard(ctx->device);
  Shape sh;
  if (!make_shape((int32_t)n, &sh)) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "vector too long");
  Args a = base_args(ctx, sh);
  a.pout = part_buf(ctx, PB_UTIL);
  k_dot<<<sh.G, kWG, 0, ctx->stream>>>(a, x, y);
  HIP_TRY(ctx, hipGetLastError());
  return finish_sum(ctx, sh, result);
}

int pbcgs_jacobi_dinv(pbcgs_ctx_t ctx, pbcgs_op_t A, double* dinv) {
  if (!ctx || !A || !dinv) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard guard(ctx->device);
  if (A->kind == OP_CV27) {
    int rc = reset_flag(ctx);
    if (rc != PBCGS_SUCCESS) return rc;
    k_dinv_conv27<<<(A->n + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(conv27_of(A), A->n, dinv, ctx->flag);
    int32_t flag = 0;
    rc = read_flag(ctx, &flag);
    if (rc != PBCGS_SUCCESS) return rc;
    if (flag & 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "zero or non-finite diagonal entry");
    return PBCGS_SUCCESS;
  }
  if (A->kind == OP_GRID) {
    int rc = reset_flag(ctx);
    if (rc != PBCGS_SUCCESS) return rc;
    GridOp<double, true> g;
    std::memset(&g, 0, sizeof g);
    g.cf = A->vcoef;
    g.nx = A->nx; g.ny = A->ny; g.nz = A->nz; g.npts = A->npts;
    k_dinv_grid<<<(int)std::min<int64_t>((A->n + 255) / 256, 8192), 256, 0, ctx->stream>>>(g, dinv, ctx->flag);
    int32_t flag = 0;
    rc = read_flag(ctx, &flag);
    if (rc != PBCGS_SUCCESS) return rc;
    if (flag & 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "zero or non-finite diagonal entry");
    return PBCGS_SUCCESS;
  }
  if (A->kind != OP_CSR) {
    const double c = stencil_centre(A);
    if (c == 0.0 || !std::isfinite(c)) return fail(ctx, PBCGS_ERR_INVALID_ARG, "zero diagonal");
    const double d = 1.0 / c;
    std::vector<double> h((size_t)A->n, d);
    HIP_TRY(ctx, hipMemcpyAsync(dinv, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PBCGS_SUCCESS;
  }
  int rc = reset_flag(ctx);
  if (rc != PBCGS_SUCCESS) return rc;
  k_dinv_csr<<<(A->n + 63) / 64, 64, 0, ctx->stream>>>(CsrOp{A->rp, A->ci, A->va, A->n}, A->n, dinv, ctx->flag);
  int32_t flag = 0;
  rc = read_flag(ctx, &flag);
  if (rc != PBCGS_SUCCESS) return rc;
  if (flag & 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "zero, non-finite or missing diagonal entry");
  return PBCGS_SUCCESS;
}

int pbcgs_solve(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, double* x, const double* dinv,
                const pbcgs_opts* opts, pbcgs_info* info) {
  if (!ctx || !A || !b || !x || !opts || !info) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (A->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "operator belongs to another context");
  const pbcgs_opts& o = *opts;
  if (o.variant < PBCGS_BICGSTAB || o.variant > PBCGS_PIPE_CG)
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown variant");
  if (o.precond != PBCGS_PRECOND_NONE && o.precond != PBCGS_PRECOND_JACOBI &&
      o.precond != PBCGS_PRECOND_JACOBI_FOLDED)
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown preconditioner");
  if (cg_family(o.variant) && o.precond == PBCGS_PRECOND_JACOBI_FOLDED)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the CG family needs a symmetric operator: use PBCGS_PRECOND_JACOBI");
  if (o.variant == PBCGS_CA_BICGSTAB && o.precond == PBCGS_PRECOND_JACOBI)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "CA-BiCGStab takes Jacobi as PBCGS_PRECOND_JACOBI_FOLDED");
  const bool folded = (o.precond == PBCGS_PRECOND_JACOBI_FOLDED);
  if (o.precision != PBCGS_FP64 && o.precision != PBCGS_FP32_RR64)
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown precision");
  const bool mp = (o.precision == PBCGS_FP32_RR64);
  if (mp && o.variant != PBCGS_PBICGSTAB_RR)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the binary32 form is p-BiCGStab with residual replacement");
  if (mp && o.precond == PBCGS_PRECOND_JACOBI)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the binary32 form takes Jacobi as PBCGS_PRECOND_JACOBI_FOLDED");
  if (o.maxit < 0 || !(o.tol >= 0.0)) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad maxit or tol");
  if (o.variant == PBCGS_PBICGSTAB_RR && o.rr_period < 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad rr_period");
  if ((const void*)b == (const void*)x) return fail(ctx, PBCGS_ERR_INVALID_ARG, "b and x must not overlap");
  if (ctx->perturb_iter >= 0 && (mp || (o.variant != PBCGS_PBICGSTAB && o.variant != PBCGS_PBICGSTAB_RR)))
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the residual perturbation hook applies to binary64 p-BiCGStab only");
  DeviceGuard guard(ctx->device);
  Shape sh;
  // the operator's own tuned shape, else one the cache holds for its key
  int32_t prefer_R = A->tuned_R[o.variant][mp ? 1 : 0][read_path(o.flags)];
  if (prefer_R == 0) prefer_R = cache_find(make_key(ctx, A, o.variant, o.precision, read_path(o.flags)));
  if (!make_shape(A->n, &sh, prefer_R))
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many rows");
  std::memset(info, 0, sizeof *info);
  PoisonScope poison_scope(ctx, (o.flags & 32) != 0);

  const size_t np = padded(A->n);
  const int nvec = 14;
  int rc = ensure_ws(ctx, np * nvec);
  if (rc != PBCGS_SUCCESS) return rc;
  poison(ctx, ctx->ws, np * nvec * sizeof(double));
  poison(ctx, ctx->part, (size_t)PB_COUNT * kMaxD * kMaxG * sizeof(double));
  Args a = base_args(ctx, sh);
  a.hist = o.history;
  a.b = b;
  a.x = x;
  // XCD-contiguous workgroup indices (see wg_index) where they measured
  // faster: p-BiCGStab in binary64 on up to 2^22 rows (128^3: 3.5 % per
  // iteration); BiCGStab at 128^3 and p-BiCGStab at 256^3 were 2-3 % slower
  // with them.  PBCGS_XCD_MAP=0 / 1 overrides.
  {
    const bool pipelined = o.variant == PBCGS_PBICGSTAB || o.variant == PBCGS_PBICGSTAB_RR;
    const int dflt = (pipelined && o.precision == PBCGS_FP64 && A->n <= (1 << 22)) ? 1 : 0;
    a.wg = env_int("PBCGS_XCD_MAP", dflt) != 0 ? -2 : -1;
  }
  double* v[nvec];
  for (int k = 0; k < nvec; ++k) v[k] = ctx->ws + (size_t)k * np;

  // preconditioner mode: none, a vector of 1/a_ii, or one constant
  int pc = PC_NONE;
  const double* dinv_vec = nullptr;  // the vector of 1/a_ii when there is one (also when constant)
  if (o.precond != PBCGS_PRECOND_NONE) {
    const double* dv = dinv;
    if (!dv && const_stencil(A)) {
      const double c = stencil_centre(A);
      if (c == 0.0 || !std::isfinite(c)) return fail(ctx, PBCGS_ERR_INVALID_ARG, "zero diagonal");
      pc = PC_SCALAR;
      a.dinv_s = 1.0 / c;
    } else {
      if (!dv) {
        rc = pbcgs_jacobi_dinv(ctx, A, v[13]);
        if (rc != PBCGS_SUCCESS) return rc;
        dv = v[13];
      }
      dinv_vec = dv;
      rc = reset_flag(ctx);
      if (rc != PBCGS_SUCCESS) return rc;
      k_dinv_const<<<(A->n + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(A->n, dv, ctx->flag);
      int32_t flag = 0;
      rc = read_flag(ctx, &flag);
      if (rc != PBCGS_SUCCESS) return rc;
      if (flag & 2) {
        pc = PC_VEC;
        a.dinv = dv;
      } else {
        pc = PC_SCALAR;
        rc = read_double(ctx, dv, &a.dinv_s);
        if (rc != PBCGS_SUCCESS) return rc;
      }
    }
  }
  if (folded && pc == PC_VEC && const_stencil(A))
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "folded Jacobi on a constant stencil needs a constant diagonal");
  const bool hat = (pc != PC_NONE) && !folded;
  // a CSR operator with a diagonal layout is read through it (same results)
  const bool use_dia = A->kind == OP_CSR && A->ndia > 0 && dia_ok(o) && !ctx->noalloc;
  if (cg_family(o.variant)) {
    // r, p, s, w, z; u = M^{-1} r in r^ and q in s^ (aliases without a preconditioner)
    a.r = v[1]; a.p = v[2]; a.s = v[3]; a.w = v[4]; a.z = v[5];
    a.rh = hat ? v[8] : a.r;
    a.sh = hat ? v[10] : a.s;
    // p-CG's alternating gather buffers: m (with Jacobi) or w itself (without)
    a.wh = hat ? v[6] : a.w;
    a.t = v[7];
  } else if (o.variant == PBCGS_BICGSTAB) {
    a.r0 = v[0]; a.r = v[1]; a.p = v[2]; a.s = v[3]; a.q = v[4]; a.y = v[5];
    a.ph = hat ? v[6] : a.p;
    a.qh = hat ? v[7] : a.q;
  } else {
    a.r0 = v[0]; a.r = v[1]; a.w = v[2]; a.t = v[3]; a.ph = v[4]; a.s = v[5]; a.z = v[6]; a.v = v[7];
    a.rh = hat ? v[8] : a.r;
    a.wh = hat ? v[9] : a.w;
    a.sh = hat ? v[10] : a.s;
    a.zh = hat ? v[11] : a.z;
  }

  if (mp) {
    // binary32 vectors, then the binary64 scratch r64, s64
    float* f32 = reinterpret_cast<float*>(ctx->ws);
    float** fv[8] = {&a.r0f, &a.rf, &a.wf, &a.tf, &a.pf, &a.sf, &a.zf, &a.vf};
    for (int k = 0; k < 8; ++k) *fv[k] = f32 + (size_t)k * np;
    a.r64 = ctx->ws + 4 * np;
    a.s64 = ctx->ws + 5 * np;
    const int xg = (A->n + kWG - 1) / kWG;
    const double* dv = dinv_vec;
    const double ds = a.dinv_s;
    a.dinv = nullptr;
    a.dinv_s = 0.0;
    if (folded && stored_values(A) > 0 && !use_dia) {
      rc = ensure_ahat(ctx, (size_t)stored_values(A));
      if (rc != PBCGS_SUCCESS) return rc;
      poison(ctx, ctx->ahat, (size_t)stored_values(A) * sizeof(double));
    }
    if (stored_values(A) > 0 && !use_dia) {
      rc = ensure_a32(ctx, (size_t)stored_values(A));
      if (rc != PBCGS_SUCCESS) return rc;
      poison(ctx, ctx->a32, (size_t)stored_values(A) * sizeof(float));
    }
    return with_op(A, [&](auto op) -> int {
      auto run_mp = [&](auto op32, auto op64) -> int {
        Driver<decltype(op32), PC_NONE, decltype(op64), true> drv(ctx, op32, op64, a, o);
        drv.true_res = !folded;
        const int st = drv.run(info);
        if (st < 0 || !folded) return st;
        if (pc == PC_VEC) k_fold_x<PC_VEC, false><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
        else k_fold_x<PC_SCALAR, false><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
        HIP_TRY(ctx, hipGetLastError());
        const int rc2 = true_relres(ctx, op, a, drv.rho0, &info->relres_true);
        if (rc2 != PBCGS_SUCCESS) return rc2;
        return st;
      };
      // run the binary32 form on op64 (A, or A M^{-1} formed); its binary32
      // operator is op64 rounded
      auto go = [&](auto op64) -> int {
        auto op32 = to_binary32(ctx, op64, A->nnz);
        HIP_TRY(ctx, hipGetLastError());
        return run_mp(op32, op64);
      };
      if constexpr (IsCsr<decltype(op)>::value) {
        if (use_dia) {
          // both operators through the diagonal layout: the binary32 values
          // and, for the replacement steps, the binary64 ones (A, or A M^{-1}
          // formed in the layout's fill, one rounding each as k_fold_csr's)
          const int pcf = folded ? pc : PC_NONE;
          DiaOpF op32;
          DiaOp op64;
          int rcd = dia_operator<float>(ctx, A, pcf, dv, ds, &op32, 0);
          if (rcd == PBCGS_SUCCESS) rcd = dia_operator<double>(ctx, A, pcf, dv, ds, &op64, 1);
          if (rcd != PBCGS_SUCCESS) return rcd;
          if (folded) {
            if (pc == PC_VEC) k_fold_x<PC_VEC, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
            else k_fold_x<PC_SCALAR, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
          }
          // both layouts value-indexed when both fit (the binary32 rounding
          // never has more distinct values than the binary64 values)
          DiaViOpF v32;
          DiaViOp v64;
          if (vi_operator(ctx, op64, &v64, 1) && vi_operator(ctx, op32, &v32, 0)) {
            info->value_codes = 1;
            return run_mp(v32, v64);
          }
          return run_mp(op32, op64);
        }
      }
      if (!folded) return go(op);
      auto fop = fold_operator(ctx, A, op, pc, dv, ds);
      if (pc == PC_VEC) k_fold_x<PC_VEC, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      else k_fold_x<PC_SCALAR, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      return go(fop);
    }, compact_ok(o));
  }

  if (folded) {
    // A M^{-1} y = b from y_0 = x_0 / dinv, then x = dinv * y (Section 3.6)
    const int xg = (A->n + kWG - 1) / kWG;
    const double* dv = dinv_vec;
    const double ds = a.dinv_s;
    a.dinv = nullptr;
    a.dinv_s = 0.0;
    if (stored_values(A) > 0 && !use_dia) {
      rc = ensure_ahat(ctx, (size_t)stored_values(A));
      if (rc != PBCGS_SUCCESS) return rc;
      poison(ctx, ctx->ahat, (size_t)stored_values(A) * sizeof(double));
    }
    return with_op(A, [&](auto op) -> int {
      auto run_folded = [&](auto fop) -> int {
      if (pc == PC_VEC) k_fold_x<PC_VEC, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      else k_fold_x<PC_SCALAR, true><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      HIP_TRY(ctx, hipGetLastError());
      Driver<decltype(fop), PC_NONE> drv(ctx, fop, a, o);
      drv.true_res = false;
      const int st = drv.run(info);
      if (st < 0) return st;
      if (pc == PC_VEC) k_fold_x<PC_VEC, false><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      else k_fold_x<PC_SCALAR, false><<<xg, kWG, 0, ctx->stream>>>(A->n, x, dv, ds);
      HIP_TRY(ctx, hipGetLastError());
      const int rc2 = true_relres(ctx, op, a, drv.rho0, &info->relres_true);
      if (rc2 != PBCGS_SUCCESS) return rc2;
      return st;
      };
      if constexpr (IsCsr<decltype(op)>::value) {
        if (use_dia) {
          DiaOp dop;
          const int rcd = dia_operator<double>(ctx, A, pc, dv, ds, &dop);
          if (rcd != PBCGS_SUCCESS) return rcd;
          DiaViOp vop;
          if (vi_operator(ctx, dop, &vop)) {
            info->value_codes = 1;
            return run_folded(vop);
          }
          if (dia_cached(A)) return run_folded(cached_loads(dop));
          return run_folded(dop);
        }
      }
      return run_folded(fold_operator(ctx, A, op, pc, dv, ds));
    }, compact_ok(o));
  }

  if (use_dia) {
    DiaOp dop;
    rc = dia_operator<double>(ctx, A, PC_NONE, nullptr, 0.0, &dop);
    if (rc != PBCGS_SUCCESS) return rc;
    // value-indexed without a preconditioner and with Jacobi by a constant
    // diagonal (a scalar); a Jacobi vector keeps the values
    DiaViOp vop;
    if (pc != PC_VEC && vi_operator(ctx, dop, &vop)) {
      info->value_codes = 1;
      if (pc == PC_NONE) return Driver<DiaViOp, PC_NONE>(ctx, vop, a, o).run(info);
      return Driver<DiaViOp, PC_SCALAR>(ctx, vop, a, o).run(info);
    }
    if (pc == PC_NONE && dia_cached(A)) return Driver<DiaOpC, PC_NONE>(ctx, cached_loads(dop), a, o).run(info);
    if (pc == PC_NONE) return Driver<DiaOp, PC_NONE>(ctx, dop, a, o).run(info);
    if (pc == PC_VEC) return Driver<DiaOp, PC_VEC>(ctx, dop, a, o).run(info);
    return Driver<DiaOp, PC_SCALAR>(ctx, dop, a, o).run(info);
  }
  return with_op(A, [&](auto op) -> int {
    using Op = decltype(op);
    if (pc == PC_NONE) return Driver<Op, PC_NONE>(ctx, op, a, o).run(info);
    if (pc == PC_VEC) return Driver<Op, PC_VEC>(ctx, op, a, o).run(info);
    return Driver<Op, PC_SCALAR>(ctx, op, a, o).run(info);
  }, compact_ok(o));
}

// The same solve with every device buffer it needs taken from `scratch`
// (see include/pbcgs.h): the context's state slots, partial sums and
// workspace are swapped for regions of the array for the duration of the call,
// and any attempt to allocate fails instead.
int pbcgs_solve_noalloc(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, double* x, const double* dinv,
                        const pbcgs_opts* opts, pbcgs_info* info) {
  if (!ctx || !A || !opts) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (!ctx->scratch) return fail(ctx, PBCGS_ERR_HIP, "no scratch array on this device: " + ctx->scratch_err);
  if (opts->precision != PBCGS_FP64)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "pbcgs_solve_noalloc runs binary64 solves only");
  if (opts->flags & 2)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "pbcgs_solve_noalloc does not time kernels (events would be created)");
  const size_t vec = padded(A->n) * 14;
  const size_t folded_vals = (opts->precond == PBCGS_PRECOND_JACOBI_FOLDED && stored_values(A) > 0)
                                 ? (size_t)std::max<int64_t>(stored_values(A), 1)
                                 : 0;
  if (vec + folded_vals > kScratchPoolDoubles)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED,
                "pbcgs_solve_noalloc needs " + std::to_string(vec + folded_vals) + " doubles of scratch (14 per row" +
                    (folded_vals ? " plus one per non-zero" : "") + "); at most " +
                    std::to_string(kScratchPoolDoubles) + " are available");
  struct View {
    pbcgs_ctx_t c;
    DevState* st;
    double *part, *ws, *ahat;
    size_t ws_cap, ahat_cap;
    explicit View(pbcgs_ctx_t c_)
        : c(c_), st(c_->st), part(c_->part), ws(c_->ws), ahat(c_->ahat), ws_cap(c_->ws_cap), ahat_cap(c_->ahat_cap) {}
    ~View() {
      c->st = st; c->part = part; c->ws = ws; c->ahat = ahat;
      c->ws_cap = ws_cap; c->ahat_cap = ahat_cap;
      c->noalloc = false;
    }
  } view(ctx);
  double* pool = reinterpret_cast<double*>(ctx->scratch + kScratchPoolOffset);
  ctx->st = reinterpret_cast<DevState*>(ctx->scratch);
  ctx->part = reinterpret_cast<double*>(ctx->scratch + kScratchPartOffset);
  ctx->ws = pool;
  ctx->ws_cap = vec;
  ctx->ahat = pool + vec;
  ctx->ahat_cap = kScratchPoolDoubles - vec;
  ctx->noalloc = true;
  return pbcgs_solve(ctx, A, b, x, dinv, opts, info);
}

// Transpose of a CSR operator (see include/pbcgs.h).
int pbcgs_op_transpose(pbcgs_ctx_t ctx, pbcgs_op_t A, pbcgs_op_t* out) {
  if (!ctx || !A || !out) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (A->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "operator belongs to another context");
  if (A->kind != OP_CSR) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "only CSR operators are transposed");
  DeviceGuard guard(ctx->device);
  const int32_t n = A->n;
  const int64_t nnz = A->nnz;
  const int32_t nchunks = (int32_t)(((int64_t)n + kScanChunk - 1) / kScanChunk);
  int32_t *rp_t = nullptr, *ci_t = nullptr, *cnt = nullptr, *orig = nullptr, *bsum = nullptr, *boff = nullptr;
  double* va_t = nullptr;
  auto cleanup = [&]() {
    if (cnt) (void)hipFree(cnt);
    if (orig) (void)hipFree(orig);
    if (bsum) (void)hipFree(bsum);
    if (boff) (void)hipFree(boff);
  };
  bool ok = hipMalloc(&rp_t, sizeof(int32_t) * ((size_t)n + 1)) == hipSuccess &&
            hipMalloc(&ci_t, sizeof(int32_t) * std::max<size_t>((size_t)nnz, 1)) == hipSuccess &&
            hipMalloc(&va_t, sizeof(double) * std::max<size_t>((size_t)nnz, 1)) == hipSuccess &&
            hipMalloc(&cnt, sizeof(int32_t) * ((size_t)n + 1)) == hipSuccess &&
            hipMalloc(&orig, sizeof(int32_t) * std::max<size_t>((size_t)nnz, 1)) == hipSuccess &&
            hipMalloc(&bsum, sizeof(int32_t) * (size_t)nchunks) == hipSuccess &&
            hipMalloc(&boff, sizeof(int32_t) * (size_t)nchunks) == hipSuccess;
  if (!ok) {
    cleanup();
    if (rp_t) (void)hipFree(rp_t);
    if (ci_t) (void)hipFree(ci_t);
    if (va_t) (void)hipFree(va_t);
    return fail(ctx, PBCGS_ERR_ALLOC, "transpose allocation failed");
  }
  hipStream_t s = ctx->stream;
  const CsrOp op{A->rp, A->ci, A->va, n};
  auto run = [&]() -> int {
    HIP_TRY(ctx, hipMemsetAsync(cnt, 0, sizeof(int32_t) * ((size_t)n + 1), s));
    const int g = (int)std::min<int64_t>((nnz + kWG - 1) / kWG, 8192);
    if (nnz > 0) k_count_cols<<<g, kWG, 0, s>>>(op, nnz, cnt);
    // row pointers of A^T: exclusive prefix sum of the column counts
    k_scan_chunks<<<nchunks, kWG, 0, s>>>(cnt, n, rp_t, bsum);
    HIP_TRY(ctx, hipGetLastError());
    std::vector<int32_t> hb((size_t)nchunks), ho((size_t)nchunks);
    HIP_TRY(ctx, hipMemcpyAsync(hb.data(), bsum, sizeof(int32_t) * hb.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int64_t run_total = 0;
    for (int32_t c = 0; c < nchunks; ++c) {
      ho[(size_t)c] = (int32_t)run_total;
      run_total += hb[(size_t)c];
    }
    if (run_total != nnz) return fail(ctx, PBCGS_ERR_INVALID_ARG, "column counts do not add up to nnz");
    HIP_TRY(ctx, hipMemcpyAsync(boff, ho.data(), sizeof(int32_t) * ho.size(), hipMemcpyHostToDevice, s));
    k_scan_add<<<(n + kWG - 1) / kWG, kWG, 0, s>>>(rp_t, n, boff);
    const int32_t last = (int32_t)nnz;
    HIP_TRY(ctx, hipMemcpyAsync(rp_t + n, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
    // cursors start at the row pointers; scatter, then order each row
    HIP_TRY(ctx, hipMemcpyAsync(cnt, rp_t, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    k_fill_t<<<(n + kWG - 1) / kWG, kWG, 0, s>>>(op, cnt, ci_t, va_t, orig);
    k_sort_t<<<(n + kWG - 1) / kWG, kWG, 0, s>>>(n, rp_t, ci_t, va_t, orig);
    k_sort_t_long<<<(int)std::min<int64_t>(n, 1024), kWG, 0, s>>>(n, rp_t, ci_t, va_t, orig);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return PBCGS_SUCCESS;
  };
  const int rc = run();
  cleanup();
  if (rc != PBCGS_SUCCESS) {
    (void)hipFree(rp_t);
    (void)hipFree(ci_t);
    (void)hipFree(va_t);
    return rc;
  }
  pbcgs_op_t T = new pbcgs_op_s();
  T->ctx = ctx;
  T->kind = OP_CSR;
  T->n = n;
  T->nnz = nnz;
  T->rp = T->own_rp = rp_t;
  T->ci = T->own_ci = ci_t;
  T->va = T->own_va = va_t;
  int rc2 = make_compact(ctx, T);
  if (rc2 == PBCGS_SUCCESS) rc2 = make_dia(ctx, T);
  if (rc2 != PBCGS_SUCCESS) {
    (void)pbcgs_op_destroy(T);
    return rc2;
  }
  *out = T;
  return PBCGS_SUCCESS;
}

// Entry gradient dL/da_ij = -lambda_i x_j (see include/pbcgs.h).
int pbcgs_csr_outer_grad(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* lambda, const double* x, double* grad) {
  if (!ctx || !A || !lambda || !x || !grad) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (A->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "operator belongs to another context");
  if (A->kind != OP_CSR) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "CSR operators only");
  DeviceGuard guard(ctx->device);
  k_outer_grad<<<(A->n + kWG - 1) / kWG, kWG, 0, ctx->stream>>>(CsrOp{A->rp, A->ci, A->va, A->n}, lambda, x, grad);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return PBCGS_SUCCESS;
}

// Batched solve (see include/pbcgs.h).
int pbcgs_solve_batched(pbcgs_ctx_t ctx, int32_t nsys, const pbcgs_op_t* A, const double* const* b,
                        double* const* x, const pbcgs_opts* opts, pbcgs_info* infos) {
  if (!ctx || !A || !b || !x || !opts || !infos) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (nsys <= 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "nsys must be positive");
  const pbcgs_opts& o = *opts;
  if (o.variant < PBCGS_BICGSTAB || o.variant > PBCGS_PIPE_CG)
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown variant");
  if (o.variant >= PBCGS_CA_BICGSTAB)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "batched solves run BiCGStab or p-BiCGStab");
  if (o.precond != PBCGS_PRECOND_NONE)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "batched solves take no preconditioner");
  if (o.precision != PBCGS_FP64) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "batched solves are binary64");
  if (o.maxit < 0 || !(o.tol >= 0.0)) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad maxit or tol");
  if (o.variant == PBCGS_PBICGSTAB_RR && o.rr_period < 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad rr_period");
  if (o.history) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "batched solves keep no history");
  if (ctx->perturb_iter >= 0)
    return fail(ctx, PBCGS_ERR_UNSUPPORTED, "the residual perturbation hook applies to single solves only");
  int gcap = env_int("PBCGS_BATCH_GCAP", ctx->batch_gcap > 0 ? ctx->batch_gcap : 64);
  if (gcap < 1 || gcap > kMaxG) gcap = 64;
  std::vector<SysDesc> desc((size_t)nsys);
  bool compact = compact_ok(o);  // every system holds compact columns
  bool dia = dia_ok(o);          // every system has a diagonal layout
  for (int32_t k = 0; k < nsys && dia; ++k) dia = A[k] && A[k]->kind == OP_CSR && A[k]->ndia > 0;
  int64_t totalG = 0;
  size_t wsneed = 0, dianeed = 0;
  for (int32_t k = 0; k < nsys; ++k) {
    const pbcgs_op_t op = A[k];
    if (!op || op->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad operator " + std::to_string(k));
    if (op->kind != OP_CSR) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "batched solves take CSR operators");
    if (!b[k] || !x[k] || (const void*)b[k] == (const void*)x[k])
      return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad b or x of system " + std::to_string(k));
    int32_t R = dia ? 2 : 1;  // the two-rows-per-lane kernels need two blocks per wave
    int64_t G = ((int64_t)op->n + 256 * (int64_t)R - 1) / (256 * (int64_t)R);
    while (G > gcap && R < kMaxR) {
      R *= 2;
      G = ((int64_t)op->n + 256 * (int64_t)R - 1) / (256 * (int64_t)R);
    }
    if (G > kMaxG) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "system " + std::to_string(k) + " too large");
    SysDesc& d = desc[(size_t)k];
    d.rp = op->rp; d.ci = op->ci; d.c16 = op->c16; d.va = op->va;
    d.x = x[k]; d.b = b[k];
    compact = compact && op->c16 != nullptr;
    d.np = (int64_t)padded(op->n);
    d.n = op->n; d.G = (int32_t)G; d.R = R;
    if (dia) {
      d.dmask = op->dmask;
      d.nd = op->ndia;
      for (int j = 0; j < op->ndia; ++j) d.doff[j] = op->dia_off[j];
      dianeed += (size_t)op->ndia * (size_t)d.np;
    }
    totalG += G;
    wsneed += (size_t)8 * (size_t)d.np;
  }
  // Workgroups are dispatched in index order: the systems whose workgroups
  // hold the most rows (largest R, then most rows) come first, so that a
  // launch does not end waiting on long workgroups dispatched last.  Each
  // system's reductions index its own workgroups, so results do not change.
  {
    std::vector<int32_t> order((size_t)nsys);
    for (int32_t k = 0; k < nsys; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) {
      const SysDesc &dp = desc[(size_t)p], &dq = desc[(size_t)q];
      return dp.R != dq.R ? dp.R > dq.R : dp.n > dq.n;
    });
    int64_t wg = 0;
    for (int32_t k : order) {
      desc[(size_t)k].wg0 = (int32_t)wg;
      wg += desc[(size_t)k].G;
    }
  }
  if (totalG > (int64_t)INT32_MAX / 2) return fail(ctx, PBCGS_ERR_UNSUPPORTED, "too many workgroups");
  DeviceGuard guard(ctx->device);
  const size_t nst = (size_t)nsys * 4;
  int rc = grow(ctx, ctx->bsys, ctx->bsys_cap, (size_t)nsys, "batch table");
  if (rc == PBCGS_SUCCESS) rc = grow(ctx, ctx->bmap, ctx->bmap_cap, (size_t)totalG, "workgroup map");
  if (rc == PBCGS_SUCCESS) rc = grow(ctx, ctx->bws, ctx->bws_cap, wsneed, "batch vectors");
  if (rc == PBCGS_SUCCESS) rc = grow(ctx, ctx->bst, ctx->bst_cap, nst, "batch states");
  if (rc == PBCGS_SUCCESS) rc = grow(ctx, ctx->bpart, ctx->bpart_cap, (size_t)PB_COUNT * kMaxD * totalG, "partials");
  if (rc == PBCGS_SUCCESS && dia) rc = grow(ctx, ctx->bdia, ctx->bdia_cap, dianeed, "diagonal-layout values");
  if (rc != PBCGS_SUCCESS) return rc;
  PoisonScope poison_scope(ctx, (o.flags & 32) != 0);
  poison(ctx, ctx->bws, wsneed * sizeof(double));
  poison(ctx, ctx->bpart, (size_t)PB_COUNT * kMaxD * (size_t)totalG * sizeof(double));
  if (dia) poison(ctx, ctx->bdia, dianeed * sizeof(double));
  if (ctx->bhst_cap < nst) {
    if (ctx->bhst) { (void)hipStreamSynchronize(ctx->stream); (void)hipHostFree(ctx->bhst); ctx->bhst = nullptr; }
    ctx->bhst_cap = 0;
    if (hipHostMalloc(&ctx->bhst, 2 * nst * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
      ctx->bhst = nullptr;
      return fail(ctx, PBCGS_ERR_ALLOC, "pinned poll buffer");
    }
    ctx->bhst_cap = nst;
  }
  std::vector<int32_t> map((size_t)totalG);
  size_t off = 0, doff = 0;
  for (int32_t k = 0; k < nsys; ++k) {
    SysDesc& d = desc[(size_t)k];
    d.ws = ctx->bws + off;
    off += (size_t)8 * (size_t)d.np;
    if (dia) {
      d.dva = ctx->bdia + doff;
      doff += (size_t)d.nd * (size_t)d.np;
    }
    d.st = ctx->bst + (size_t)k * 4;
    for (int32_t g = 0; g < d.G; ++g) map[(size_t)d.wg0 + g] = k;
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->bsys, desc.data(), desc.size() * sizeof(SysDesc), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->bmap, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the host tables may go away after this
  const int st = dia       ? BatchDriver<DiaOpB>(ctx, o, nsys, (int32_t)totalG).run(infos)
                 : compact ? BatchDriver<CsrOp16>(ctx, o, nsys, (int32_t)totalG).run(infos)
                           : BatchDriver<CsrOp>(ctx, o, nsys, (int32_t)totalG).run(infos);
  if (st >= 0)
    for (int32_t k = 0; k < nsys; ++k) {
      infos[k].rows_per_wave_blocks = desc[(size_t)k].R;
      infos[k].workgroups = desc[(size_t)k].G;
    }
  return st;
}

// Autotuner of the launch shape (see include/pbcgs.h).
int pbcgs_tune(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, const pbcgs_opts* opts, int32_t iters,
               pbcgs_tune_report* rep) {
  if (!ctx || !A || !b || !opts || !rep) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (iters < 1) return fail(ctx, PBCGS_ERR_INVALID_ARG, "iters must be positive");
  if (opts->variant < PBCGS_BICGSTAB || opts->variant > PBCGS_PIPE_CG ||
      (opts->precision != PBCGS_FP64 && opts->precision != PBCGS_FP32_RR64))
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown variant or precision");
  DeviceGuard guard(ctx->device);
  std::memset(rep, 0, sizeof *rep);
  double* xs = nullptr;
  if (hipMalloc(&xs, sizeof(double) * (size_t)A->n) != hipSuccess) return fail(ctx, PBCGS_ERR_ALLOC, "tune scratch");
  pbcgs_opts o = *opts;
  o.tol = 0.0;
  o.maxit = iters;
  o.history = nullptr;
  o.flags = opts->flags & (4 | 8 | 16);  // keep the alpha form and the read path; graph replay, no timing
  o.check_every = 0;
  int32_t& slot = A->tuned_R[o.variant][o.precision == PBCGS_FP32_RR64 ? 1 : 0][read_path(o.flags)];
  const int32_t saved = slot;
  double best = -1.0;
  int rc = PBCGS_SUCCESS;
  for (int R = 1; R <= kMaxR && rep->ncand < 12; R *= 2) {
    const int64_t G = ((int64_t)A->n + 256 * (int64_t)R - 1) / (256 * (int64_t)R);
    if (G > kMaxG) continue;
    if (rep->ncand > 0 && G < 64) break;  // fewer workgroups than a quarter of the CUs: not a candidate
    slot = R;
    double ms = 0.0;
    // the first run captures the graphs; the fastest of the next three counts
    for (int t = 0; t < 4 && rc >= 0; ++t) {
      pbcgs_info info;
      HIP_TRY(ctx, hipMemsetAsync(xs, 0, sizeof(double) * (size_t)A->n, ctx->stream));
      rc = pbcgs_solve(ctx, A, b, xs, nullptr, &o, &info);
      if (t == 1 || (t > 1 && info.ms < ms)) ms = info.ms;
    }
    if (rc < 0) break;
    const double per = ms / iters;
    rep->cand[rep->ncand] = R;
    rep->ms_per_iter[rep->ncand] = per;
    ++rep->ncand;
    if (best < 0.0 || per < best) { best = per; rep->best = R; }
    if (G <= 1) break;  // larger R only adds idle waves
  }
  (void)hipFree(xs);
  if (rc < 0) {
    slot = saved;
    return rc;
  }
  slot = rep->best;
  rep->best_ms_per_iter = best;
  pbcgs_tune_entry e = make_key(ctx, A, o.variant, o.precision, read_path(o.flags));
  e.best = rep->best;
  cache_store(e);
  return PBCGS_SUCCESS;
}

// The launch-shape cache (see include/pbcgs.h).
int32_t pbcgs_tune_cache_size(void) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  return (int32_t)c.entries.size();
}

int pbcgs_tune_cache_get(int32_t i, pbcgs_tune_entry* out) {
  if (!out) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "out is NULL");
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  if (i < 0 || (size_t)i >= c.entries.size()) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "no cache entry at this index");
  *out = c.entries[(size_t)i];
  return PBCGS_SUCCESS;
}

int pbcgs_tune_cache_put(const pbcgs_tune_entry* e) {
  if (!e) return fail(nullptr, PBCGS_ERR_INVALID_ARG, "entry is NULL");
  if (std::memchr(e->device, 0, sizeof e->device) == nullptr || std::memchr(e->build, 0, sizeof e->build) == nullptr)
    return fail(nullptr, PBCGS_ERR_INVALID_ARG, "device and build must be NUL-terminated");
  if (e->variant < PBCGS_BICGSTAB || e->variant > PBCGS_PIPE_CG ||
      (e->precision != PBCGS_FP64 && e->precision != PBCGS_FP32_RR64) || e->op_kind < OP_CSR ||
      e->op_kind > OP_GRID || e->nnz < 0 || e->read_path < 0 || e->read_path > 2)
    return fail(nullptr, PBCGS_ERR_INVALID_ARG, "bad variant, precision, operator kind, nnz or read path");
  if (!shape_fits(e->n, e->best))
    return fail(nullptr, PBCGS_ERR_INVALID_ARG, "best must be a power of two whose grid fits n rows");
  pbcgs_tune_entry c;
  std::memset(&c, 0, sizeof c);
  std::memcpy(c.device, e->device, sizeof c.device);
  std::memcpy(c.build, e->build, sizeof c.build);
  c.nnz = e->nnz;
  c.n = e->n;
  c.op_kind = e->op_kind;
  c.variant = e->variant;
  c.precision = e->precision;
  c.read_path = e->read_path;
  c.best = e->best;
  cache_store(c);
  return PBCGS_SUCCESS;
}

int pbcgs_tune_cache_clear(void) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.entries.clear();
  return PBCGS_SUCCESS;
}

int pbcgs_tune_cache_key(pbcgs_ctx_t ctx, pbcgs_op_t A, int32_t variant, int32_t precision, int32_t flags,
                         pbcgs_tune_entry* out) {
  if (!ctx || !A || !out) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL argument");
  if (A->ctx != ctx) return fail(ctx, PBCGS_ERR_INVALID_ARG, "operator belongs to another context");
  if (variant < PBCGS_BICGSTAB || variant > PBCGS_PIPE_CG || (precision != PBCGS_FP64 && precision != PBCGS_FP32_RR64))
    return fail(ctx, PBCGS_ERR_INVALID_ARG, "unknown variant or precision");
  *out = make_key(ctx, A, variant, precision, read_path(flags));
  out->best = cache_find(*out);
  return PBCGS_SUCCESS;
}

int pbcgs_tune_batched(pbcgs_ctx_t ctx, int32_t nsys, const pbcgs_op_t* A, const double* const* b,
                       const pbcgs_opts* opts, int32_t iters, pbcgs_tune_report* rep) {
  if (!ctx || !A || !b || !opts || !rep || nsys <= 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "bad argument");
  if (iters < 0) return fail(ctx, PBCGS_ERR_INVALID_ARG, "iters must not be negative");
  // iters = 0: time complete solves at the caller's tol and maxit.  Systems
  // stop at different iterations, so the best cap for the whole solve (many
  // systems at first, a few large ones at the end) differs from the best cap
  // for its first iterations.
  const bool complete = (iters == 0);
  DeviceGuard guard(ctx->device);
  std::memset(rep, 0, sizeof *rep);
  size_t tot = 0;
  for (int32_t k = 0; k < nsys; ++k) {
    if (!A[k]) return fail(ctx, PBCGS_ERR_INVALID_ARG, "NULL operator");
    tot += padded(A[k]->n);
  }
  double* xs = nullptr;
  if (hipMalloc(&xs, sizeof(double) * std::max<size_t>(tot, 1)) != hipSuccess)
    return fail(ctx, PBCGS_ERR_ALLOC, "tune scratch");
  std::vector<double*> xp((size_t)nsys);
  size_t off = 0;
  for (int32_t k = 0; k < nsys; ++k) {
    xp[(size_t)k] = xs + off;
    off += padded(A[k]->n);
  }
  pbcgs_opts o = *opts;
  if (!complete) {
    o.tol = 0.0;
    o.maxit = iters;
  }
  o.history = nullptr;
  o.flags = 0;
  const int32_t saved = ctx->batch_gcap;
  std::vector<pbcgs_info> infos((size_t)nsys);
  double best = -1.0;
  int rc = PBCGS_SUCCESS;
  for (int gcap = 8; gcap <= 512 && rep->ncand < 12; gcap *= 2) {
    ctx->batch_gcap = gcap;
    double ms = 0.0;
    for (int t = 0; t < 2 && rc >= 0; ++t) {
      HIP_TRY(ctx, hipMemsetAsync(xs, 0, sizeof(double) * std::max<size_t>(tot, 1), ctx->stream));
      rc = pbcgs_solve_batched(ctx, nsys, A, b, xp.data(), &o, infos.data());
      ms = infos[0].ms;
    }
    if (rc < 0) break;
    const double per = complete ? ms : ms / iters;
    rep->cand[rep->ncand] = gcap;
    rep->ms_per_iter[rep->ncand] = per;
    ++rep->ncand;
    if (best < 0.0 || per < best) { best = per; rep->best = gcap; }
  }
  (void)hipFree(xs);
  if (rc < 0) {
    ctx->batch_gcap = saved;
    return rc;
  }
  ctx->batch_gcap = rep->best;
  rep->best_ms_per_iter = best;
  return PBCGS_SUCCESS;
}

}  // extern "C"
