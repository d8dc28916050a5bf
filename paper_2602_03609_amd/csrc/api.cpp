// Host side of the C ABI declared in include/vif.h: argument validation,
// workspace layout, per-lag tables for the neighbor key, launch sequencing and
// error reporting. No device memory is allocated here.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <algorithm>
#include <functional>
#include <memory>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "vif.h"
#include "vif_learn.h"
#include "vif_batch.h"
#include "vif_residual.h"
#include "vif_grad.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int32_t ok() {
  g_err.clear();
  return VIF_OK;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(VIF_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace vif {
int32_t report_error(int32_t code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace vif

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- optional stage timing: HIP events on the caller's stream ----------------
struct Prof {
  bool on = false;
  hipEvent_t beg[VIF_NSTAGES] = {}, end[VIF_NSTAGES] = {};
  bool used[VIF_NSTAGES] = {};
  double total_ms[VIF_NSTAGES] = {};
  int32_t calls[VIF_NSTAGES] = {};
};
Prof g_prof;

int32_t prof_mark(int st, bool at_end, hipStream_t s) {
  if (!g_prof.on) return VIF_OK;
  hipEvent_t* ev = at_end ? &g_prof.end[st] : &g_prof.beg[st];
  if (!*ev) {
    hipError_t e = hipEventCreate(ev);
    if (e != hipSuccess) return fail(VIF_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
  }
  hipError_t e = hipEventRecord(*ev, s);
  if (e != hipSuccess) return fail(VIF_E_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  if (at_end) g_prof.used[st] = true;
  return VIF_OK;
}

// Called after the stream has been synchronised.
void prof_collect() {
  if (!g_prof.on) return;
  for (int st = 0; st < VIF_NSTAGES; ++st) {
    if (!g_prof.used[st]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_prof.beg[st], g_prof.end[st]) == hipSuccess) {
      g_prof.total_ms[st] += ms;
      g_prof.calls[st] += 1;
    }
    g_prof.used[st] = false;
  }
}

#define PROF(st, end)                          \
  do {                                         \
    int32_t p_ = prof_mark((st), (end), s);    \
    if (p_) return p_;                         \
  } while (0)

int kpad_of(int k) { return k > 0 ? ((k + 1 + 63) / 64) * 64 : 0; }

struct Layout {
  size_t c2 = 0, f2 = 0, b2 = 0, k2 = 0, px2 = 0, py2 = 0, pi2 = 0, pflag = 0, plist = 0,
         pcount = 0, pemb = 0;  // proposal search
  size_t lag = 0;  // per-lag Gneiting factors (VIF per-point kernel)
  size_t flags = 0, out = 0, part = 0, sums = 0, logD = 0, z = 0, Sk = 0, P = 0, Pb = 0, U = 0, W = 0,
         syrk = 0, M = 0, q = 0, dscr = 0, tab1 = 0, tab2 = 0, bnd = 0, bbox = 0, counts = 0,
         fill = 0, bsum = 0, key = 0, px = 0, py = 0, pidx = 0, total = 0;
  int kpad = 0, splits = 0;
};

// Flags block: [0] fail_points, [1] fail_sigma_k, [2] fail_M, [3] bad_nbr (uint64 each),
// [4] time flags (uint32).
constexpr size_t kFlagBytes = 256;

// Average number of points of one time slab per grid cell of the neighbor index
// (search time on a 1.1M-point network of 365 daily slabs: 16 -> 4.62 ms, 24 -> 4.65,
// 32 -> 4.74, 64 -> 5.22).
constexpr double kCellTarget = 16.0;

// Real-valued times: the search's time bins hold about this many points each.
constexpr int64_t kBinPoints = 2048;

Layout make_layout(int64_t n, int m, int k, int prec, int op, int chunk_rows = 4096) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  const size_t es = prec == VIF_PREC_FP64 ? 8 : 4;
  L.flags = take(kFlagBytes);
  if (op == VIF_OP_NEIGHBORS) {
    L.tab1 = take(sizeof(double) * VIF_MAX_LAGS);
    L.tab2 = take(sizeof(double) * VIF_MAX_LAGS);
    L.bnd = take(sizeof(double) * VIF_MAX_LAGS);
    L.bbox = take(sizeof(double) * (4 * 256 + 4));
    L.counts = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
    L.fill = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
    L.bsum = take(sizeof(int32_t) * ((size_t)vif::kMaxCells / 1024 + 2));
    L.key = take(sizeof(int32_t) * (size_t)n);
    L.px = take(sizeof(double) * (size_t)n);
    L.py = take(sizeof(double) * (size_t)n);
    L.pidx = take(sizeof(int32_t) * (size_t)n);
    L.total = off;
    return L;
  }
  (void)m;
  L.out = take(sizeof(double) * 8);
  L.part = take(sizeof(double) * 256);
  L.sums = take(sizeof(double) * 8);
  if (op == VIF_OP_NLL) {
    L.logD = take(sizeof(double) * (size_t)n);
    L.z = take(sizeof(double) * (size_t)n);
  }
  if (k > 0) {
    // processing order of the per-point kernel (Z order of a fine grid per time slab)
    L.bbox = take(sizeof(double) * (4 * 256 + 4));
    L.counts = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
    L.fill = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
    L.bsum = take(sizeof(int32_t) * ((size_t)vif::kMaxCells / 1024 + 2));
    L.key = take(sizeof(int32_t) * (size_t)n);
    L.pidx = take(sizeof(int32_t) * (size_t)n);
    L.kpad = kpad_of(k);
    const size_t kk = (size_t)L.kpad * L.kpad;
    L.Sk = take(sizeof(double) * kk);
    L.P = take(sizeof(double) * kk);
    if (prec >= VIF_PREC_BF16X3) L.Pb = take((prec == VIF_PREC_BF16X6 ? 6 : 4) * kk);
    L.dscr = take(std::max(sizeof(double) * 64 * 64, vif::trinv_scratch_bytes(L.kpad)));
    L.lag = take(sizeof(double) * 2 * VIF_MAX_LAGS);
    L.U = take(es * (size_t)n * L.kpad);
    if (op == VIF_OP_NLL) {
      if (prec >= VIF_PREC_BF16X3) {
        // bfloat16 term planes of W (2 or 3), rows padded to a multiple of 16.
        const int64_t wr = vif::w_plane_rows(n);
        const size_t nsp = prec == VIF_PREC_BF16X6 ? 3 : 2;
        L.W = take(2 * nsp * (size_t)wr * L.kpad);
        L.splits = vif::syrk_chunks(wr, L.kpad, prec, chunk_rows);
        L.syrk = take(vif::syrk_part_bytes(wr, L.kpad, prec, chunk_rows));
      } else {
        L.W = take(es * (size_t)n * L.kpad);
        L.splits = vif::syrk_chunks(n, L.kpad, prec);
        L.syrk = take(vif::syrk_part_bytes(n, L.kpad, prec));
      }
      L.M = take(sizeof(double) * kk);
      L.q = take(sizeof(double) * L.kpad);
    }
  }
  L.total = off;
  return L;
}

// Low-rank factor in FP64 (Sigma_k, L_k^-1, U) plus the residual variances.
Layout make_residual_layout(int64_t n, int k) {
  Layout L = make_layout(n, 0, k, VIF_PREC_FP64, VIF_OP_FACTOR);
  L.logD = L.total;  // residual variances r(j, j)
  L.total += align256(sizeof(double) * (size_t)n);
  L.tab1 = L.total;  // per-lag factors of the Gneiting kernel
  L.total += align256(sizeof(double) * 2 * VIF_MAX_LAGS);
  return L;
}

// Exact-search layout plus the proposal grid, fallback flags and list.
Layout make_propose_layout(int64_t n) {
  Layout L = make_layout(n, 1, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS);
  size_t off = L.total;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  L.c2 = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
  L.f2 = take(sizeof(int32_t) * ((size_t)vif::kMaxCells + 1));
  L.b2 = take(sizeof(int32_t) * ((size_t)vif::kMaxCells / 1024 + 2));
  L.k2 = take(sizeof(int32_t) * (size_t)n);
  L.px2 = take(sizeof(double) * (size_t)n);
  L.py2 = take(sizeof(double) * (size_t)n);
  L.pi2 = take(sizeof(int32_t) * (size_t)n);
  L.pflag = take(sizeof(int32_t) * (size_t)n);
  L.plist = take(sizeof(int32_t) * (size_t)n);
  L.pcount = take(256);
  L.pemb = take(sizeof(float) * 16 * (size_t)n);
  L.total = off;
  return L;
}

bool finite(double x) { return isfinite(x); }

int nu_code(double nu) {
  if (nu == 0.5) return 0;
  if (nu == 1.5) return 1;
  if (nu == 2.5) return 2;
  return -1;
}

int32_t check_kernel(const vif_kernel* K) {
  if (!K) return fail(VIF_E_ARG, "kern is NULL");
  if (!finite(K->sigma2) || !(K->sigma2 > 0)) return fail(VIF_E_ARG, "sigma2 must be finite and > 0");
  if (!finite(K->nugget) || K->nugget < 0) return fail(VIF_E_ARG, "nugget must be finite and >= 0");
  if (!finite(K->jitter) || K->jitter < 0) return fail(VIF_E_ARG, "jitter must be finite and >= 0");
  switch (K->kind) {
    case VIF_KERNEL_GNEITING:
      if (!finite(K->a) || !(K->a > 0)) return fail(VIF_E_ARG, "a must be > 0");
      if (!finite(K->c) || !(K->c > 0)) return fail(VIF_E_ARG, "c must be > 0");
      if (!(K->alpha > 0 && K->alpha <= 1)) return fail(VIF_E_ARG, "alpha must be in (0,1]");
      if (!(K->gamma > 0 && K->gamma <= 1)) return fail(VIF_E_ARG, "gamma must be in (0,1]");
      if (!(K->beta >= 0 && K->beta <= 1)) return fail(VIF_E_ARG, "beta must be in [0,1]");
      if (!finite(K->tau) || K->tau < 0) return fail(VIF_E_ARG, "tau must be >= 0");
      return VIF_OK;
    case VIF_KERNEL_GNEITING_MATERN:
      if (!finite(K->a) || !(K->a > 0)) return fail(VIF_E_ARG, "a must be > 0");
      if (!finite(K->c) || !(K->c > 0)) return fail(VIF_E_ARG, "c must be > 0");
      if (!(K->alpha > 0 && K->alpha <= 1)) return fail(VIF_E_ARG, "alpha must be in (0,1]");
      if (!(K->gamma >= 0 && K->gamma <= 1)) return fail(VIF_E_ARG, "gamma must be in [0,1]");
      if (!finite(K->delta) || K->delta < 0) return fail(VIF_E_ARG, "delta must be >= 0");
      if (nu_code(K->nu) < 0)
        return fail(VIF_E_UNSUPPORTED, "nu must be 0.5, 1.5 or 2.5 (closed forms only)");
      return VIF_OK;
    case VIF_KERNEL_MATERN_ANISO:
      if (!finite(K->range_s) || !(K->range_s > 0)) return fail(VIF_E_ARG, "range_s must be > 0");
      if (!finite(K->range_t) || !(K->range_t > 0)) return fail(VIF_E_ARG, "range_t must be > 0");
      if (nu_code(K->nu) < 0)
        return fail(VIF_E_UNSUPPORTED, "nu must be 0.5, 1.5 or 2.5 (closed forms only)");
      return VIF_OK;
    default:
      return fail(VIF_E_ARG, "unknown kernel kind %d", (int)K->kind);
  }
}

vif::KernDev to_dev(const vif_kernel* K) {
  vif::KernDev d{};
  d.kind = K->kind;
  d.nu_code = (K->kind == VIF_KERNEL_GNEITING) ? 0 : nu_code(K->nu);
  d.gamma_half = (K->kind == VIF_KERNEL_GNEITING && K->gamma == 0.5) ? 1 : 0;
  d.sigma2 = K->sigma2;
  d.nugget = K->nugget;
  d.a = K->a;
  d.c = K->c;
  d.two_alpha = 2.0 * K->alpha;
  d.tau = K->tau;
  d.bg = K->beta * K->gamma;
  d.gamma = K->gamma;
  d.half_gamma = K->gamma / 2.0;
  d.dpg = K->delta + K->gamma;
  if (K->kind == VIF_KERNEL_MATERN_ANISO) {
    d.ir_s2 = 1.0 / (K->range_s * K->range_s);
    d.ir_t2 = 1.0 / (K->range_t * K->range_t);
  }
  return d;
}

int32_t check_points(const vif_points* p, const char* what) {
  if (!p) return fail(VIF_E_ARG, "%s is NULL", what);
  if (p->n < 0 || p->n >= (int64_t)INT32_MAX) return fail(VIF_E_ARG, "%s->n out of range", what);
  if (p->n > 0 && (!p->sx || !p->sy || !p->t)) return fail(VIF_E_ARG, "%s has NULL arrays", what);
  return VIF_OK;
}

int32_t check_common(const vif_points* p, const vif_kernel* kern, int32_t m, void* ws,
                     size_t ws_bytes, size_t need) {
  int32_t st = check_points(p, "points");
  if (st) return st;
  if (p->n < 1) return fail(VIF_E_ARG, "n must be >= 1");
  st = check_kernel(kern);
  if (st) return st;
  if (m < 0) return fail(VIF_E_ARG, "m must be >= 0");
  if (m > VIF_MAX_M) return fail(VIF_E_UNSUPPORTED, "m = %d exceeds VIF_MAX_M = %d", m, VIF_MAX_M);
  if (!ws) return fail(VIF_E_ARG, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(VIF_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(VIF_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return VIF_OK;
}

struct Flags {
  unsigned long long fail_pts, fail_sk, fail_m, bad_nbr;
  uint32_t tflag, pad;
};

int32_t init_flags(char* ws, const Layout& L, hipStream_t s) {
  HIPCHK(vif::launch_init_flags(ws + L.flags, s));
  return VIF_OK;
}

int32_t read_flags(char* ws, const Layout& L, Flags* f, double* out, int nout, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(f, ws + L.flags, sizeof(Flags), hipMemcpyDeviceToHost, s));
  if (nout > 0) HIPCHK(hipMemcpyAsync(out, ws + L.out, sizeof(double) * nout, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return VIF_OK;
}

int32_t report_flags(const Flags& f) {
  if (f.bad_nbr != ~0ull)
    return fail(VIF_E_ARG, "neighbor row %llu has an index that is not an earlier point, or -1 padding before a valid entry",
                f.bad_nbr);
  if (f.fail_sk != ~0ull)
    return fail(VIF_E_NOT_PD, "Sigma_k (inducing-point covariance) is not positive definite at row %llu", f.fail_sk);
  if (f.fail_pts != ~0ull)
    return fail(VIF_E_NOT_PD, "conditioning block of point %llu is not positive definite", f.fail_pts);
  if (f.fail_m != ~0ull)
    return fail(VIF_E_NOT_PD, "Woodbury matrix M is not positive definite at row %llu", f.fail_m);
  return VIF_OK;
}

// Processing order for the per-point VIF kernel: points sorted by time slab and
// then by the Z order of a fine spatial grid, so that consecutive points (and
// the workgroups one XCD runs together) share most of their neighbors' U rows.
int32_t build_order(const vif_points* p, char* ws, const Layout& L, hipStream_t s,
                    const int32_t** ord, int* nlag) {
  Flags* dflags = reinterpret_cast<Flags*>(ws + L.flags);
  double* bbox = reinterpret_cast<double*>(ws + L.bbox);
  HIPCHK(vif::launch_validate_times(p->n, p->t, &dflags->tflag, s));
  HIPCHK(vif::launch_bbox(p->n, p->sx, p->sy, bbox, bbox + 4 * 256, s));
  Flags f;
  double tt[2], bb[4];
  HIPCHK(hipMemcpyAsync(&f, ws + L.flags, sizeof(f), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&tt[0], p->t, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&tt[1], p->t + (p->n - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(bb, bbox + 4 * 256, sizeof(bb), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *ord = nullptr;
  if (f.tflag & 1u) return fail(VIF_E_ARG, "times must be finite");
  if (!isfinite(bb[0]) || !isfinite(bb[1]) || !isfinite(bb[2]) || !isfinite(bb[3]))
    return fail(VIF_E_ARG, "coordinates must be finite");
  // Integer, nondecreasing times: one slab per time value; otherwise one slab.
  int nslab = 1;
  const double span = tt[1] - tt[0];
  if (!(f.tflag & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) nslab = (int)span + 1;
  *nlag = (!(f.tflag & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) ? nslab : 0;
  const double per = (double)p->n / nslab;
  int bits = 0;
  while (bits < 10 && (double)(1 << (2 * (bits + 1))) * 3.0 <= per &&
         (int64_t)(1 << (2 * (bits + 1))) * nslab <= vif::kMaxCells)
    ++bits;
  const double w = bb[1] - bb[0], h = bb[3] - bb[2];
  vif::GridArgs g{};
  g.gx = g.gy = 1 << bits;
  g.ncell = g.gx * g.gy;
  g.nslab = nslab;
  g.morton = 1;
  g.xmin = bb[0];
  g.ymin = bb[2];
  g.cw = w > 0 ? w / g.gx : 1.0;
  g.ch = h > 0 ? h / g.gy : 1.0;
  g.icw = w > 0 ? g.gx / w : 0.0;
  g.ich = h > 0 ? g.gy / h : 0.0;
  HIPCHK(vif::launch_grid_build(p->n, p->sx, p->sy, p->t, tt[0], g,
                                reinterpret_cast<int32_t*>(ws + L.counts),
                                reinterpret_cast<int32_t*>(ws + L.fill),
                                reinterpret_cast<int32_t*>(ws + L.bsum),
                                reinterpret_cast<int32_t*>(ws + L.key), nullptr, nullptr,
                                reinterpret_cast<int32_t*>(ws + L.pidx), s));
  *ord = reinterpret_cast<const int32_t*>(ws + L.pidx);
  return VIF_OK;
}

// Sigma_k, its Cholesky factor and inverse, then U = C(X,Z) L_k^-T.
vif::LowRankArgs lowrank_args(const vif_points* p, const vif_points* ind, const vif_kernel* kern,
                              const Layout& L) {
  vif::LowRankArgs a{};
  a.n = p->n;
  a.k = (int)ind->n;
  a.kpad = L.kpad;
  a.K = to_dev(kern);
  a.jitter = kern->jitter;
  a.sx = p->sx; a.sy = p->sy; a.t = p->t;
  a.zx = ind->sx; a.zy = ind->sy; a.zt = ind->t;
  return a;
}

// U from L_k^-1 (in L.P): fused on chip in the split modes, else cross-covariance
// then an in-place product.
int32_t run_u(const vif::LowRankArgs& a, int prec, char* ws, const Layout& L, hipStream_t s) {
  const double* P = reinterpret_cast<const double*>(ws + L.P);
  if (prec >= VIF_PREC_BF16X3 && vif::lowrank_fused_ok(L.kpad, prec)) {
    // Cross-covariance evaluated on chip inside the product.
    PROF(VIF_STAGE_TRMM, false);
    HIPCHK(vif::launch_lowrank_fused(a, P, ws + L.Pb, reinterpret_cast<float*>(ws + L.U), prec, s));
    PROF(VIF_STAGE_TRMM, true);
    return VIF_OK;
  }
  PROF(VIF_STAGE_CROSSCOV, false);
  HIPCHK(vif::launch_crosscov(a, ws + L.U, prec, s));
  PROF(VIF_STAGE_CROSSCOV, true);
  PROF(VIF_STAGE_TRMM, false);
  HIPCHK(vif::launch_trmm(a, P, ws + L.U, prec, s));
  PROF(VIF_STAGE_TRMM, true);
  return VIF_OK;
}

// Sigma_k, its Cholesky factor and L_k^-1 (in L.P).
int32_t run_sigma_k(const vif::LowRankArgs& a, char* ws, const Layout& L, hipStream_t s) {
  double* Sk = reinterpret_cast<double*>(ws + L.Sk);
  double* P = reinterpret_cast<double*>(ws + L.P);
  auto* fl = reinterpret_cast<unsigned long long*>(ws + L.flags);
  PROF(VIF_STAGE_SIGMA_K, false);
  HIPCHK(vif::launch_cov_kk(a, Sk, s));
  HIPCHK(vif::launch_cholesky(L.kpad, Sk, reinterpret_cast<double*>(ws + L.dscr), fl + 1, s));
  HIPCHK(vif::launch_trinv(L.kpad, Sk, P, reinterpret_cast<double*>(ws + L.dscr), s));
  PROF(VIF_STAGE_SIGMA_K, true);
  return VIF_OK;
}

int32_t run_lowrank(const vif_points* p, const vif_points* ind, const vif_kernel* kern, int prec,
                    char* ws, const Layout& L, hipStream_t s) {
  const vif::LowRankArgs a = lowrank_args(p, ind, kern, L);
  const int32_t st = run_sigma_k(a, ws, L, s);
  return st ? st : run_u(a, prec, ws, L, s);
}

int32_t check_ind(const vif_points* ind, int* k) {
  *k = 0;
  if (!ind) return VIF_OK;
  int32_t st = check_points(ind, "ind");
  if (st) return st;
  if (ind->n > VIF_MAX_K) return fail(VIF_E_UNSUPPORTED, "k = %lld exceeds VIF_MAX_K = %d", (long long)ind->n, VIF_MAX_K);
  *k = (int)ind->n;
  return VIF_OK;
}

// Work that another stream runs while the NLL builds its low-rank factor: start()
// queues it behind the NLL stream's work so far, and `done` is recorded after it;
// the NLL stream waits on `done` before the per-point kernel reads the neighbors.
struct SideWork {
  std::function<int32_t(hipStream_t)> start;
  hipEvent_t done = nullptr;
};

int32_t nll_impl(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                 const int32_t* nbr, const vif_points* ind, int32_t prec, double* nll,
                 double* terms, void* wsv, size_t ws_bytes, void* hip_stream,
                 const SideWork* side = nullptr, double* lout = nullptr) {
  int k = 0;
  int32_t st = check_ind(ind, &k);
  if (st) return st;
  if (prec < VIF_PREC_FP64 || prec > VIF_PREC_BF16X6) return fail(VIF_E_ARG, "unknown precision %d", prec);
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const Layout L = make_layout(p->n, m, k, prec, VIF_OP_NLL);
  st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  if (!y) return fail(VIF_E_ARG, "y is NULL");
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (!nll) return fail(VIF_E_ARG, "nll is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  auto* fl = reinterpret_cast<unsigned long long*>(ws + L.flags);
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* out = reinterpret_cast<double*>(ws + L.out);
  if ((st = init_flags(ws, L, s))) return st;

  vif::FactorArgs fa{};
  fa.n = p->n;
  fa.m = m;
  fa.k = k;
  fa.ldu = L.kpad;
  fa.K = to_dev(kern);
  fa.sx = p->sx; fa.sy = p->sy; fa.t = p->t; fa.y = y;
  fa.nbr = nbr;
  fa.logD = reinterpret_cast<double*>(ws + L.logD);
  fa.fail = fl;
  fa.bad_nbr = fl + 3;
  fa.Lout = lout;
  if (k > 0) {
    int nlag = 0;
    if ((st = build_order(p, ws, L, s, &fa.ord, &nlag))) return st;
    if (kern->kind == VIF_KERNEL_GNEITING && nlag > 0) {
      HIPCHK(vif::launch_lag_table(to_dev(kern), nlag, prec, ws + L.lag, s));
      fa.lagtab = ws + L.lag;
    }
    // The side work (the neighbor search) starts first and runs beside the chain
    // of small Sigma_k kernels, which use the CUs its stream leaves free, and U.
    const vif::LowRankArgs la = lowrank_args(p, ind, kern, L);
    if (side && (st = side->start(s))) return st;
    if ((st = run_sigma_k(la, ws, L, s))) return st;
    if ((st = run_u(la, prec, ws, L, s))) return st;
    if (side) HIPCHK(hipStreamWaitEvent(s, side->done, 0));
    fa.U = ws + L.U;
    fa.W = ws + L.W;
    fa.z = reinterpret_cast<double*>(ws + L.z);
    fa.wrb = vif::w_plane_rows(p->n) / 8;
    PROF(VIF_STAGE_POINT_FACTOR, false);
    HIPCHK(vif::launch_point_factor(fa, 0, prec, s));
    PROF(VIF_STAGE_POINT_FACTOR, true);
    void* syrk = ws + L.syrk;
    double* M = reinterpret_cast<double*>(ws + L.M);
    double* q = reinterpret_cast<double*>(ws + L.q);
    PROF(VIF_STAGE_SYRK, false);
    const int64_t wrows = prec >= VIF_PREC_BF16X3 ? vif::w_plane_rows(p->n) : p->n;
    HIPCHK(vif::launch_syrk(wrows, L.kpad, ws + L.W, prec, syrk, L.splits, s));
    PROF(VIF_STAGE_SYRK, true);
    PROF(VIF_STAGE_ASSEMBLY, false);
    // z'z is summed in FP64 from the per-point z (sums[1]); the Gram's own (k, k)
    // entry goes to sums[2] unused.
    HIPCHK(vif::launch_syrk_reduce(k, L.kpad, syrk, prec, L.splits, M, q, sums + 2, s));
    HIPCHK(vif::launch_cholesky(L.kpad, M, reinterpret_cast<double*>(ws + L.dscr), fl + 2, s));
    HIPCHK(vif::launch_sum(p->n, fa.logD, 0, part, sums + 0, s));
    HIPCHK(vif::launch_sum(p->n, fa.z, 1, part, sums + 1, s));
    HIPCHK(vif::launch_finalize(p->n, k, L.kpad, M, sums + 0, sums + 1, out, s));
    PROF(VIF_STAGE_ASSEMBLY, true);
  } else {
    if (side) {
      if ((st = side->start(s))) return st;
      HIPCHK(hipStreamWaitEvent(s, side->done, 0));
    }
    fa.z = reinterpret_cast<double*>(ws + L.z);
    PROF(VIF_STAGE_POINT_FACTOR, false);
    HIPCHK(vif::launch_point_factor(fa, 0, prec, s));
    PROF(VIF_STAGE_POINT_FACTOR, true);
    PROF(VIF_STAGE_ASSEMBLY, false);
    HIPCHK(vif::launch_sum(p->n, fa.logD, 0, part, sums + 0, s));
    HIPCHK(vif::launch_sum(p->n, fa.z, 1, part, sums + 1, s));
    HIPCHK(vif::launch_finalize(p->n, 0, 0, nullptr, sums + 0, sums + 1, out, s));
    PROF(VIF_STAGE_ASSEMBLY, true);
  }
  Flags f;
  double h[5];
  if ((st = read_flags(ws, L, &f, h, 5, s))) return st;
  prof_collect();
  if ((st = report_flags(f))) return st;
  *nll = h[0];
  if (terms) {
    terms[0] = h[1];
    terms[1] = h[2];
    terms[2] = h[3];
    terms[3] = h[4];
  }
  return ok();
}

}  // namespace

namespace vif {
// Host tables of the neighbor search (pure host code): Lmax + 1 entries each of
// tab1, tab2 and bnd in *tab, the key mode and, for real-valued times
// (general), the time-bin width. Integer times: one slab per time value.
int32_t search_tables(const vif_kernel* kern, bool general, double span, int64_t n,
                      std::vector<double>* tab, int* Lmax_out, double* width_out, int* mode_out) {
  int Lmax = 0;
  double width = 1.0;  // slab width in time
  if (!general) {
    if (!(span >= 0) || span >= (double)VIF_MAX_LAGS)
      return fail(VIF_E_UNSUPPORTED, "time span %g exceeds VIF_MAX_LAGS - 1", span);
    Lmax = (int)span;
  } else if (span > 0) {
    // time bins of about kBinPoints points (at most VIF_MAX_LAGS of them)
    const int64_t nb = std::min<int64_t>(std::max<int64_t>(n / kBinPoints, 1), VIF_MAX_LAGS);
    Lmax = (int)nb - 1;
    width = span / (double)nb;
  }

  // Per-lag factors from the host C math library, in the operation order the
  // ranking key specifies; bnd is the suffix maximum of -tab1. For real-valued
  // times, entry L holds f1 at the smallest and f2 at the largest lag of two
  // bins L apart (widened by a relative 1e-9), the bounds the search needs.
  tab->assign((size_t)3 * (Lmax + 1), 0.0);
  double* tab1 = tab->data();
  double* tab2 = tab1 + (Lmax + 1);
  double* bnd = tab2 + (Lmax + 1);
  auto lag_lo = [&](int l) {
    return general ? std::max(0.0, (double)(l - 1) * width * (1.0 - 1e-9)) : (double)l;
  };
  auto lag_hi = [&](int l) { return general ? (double)(l + 1) * width * (1.0 + 1e-9) : (double)l; };
  int mode;
  const vif::KernDev kd = to_dev(kern);
  if (kern->kind == VIF_KERNEL_MATERN_ANISO) {
    mode = 1;
    const double ir_t = 1.0 / kern->range_t;
    for (int l = 0; l <= Lmax; ++l) {
      const double w = lag_lo(l) * ir_t;
      tab1[l] = w * w;
    }
  } else {
    const double two_alpha = 2.0 * kern->alpha;
    auto factors = [&](double lag, double* f1, double* f2) {
      const double pw = pow(lag, two_alpha);
      const double psi = kern->a * pw + 1.0;
      if (kern->kind == VIF_KERNEL_GNEITING) {
        *f1 = kern->tau * log(psi);
        *f2 = kern->c * pow(psi, -(kern->beta * kern->gamma));
      } else {
        *f1 = (kern->delta + kern->gamma) * log(psi);
        *f2 = kern->c * pow(psi, -(kern->gamma / 2.0));
      }
    };
    for (int l = 0; l <= Lmax; ++l) {
      double f2 = 0.0;
      factors(lag_lo(l), &tab1[l], &f2);
      if (general) factors(lag_hi(l), &f2, &tab2[l]); else tab2[l] = f2;
    }
    if (kern->kind == VIF_KERNEL_GNEITING)
      mode = kern->gamma == 0.5 ? 0 : 2;
    else
      mode = kd.nu_code == 0 ? 0 : 3;
  }
  double run = -INFINITY;
  for (int l = Lmax; l >= 0; --l) {
    const double b = -tab1[l];
    run = b > run ? b : run;
    bnd[l] = run;
  }
  *Lmax_out = Lmax;
  *width_out = width;
  *mode_out = mode;
  return VIF_OK;
}
}  // namespace vif

// Shared by the exact and the proposal search: validates times, reads the
// bounding box, uploads the per-lag tables and fills the search arguments.
struct SearchSetup {
  double tt[2], bb[4];
  int Lmax = 0;
  int mode = 0;
  bool general = false;  // real-valued times: slabs are time bins
  std::vector<double> tab;  // host tables; must outlive the copies (caller syncs)
  vif::NbrArgs a{};
};

int32_t search_setup(const vif_points* p, const vif_kernel* kern, int32_t m, int32_t* nbr,
                     char* ws, const Layout& L, hipStream_t s, SearchSetup* S) {
  int32_t st;
  if ((st = init_flags(ws, L, s))) return st;
  Flags* dflags = reinterpret_cast<Flags*>(ws + L.flags);
  double* bbox = reinterpret_cast<double*>(ws + L.bbox);
  HIPCHK(vif::launch_validate_times(p->n, p->t, &dflags->tflag, s));
  HIPCHK(vif::launch_bbox(p->n, p->sx, p->sy, bbox, bbox + 4 * 256, s));
  Flags f;
  HIPCHK(hipMemcpyAsync(&f, ws + L.flags, sizeof(f), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&S->tt[0], p->t, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&S->tt[1], p->t + (p->n - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(S->bb, bbox + 4 * 256, sizeof(S->bb), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!isfinite(S->bb[0]) || !isfinite(S->bb[1]) || !isfinite(S->bb[2]) || !isfinite(S->bb[3]))
    return fail(VIF_E_ARG, "coordinates must be finite");
  if (f.tflag & 1u) return fail(VIF_E_ARG, "times must be finite");
  if (f.tflag & 4u) return fail(VIF_E_ARG, "times must be nondecreasing in index");
  const bool general = (f.tflag & 2u) != 0;  // some time is not an integer
  const double span = S->tt[1] - S->tt[0];
  int Lmax = 0, mode = 0;
  double width = 1.0;
  if ((st = vif::search_tables(kern, general, span, p->n, &S->tab, &Lmax, &width, &mode))) return st;
  S->Lmax = Lmax;
  S->general = general;
  const double* tab1 = S->tab.data();
  const double* tab2 = tab1 + (Lmax + 1);
  const double* bnd = tab2 + (Lmax + 1);
  HIPCHK(hipMemcpyAsync(ws + L.tab1, tab1, sizeof(double) * (Lmax + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + L.tab2, tab2, sizeof(double) * (Lmax + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + L.bnd, bnd, sizeof(double) * (Lmax + 1), hipMemcpyHostToDevice, s));
  S->mode = mode;
  vif::NbrArgs& a = S->a;
  a.n = p->n;
  a.m = m;
  a.mode = mode;
  a.nu_code = to_dev(kern).nu_code;
  a.ir_s = kern->kind == VIF_KERNEL_MATERN_ANISO ? 1.0 / kern->range_s : 0.0;
  a.gamma = kern->gamma;
  a.t0 = S->tt[0];
  a.general = general ? 1 : 0;
  a.islab = general ? (span > 0 ? 1.0 / width : 0.0) : 1.0;
  a.a = kern->a;
  a.two_alpha = 2.0 * kern->alpha;
  a.c = kern->c;
  if (kern->kind == VIF_KERNEL_GNEITING) {
    a.c1 = kern->tau;
    a.e2 = -(kern->beta * kern->gamma);
  } else {
    a.c1 = kern->delta + kern->gamma;
    a.e2 = -(kern->gamma / 2.0);
  }
  a.ir_t = kern->kind == VIF_KERNEL_MATERN_ANISO ? 1.0 / kern->range_t : 0.0;
  a.sx = p->sx; a.sy = p->sy; a.t = p->t;
  a.tab1 = reinterpret_cast<const double*>(ws + L.tab1);
  a.tab2 = reinterpret_cast<const double*>(ws + L.tab2);
  a.bnd = reinterpret_cast<const double*>(ws + L.bnd);
  a.nbr = nbr;
  return VIF_OK;
}

// The exact search's grid: about kCellTarget points of one time slab per cell.
int32_t exact_grid(const vif_points* p, char* ws, const Layout& L, hipStream_t s,
                   const SearchSetup& S, vif::GridArgs* out) {
  const int Lmax = S.Lmax;
  const double* bb = S.bb;
  const double* tt = S.tt;
  vif::GridArgs g{};
  {
    const int nslab = Lmax + 1;
    const double w = bb[1] - bb[0], h = bb[3] - bb[2];
    const double per_slab = (double)p->n / nslab;
    double cells = per_slab / kCellTarget;
    const double cap = (double)vif::kMaxCells / nslab;
    if (cells > cap) cells = cap;
    if (cells > 65536.0) cells = 65536.0;
    if (cells < 1.0) cells = 1.0;
    int gx = 1, gy = 1;
    if (w > 0 && h > 0) {
      gx = (int)lround(sqrt(cells * w / h));
      if (gx < 1) gx = 1;
      gy = (int)ceil(cells / gx);
      if (gy < 1) gy = 1;
    } else if (w > 0) {
      gx = (int)cells;
    } else if (h > 0) {
      gy = (int)cells;
    }
    while ((int64_t)gx * gy * nslab > vif::kMaxCells) {
      if (gx >= gy && gx > 1) --gx; else if (gy > 1) --gy; else break;
    }
    g.gx = gx;
    g.gy = gy;
    g.ncell = gx * gy;
    g.nslab = nslab;
    g.islab = S.a.islab;
    g.xmin = bb[0];
    g.ymin = bb[2];
    g.cw = w > 0 ? w / gx : 1.0;
    g.ch = h > 0 ? h / gy : 1.0;
    g.icw = w > 0 ? gx / w : 0.0;
    g.ich = h > 0 ? gy / h : 0.0;
    const double scale = fabs(bb[0]) + fabs(bb[1]) + fabs(bb[2]) + fabs(bb[3]) + w + h + 1.0;
    g.margin = 1e-9 * scale;
    g.off = reinterpret_cast<const int32_t*>(ws + L.counts);
    g.px = reinterpret_cast<const double*>(ws + L.px);
    g.py = reinterpret_cast<const double*>(ws + L.py);
    g.pidx = reinterpret_cast<const int32_t*>(ws + L.pidx);
  }
  HIPCHK(vif::launch_grid_build(p->n, p->sx, p->sy, p->t, tt[0], g,
                                reinterpret_cast<int32_t*>(ws + L.counts),
                                reinterpret_cast<int32_t*>(ws + L.fill),
                                reinterpret_cast<int32_t*>(ws + L.bsum),
                                reinterpret_cast<int32_t*>(ws + L.key),
                                reinterpret_cast<double*>(ws + L.px),
                                reinterpret_cast<double*>(ws + L.py),
                                reinterpret_cast<int32_t*>(ws + L.pidx), s));
  *out = g;
  return VIF_OK;
}

// Per device, for vif_neighbors_nll: the stream of the neighbor search, which runs
// beside the Sigma_k chain and U (default priority, restricted to all but
// kSearchFreeCUs compute units, so that the chain's small launches find free CUs
// while the search fills the rest); a non-blocking stream that takes the NLL's
// work when the caller passes the null stream (a stream with a CU mask is a
// blocking stream, which null-stream work would otherwise serialise with); and
// three events. The lock serialises such calls on one device, which share them.
constexpr int kSearchFreeCUs = 32;
struct SideStream {
  std::mutex mu;
  hipStream_t s = nullptr, main = nullptr;
  hipEvent_t fork = nullptr, done = nullptr, enter = nullptr;
};

constexpr int kMaxDevices = 64;

// The side stream and events of the device that runs `main` (the current device
// for the null stream), created on first use with that device current.
int32_t side_stream(hipStream_t main, SideStream** out) {
  static SideStream slots[kMaxDevices];
  int dev = 0;
  if (main) {
    hipDevice_t d = 0;
    HIPCHK(hipStreamGetDevice(main, &d));
    dev = (int)d;
  } else {
    HIPCHK(hipGetDevice(&dev));
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(VIF_E_UNSUPPORTED, "device index %d", dev);
  SideStream* ss = &slots[dev];
  std::lock_guard<std::mutex> lock(ss->mu);
  if (!ss->s) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    hipStream_t st = nullptr, sm = nullptr;
    hipEvent_t a = nullptr, b = nullptr, c = nullptr;
    int ncu = 0;
    hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && ncu > 2 * kSearchFreeCUs) {
      uint32_t mask[(4096 + 31) / 32] = {};
      const int used = (ncu < 4096 ? ncu : 4096) - kSearchFreeCUs;
      for (int cu = 0; cu < used; ++cu) mask[cu >> 5] |= 1u << (cu & 31);
      if (hipExtStreamCreateWithCUMask(&st, (uint32_t)((used + kSearchFreeCUs + 31) / 32), mask) !=
          hipSuccess) {
        (void)hipGetLastError();  // fall back to a stream on every CU
        st = nullptr;
      }
    }
    if (e == hipSuccess && !st) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sm, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (c) (void)hipEventDestroy(c);
      if (b) (void)hipEventDestroy(b);
      if (a) (void)hipEventDestroy(a);
      if (sm) (void)hipStreamDestroy(sm);
      if (st) (void)hipStreamDestroy(st);
    }
    if (cur != dev) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess) return fail(VIF_E_DEVICE, "side stream set-up: %s", hipGetErrorString(e));
    ss->s = st;
    ss->main = sm;
    ss->fork = a;
    ss->done = b;
    ss->enter = c;
  }
  *out = ss;
  return VIF_OK;
}

extern "C" {

size_t vif_workspace_bytes(int64_t n, int32_t m, int32_t k, int32_t prec, int32_t op) {
  if (n < 1 || m < 0 || m > VIF_MAX_M || k < 0 || k > VIF_MAX_K) return 0;
  if (prec < VIF_PREC_FP64 || prec > VIF_PREC_BF16X6) return 0;
  if (op < VIF_OP_NEIGHBORS || op > VIF_OP_NEIGHBORS_NLL) return 0;
  if (op == VIF_OP_NEIGHBORS_NLL)
    return align256(make_layout(n, m, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS).total) +
           make_layout(n, m, k, prec, VIF_OP_NLL).total;
  return make_layout(n, m, k, prec, op).total;
}

const char* vif_last_error(void) { return g_err.c_str(); }

int32_t vif_profile(int32_t enable) {
  g_prof.on = enable != 0;
  for (int st = 0; st < VIF_NSTAGES; ++st) {
    g_prof.total_ms[st] = 0.0;
    g_prof.calls[st] = 0;
    g_prof.used[st] = false;
  }
  return ok();
}

int32_t vif_profile_read(double* total_ms, int32_t* calls, int32_t cap) {
  if (!total_ms || !calls || cap < 0) return fail(VIF_E_ARG, "NULL output or negative cap");
  const int nst = cap < VIF_NSTAGES ? cap : VIF_NSTAGES;
  for (int st = 0; st < nst; ++st) {
    total_ms[st] = g_prof.total_ms[st];
    calls[st] = g_prof.calls[st];
  }
  return ok();
}

int32_t vif_neighbors(const vif_points* p, const vif_kernel* kern, int32_t m, int32_t* nbr,
                      void* wsv, size_t ws_bytes, void* hip_stream) {
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const Layout L = make_layout(p->n, m, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS);
  int32_t st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (m == 0) return ok();
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  SearchSetup S;
  if ((st = search_setup(p, kern, m, nbr, ws, L, s, &S))) return st;
  PROF(VIF_STAGE_NEIGHBORS, false);
  vif::GridArgs g{};
  if ((st = exact_grid(p, ws, L, s, S, &g))) return st;
  HIPCHK(vif::launch_neighbors(S.a, g, s));
  PROF(VIF_STAGE_NEIGHBORS, true);
  // The host tables must outlive the copies above.
  HIPCHK(hipStreamSynchronize(s));
  prof_collect();
  return ok();
}

int32_t vif_neighbors_nll(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                          int32_t* nbr, const vif_points* ind, int32_t prec, double* nll, void* wsv,
                          size_t ws_bytes, void* hip_stream) {
  int k = 0;
  int32_t st = check_ind(ind, &k);
  if (st) return st;
  if (prec < VIF_PREC_FP64 || prec > VIF_PREC_BF16X6) return fail(VIF_E_ARG, "unknown precision %d", prec);
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const Layout Ln = make_layout(p->n, m, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS);
  const size_t off = align256(Ln.total);
  const size_t need = off + make_layout(p->n, m, k, prec, VIF_OP_NLL).total;
  if ((st = check_common(p, kern, m, wsv, ws_bytes, need))) return st;
  if (!y) return fail(VIF_E_ARG, "y is NULL");
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (!nll) return fail(VIF_E_ARG, "nll is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  if (m == 0)
    return nll_impl(p, y, kern, 0, nullptr, ind, prec, nll, nullptr, ws + off, ws_bytes - off, hip_stream);
  SideStream* ss = nullptr;
  if ((st = side_stream(s, &ss))) return st;
  std::lock_guard<std::mutex> lock(ss->mu);
  if (!s) {
    // null stream: the work runs on the library's non-blocking stream, after what
    // the caller enqueued before (the call returns with both streams drained)
    HIPCHK(hipEventRecord(ss->enter, nullptr));
    HIPCHK(hipStreamWaitEvent(ss->main, ss->enter, 0));
    s = ss->main;
  }
  SearchSetup S;
  if ((st = search_setup(p, kern, m, nbr, ws, Ln, s, &S))) return st;
  SideWork side;
  side.done = ss->done;
  side.start = [&](hipStream_t main) -> int32_t {
    HIPCHK(hipEventRecord(ss->fork, main));
    HIPCHK(hipStreamWaitEvent(ss->s, ss->fork, 0));
    int32_t r = prof_mark(VIF_STAGE_NEIGHBORS, false, ss->s);
    if (r) return r;
    vif::GridArgs g{};
    if ((r = exact_grid(p, ws, Ln, ss->s, S, &g))) return r;
    HIPCHK(vif::launch_neighbors(S.a, g, ss->s));
    if ((r = prof_mark(VIF_STAGE_NEIGHBORS, true, ss->s))) return r;
    HIPCHK(hipEventRecord(ss->done, ss->s));
    return VIF_OK;
  };
  st = nll_impl(p, y, kern, m, nbr, ind, prec, nll, nullptr, ws + off, ws_bytes - off, s, &side);
  // The search's host tables and the workspace are in use until both streams drain,
  // also when the NLL stopped early with an error.
  const hipError_t e_side = hipStreamSynchronize(ss->s);
  const hipError_t e_main = hipStreamSynchronize(s);
  if (st) return st;
  if (e_side != hipSuccess) return fail(VIF_E_DEVICE, "side stream: %s", hipGetErrorString(e_side));
  if (e_main != hipSuccess) return fail(VIF_E_DEVICE, "stream: %s", hipGetErrorString(e_main));
  return ok();
}

int32_t vif_factor(const vif_points* p, const vif_kernel* kern, int32_t m, const int32_t* nbr,
                   const vif_points* ind, int32_t prec, double* B, double* D, void* wsv,
                   size_t ws_bytes, void* hip_stream) {
  int k = 0;
  int32_t st = check_ind(ind, &k);
  if (st) return st;
  if (prec < VIF_PREC_FP64 || prec > VIF_PREC_BF16X6) return fail(VIF_E_ARG, "unknown precision %d", prec);
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const Layout L = make_layout(p->n, m, k, prec, VIF_OP_FACTOR);
  st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  if (m > 0 && (!nbr || !B)) return fail(VIF_E_ARG, "nbr or B is NULL");
  if (!D) return fail(VIF_E_ARG, "D is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  auto* fl = reinterpret_cast<unsigned long long*>(ws + L.flags);
  if ((st = init_flags(ws, L, s))) return st;
  vif::FactorArgs fa{};
  fa.n = p->n;
  fa.m = m;
  fa.k = k;
  fa.ldu = L.kpad;
  fa.K = to_dev(kern);
  fa.sx = p->sx; fa.sy = p->sy; fa.t = p->t; fa.y = nullptr;
  fa.nbr = nbr;
  fa.B = B;
  fa.D = D;
  fa.fail = fl;
  fa.bad_nbr = fl + 3;
  if (k > 0) {
    int nlag = 0;
    if ((st = build_order(p, ws, L, s, &fa.ord, &nlag))) return st;
    if (kern->kind == VIF_KERNEL_GNEITING && nlag > 0) {
      HIPCHK(vif::launch_lag_table(to_dev(kern), nlag, prec, ws + L.lag, s));
      fa.lagtab = ws + L.lag;
    }
    if ((st = run_lowrank(p, ind, kern, prec, ws, L, s))) return st;
    fa.U = ws + L.U;
  }
  PROF(VIF_STAGE_POINT_FACTOR, false);
  HIPCHK(vif::launch_point_factor(fa, 1, prec, s));
  PROF(VIF_STAGE_POINT_FACTOR, true);
  Flags f;
  if ((st = read_flags(ws, L, &f, nullptr, 0, s))) return st;
  prof_collect();
  if ((st = report_flags(f))) return st;
  return ok();
}

int32_t vif_nll(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                const int32_t* nbr, const vif_points* ind, int32_t prec, double* nll, void* ws,
                size_t ws_bytes, void* hip_stream) {
  return nll_impl(p, y, kern, m, nbr, ind, prec, nll, nullptr, ws, ws_bytes, hip_stream);
}

int32_t vif_nll_terms(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                      const int32_t* nbr, const vif_points* ind, int32_t prec, double* nll,
                      double* terms, void* ws, size_t ws_bytes, void* hip_stream) {
  return nll_impl(p, y, kern, m, nbr, ind, prec, nll, terms, ws, ws_bytes, hip_stream);
}


// ---------------------------------------------------------- learned proposal ----
int32_t vif_mlp_features(const vif_points* p, const vif_kernel* kern, const double* centre,
                         float* X, void* hip_stream) {
  if (!p || !kern || !centre || !X) return fail(VIF_E_ARG, "NULL argument");
  int32_t st = check_points(p, "points");
  if (st) return st;
  if (kern->kind != VIF_KERNEL_GNEITING)
    return fail(VIF_E_UNSUPPORTED, "features need the Gneiting kernel (log a, c, alpha, beta, gamma)");
  if (!(kern->a > 0) || !(kern->c > 0) || !(kern->alpha > 0) || !(kern->beta > 0) ||
      !(kern->gamma > 0))
    return fail(VIF_E_ARG, "a, c, alpha, beta, gamma must be positive");
  if (!(centre[3] > 0) || !(centre[4] > 0)) return fail(VIF_E_ARG, "scales must be positive");
  vif::FeatArgs f{};
  f.cx = centre[0]; f.cy = centre[1]; f.ct = centre[2]; f.ss = centre[3]; f.st = centre[4];
  const double hp[5] = {kern->a, kern->c, kern->alpha, kern->beta, kern->gamma};
  for (int c = 0; c < 5; ++c) f.hyper[c] = log(hp[c]) - centre[5 + c];
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_features(p->n, p->sx, p->sy, p->t, f, X, s));
  return ok();
}

int32_t vif_mlp_forward(const float* params, const float* X, int64_t rows, float* E, float* H,
                        void* hip_stream) {
  if (rows < 0) return fail(VIF_E_ARG, "rows < 0");
  if (rows > 0 && (!params || !X || !E)) return fail(VIF_E_ARG, "NULL argument");
  if (rows > ((int64_t)1 << 31) / 192) return fail(VIF_E_UNSUPPORTED, "too many rows");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_mlp_forward(rows, params, X, E, H, s));
  return ok();
}

size_t vif_mlp_backward_ws(int64_t rows) {
  if (rows < 0) return 0;
  return align256(sizeof(float) * (size_t)(vif::mlp_backward_blocks(rows) + 1) * VIF_MLP_PARAMS);
}

int32_t vif_mlp_backward(const float* params, const float* X, const float* H, const float* dE,
                         int64_t rows, float* grad, void* ws, size_t ws_bytes, void* hip_stream) {
  if (rows < 0) return fail(VIF_E_ARG, "rows < 0");
  if (!params || !grad || (rows > 0 && (!X || !H || !dE))) return fail(VIF_E_ARG, "NULL argument");
  if (rows > ((int64_t)1 << 31) / 192) return fail(VIF_E_UNSUPPORTED, "too many rows");
  if (!ws || ws_bytes < vif_mlp_backward_ws(rows))
    return fail(VIF_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes,
                vif_mlp_backward_ws(rows));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_mlp_backward(rows, params, X, H, dE, reinterpret_cast<float*>(ws), grad, s));
  return ok();
}

int32_t vif_mlp_pair_loss(const float* E, int64_t groups, int32_t npos, int32_t nneg, float tau,
                          float* dE, float* loss, void* hip_stream) {
  if (groups < 0 || npos < 1 || nneg < 1 || npos + nneg > 128 || !(tau > 0))
    return fail(VIF_E_ARG, "need groups >= 0, npos, nneg >= 1, npos + nneg <= 128, tau > 0");
  if (groups > 0 && (!E || !dE || !loss)) return fail(VIF_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_pair_loss(groups, npos, nneg, tau, E, dE, loss, s));
  return ok();
}

int32_t vif_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t count,
                     int32_t step, float lr, float beta1, float beta2, float eps,
                     void* hip_stream) {
  if (count < 0 || step < 1) return fail(VIF_E_ARG, "need count >= 0 and step >= 1");
  if (count > 0 && (!params || !grad || !m || !v)) return fail(VIF_E_ARG, "NULL argument");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(VIF_E_ARG, "bad Adam constants");
  const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_adam(count, params, grad, m, v, lr, beta1, beta2, eps, c1, c2, s));
  return ok();
}

int32_t vif_mlp_batch(const float* X, const int32_t* queries, int64_t nq, const int32_t* nbr_ext,
                      int32_t m_ext, int32_t npos, int32_t nhard, int32_t nrand,
                      const uint32_t* rnd, int32_t rand_window, float* Xb, void* hip_stream) {
  if (nq < 0 || npos < 1 || nhard < 0 || nrand < 0 || m_ext < npos + nhard || rand_window < 1)
    return fail(VIF_E_ARG, "bad batch sizes");
  if (nhard == 0 && nrand > 0)
    return fail(VIF_E_ARG, "random negatives need at least one hard negative");
  if (nq > 0 && (!X || !queries || !nbr_ext || !Xb || (nrand > 0 && !rnd)))
    return fail(VIF_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHK(vif::launch_batch(nq, queries, nbr_ext, m_ext, npos, nhard, nrand, rnd, rand_window, X,
                           Xb, s));
  return ok();
}

size_t vif_propose_ws(int64_t n) {
  if (n < 1) return 0;
  return make_propose_layout(n).total;
}

int32_t vif_propose_neighbors(const vif_points* p, const vif_kernel* kern, int32_t m,
                              const float* E, int32_t ncand, double cell, int32_t lags,
                              int32_t wmin, int32_t rmax, int32_t cmax, int32_t* nbr,
                              int64_t* n_fallback, void* wsv, size_t ws_bytes,
                              void* hip_stream) {
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const Layout L = make_propose_layout(p->n);
  int32_t st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (ncand < m || ncand > 128) return fail(VIF_E_ARG, "need m <= ncand <= 128");
  if (!(cell > 0) || !isfinite(cell)) return fail(VIF_E_ARG, "cell must be positive");
  if (lags < 0) return fail(VIF_E_ARG, "lags < 0");
  if (wmin < 0 || rmax < 1 || (int64_t)(lags + 1) * (2 * rmax + 1) > 256)
    return fail(VIF_E_ARG, "need wmin >= 0, rmax >= 1 and (lags + 1)(2 rmax + 1) <= 256");
  if (cmax < 1 || cmax > vif::kProposeCmax)
    return fail(VIF_E_ARG, "cmax must be in 1..%d", vif::kProposeCmax);
  if (reinterpret_cast<uintptr_t>(E) % 16 != 0) return fail(VIF_E_ARG, "E must be 16-byte aligned");
  if (n_fallback) *n_fallback = 0;
  if (m == 0) return ok();
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  SearchSetup S;
  if ((st = search_setup(p, kern, m, nbr, ws, L, s, &S))) return st;
  if (S.general) {
    HIPCHK(hipStreamSynchronize(s));  // the host tables outlive their copies
    return fail(VIF_E_UNSUPPORTED, "the proposal search requires integer-valued times");
  }
  // proposal grid: square cells of side `cell`
  const double ih = 1.0 / cell;
  const double gxd = (S.bb[1] - S.bb[0]) * ih + 1.0, gyd = (S.bb[3] - S.bb[2]) * ih + 1.0;
  const int nslab = S.Lmax + 1;
  if (gxd * gyd * nslab > (double)vif::kMaxCells)
    return fail(VIF_E_UNSUPPORTED, "cell too small: %.0f cells exceed %d", gxd * gyd * nslab,
                vif::kMaxCells);
  vif::GridArgs g2{};
  g2.gx = (int)((S.bb[1] - S.bb[0]) * ih) + 1;
  g2.gy = (int)((S.bb[3] - S.bb[2]) * ih) + 1;
  g2.ncell = g2.gx * g2.gy;
  g2.nslab = nslab;
  g2.morton = 0;
  g2.xmin = S.bb[0];
  g2.ymin = S.bb[2];
  g2.cw = cell;
  g2.ch = cell;
  g2.icw = ih;
  g2.ich = ih;
  g2.off = reinterpret_cast<const int32_t*>(ws + L.c2);
  g2.px = reinterpret_cast<const double*>(ws + L.px2);
  g2.py = reinterpret_cast<const double*>(ws + L.py2);
  g2.pidx = reinterpret_cast<const int32_t*>(ws + L.pi2);
  HIPCHK(vif::launch_grid_build(p->n, p->sx, p->sy, p->t, S.tt[0], g2,
                                reinterpret_cast<int32_t*>(ws + L.c2),
                                reinterpret_cast<int32_t*>(ws + L.f2),
                                reinterpret_cast<int32_t*>(ws + L.b2),
                                reinterpret_cast<int32_t*>(ws + L.k2),
                                reinterpret_cast<double*>(ws + L.px2),
                                reinterpret_cast<double*>(ws + L.py2),
                                reinterpret_cast<int32_t*>(ws + L.pi2), s));
  vif::ProposeArgs pa{};
  pa.ncand = ncand;
  pa.lags = lags;
  pa.wmin = wmin;
  pa.rmax = rmax;
  pa.cmax = cmax;
  pa.E = E;
  pa.Ecsr = reinterpret_cast<const float*>(ws + L.pemb);
  pa.fallback = reinterpret_cast<int32_t*>(ws + L.pflag);
  int32_t* count = reinterpret_cast<int32_t*>(ws + L.pcount);
  PROF(VIF_STAGE_NEIGHBORS, false);
  if (E)
    HIPCHK(vif::launch_permute16(p->n, g2.pidx, E, reinterpret_cast<float*>(ws + L.pemb), s));
  HIPCHK(vif::launch_propose(S.a, g2, pa, s));
  HIPCHK(vif::launch_zero_i32(count, 1, s));
  HIPCHK(vif::launch_compact(p->n, pa.fallback, reinterpret_cast<int32_t*>(ws + L.plist), count,
                             s));
  int32_t nfb = 0;
  HIPCHK(hipMemcpyAsync(&nfb, count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (nfb > 0) {
    vif::GridArgs g{};
    if ((st = exact_grid(p, ws, L, s, S, &g))) return st;
    vif::NbrArgs a = S.a;
    a.qlist = reinterpret_cast<const int32_t*>(ws + L.plist);
    a.n = nfb;
    HIPCHK(vif::launch_neighbors(a, g, s));
  }
  PROF(VIF_STAGE_NEIGHBORS, true);
  HIPCHK(hipStreamSynchronize(s));
  prof_collect();
  if (n_fallback) *n_fallback = nfb;
  return ok();
}


// --------------------------------------------------------------- NLL gradient ----
}  // extern "C"

namespace {

struct GradLayout {
  size_t flags, g, logD, z, part, sums, tab, total;
};

GradLayout make_grad_layout(int64_t n) {
  GradLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  L.flags = take(kFlagBytes);
  L.g = take(sizeof(double) * vif::kGradMaxParams * (size_t)n);
  L.logD = take(sizeof(double) * (size_t)n);
  L.z = take(sizeof(double) * (size_t)n);
  L.part = take(sizeof(double) * 256);
  L.sums = take(sizeof(double) * (vif::kGradMaxParams + 2));
  L.tab = take(sizeof(double) * vif::kGradLagVals * VIF_MAX_LAGS);
  L.total = off;
  return L;
}

}  // namespace

namespace {

// ------------------------------------------------------------ VIF gradient ----
// Workspace of vif_nll_grad_vif: the FP64 VIF NLL's, then the gradient's buffers.
struct VifGradLayout {
  size_t lfac = 0, e = 0, H = 0, Gam = 0, LMi = 0, Minv = 0, v = 0, psi = 0, part = 0, dSk = 0,
         T = 0, X = 0, blk = 0, cross = 0, phi = 0, sums = 0, bw = 0, key = 0, cnt = 0, fill = 0,
         list = 0, bsum = 0, total = 0;
  int Q = 16, S = 32, splits = 1;  // Q: factor block width; S: gradient slots per point
  Layout fwd;
};

VifGradLayout make_vif_grad_layout(int64_t n, int m, int k) {
  VifGradLayout G;
  G.fwd = make_layout(n, m, k, VIF_PREC_FP64, VIF_OP_NLL);
  size_t off = G.fwd.total;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  const size_t kp = (size_t)G.fwd.kpad, kk = kp * kp, P = vif::kGradMaxParams;
  // the per-point kernel's block width (rows of q = m + 1 lanes: 16, 32 or 64)
  G.Q = m < 16 ? 16 : (m < 32 ? 32 : 64);
  // split K of Gamma' U: about 64k rows per split, at most 64 splits
  G.splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, n / 65536));
  G.lfac = take(sizeof(double) * (size_t)n * G.Q * G.Q);
  G.e = take(sizeof(double) * (size_t)n);
  G.H = take(sizeof(double) * (size_t)n * kp);
  G.Gam = take(sizeof(double) * (size_t)n * kp);
  G.LMi = take(sizeof(double) * kk);
  G.Minv = take(sizeof(double) * kk);
  G.v = take(sizeof(double) * kp);
  G.psi = take(sizeof(double) * kk);
  G.part = take(sizeof(double) * kk * G.splits);
  G.dSk = take(sizeof(double) * kk * P);
  G.T = take(sizeof(double) * kk);
  G.X = take(sizeof(double) * kk * P);
  G.blk = take(sizeof(double) * (size_t)n * P);
  G.cross = take(sizeof(double) * (size_t)n * P);
  G.phi = take(sizeof(double) * (size_t)vif::phi_dot_blocks(G.fwd.kpad) * P);
  G.sums = take(sizeof(double) * 3 * P);
  // the gradient's per-point kernel works in blocks of 32 (m < 32) or 64 lanes
  G.S = m < 32 ? 32 : 64;
  const size_t slots = (size_t)n * G.S;
  G.bw = take(sizeof(double) * 2 * slots);
  G.key = take(sizeof(int32_t) * slots);
  G.cnt = take(sizeof(int32_t) * ((size_t)n + 1));
  G.fill = take(sizeof(int32_t) * ((size_t)n + 1));
  G.list = take(sizeof(int32_t) * slots);
  G.bsum = take(sizeof(int32_t) * (((size_t)n + 1 + 1023) / 1024 + 1));
  G.total = off;
  return G;
}

vif::GradKern grad_kern(const vif_kernel* kern) {
  vif::GradKern G{};
  G.kind = kern->kind;
  G.nu_code = kern->kind != VIF_KERNEL_GNEITING ? nu_code(kern->nu) : 0;
  G.sigma2 = kern->sigma2;
  G.a = kern->a;
  G.c = kern->c;
  G.two_alpha = 2.0 * kern->alpha;
  G.beta = kern->beta;
  G.gamma = kern->gamma;
  G.bg = kern->beta * kern->gamma;
  G.tau = kern->tau;
  G.delta = kern->delta;
  if (kern->kind == VIF_KERNEL_MATERN_ANISO) {
    G.ir_s2 = 1.0 / (kern->range_s * kern->range_s);
    G.ir_t2 = 1.0 / (kern->range_t * kern->range_t);
    G.inv_rs = 1.0 / kern->range_s;
    G.inv_rt = 1.0 / kern->range_t;
  }
  return G;
}

}  // namespace

extern "C" {

int32_t vif_grad_params(int32_t kind) {
  if (kind == VIF_KERNEL_GNEITING) return 8;
  if (kind == VIF_KERNEL_GNEITING_MATERN) return 7;
  if (kind == VIF_KERNEL_MATERN_ANISO) return 4;
  return 0;
}

size_t vif_grad_ws(int64_t n) {
  if (n < 1 || n >= (int64_t)INT32_MAX) return 0;
  return make_grad_layout(n).total;
}

int32_t vif_nll_grad(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                     const int32_t* nbr, double* nll, double* grad, void* wsv, size_t ws_bytes,
                     void* hip_stream) {
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  const GradLayout L = make_grad_layout(p->n > 0 ? p->n : 1);
  int32_t st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  const int P = vif_grad_params(kern->kind);
  if (P == 0) return fail(VIF_E_UNSUPPORTED, "gradient not available for kernel kind %d", kern->kind);
  if (!y) return fail(VIF_E_ARG, "y is NULL");
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (!nll || !grad) return fail(VIF_E_ARG, "nll or grad is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  HIPCHK(vif::launch_init_flags(ws + L.flags, s));
  auto* fl = reinterpret_cast<unsigned long long*>(ws + L.flags);
  vif::GradArgs a{};
  a.n = p->n;
  a.m = m;
  a.P = P;
  a.K = to_dev(kern);
  a.G.kind = kern->kind;
  a.G.nu_code = kern->kind != VIF_KERNEL_GNEITING ? nu_code(kern->nu) : 0;
  a.G.sigma2 = kern->sigma2;
  a.G.a = kern->a;
  a.G.c = kern->c;
  a.G.two_alpha = 2.0 * kern->alpha;
  a.G.beta = kern->beta;
  a.G.gamma = kern->gamma;
  a.G.bg = kern->beta * kern->gamma;
  a.G.tau = kern->tau;
  a.G.delta = kern->delta;
  if (kern->kind == VIF_KERNEL_MATERN_ANISO) {
    a.G.ir_s2 = 1.0 / (kern->range_s * kern->range_s);
    a.G.ir_t2 = 1.0 / (kern->range_t * kern->range_t);
    a.G.inv_rs = 1.0 / kern->range_s;
    a.G.inv_rt = 1.0 / kern->range_t;
  }
  a.nugget = kern->nugget;
  a.sx = p->sx; a.sy = p->sy; a.t = p->t; a.y = y;
  a.nbr = nbr;
  a.g = reinterpret_cast<double*>(ws + L.g);
  a.logD = reinterpret_cast<double*>(ws + L.logD);
  a.z = reinterpret_cast<double*>(ws + L.z);
  a.fail = fl;
  a.bad_nbr = fl + 3;
  a.lagtab = nullptr;
  if (kern->kind == VIF_KERNEL_GNEITING) {
    // Integer, nondecreasing times: the lag-only factors from a table.
    Flags* dflags = reinterpret_cast<Flags*>(ws + L.flags);
    HIPCHK(vif::launch_validate_times(p->n, p->t, &dflags->tflag, s));
    Flags f0;
    double tt[2];
    HIPCHK(hipMemcpyAsync(&f0, ws + L.flags, sizeof(f0), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tt[0], p->t, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tt[1], p->t + (p->n - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (f0.tflag & 1u) return fail(VIF_E_ARG, "times must be finite");
    const double span = tt[1] - tt[0];
    if (!(f0.tflag & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) {
      double* tab = reinterpret_cast<double*>(ws + L.tab);
      HIPCHK(vif::launch_grad_lags(a.G, (int)span + 1, tab, s));
      a.lagtab = tab;
    }
  }
  HIPCHK(vif::launch_vecchia_grad(a, s));
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  double* part = reinterpret_cast<double*>(ws + L.part);
  HIPCHK(vif::launch_sum(p->n, a.logD, 0, part, sums + 0, s));
  HIPCHK(vif::launch_sum(p->n, a.z, 1, part, sums + 1, s));
  for (int q = 0; q < P; ++q) HIPCHK(vif::launch_sum(p->n, a.g + (int64_t)q * p->n, 0, part, sums + 2 + q, s));
  Flags f;
  double h[vif::kGradMaxParams + 2];
  HIPCHK(hipMemcpyAsync(&f, ws + L.flags, sizeof(Flags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(h, sums, sizeof(double) * (P + 2), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if ((st = report_flags(f))) return st;
  *nll = 0.5 * (double)p->n * 1.8378770664093454836 + 0.5 * (h[0] + h[1]);
  for (int q = 0; q < P; ++q) grad[q] = h[2 + q];
  return ok();
}

// ------------------------------------------------------- residual neighbors ----
size_t vif_grad_vif_ws(int64_t n, int32_t m, int32_t k) {
  if (n < 1 || m < 0 || m > VIF_MAX_M || k < 1 || k > VIF_MAX_K) return 0;
  return make_vif_grad_layout(n, m, k).total;
}

int32_t vif_nll_grad_vif(const vif_points* p, const double* y, const vif_kernel* kern, int32_t m,
                         const int32_t* nbr, const vif_points* ind, double* nll, double* grad,
                         void* wsv, size_t ws_bytes, void* hip_stream) {
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  int k = 0;
  int32_t st = check_ind(ind, &k);
  if (st) return st;
  if (k < 1) return fail(VIF_E_ARG, "inducing points required (vif_nll_grad covers k = 0)");
  const VifGradLayout G = make_vif_grad_layout(p->n > 0 ? p->n : 1, m, k);
  if ((st = check_common(p, kern, m, wsv, ws_bytes, G.total))) return st;
  const int P = vif_grad_params(kern->kind);
  if (P == 0) return fail(VIF_E_UNSUPPORTED, "gradient not available for kernel kind %d", kern->kind);
  if (!y) return fail(VIF_E_ARG, "y is NULL");
  if (m > 0 && !nbr) return fail(VIF_E_ARG, "nbr is NULL");
  if (!nll || !grad) return fail(VIF_E_ARG, "nll or grad is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  const Layout& L = G.fwd;
  const int kpad = L.kpad;
  const int64_t n = p->n;
  const int64_t kk = (int64_t)kpad * kpad;
  auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
  // forward: the FP64 VIF NLL, keeping each point's residual-block factor
  double terms[4];
  if ((st = nll_impl(p, y, kern, m, nbr, ind, VIF_PREC_FP64, nll, terms, wsv, ws_bytes, hip_stream,
                     nullptr, D(G.lfac))))
    return st;
  double* U = D(L.U);
  double* W = D(L.W);
  double* z = D(L.z);
  double* q = D(L.q);
  double* Pk = D(L.P);  // L_k^-1, identity on the padding
  // M^-1 from the factor of the augmented Woodbury matrix (its leading k x k block)
  HIPCHK(vif::launch_lead_block(k, kpad, D(L.M), D(G.T), s));
  HIPCHK(vif::launch_trinv(kpad, D(G.T), D(G.LMi), D(L.dscr), s));
  auto gemm = [&](int64_t M_, int N_, int64_t K_, const double* A_, int64_t lda, int ta,
                  const double* B_, int64_t ldb, int tb, double* C_, int64_t ldc, const double* eu,
                  const double* ev, double gam, int splits, int64_t cstride, int b_lower = 0,
                  int c_lower = 0) {
    vif::GemmF64 g{};
    g.b_lower = b_lower;
    g.c_lower = c_lower;
    g.M = M_; g.N = N_; g.K = K_;
    g.A = A_; g.lda = lda; g.ta = ta;
    g.B = B_; g.ldb = ldb; g.tb = tb;
    g.C = C_; g.ldc = ldc;
    g.alpha = 1.0;
    g.eu = eu; g.ev = ev; g.gamma = gam;
    g.kchunk = ((K_ + splits - 1) / splits + 15) / 16 * 16;
    g.cstride = cstride;
    return vif::launch_gemm_f64(g, splits, s);
  };
  HIPCHK(gemm(kpad, kpad, kpad, D(G.LMi), kpad, 1, D(G.LMi), kpad, 0, D(G.Minv), kpad, nullptr,
              nullptr, 0.0, 1, 0, /*b_lower=*/1));
  HIPCHK(vif::launch_clip_kk(k, kpad, D(G.Minv), s));
  HIPCHK(vif::launch_fill_f64(q + k, kpad - k, 0.0, s));
  HIPCHK(vif::launch_matvec(kpad, D(G.Minv), q, D(G.v), s));          // v = M^-1 q
  HIPCHK(vif::launch_resid_e(n, k, kpad, W, z, D(G.v), D(G.e), s));  // e = z - W v
  // H = W M^-1 - e v'
  HIPCHK(gemm(n, kpad, kpad, W, kpad, 0, D(G.Minv), kpad, 0, D(G.H), kpad, D(G.e), D(G.v), -1.0, 1, 0));
  // per-point terms; Gamma's terms per conditioning slot
  auto I32 = [&](size_t off) { return reinterpret_cast<int32_t*>(ws + off); };
  HIPCHK(vif::launch_zero_i32(I32(G.cnt), n + 1, s));
  HIPCHK(vif::launch_zero_i32(I32(G.fill), n + 1, s));
  vif::VifGradArgs a{};
  a.n = n;
  a.m = m;
  a.k = k;
  a.kpad = kpad;
  a.P = P;
  a.G = grad_kern(kern);
  a.sx = p->sx; a.sy = p->sy; a.st = p->t; a.y = y;
  a.nbr = nbr;
  a.lrows = G.Q;
  a.Lfac = D(G.lfac);
  a.U = U;
  a.W = W;
  a.H = D(G.H);
  a.e = D(G.e);
  a.blk = D(G.blk);
  a.bw = D(G.bw);
  a.key = I32(G.key);
  a.cnt = I32(G.cnt);
  HIPCHK(vif::launch_vif_grad_points(a, s));
  // Gamma by rows: the slots of each row j listed (counts -> offsets -> fill), then
  // summed in slot order
  HIPCHK(vif::launch_exclusive_scan(I32(G.cnt), n + 1, I32(G.bsum), s));
  HIPCHK(vif::launch_slot_fill(n * (int64_t)G.S, I32(G.key), I32(G.cnt), I32(G.fill), I32(G.list), s));
  vif::GammaArgs ga{};
  ga.n = n;
  ga.k = k;
  ga.kpad = kpad;
  ga.qmax = G.S;
  ga.phi = D(G.H);
  ga.W = W;
  ga.bw = D(G.bw);
  ga.off = I32(G.cnt);
  ga.list = I32(G.list);
  ga.Gam = D(G.Gam);
  HIPCHK(vif::launch_gamma_gather(ga, s));
  // <Gamma L_k^-1, dC_nk>: Gamma L_k^-1 into H's buffer
  double* Gt = D(G.H);
  HIPCHK(gemm(n, kpad, kpad, D(G.Gam), kpad, 0, Pk, kpad, 0, Gt, kpad, nullptr, nullptr, 0.0, 1, 0,
              /*b_lower=*/1));
  HIPCHK(vif::launch_cross_deriv(a.G, P, n, k, kpad, p->sx, p->sy, p->t, ind->sx, ind->sy, ind->t,
                                 Gt, D(G.cross), s));
  // Psi = Gamma' U (split over the rows), and <Phi(L_k^-1 dSigma_k L_k^-T), Psi> per parameter;
  // Phi is lower triangular, so only Psi's lower triangle is formed
  HIPCHK(gemm(kpad, kpad, n, D(G.Gam), kpad, 1, U, kpad, 0, D(G.part), kpad, nullptr, nullptr, 0.0,
              G.splits, kk, 0, /*c_lower=*/1));
  HIPCHK(vif::launch_splitk_reduce(kk, G.splits, kk, D(G.part), D(G.psi), s));
  HIPCHK(vif::launch_kk_deriv(a.G, P, k, kpad, ind->sx, ind->sy, ind->t, D(G.dSk), s));
  for (int pp = 0; pp < P; ++pp) {
    HIPCHK(gemm(kpad, kpad, kpad, Pk, kpad, 0, D(G.dSk) + pp * kk, kpad, 0, D(G.T), kpad, nullptr,
                nullptr, 0.0, 1, 0));
    HIPCHK(gemm(kpad, kpad, kpad, D(G.T), kpad, 0, Pk, kpad, 1, D(G.X) + pp * kk, kpad, nullptr,
                nullptr, 0.0, 1, 0));
  }
  const int nb = vif::phi_dot_blocks(kpad);
  HIPCHK(vif::launch_phi_dot(kpad, P, D(G.X), D(G.psi), D(G.phi), s));
  double* part = D(L.part);
  double* sm = D(G.sums);
  for (int pp = 0; pp < P; ++pp) {
    HIPCHK(vif::launch_sum(n, D(G.blk) + pp * n, 0, part, sm + pp, s));
    HIPCHK(vif::launch_sum(n, D(G.cross) + pp * n, 0, part, sm + P + pp, s));
    HIPCHK(vif::launch_sum(nb, D(G.phi) + (int64_t)pp * nb, 0, part, sm + 2 * P + pp, s));
  }
  double h[3 * vif::kGradMaxParams];
  HIPCHK(hipMemcpyAsync(h, sm, sizeof(double) * 3 * P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int pp = 0; pp < P; ++pp) grad[pp] = h[pp] + h[P + pp] - h[2 * P + pp];
  return ok();
}

size_t vif_residual_ws(int64_t n, int32_t k) {
  if (n < 1 || n >= (int64_t)INT32_MAX || k < 0 || k > VIF_MAX_K) return 0;
  return make_residual_layout(n, k).total;
}

int32_t vif_residual_neighbors(const vif_points* p, const vif_kernel* kern, int32_t m,
                               const vif_points* ind, int32_t* nbr, void* wsv, size_t ws_bytes,
                               void* hip_stream) {
  int k = 0;
  int32_t st = check_ind(ind, &k);
  if (st) return st;
  if (!p) return fail(VIF_E_ARG, "points is NULL");
  if (m < 1) return fail(VIF_E_ARG, "m must be >= 1");
  const Layout L = make_residual_layout(p->n, k);
  st = check_common(p, kern, m, wsv, ws_bytes, L.total);
  if (st) return st;
  if (!nbr) return fail(VIF_E_ARG, "nbr is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(wsv);
  if ((st = init_flags(ws, L, s))) return st;
  double* d = reinterpret_cast<double*>(ws + L.logD);
  const double* U = nullptr;
  if (k > 0) {
    if ((st = run_lowrank(p, ind, kern, VIF_PREC_FP64, ws, L, s))) return st;
    U = reinterpret_cast<const double*>(ws + L.U);
  }
  HIPCHK(vif::launch_resid_var(p->n, L.kpad, kern->sigma2, U, d, s));
  // Gneiting kernel with integer times: per-lag factors in a table.
  const double* lagtab = nullptr;
  if (kern->kind == VIF_KERNEL_GNEITING) {
    Flags* dflags = reinterpret_cast<Flags*>(ws + L.flags);
    HIPCHK(vif::launch_validate_times(p->n, p->t, &dflags->tflag, s));
    Flags f;
    double tt[2];
    HIPCHK(hipMemcpyAsync(&f, ws + L.flags, sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tt[0], p->t, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tt[1], p->t + (p->n - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (f.tflag & 1u) return fail(VIF_E_ARG, "times must be finite");
    const double span = tt[1] - tt[0];
    if (!(f.tflag & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) {
      double* tab = reinterpret_cast<double*>(ws + L.tab1);
      HIPCHK(vif::launch_resid_lags(to_dev(kern), (int)span + 1, tab, s));
      lagtab = tab;
    }
  }
  vif::ResidArgs a{};
  a.lagtab = lagtab;
  a.n = p->n;
  a.m = m;
  a.kpad = L.kpad;
  a.K = to_dev(kern);
  a.sx = p->sx; a.sy = p->sy; a.t = p->t;
  a.U = U;
  a.d = d;
  a.nbr = nbr;
  HIPCHK(vif::launch_resid_topm(a, s));
  Flags f;
  if ((st = read_flags(ws, L, &f, nullptr, 0, s))) return st;
  if ((st = report_flags(f))) return st;
  return ok();
}

// ------------------------------------------------------------------- batches ----
}  // extern "C"

namespace {

struct ProbPlan {
  vif_points p{};
  const double* y = nullptr;
  vif_kernel kern{};
  int m = 0;
  const int32_t* nbr = nullptr;
  vif_points ind{};
  int k = 0;
  Layout L;
  size_t off = 0;
  vif::GridArgs og{};  // processing-order grid (k > 0)
  double t0 = 0.0;
  int nlag = 0;  // > 0: integer, sorted times spanning nlag lags (Gneiting lag table)
};

constexpr int kBatchMaxStreams = 4;
constexpr int kBatchPlanScratch = VIF_BATCH_PLAN_SCRATCH;

}  // namespace

struct vif_batch {
  int prec = 0;
  std::vector<ProbPlan> probs;
  size_t total = 0;
  int streams = 1;
  int chunk_rows = 4096;
  hipStream_t side[kBatchMaxStreams] = {};
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kBatchMaxStreams] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* g_ws = nullptr;
  double* g_nll = nullptr;
  int g_streams = 0, g_chunk = 0;
};

namespace {

void drop_graph(vif_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// One problem's NLL, kernels only (capturable): the path of vif_nll with the
// host-side quantities taken from the plan, in three stages so that the batch can
// factor every problem's Sigma_k (after stage 0) and M (after stage 1) together:
//   stage 0: flags; with inducing points, the processing order, the lag table and Sigma_k;
//   stage 1: with inducing points, L_k^-1, U, the per-point factor, the Gram and M;
//            without, the whole NLL;
//   stage 2: with inducing points, the sums and the finalisation.
int32_t enqueue_problem(const ProbPlan& P, int prec, int chunk_rows, char* wsb, double* nll_out,
                        int stage, hipStream_t s) {
  const Layout& L = P.L;
  char* ws = wsb + P.off;
  auto* fl = reinterpret_cast<unsigned long long*>(ws + L.flags);
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* out = reinterpret_cast<double*>(ws + L.out);
  vif::FactorArgs fa{};
  fa.n = P.p.n;
  fa.m = P.m;
  fa.k = P.k;
  fa.ldu = L.kpad;
  fa.K = to_dev(&P.kern);
  fa.sx = P.p.sx; fa.sy = P.p.sy; fa.t = P.p.t; fa.y = P.y;
  fa.nbr = P.nbr;
  fa.logD = reinterpret_cast<double*>(ws + L.logD);
  fa.z = reinterpret_cast<double*>(ws + L.z);
  fa.fail = fl;
  fa.bad_nbr = fl + 3;
  if (P.k > 0) {
    const vif::LowRankArgs a = lowrank_args(&P.p, &P.ind, &P.kern, L);
    if (stage == 0) {
      HIPCHK(vif::launch_init_flags(ws + L.flags, s));
      vif::GridArgs g = P.og;
      HIPCHK(vif::launch_grid_build(P.p.n, P.p.sx, P.p.sy, P.p.t, P.t0, g,
                                    reinterpret_cast<int32_t*>(ws + L.counts),
                                    reinterpret_cast<int32_t*>(ws + L.fill),
                                    reinterpret_cast<int32_t*>(ws + L.bsum),
                                    reinterpret_cast<int32_t*>(ws + L.key), nullptr, nullptr,
                                    reinterpret_cast<int32_t*>(ws + L.pidx), s));
      if (P.kern.kind == VIF_KERNEL_GNEITING && P.nlag > 0)
        HIPCHK(vif::launch_lag_table(to_dev(&P.kern), P.nlag, prec, ws + L.lag, s));
      HIPCHK(vif::launch_cov_kk(a, reinterpret_cast<double*>(ws + L.Sk), s));
      return VIF_OK;
    }
    if (stage == 1) {
      HIPCHK(vif::launch_trinv(L.kpad, reinterpret_cast<double*>(ws + L.Sk),
                               reinterpret_cast<double*>(ws + L.P),
                               reinterpret_cast<double*>(ws + L.dscr), s));
      int32_t st = run_u(a, prec, ws, L, s);
      if (st) return st;
      fa.ord = reinterpret_cast<const int32_t*>(ws + L.pidx);
      if (P.kern.kind == VIF_KERNEL_GNEITING && P.nlag > 0) fa.lagtab = ws + L.lag;
      fa.U = ws + L.U;
      fa.W = ws + L.W;
      fa.wrb = vif::w_plane_rows(P.p.n) / 8;
      HIPCHK(vif::launch_point_factor(fa, 0, prec, s));
      double* M = reinterpret_cast<double*>(ws + L.M);
      double* q = reinterpret_cast<double*>(ws + L.q);
      const int64_t wrows = prec >= VIF_PREC_BF16X3 ? vif::w_plane_rows(P.p.n) : P.p.n;
      const int nchunk = vif::syrk_chunks(wrows, L.kpad, prec, chunk_rows);
      HIPCHK(vif::launch_syrk(wrows, L.kpad, ws + L.W, prec, ws + L.syrk, nchunk, s, chunk_rows));
      HIPCHK(vif::launch_syrk_reduce(P.k, L.kpad, ws + L.syrk, prec, nchunk, M, q, sums + 2, s));
      return VIF_OK;
    }
    HIPCHK(vif::launch_sum(P.p.n, fa.logD, 0, part, sums + 0, s));
    HIPCHK(vif::launch_sum(P.p.n, fa.z, 1, part, sums + 1, s));
    HIPCHK(vif::launch_finalize(P.p.n, P.k, L.kpad, reinterpret_cast<double*>(ws + L.M), sums + 0,
                                sums + 1, out, s));
    HIPCHK(vif::launch_copy_f64(out, nll_out, s));
    return VIF_OK;
  }
  if (stage == 0) {
    HIPCHK(vif::launch_init_flags(ws + L.flags, s));
    return VIF_OK;
  }
  if (stage == 2) return VIF_OK;
  HIPCHK(vif::launch_point_factor(fa, 0, prec, s));
  HIPCHK(vif::launch_sum(P.p.n, fa.logD, 0, part, sums + 0, s));
  HIPCHK(vif::launch_sum(P.p.n, fa.z, 1, part, sums + 1, s));
  HIPCHK(vif::launch_finalize(P.p.n, 0, 0, nullptr, sums + 0, sums + 1, out, s));
  HIPCHK(vif::launch_copy_f64(out, nll_out, s));
  return VIF_OK;
}

// The factorisations of every problem's Sigma_k (which = 1) or M (which = 2) as
// one set: one panel and one update launch per step for all of them.
int32_t batch_cholesky(const vif_batch* b, char* wsb, int which, hipStream_t s) {
  std::vector<double*> A, scr;
  std::vector<int> N;
  std::vector<unsigned long long*> fl;
  for (const ProbPlan& P : b->probs) {
    if (P.k == 0) continue;
    char* ws = wsb + P.off;
    A.push_back(reinterpret_cast<double*>(ws + (which == 1 ? P.L.Sk : P.L.M)));
    N.push_back(P.L.kpad);
    scr.push_back(reinterpret_cast<double*>(ws + P.L.dscr));
    fl.push_back(reinterpret_cast<unsigned long long*>(ws + P.L.flags) + which);
  }
  if (A.empty()) return VIF_OK;
  HIPCHK(vif::launch_cholesky_set((int)A.size(), A.data(), N.data(), scr.data(), fl.data(), s));
  return VIF_OK;
}

int32_t batch_enqueue(vif_batch* b, char* ws, double* nll, hipStream_t s) {
  const int ns = b->streams;
  const int np = (int)b->probs.size();
  auto fork = [&]() -> int32_t {
    if (ns > 1) {
      HIPCHK(hipEventRecord(b->ev_fork, s));
      for (int j = 0; j < ns; ++j) HIPCHK(hipStreamWaitEvent(b->side[j], b->ev_fork, 0));
    }
    return VIF_OK;
  };
  auto join = [&]() -> int32_t {
    if (ns > 1) {
      for (int j = 0; j < ns; ++j) {
        HIPCHK(hipEventRecord(b->ev_join[j], b->side[j]));
        HIPCHK(hipStreamWaitEvent(s, b->ev_join[j], 0));
      }
    }
    return VIF_OK;
  };
  int32_t st = VIF_OK;
  for (int stage = 0; stage < 3 && !st; ++stage) {
    // problems round-robin over the streams, largest first
    if ((st = fork())) break;
    for (int i = 0; i < np && !st; ++i)
      st = enqueue_problem(b->probs[i], b->prec, b->chunk_rows, ws, nll + i, stage,
                           ns > 1 ? b->side[i % ns] : s);
    if (st || (st = join())) break;
    if (stage < 2) st = batch_cholesky(b, ws, stage + 1, s);
  }
  return st;
}

int32_t batch_check(const vif_batch* b, void* ws, size_t ws_bytes, const double* nll) {
  if (!b) return fail(VIF_E_ARG, "batch is NULL");
  if (!ws) return fail(VIF_E_ARG, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(VIF_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < b->total)
    return fail(VIF_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, b->total);
  if (!nll) return fail(VIF_E_ARG, "nll is NULL");
  return VIF_OK;
}

}  // namespace

extern "C" {

vif_batch* vif_batch_create(const vif_problem* probs, int32_t count, int32_t prec, void* scratch,
                            size_t scratch_bytes, void* hip_stream) {
  if (!probs || count < 1) {
    fail(VIF_E_ARG, "need at least one problem");
    return nullptr;
  }
  if (prec < VIF_PREC_FP64 || prec > VIF_PREC_BF16X6) {
    fail(VIF_E_ARG, "unknown precision %d", prec);
    return nullptr;
  }
  if (!scratch || scratch_bytes < (size_t)kBatchPlanScratch ||
      (reinterpret_cast<uintptr_t>(scratch) & 255) != 0) {
    fail(VIF_E_WORKSPACE, "plan scratch must hold %d bytes, 256-byte aligned", kBatchPlanScratch);
    return nullptr;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  std::unique_ptr<vif_batch> b(new vif_batch());
  b->prec = prec;
  size_t off = 0;
  char* scr = reinterpret_cast<char*>(scratch);
  for (int i = 0; i < count; ++i) {
    const vif_problem& q = probs[i];
    ProbPlan P;
    P.p = q.points;
    P.y = q.y;
    P.kern = q.kern;
    P.m = q.m;
    P.nbr = q.nbr;
    P.ind = q.ind;
    int k = 0;
    if (q.ind.n != 0 && check_ind(&q.ind, &k)) return nullptr;
    P.k = k;
    P.L = make_layout(q.points.n, q.m, k, prec, VIF_OP_NLL, 1024);
    if (check_common(&q.points, &q.kern, q.m, scr, (size_t)-1, 0)) return nullptr;  // ws unused
    if (!q.y || (q.m > 0 && !q.nbr)) {
      fail(VIF_E_ARG, "problem %d: y or nbr is NULL", i);
      return nullptr;
    }
    if (k > 0) {
      // the processing-order grid, as in vif_nll, from the problem's bounding box
      double* bbox = reinterpret_cast<double*>(scr + 256);
      uint32_t* tflag = reinterpret_cast<uint32_t*>(scr);
      if (vif::launch_zero_i32(reinterpret_cast<int32_t*>(scr), 64, s) != hipSuccess ||
          vif::launch_validate_times(q.points.n, q.points.t, tflag, s) != hipSuccess ||
          vif::launch_bbox(q.points.n, q.points.sx, q.points.sy, bbox, bbox + 4 * 256, s) !=
              hipSuccess) {
        fail(VIF_E_DEVICE, "problem %d: launch failed", i);
        return nullptr;
      }
      uint32_t tf = 0;
      double tt[2], bb[4];
      if (hipMemcpyAsync(&tf, tflag, sizeof(tf), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(&tt[0], q.points.t, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(&tt[1], q.points.t + (q.points.n - 1), sizeof(double),
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipMemcpyAsync(bb, bbox + 4 * 256, sizeof(bb), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        fail(VIF_E_DEVICE, "problem %d: readback failed", i);
        return nullptr;
      }
      if (tf & 1u) {
        fail(VIF_E_ARG, "problem %d: times must be finite", i);
        return nullptr;
      }
      if (!isfinite(bb[0]) || !isfinite(bb[1]) || !isfinite(bb[2]) || !isfinite(bb[3])) {
        fail(VIF_E_ARG, "problem %d: coordinates must be finite", i);
        return nullptr;
      }
      int nslab = 1;
      const double span = tt[1] - tt[0];
      if (!(tf & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) nslab = (int)span + 1;
      P.nlag = (!(tf & 6u) && span >= 0 && span < (double)VIF_MAX_LAGS) ? nslab : 0;
      const double per = (double)q.points.n / nslab;
      int bits = 0;
      while (bits < 10 && (double)(1 << (2 * (bits + 1))) * 3.0 <= per &&
             (int64_t)(1 << (2 * (bits + 1))) * nslab <= vif::kMaxCells)
        ++bits;
      const double w = bb[1] - bb[0], h = bb[3] - bb[2];
      vif::GridArgs& g = P.og;
      g.gx = g.gy = 1 << bits;
      g.ncell = g.gx * g.gy;
      g.nslab = nslab;
      g.morton = 1;
      g.xmin = bb[0];
      g.ymin = bb[2];
      g.cw = w > 0 ? w / g.gx : 1.0;
      g.ch = h > 0 ? h / g.gy : 1.0;
      g.icw = w > 0 ? g.gx / w : 0.0;
      g.ich = h > 0 ? g.gy / h : 0.0;
      P.t0 = tt[0];
    }
    P.off = off;
    off += align256(P.L.total);
    b->probs.push_back(P);
  }
  b->total = off;
  if (vif::prepare_lowrank_fused() != hipSuccess) {
    fail(VIF_E_DEVICE, "kernel attribute could not be set");
    return nullptr;
  }
  for (int j = 0; j < kBatchMaxStreams; ++j) {
    if (hipStreamCreateWithFlags(&b->side[j], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join[j], hipEventDisableTiming) != hipSuccess) {
      fail(VIF_E_DEVICE, "stream or event creation failed");
      vif_batch_destroy(b.release());
      return nullptr;
    }
  }
  if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    fail(VIF_E_DEVICE, "stream or event creation failed");
    vif_batch_destroy(b.release());
    return nullptr;
  }
  ok();
  return b.release();
}

size_t vif_batch_workspace_bytes(const vif_batch* b) { return b ? b->total : 0; }

int32_t vif_batch_enqueue(vif_batch* b, void* ws, size_t ws_bytes, double* nll, void* hip_stream) {
  int32_t st = batch_check(b, ws, ws_bytes, nll);
  if (st) return st;
  if ((st = batch_enqueue(b, reinterpret_cast<char*>(ws), nll,
                          reinterpret_cast<hipStream_t>(hip_stream))))
    return st;
  return ok();
}

int32_t vif_batch_graph_launch(vif_batch* b, void* ws, size_t ws_bytes, double* nll,
                               void* hip_stream) {
  int32_t st = batch_check(b, ws, ws_bytes, nll);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (!b->exec || b->g_ws != ws || b->g_nll != nll || b->g_streams != b->streams ||
      b->g_chunk != b->chunk_rows) {
    drop_graph(b);
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    st = batch_enqueue(b, reinterpret_cast<char*>(ws), nll, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(VIF_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_ws = ws;
    b->g_nll = nll;
    b->g_streams = b->streams;
    b->g_chunk = b->chunk_rows;
  }
  HIPCHK(hipGraphLaunch(b->exec, s));
  return ok();
}

int32_t vif_batch_autotune(vif_batch* b, void* ws, size_t ws_bytes, double* nll, int32_t reps,
                           double* best_ms, void* hip_stream) {
  int32_t st = batch_check(b, ws, ws_bytes, nll);
  if (st) return st;
  if (reps < 1) return fail(VIF_E_ARG, "reps < 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int cand_streams[3] = {1, 2, 4};
  const int cand_chunk[2] = {1024, 4096};
  const int nchunk_cand = b->prec >= VIF_PREC_BF16X3 ? 2 : 1;  // rows per partial: split modes
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIPCHK(hipEventCreate(&ev.e0));
  HIPCHK(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  double best = INFINITY;
  const int s0 = b->streams, c0 = b->chunk_rows;  // restored if a candidate fails
  int bs = s0, bc = c0;
  auto dev_err = [&](hipError_t e) {
    return e == hipSuccess ? VIF_OK : fail(VIF_E_DEVICE, "autotune: %s", hipGetErrorString(e));
  };
  for (int a = 0; a < 3 && !st; ++a) {
    for (int c = 0; c < nchunk_cand && !st; ++c) {
      b->streams = cand_streams[a];
      b->chunk_rows = nchunk_cand == 2 ? cand_chunk[c] : 4096;
      if ((st = vif_batch_graph_launch(b, ws, ws_bytes, nll, hip_stream))) break;  // warm-up
      if ((st = dev_err(hipEventRecord(e0, s)))) break;
      for (int r = 0; r < reps && !st; ++r) st = vif_batch_graph_launch(b, ws, ws_bytes, nll, hip_stream);
      if (st) break;
      float ms = 0.f;
      if ((st = dev_err(hipEventRecord(e1, s))) || (st = dev_err(hipEventSynchronize(e1))) ||
          (st = dev_err(hipEventElapsedTime(&ms, e0, e1))))
        break;
      const double per = ms / reps;
      if (per < best) {
        best = per;
        bs = b->streams;
        bc = b->chunk_rows;
      }
    }
  }
  b->streams = st ? s0 : bs;
  b->chunk_rows = st ? c0 : bc;
  drop_graph(b);
  if (st) return st;
  if (best_ms) *best_ms = best;
  return ok();
}

int32_t vif_batch_schedule(const vif_batch* b, int32_t* streams, int32_t* chunk_rows) {
  if (!b) return fail(VIF_E_ARG, "batch is NULL");
  if (streams) *streams = b->streams;
  if (chunk_rows) *chunk_rows = b->chunk_rows;
  return ok();
}

int32_t vif_batch_set_schedule(vif_batch* b, int32_t streams, int32_t chunk_rows) {
  if (!b) return fail(VIF_E_ARG, "batch is NULL");
  if (streams < 1 || streams > kBatchMaxStreams)
    return fail(VIF_E_ARG, "streams must be in 1 .. %d", kBatchMaxStreams);
  if (chunk_rows < 1024 || chunk_rows > 65536 || chunk_rows % 8)
    return fail(VIF_E_ARG, "chunk_rows must be a multiple of 8 in 1024 .. 65536");
  b->streams = streams;
  b->chunk_rows = chunk_rows;
  drop_graph(b);
  return ok();
}

int32_t vif_batch_status(vif_batch* b, void* ws, int32_t* status, void* hip_stream) {
  if (!b || !ws) return fail(VIF_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int np = (int)b->probs.size();
  std::vector<Flags> f((size_t)np);
  for (int i = 0; i < np; ++i)
    HIPCHK(hipMemcpyAsync(&f[i], reinterpret_cast<char*>(ws) + b->probs[i].off + b->probs[i].L.flags,
                          sizeof(Flags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int32_t first = VIF_OK;
  for (int i = 0; i < np; ++i) {
    const int32_t st = report_flags(f[i]);
    if (status) status[i] = st;
    if (st && first == VIF_OK) first = st;
  }
  if (first == VIF_OK) return ok();
  return first;
}

void vif_batch_destroy(vif_batch* b) {
  if (!b) return;
  drop_graph(b);
  for (int j = 0; j < kBatchMaxStreams; ++j) {
    if (b->side[j]) (void)hipStreamDestroy(b->side[j]);
    if (b->ev_join[j]) (void)hipEventDestroy(b->ev_join[j]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}
}  // extern "C"
