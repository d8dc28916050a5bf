// Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure; built and run by tests/test_abi_sanitize.py on a machine
// without a GPU). Every call below must be refused by the host-side validation
// before any device work, so no device pointer is ever dereferenced; the search
// tables (pure host code) are checked for every kernel family and time layout.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include <hip/hip_runtime_api.h>

#include "vif.h"
#include "vif_batch.h"
#include "vif_grad.h"
#include "vif_learn.h"
#include "vif_residual.h"

namespace vif {
int32_t search_tables(const vif_kernel* kern, bool general, double span, int64_t n,
                      std::vector<double>* tab, int* Lmax_out, double* width_out, int* mode_out);
}

static int g_fail = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);       \
      ++g_fail;                                                             \
    }                                                                       \
  } while (0)

static void* const FAKE = reinterpret_cast<void*>(0x100000);  // never dereferenced

static vif_kernel gneiting() {
  vif_kernel k;
  memset(&k, 0, sizeof(k));
  k.kind = VIF_KERNEL_GNEITING;
  k.sigma2 = 1.0; k.nugget = 0.1; k.a = 0.5; k.c = 20.0; k.alpha = 0.75; k.beta = 0.5;
  k.gamma = 0.5; k.tau = 1.0;
  return k;
}
static vif_kernel gneiting_matern(double nu) {
  vif_kernel k = gneiting();
  k.kind = VIF_KERNEL_GNEITING_MATERN;
  k.gamma = 0.4; k.delta = 0.2; k.alpha = 0.4; k.nu = nu;
  return k;
}
static vif_kernel aniso() {
  vif_kernel k;
  memset(&k, 0, sizeof(k));
  k.kind = VIF_KERNEL_MATERN_ANISO;
  k.sigma2 = 1.0; k.nugget = 0.05; k.range_s = 0.2; k.range_t = 3.0; k.nu = 1.5;
  return k;
}

static void check_workspace_sizes() {
  const int64_t ns[] = {-5, 0, 1, 2, 63, 64, 65, 1000, 1 << 20, 1097040, (int64_t)1 << 31,
                        (int64_t)1 << 40};
  const int32_t ms[] = {-1, 0, 1, 30, VIF_MAX_M, VIF_MAX_M + 1};
  const int32_t ks[] = {-1, 0, 1, 63, 64, 1000, VIF_MAX_K, VIF_MAX_K + 1};
  for (int64_t n : ns)
    for (int32_t m : ms)
      for (int32_t k : ks)
        for (int32_t prec = -1; prec <= 4; ++prec)
          for (int32_t op = -1; op <= 4; ++op) {
            const size_t b = vif_workspace_bytes(n, m, k, prec, op);
            const bool bad = n < 1 || m < 0 || m > VIF_MAX_M || k < 0 || k > VIF_MAX_K ||
                             prec < 0 || prec > 3 || op < 0 || op > 3;
            if (bad) CHECK(b == 0);
            if (!bad && n <= (1 << 20)) CHECK(b > 0);
          }
  // monotone in n for a valid shape
  size_t prev = 0;
  for (int64_t n = 1; n <= (1 << 22); n *= 2) {
    const size_t b = vif_workspace_bytes(n, 30, 1000, VIF_PREC_BF16X3, VIF_OP_NLL);
    CHECK(b >= prev);
    prev = b;
  }
}

static void check_argument_errors() {
  vif_kernel K = gneiting();
  vif_points P{100, (const double*)FAKE, (const double*)FAKE, (const double*)FAKE};
  vif_points Z{20, (const double*)FAKE, (const double*)FAKE, (const double*)FAKE};
  int32_t* nbr = (int32_t*)FAKE;
  double out = 0.0, terms[4];
  const size_t big = (size_t)1 << 40;
  // NULL arguments
  CHECK(vif_neighbors(nullptr, &K, 5, nbr, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors(&P, nullptr, 5, nbr, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors(&P, &K, 5, nullptr, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors(&P, &K, 5, nbr, nullptr, big, nullptr) == VIF_E_ARG);
  CHECK(strlen(vif_last_error()) > 0);
  // workspace: misaligned, too small
  CHECK(vif_neighbors(&P, &K, 5, nbr, (char*)FAKE + 8, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors(&P, &K, 5, nbr, FAKE, 16, nullptr) == VIF_E_WORKSPACE);
  // m, n
  CHECK(vif_neighbors(&P, &K, -1, nbr, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors(&P, &K, VIF_MAX_M + 1, nbr, FAKE, big, nullptr) == VIF_E_UNSUPPORTED);
  vif_points P0 = P;
  P0.n = 0;
  CHECK(vif_neighbors(&P0, &K, 5, nbr, FAKE, big, nullptr) == VIF_E_ARG);
  vif_points Pn = P;
  Pn.sx = nullptr;
  CHECK(vif_neighbors(&Pn, &K, 5, nbr, FAKE, big, nullptr) == VIF_E_ARG);
  // every hyperparameter the Gneiting kernel uses, outside its range, NaN or infinite
  struct Bad { int field; double v[4]; int nv; };
  const Bad bads[] = {
      {0, {NAN, INFINITY, -1.0, 0.0}, 4},   // sigma2 > 0
      {1, {NAN, INFINITY, -1.0, 0.0}, 3},   // nugget >= 0
      {2, {NAN, INFINITY, -1.0, 0.0}, 4},   // a > 0
      {3, {NAN, INFINITY, -1.0, 0.0}, 4},   // c > 0
      {4, {NAN, -1.0, 0.0, 1.5}, 4},        // alpha in (0, 1]
      {5, {NAN, -1.0, 1.5, INFINITY}, 4},   // beta in [0, 1]
      {6, {NAN, -1.0, 0.0, 1.5}, 4},        // gamma in (0, 1]
      {7, {NAN, -1.0, INFINITY, -0.5}, 4},  // tau >= 0
  };
  for (const Bad& b : bads)
    for (int e = 0; e < b.nv; ++e) {
      vif_kernel B = gneiting();
      double* f = &B.sigma2 + b.field;  // sigma2 .. jitter are consecutive doubles
      *f = b.v[e];
      const int32_t st = vif_nll(&P, (const double*)FAKE, &B, 5, nbr, nullptr, VIF_PREC_FP64, &out,
                                 FAKE, big, nullptr);
      if (st != VIF_E_ARG) {
        fprintf(stderr, "field %d = %g: status %d (expected VIF_E_ARG)\n", b.field, b.v[e], st);
        ++g_fail;
      }
    }
  vif_kernel Bk = K;
  Bk.kind = 9;
  CHECK(vif_nll(&P, (const double*)FAKE, &Bk, 5, nbr, nullptr, VIF_PREC_FP64, &out, FAKE, big,
                nullptr) == VIF_E_ARG);
  vif_kernel Gm = gneiting_matern(1.0);  // no closed form
  CHECK(vif_nll(&P, (const double*)FAKE, &Gm, 5, nbr, nullptr, VIF_PREC_FP64, &out, FAKE, big,
                nullptr) == VIF_E_UNSUPPORTED);
  // precision, inducing points, outputs
  CHECK(vif_nll(&P, (const double*)FAKE, &K, 5, nbr, &Z, 7, &out, FAKE, big, nullptr) == VIF_E_ARG);
  vif_points Zk = Z;
  Zk.n = VIF_MAX_K + 1;
  CHECK(vif_nll(&P, (const double*)FAKE, &K, 5, nbr, &Zk, 0, &out, FAKE, big, nullptr) ==
        VIF_E_UNSUPPORTED);
  CHECK(vif_nll(&P, nullptr, &K, 5, nbr, &Z, 0, &out, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_nll(&P, (const double*)FAKE, &K, 5, nbr, &Z, 0, nullptr, FAKE, big, nullptr) ==
        VIF_E_ARG);
  CHECK(vif_nll_terms(&P, (const double*)FAKE, &K, 5, nullptr, &Z, 0, &out, terms, FAKE, big,
                      nullptr) == VIF_E_ARG);
  CHECK(vif_factor(&P, &K, 5, nbr, &Z, 0, nullptr, (double*)FAKE, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_factor(&P, &K, 5, nbr, &Z, 0, (double*)FAKE, (double*)FAKE, FAKE, 8, nullptr) ==
        VIF_E_WORKSPACE);
  CHECK(vif_neighbors_nll(&P, nullptr, &K, 5, nbr, &Z, 0, &out, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_neighbors_nll(&P, (const double*)FAKE, &K, 5, nbr, &Z, 9, &out, FAKE, big, nullptr) ==
        VIF_E_ARG);
  // the static-scratch search refuses sizes beyond its array before any launch
  vif_points Ph = P;
  Ph.n = (int64_t)1 << 30;
  CHECK(vif_neighbors_noalloc(&Ph, &K, 5, nbr, nullptr) == VIF_E_WORKSPACE);
  CHECK(vif_neighbors_noalloc(nullptr, &K, 5, nbr, nullptr) == VIF_E_ARG);
  // gradient, residual search, learned proposal, batch
  CHECK(vif_grad_params(99) < 0 || vif_grad_params(99) == 0);
  CHECK(vif_nll_grad(&P, nullptr, &K, 5, nbr, &out, terms, FAKE, big, nullptr) == VIF_E_ARG);
  CHECK(vif_residual_neighbors(&P, &K, 5, nullptr, nbr, nullptr, big, nullptr) == VIF_E_ARG);
  CHECK(vif_propose_neighbors(&P, &K, 5, nullptr, 4, -1.0, 1, 64, 3, 8, nbr, nullptr, FAKE, big,
                              nullptr) == VIF_E_ARG);
  CHECK(vif_mlp_forward(nullptr, nullptr, 10, nullptr, nullptr, nullptr) == VIF_E_ARG);
  vif_problem prob;
  memset(&prob, 0, sizeof(prob));
  prob.points = P;
  prob.y = nullptr;  // invalid
  prob.kern = K;
  prob.m = 5;
  prob.nbr = nbr;
  CHECK(vif_batch_create(&prob, 1, VIF_PREC_FP32, FAKE, VIF_BATCH_PLAN_SCRATCH, nullptr) == nullptr);
  CHECK(vif_batch_create(nullptr, 1, VIF_PREC_FP32, FAKE, VIF_BATCH_PLAN_SCRATCH, nullptr) == nullptr);
  prob.y = (const double*)FAKE;
  prob.m = VIF_MAX_M + 1;  // invalid
  CHECK(vif_batch_create(&prob, 1, VIF_PREC_FP32, FAKE, VIF_BATCH_PLAN_SCRATCH, nullptr) == nullptr);
  CHECK(vif_batch_workspace_bytes(nullptr) == 0);
  vif_batch_destroy(nullptr);
}

static void check_tables(const vif_kernel& K, bool general, double span, int64_t n) {
  std::vector<double> tab;
  int Lmax = -1, mode = -1;
  double width = 0.0;
  const int32_t st = vif::search_tables(&K, general, span, n, &tab, &Lmax, &width, &mode);
  if (!general && span >= VIF_MAX_LAGS) {
    CHECK(st == VIF_E_UNSUPPORTED);
    return;
  }
  CHECK(st == VIF_OK);
  if (st != VIF_OK) return;
  CHECK(Lmax >= 0 && Lmax < VIF_MAX_LAGS);
  CHECK(tab.size() == (size_t)3 * (Lmax + 1));
  CHECK(mode >= 0 && mode <= 3);
  CHECK(width > 0.0);
  const double* t1 = tab.data();
  const double* t2 = t1 + (Lmax + 1);
  const double* bd = t2 + (Lmax + 1);
  for (int l = 0; l <= Lmax; ++l) {
    CHECK(isfinite(t1[l]) && isfinite(t2[l]) && isfinite(bd[l]));
    CHECK(t1[l] >= 0.0 && t2[l] >= 0.0);
    CHECK(bd[l] >= -t1[l]);
    if (l > 0) {
      CHECK(t1[l] >= t1[l - 1]);             // f1 nondecreasing in the lag
      CHECK(t2[l] <= t2[l - 1]);             // f2 nonincreasing in the lag
      CHECK(bd[l] <= bd[l - 1]);             // suffix maximum
    }
  }
  if (!general) CHECK(Lmax == (int)span);
}

static void check_search_tables() {
  const vif_kernel kerns[] = {gneiting(), gneiting_matern(0.5), gneiting_matern(1.5),
                              gneiting_matern(2.5), aniso()};
  vif_kernel g4 = gneiting();
  g4.gamma = 0.4;
  const double spans[] = {0.0, 0.5, 1.0, 9.0, 364.0, 65535.0, 65536.0, 1e6};
  const int64_t ns[] = {1, 2047, 2048, 1 << 20, (int64_t)1 << 30};
  for (const vif_kernel& K : kerns)
    for (double sp : spans)
      for (int64_t n : ns) {
        check_tables(K, false, floor(sp), n);
        check_tables(K, true, sp, n);
      }
  for (double sp : spans) check_tables(g4, true, sp, 1 << 20);
}

int main() {
  // Nothing here may reach a GPU: the argument checks pass fake device pointers.
  int devices = 0;
  if (hipGetDeviceCount(&devices) == hipSuccess && devices > 0) {
    printf("abi_sanitize: a GPU is present; these host-only checks are skipped\n");
    return 77;
  }
  check_workspace_sizes();
  check_argument_errors();
  check_search_tables();
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("abi_sanitize: all checks passed\n");
  return 0;
}
