// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no GPU is touched): parameter
// validation over valid and out-of-range settings of every field, workspace
// sizing over sizes, precisions, sub-steps and diagnostics, batch sizing, the
// status strings and the rejection of a workspace that is too small before
// any device call.  Exits 0 when every return code is the expected one.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "lbdps.h"

static int failures = 0;
static void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, lbdps_last_error());
    ++failures;
  }
}

static lbdps_params base() {
  lbdps_params p;
  std::memset(&p, 0, sizeof p);
  p.nx = 64;
  p.ny = 256;
  p.bc[0] = p.bc[1] = LBDPS_BC_PERIODIC;
  p.bc[2] = LBDPS_BC_INLET;
  p.bc[3] = LBDPS_BC_OUTLET;
  p.tau = 0.6;
  p.rho_g = 1.0;
  p.rho_s = 788.5;
  p.d_p = 0.5;
  p.e_pp = p.e_pw = 0.9;
  p.g[1] = -1e-5;
  p.pressure_force_sign = -1;
  p.omega_dense = 1.0;
  p.precision = LBDPS_FP32;
  return p;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  lbdps_params p = base();
  expect(lbdps_validate_params(&p, 2000) == LBDPS_OK, "base params");
  expect(lbdps_validate_params(nullptr, 1) == LBDPS_E_INVALID, "NULL params");
  struct Bad {
    const char *name;
    void (*set)(lbdps_params &);
    lbdps_status want;
  } bad[] = {
      {"nx 2", [](lbdps_params &q) { q.nx = 2; }, LBDPS_E_SHAPE},
      {"ny -5", [](lbdps_params &q) { q.ny = -5; }, LBDPS_E_SHAPE},
      {"nx*ny 2^29", [](lbdps_params &q) { q.nx = 1 << 15; q.ny = 1 << 14; }, LBDPS_E_SHAPE},
      {"bc 4", [](lbdps_params &q) { q.bc[2] = 4; }, LBDPS_E_INVALID},
      {"x inlet", [](lbdps_params &q) { q.bc[0] = q.bc[1] = LBDPS_BC_INLET; }, LBDPS_E_INVALID},
      {"half periodic", [](lbdps_params &q) { q.bc[1] = LBDPS_BC_WALL; }, LBDPS_E_INVALID},
      {"tau 0.5", [](lbdps_params &q) { q.tau = 0.5; }, LBDPS_E_INVALID},
      {"rho_g 0", [](lbdps_params &q) { q.rho_g = 0; }, LBDPS_E_INVALID},
      {"d_p 1", [](lbdps_params &q) { q.d_p = 1.0; }, LBDPS_E_INVALID},
      {"e_pp 2", [](lbdps_params &q) { q.e_pp = 2; }, LBDPS_E_INVALID},
      {"drag mode 3", [](lbdps_params &q) { q.drag_ratio_mode = 3; }, LBDPS_E_INVALID},
      {"porosity 5", [](lbdps_params &q) { q.u_gas_porosity = 5; }, LBDPS_E_INVALID},
      {"omega mode -1", [](lbdps_params &q) { q.omega_mode = -1; }, LBDPS_E_INVALID},
      {"pressure sign 2", [](lbdps_params &q) { q.pressure_force_sign = 2; }, LBDPS_E_INVALID},
      {"n_sub 65", [](lbdps_params &q) { q.n_sub = LBDPS_MAX_SUBSTEPS + 1; }, LBDPS_E_INVALID},
      {"precision 9", [](lbdps_params &q) { q.precision = 9; }, LBDPS_E_INVALID},
      {"diagnostics 2", [](lbdps_params &q) { q.diagnostics = 2; }, LBDPS_E_INVALID},
      {"loop 3", [](lbdps_params &q) { q.particles_periodic_y = 3; }, LBDPS_E_INVALID},
  };
  for (const Bad &b : bad) {
    lbdps_params q = base();
    b.set(q);
    expect(lbdps_validate_params(&q, 100) == b.want, b.name);
  }
  lbdps_params q = base();
  q.tau = nan;
  expect(lbdps_validate_params(&q, 100) == LBDPS_E_INVALID, "tau NaN");
  q = base();
  q.cs_smag = inf;
  expect(lbdps_validate_params(&q, 100) == LBDPS_E_INVALID, "cs_smag inf");
  q = base();
  q.g[0] = nan;
  expect(lbdps_validate_params(&q, 100) == LBDPS_E_INVALID, "g NaN");
  expect(lbdps_validate_params(&p, -1) == LBDPS_E_SHAPE, "negative particle count");
  expect(lbdps_validate_params(&p, 1ll << 29) == LBDPS_E_SHAPE, "2^29 particles");

  // workspace sizes: positive, growing with the work, for every precision and option
  size_t prev = 0;
  for (int prec = 0; prec < 4; ++prec)
    for (int diag = 0; diag < 2; ++diag)
      for (int nsub = 0; nsub <= 4; nsub += 4)
        for (long long n : {0ll, 1ll, 255ll, 256ll, 257ll, 200000ll}) {
          lbdps_params w = base();
          w.precision = prec;
          w.diagnostics = diag;
          w.n_sub = nsub;
          size_t b0 = 0, b1 = 0;
          expect(lbdps_workspace_bytes(&w, n, &b0) == LBDPS_OK, "workspace bytes");
          expect(lbdps_workspace_bytes(&w, n + 1000, &b1) == LBDPS_OK && b1 > b0, "more particles, more bytes");
          expect(b0 % 256 == 0 || b0 > 0, "workspace size");
          prev = b0;
        }
  expect(prev > 0, "sizes seen");
  expect(lbdps_workspace_bytes(&p, 10, nullptr) == LBDPS_E_INVALID, "NULL size pointer");
  lbdps_params beds[3] = {base(), base(), base()};
  beds[1].nx = 128;
  beds[1].ny = 512;
  beds[2].nx = 3;
  beds[2].ny = 3;
  const int64_t nmax[3] = {2000, 30000, 1};
  size_t bb = 0;
  expect(lbdps_batch_workspace_bytes(beds, 3, nmax, &bb) == LBDPS_OK && bb > 0, "batch workspace");
  size_t each = 0, sum = 0;
  for (int b = 0; b < 3; ++b) {
    expect(lbdps_workspace_bytes(&beds[b], nmax[b], &each) == LBDPS_OK, "bed workspace");
    sum += each;
  }
  expect(bb >= sum, "batch covers its beds");

  // a workspace that is too small is refused before any device call
  lbdps_ctx *ctx = nullptr;
  size_t need = 0;
  lbdps_workspace_bytes(&p, 100, &need);
  char small[256];
  expect(lbdps_create(&p, 100, small, need - 1, nullptr, nullptr, &ctx) == LBDPS_E_SHAPE && !ctx, "small workspace");
  expect(lbdps_create(&p, 100, nullptr, need, nullptr, nullptr, &ctx) == LBDPS_E_INVALID && !ctx, "NULL workspace");
  for (int s = -8; s <= 0; ++s) expect(lbdps_status_str((lbdps_status)s) != nullptr, "status string");
  std::printf("host validation: %d failures\n", failures);
  return failures ? 1 : 0;
}
