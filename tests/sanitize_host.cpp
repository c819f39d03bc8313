// Host-side exercise of libsip's engine for a sanitizer build (address and
// undefined-behaviour checks on the CPU; no GPU call is made): validation,
// operator row counts, workspace and plan sizes (which build the work tables
// on the host), multilevel grids and set lists, option defaults and status
// strings, over a seeded sweep of grids, set lists and tiles, valid and not.
// Prints one line per check group and exits non-zero on an inconsistency.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "sip.h"

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  auto uni = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
  auto unif = [&](double lo, double hi) { return std::uniform_real_distribution<double>(lo, hi)(rng); };

  for (int st = -8; st <= 1; ++st) CHECK(sip_strerror(st) != nullptr && std::strlen(sip_strerror(st)) > 0);
  sip_opts o;
  CHECK(sip_opts_default(&o) == SIP_OK);
  CHECK(sip_opts_default(nullptr) == SIP_EINVAL);
  sip_tiles td;
  CHECK(sip_tiles_default(&td) == SIP_OK);

  int valid = 0, invalid = 0;
  for (int trial = 0; trial < 3000; ++trial) {
    sip_grid g{};
    g.ndim = uni(0, 9) < 7 ? 2 : 3;
    for (int a = 0; a < g.ndim; ++a) {
      g.n[a] = uni(0, 9) == 0 ? uni(-1, 1) : uni(1, g.ndim == 2 ? 700 : 60);
      g.h[a] = uni(0, 20) == 0 ? 0.0 : unif(0.1, 30.0);
    }
    if (uni(0, 30) == 0) g.ndim = uni(-1, 5);
    const int nsets = uni(0, 30) == 0 ? uni(-2, SIP_MAX_SETS + 2) : uni(0, 6);
    sip_set sets[SIP_MAX_SETS + 2];
    std::memset(sets, 0, sizeof(sets));
    for (int i = 0; i < SIP_MAX_SETS + 2; ++i) {
      sip_set& s = sets[i];
      s.kind = uni(0, 80) == 0 ? uni(-1, 7) : uni(0, 4);
      s.op = uni(0, 80) == 0 ? uni(-1, 8) : uni(0, 5);
      s.lo = unif(-2, 0.5);
      s.hi = s.lo + unif(uni(0, 80) == 0 ? -1.0 : 0.0, 2.0);
      if (uni(0, 10) == 0) s.hi = INFINITY;
      if (uni(0, 10) == 0) s.lo = -INFINITY;
      if (uni(0, 200) == 0) s.lo = NAN;
      s.tau = uni(0, 80) == 0 ? -1.0 : unif(0.0, 100.0);
      s.k = uni(0, 80) == 0 ? uni(-5, 0) : uni(1, 400);
      s.line = uni(0, 4) == 0 ? uni(0, 3) : 0;
      if (uni(0, 200) == 0) s.line = uni(-2, 6);
    }
    o.field = uni(0, 1);
    o.reduce = uni(0, 10) == 0 ? SIP_F32 : SIP_F64;
    o.stop_every = uni(0, 2) == 0 ? 5 : 0;
    o.adapt_every = uni(0, 5) == 0 ? 0 : 2;
    o.evol_hist = uni(0, 20) == 0 ? uni(-1, 12) : 5;
    o.log_schedule = uni(0, 1);
    o.max_iter = uni(0, 20) == 0 ? uni(-3, 0) : uni(1, 300);
    const int32_t v = sip_validate(&g, sets, nsets, &o);
    const int64_t ws = sip_workspace_bytes(&g, sets, nsets, &o);
    sip_tiles t = td;
    if (uni(0, 1)) {
      t.pt_points = 256 * uni(0, 16);
      t.thr_points = 256 * uni(0, 16);
      t.pt_max_items = uni(0, 4096);
      t.thr_max_items = uni(0, 4096);
      t.pt_threads = uni(0, 10) == 0 ? 384 : (uni(0, 1) ? 256 : 512);
      t.cg_form = uni(0, 10) == 0 ? 3 : uni(0, 2);
    }
    const bool tiles_ok = t.pt_points >= 256 && t.thr_points >= 256 && t.pt_max_items >= 1 &&
                          t.thr_max_items >= 1 && (t.pt_threads == 256 || t.pt_threads == 512) &&
                          (t.cg_form >= 0 && t.cg_form <= 2);
    const int64_t pb = sip_plan_bytes(&g, sets, nsets, &o, &t);
    if (v == SIP_OK) {
      ++valid;
      CHECK(ws > 0 && ws % 256 == 0);
      CHECK(tiles_ok ? (pb >= ws && pb % 256 == 0) : pb == -1);
      for (int i = 0; i < nsets; ++i) CHECK(sip_set_rows(&g, &sets[i]) >= 0);
      sip_grid gl{};
      sip_set sl[SIP_MAX_SETS];
      for (int lev = 0; lev < 4; ++lev) {
        if (sip_level(&g, sets, nsets, lev, &gl, sl) != SIP_OK) break;
        for (int a = 0; a < gl.ndim; ++a) CHECK(gl.n[a] >= 1 && gl.n[a] <= g.n[a]);
        (void)sip_workspace_bytes(&gl, sl, nsets, &o);
      }
    } else {
      ++invalid;
      CHECK(v == SIP_EINVAL || v == SIP_EUNSUPPORTED);
      CHECK(ws == -1 && pb == -1);
    }
  }
  std::printf("host sweep: %d valid, %d invalid configurations, %d failed checks\n", valid, invalid, failures);
  CHECK(sip_validate(nullptr, nullptr, 0, &o) == SIP_EINVAL);
  CHECK(sip_plan_bytes(nullptr, nullptr, 0, &o, nullptr) == -1);
  CHECK(sip_set_rows(nullptr, nullptr) == -1);
  return failures == 0 ? 0 : 1;
}
