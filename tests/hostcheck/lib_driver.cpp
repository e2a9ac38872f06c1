// Drives the host half of the library (include/lisaresp.h) under the host
// sanitizers: the orbit spline fit, the padding rules, argument checks of the
// per-template calls and the batch planner (ragged and empty templates,
// overlaps, ranges, groups), with the kernel launchers stubbed out.  Calls
// that would copy to a device either fail cleanly (no GPU) or reach the
// stubs.  Exit status 0 and "ok" when every call returned as expected.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/lisaresp.h"

extern int g_launches;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

int main() {
  // coarse samples of a rigid triangle circling on 1 AU (light times ~8.3 s)
  const int64_t n = 40;
  const double dto = 1e4, AU = 1.495978707e11, L = 2.5e9;
  std::vector<double> x(n * 9), ltt(n * 6);
  for (int64_t k = 0; k < n; ++k) {
    const double a = 2e-7 * k * dto;
    for (int s = 0; s < 3; ++s) {
      const double b = a + 2.0943951023931953 * s;
      x[k * 9 + s * 3 + 0] = AU * std::cos(a) + L / std::sqrt(3.0) * std::cos(b);
      x[k * 9 + s * 3 + 1] = AU * std::sin(a) + L / std::sqrt(3.0) * std::sin(b);
      x[k * 9 + s * 3 + 2] = 0.0;
    }
    for (int l = 0; l < 6; ++l) ltt[k * 6 + l] = L / 299792458.0 + 1e-4 * std::sin(0.1 * k + l);
  }
  const size_t nb = lr_orbits_bytes(n);
  CHECK(nb > 0 && lr_orbits_bytes(3) == 0);
  std::vector<double> store(nb / sizeof(double) + 1);
  lr_orbits orb{};
  // arguments the fit rejects
  CHECK(lr_orbits_init(0.0, dto, 3, x.data(), ltt.data(), store.data(), nb, &orb, nullptr) == LR_E_ARG);
  CHECK(lr_orbits_init(0.0, -1.0, n, x.data(), ltt.data(), store.data(), nb, &orb, nullptr) == LR_E_ARG);
  CHECK(lr_orbits_init(0.0, dto, n, x.data(), ltt.data(), store.data(), nb - 8, &orb, nullptr) == LR_E_WORKSPACE);
  std::vector<double> xnan = x;
  xnan[17] = NAN;
  CHECK(lr_orbits_init(0.0, dto, n, xnan.data(), ltt.data(), store.data(), nb, &orb, nullptr) == LR_E_ARG);
  // the fit runs; the copy to the (absent) device then fails cleanly or succeeds
  const int st = lr_orbits_init(0.0, dto, n, x.data(), ltt.data(), store.data(), nb, &orb, nullptr);
  CHECK(st == LR_OK || st == LR_E_HIP);
  // the host-only fit: bounds without a device, enough for the padding rules
  lr_orbits hb{};
  CHECK(lr_orbits_bounds(0.0, dto, 3, x.data(), ltt.data(), &hb) == LR_E_ARG);
  CHECK(lr_orbits_bounds(0.0, dto, n, xnan.data(), ltt.data(), &hb) == LR_E_ARG);
  CHECK(lr_orbits_bounds(0.0, dto, n, x.data(), ltt.data(), nullptr) == LR_E_ARG);
  CHECK(lr_orbits_bounds(0.0, dto, n, x.data(), ltt.data(), &hb) == LR_OK);
  CHECK(hb.coef == nullptr && hb.L_min <= hb.L_max && hb.L_max < 8.5 && hb.R_max > AU);
  {
    int64_t hf = 0, hbk = 0;
    CHECK(lr_tdi_padding(&hb, 25, 2, 10.0, &hf, &hbk) == LR_OK && hf > 13 && hbk >= 13);
    CHECK(lr_projection_padding(&hb, 25, 10.0, &hf, &hbk) == LR_OK && hf > 13 && hbk > 13);
  }
  // a handle as lr_orbits_init fills it, for the host-only calls below
  orb.t0 = 0.0; orb.dt = dto; orb.n = n; orb.coef = store.data();
  orb.L_min = 8.3; orb.L_max = 8.4; orb.R_max = 1.02 * AU;
  int64_t f = 0, b = 0;
  for (int order = 1; order <= 31; order += 2) {
    CHECK(lr_projection_padding(&orb, order, 10.0, &f, &b) == LR_OK && f > 0 && b > 0);
    for (int gen = 1; gen <= 2; ++gen)
      CHECK(lr_tdi_padding(&orb, order, gen, 10.0, &f, &b) == LR_OK && f > 0 && b > 0);
  }
  CHECK(lr_projection_padding(&orb, 4, 10.0, &f, &b) == LR_E_UNSUPPORTED);
  CHECK(lr_tdi_padding(&orb, 25, 3, 10.0, &f, &b) != LR_OK);
  CHECK(lr_projection_padding(&orb, 25, 0.0, &f, &b) != LR_OK);

  // per-template calls: argument errors are caught before any launch
  const int before = g_launches;
  double dummy[16];
  CHECK(lr_project_links(&orb, 1e5, 10.0, 100, dummy, dummy, dummy, 25, 0, 50, dummy, nullptr) != LR_OK);
  CHECK(lr_tdi_combine(&orb, 1e5, 10.0, 100, dummy, 2, 6, 0, 20, 10, dummy, nullptr) != LR_OK);
  CHECK(lr_loglike(dummy, dummy, -1, 1.0, dummy, nullptr, dummy, 0, nullptr) == LR_E_ARG);
  CHECK(lr_loglike(dummy, dummy, 4, 0.0, dummy, nullptr, dummy, 8192, nullptr) == LR_E_ARG);
  CHECK(g_launches == before);

  // batch planner: ragged templates, an empty one, groups 1, 2, 4

  int64_t fp = 0, bp = 0, ft = 0, bt = 0;
  CHECK(lr_projection_padding(&orb, 25, 10.0, &fp, &bp) == LR_OK);
  CHECK(lr_tdi_padding(&orb, 25, 2, 10.0, &ft, &bt) == LR_OK);
  std::vector<lr_template> t;
  int64_t hoff = 0, ooff = 0;
  for (int64_t nout : {3000, 0, 1, 33, 481, 1000, 2999}) {
    lr_template T;
    T.n_out = nout;
    T.out_start = fp + ft;
    T.n_h = nout > 0 ? fp + ft + nout + bt + bp : 0;
    T.h_offset = hoff;
    T.out_offset = ooff;
    hoff += T.n_h;
    ooff += 3 * nout;
    t.push_back(T);
  }
  for (int group : {1, 2, 4})
    for (int tile : {0, 256, 512, 1024})
      for (int segment : {0, 1, 3, 64}) {
        const size_t ws = lr_batch_workspace(t.data(), (int64_t)t.size(), &orb, 10.0, 25, 2,
                                             LR_AET, group, tile, segment, 1);
        if (group == 4 && tile == 1024) {             // not compiled
          CHECK(ws == 0);
          continue;
        }
        CHECK(ws > 0);
        std::vector<char> w(ws);
        lr_batch bt_{};
        const int s2 = lr_batch_prepare(t.data(), (int64_t)t.size(), &orb, &orb, 2e4, 10.0, 25,
                                        2, LR_AET, group, tile, segment, 1, w.data(), ws, &bt_,
                                        nullptr);
        CHECK(s2 == LR_OK || s2 == LR_E_HIP);
        // too small a workspace, bad group, overlapping outputs, short h
        CHECK(lr_batch_prepare(t.data(), (int64_t)t.size(), &orb, &orb, 2e4, 10.0, 25, 2, LR_AET,
                               group, tile, segment, 1, w.data(), ws - 1, &bt_,
                               nullptr) == LR_E_WORKSPACE);
      }
  CHECK(lr_batch_workspace(t.data(), (int64_t)t.size(), &orb, 10.0, 25, 2, LR_AET, 3, 0, 0, 0) ==
        0);
  CHECK(lr_batch_workspace(t.data(), (int64_t)t.size(), &orb, 10.0, 25, 2, LR_AET, 2, 768, 0,
                           0) == 0);
  CHECK(lr_batch_workspace(t.data(), (int64_t)t.size(), &orb, 10.0, 25, 2, LR_AET, 2, 0, 65,
                           0) == 0);
  CHECK(lr_batch_workspace(t.data(), (int64_t)t.size(), &orb, 10.0, 25, 2, LR_AET, 2, 0, -1,
                           0) == 0);
  std::vector<lr_template> bad = t;
  bad[2].out_offset = bad[0].out_offset;
  {
    const size_t ws = lr_batch_workspace(bad.data(), (int64_t)bad.size(), &orb, 10.0, 25, 2,
                                         LR_AET, 2, 0, 0, 0);
    std::vector<char> w(ws);
    lr_batch bt_{};
    CHECK(lr_batch_prepare(bad.data(), (int64_t)bad.size(), &orb, &orb, 2e4, 10.0, 25, 2,
                           LR_AET, 2, 0, 0, 0, w.data(), ws, &bt_, nullptr) == LR_E_ARG);
    bad = t;
    bad[0].n_h -= 1;
    CHECK(lr_batch_prepare(bad.data(), (int64_t)bad.size(), &orb, &orb, 2e4, 10.0, 25, 2,
                           LR_AET, 2, 0, 0, 0, w.data(), ws, &bt_, nullptr) == LR_E_RANGE);
  }
  CHECK(lr_status_str(LR_E_RANGE) != nullptr && lr_status_str(99) != nullptr);
  CHECK(lr_last_error() != nullptr);
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
