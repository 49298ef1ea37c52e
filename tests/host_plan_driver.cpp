// Host-side plan building under AddressSanitizer and UndefinedBehaviorSanitizer: every
// supported shape, precision, LED grid, multiplexing and flag combination, plus malformed
// problems, through elfpie_workspace_bytes (the plan tables are built on the host only;
// nothing touches a GPU).  Built and run by test_host_sanitizers.py; a sanitizer report
// aborts the process with a nonzero status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "elfpie.h"

namespace {

unsigned long long g_rng = 0x9e3779b97f4a7c15ull;
double uniform() {  // in [-0.5, 0.5)
  g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
  return double(g_rng >> 11) / double(1ull << 53) - 0.5;
}

// A g x g LED grid whose windows reach at most `reach` of the room (n_hi - n_lo) / 2, with
// sub-pixel jitter: led_k = offset_px / FOV.
std::vector<double> grid(int g, int n_lo, int up, double dx, double reach) {
  const double fov = n_lo * dx;
  const double room = 0.5 * (n_lo * up - n_lo);
  const double step = g > 1 ? 2.0 * reach * room / (g - 1) : 0.0;
  std::vector<double> k;
  for (int i = 0; i < g; ++i)
    for (int j = 0; j < g; ++j) {
      const double ox = (j - 0.5 * (g - 1)) * step + 0.4 * uniform();
      const double oy = (i - 0.5 * (g - 1)) * step + 0.4 * uniform();
      k.push_back(ox / fov);
      k.push_back(oy / fov);
    }
  return k;
}

int g_ok = 0, g_rejected = 0, g_bad = 0;

void check(const elfpie_problem& p, bool expect_ok, const char* what) {
  size_t bytes = 0;
  const elfpie_status s = elfpie_workspace_bytes(&p, &bytes);
  const bool ok = s == ELFPIE_OK;
  if (s < ELFPIE_OK || s > ELFPIE_E_NONFINITE) {
    std::printf("unknown status %d (%s)\n", int(s), what);
    ++g_bad;
  }
  if (ok && (bytes == 0 || bytes > (size_t(64) << 30))) {
    std::printf("implausible workspace %zu bytes (%s)\n", bytes, what);
    ++g_bad;
  }
  if (expect_ok && !ok) {
    std::printf("rejected %s: n_lo %d up %d K %d mux %d prec %d: %s\n", what, p.n_lo, p.upsample, p.K, p.mux,
                p.precision, elfpie_last_error(nullptr));
    ++g_bad;
  }
  if (!expect_ok && ok) {
    std::printf("accepted malformed problem (%s)\n", what);
    ++g_bad;
  }
  (ok ? g_ok : g_rejected)++;
}

}  // namespace

int main() {
  const int lows[] = {32, 64, 96, 128, 192, 256};
  const int ups[] = {2, 4};
  const int grids[] = {1, 3, 5, 7, 9, 11, 15};
  const int precs[] = {ELFPIE_F32, ELFPIE_F64, ELFPIE_F32_MFMA_BF16X3};
  for (int n_lo : lows)
    for (int up : ups)
      for (int prec : precs)
        for (int g : grids)
          for (int mux = 1; mux <= 3; ++mux)
            for (unsigned flags = 0; flags < 8; flags += 7) {
              const long long nh = (long long)n_lo * up;
              const bool shape_ok = (nh == 128 || nh == 256 || nh == 384 || nh == 512 || nh == 768 || nh == 1024) &&
                                    (prec == ELFPIE_F64 ? (n_lo == 32 || n_lo == 64)
                                                        : prec == ELFPIE_F32 || n_lo == 256);
              const int K = g * g;
              const bool mux_ok = K % mux == 0 && (mux == 1 || n_lo < 192);
              elfpie_problem p;
              elfpie_problem_defaults(&p);
              p.n_lo = n_lo;
              p.upsample = up;
              p.K = K;
              p.wavelength_um = 0.52;
              p.na = 0.1;
              p.dx_lo_um = 1.625;
              const std::vector<double> k = grid(g, n_lo, up, p.dx_lo_um, 0.8);
              p.led_k = k.data();
              p.precision = prec;
              p.flags = flags;
              p.mux = mux;
              p.norm = (g + mux) % 2;
              p.fidelity = (g + flags) % 2;
              // shapes the library does not take are rejected, never mis-built
              check(p, shape_ok && mux_ok, "grid");
            }
  // malformed problems of a valid shape: each must be rejected
  elfpie_problem base;
  elfpie_problem_defaults(&base);
  base.n_lo = 64;
  base.upsample = 4;
  base.K = 9;
  base.wavelength_um = 0.52;
  base.na = 0.1;
  base.dx_lo_um = 1.625;
  const std::vector<double> k9 = grid(3, 64, 4, 1.625, 0.8);
  base.led_k = k9.data();
  check(base, true, "base");
  std::vector<double> knan = k9;
  knan[5] = std::nan("");
  std::vector<double> kfar = k9;
  kfar[0] = 1e3;
  struct Bad {
    const char* what;
    void (*edit)(elfpie_problem&);
  };
  const Bad bads[] = {
      {"K = 0", [](elfpie_problem& p) { p.K = 0; }},
      {"n_lo = 48", [](elfpie_problem& p) { p.n_lo = 48; }},
      {"upsample = 3", [](elfpie_problem& p) { p.upsample = 3; }},
      {"negative wavelength", [](elfpie_problem& p) { p.wavelength_um = -0.5; }},
      {"zero NA", [](elfpie_problem& p) { p.na = 0.0; }},
      {"NaN pixel", [](elfpie_problem& p) { p.dx_lo_um = std::nan(""); }},
      {"negative alpha", [](elfpie_problem& p) { p.alpha = -1.0; }},
      {"gamma1 = 1", [](elfpie_problem& p) { p.gamma1 = 1.0; }},
      {"bad fidelity", [](elfpie_problem& p) { p.fidelity = 17; }},
      {"bad norm", [](elfpie_problem& p) { p.norm = -1; }},
      {"bad precision", [](elfpie_problem& p) { p.precision = 9; }},
      {"mux not dividing K", [](elfpie_problem& p) { p.mux = 2; }},
      {"NULL led_k", [](elfpie_problem& p) { p.led_k = nullptr; }},
  };
  for (const Bad& b : bads) {
    elfpie_problem p = base;
    b.edit(p);
    check(p, false, b.what);
  }
  elfpie_problem p = base;
  p.led_k = knan.data();
  check(p, false, "NaN LED frequency");
  p.led_k = kfar.data();
  check(p, false, "window off the spectrum");
  size_t bytes = 0;
  if (elfpie_workspace_bytes(nullptr, &bytes) == ELFPIE_OK || elfpie_workspace_bytes(&base, nullptr) == ELFPIE_OK) {
    std::printf("accepted NULL arguments\n");
    ++g_bad;
  }
  std::printf("plans built %d, rejected %d, problems %d\n", g_ok, g_rejected, g_bad);
  return g_bad == 0 ? 0 : 1;
}
