// Runs every entry point of the CPU oracle (oracle/lbm_oracle.cpp, compiled into this program) on
// small inputs that reach its edge cases: every face rule, odd lattice extents, windows clipped at
// walls and wrapped on periodic axes, point-sampled and cell-integral weights, every coupling
// variant, bubbles that reach the top, invalid arguments. Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py; any report fails the test.
#include "../oracle/lbm_oracle.cpp"

#include <cstdio>
#include <cstdlib>

namespace {

unsigned long long rng_state = 1710;
double uniform(double lo, double hi) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return lo + (hi - lo) * (double)(rng_state >> 11) / 9007199254740992.0;
}

int fail(const char* what) {
  std::fprintf(stderr, "oracle call failed: %s\n", what);
  return 1;
}

}  // namespace

int main() {
  int32_t c[57], opp[19];
  double w[19];
  orc_lattice(c, w, opp);
  const double u[3] = {0.05, -0.02, 0.01}, F[3] = {1e-3, 2e-3, -1e-3};
  double feq[19], S[19], g[19], out[19], rho, uo[3];
  orc_equilibrium(1.01, u, feq);
  orc_guo_source(1.3, u, F, S);
  for (int q = 0; q < 19; ++q) g[q] = uniform(-1e-3, 1e-3);
  orc_collide_node(1.7, g, F, out, &rho, uo);
  for (double r : {-2.0, -0.5, 0.0, 0.7, 3.0}) (void)orc_kernel_Z(r, 1.2), (void)orc_kernel_P(r);
  for (int per = 0; per < 2; ++per)
    for (int point = 0; point < 2; ++point)
      for (double x : {0.0, 0.3, 2.5, 6.0, 6.9}) {
        int32_t idx[64];
        double wt[64];
        (void)orc_axis_weights(x, 2.7, 7, per, idx, wt, 64, point);
      }
  const int faces[4][6] = {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 1}, {2, 2, 2, 2, 0, 1}, {1, 1, 2, 2, 2, 2}};
  const int nx = 7, ny = 6, nz = 11;
  const long N = (long)nx * ny * nz;
  std::vector<double> pop(19 * N), tmp(19 * N), Fv(3 * N), U(3 * N), pre(19 * N), rhof(N), uf(3 * N),
      curl(3 * N);
  for (const auto& f : faces) {
    const int32_t bc[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
    for (auto& v : pop) v = uniform(-1e-3, 1e-3);
    for (auto& v : Fv) v = uniform(-1e-4, 1e-4);
    if (orc_lbm_step(nx, ny, nz, bc, 1.6, pop.data(), tmp.data(), Fv.data(), U.data(), 1))
      return fail("lbm_step");
    if (orc_lbm_step(nx, ny, nz, bc, 0.9, pop.data(), tmp.data(), nullptr, nullptr, 2))
      return fail("lbm_step without force");
    if (orc_stream(nx, ny, nz, bc, pop.data(), pre.data())) return fail("stream");
    double sums[4];
    if (orc_moments(nx, ny, nz, pop.data(), rhof.data(), uf.data(), sums)) return fail("moments");
    if (orc_curl(nx, ny, nz, bc, uf.data(), curl.data())) return fail("curl");
    for (int point = 0; point < 2; ++point)
      for (double x : {0.0, 0.4, 3.0, 6.0}) {
        const double xb[3] = {x, 0.5 * x, 10.0 - x}, psi[3] = {1e-4, -2e-4, 3e-4};
        double ul[3], wl[3];
        if (orc_interpolate(nx, ny, nz, bc, uf.data(), xb, 1.6, ul, wl, point)) return fail("interpolate");
        if (orc_spread(nx, ny, nz, bc, xb, 1.6, psi, Fv.data(), point)) return fail("spread");
      }
    for (int coupling : {0, 1, 2, 4, 8, 9}) {
      orc_bubble_params P{1e-3, 1.0, 1e-3, 1e-3, 0.5, 1.0, 1.0, 1.5, 0.15, 0.474, 10, coupling};
      const int nb = 12;
      std::vector<double> pos(3 * nb), vel(3 * nb), d(nb), ulp(3 * nb), psi(3 * nb);
      std::vector<int32_t> state(nb, 1);
      for (int b = 0; b < nb; ++b) {
        pos[b] = uniform(0.0, nx - 1.0);
        pos[nb + b] = uniform(0.0, ny - 1.0);
        pos[2 * nb + b] = b < 2 ? nz - 1.2 : uniform(0.0, nz - 1.0);  // two reach the top
        vel[2 * nb + b] = b < 2 ? 0.5 : 0.0;
        d[b] = uniform(0.8, 2.4);
      }
      for (auto& v : pop) v = 0.0;
      for (int step = 0; step < 20; ++step)
        if (orc_method_step(nx, ny, nz, bc, 1.3, &P, nb, pos.data(), vel.data(), d.data(), ulp.data(),
                            state.data(), pop.data(), tmp.data(), Fv.data(), U.data(), psi.data(), 2))
          return fail("method_step");
    }
  }
  // argument checks
  const int32_t bad[6] = {2, 0, 0, 0, 0, 0};
  if (orc_lbm_step(nx, ny, nz, bad, 1.0, pop.data(), tmp.data(), nullptr, nullptr, 1) == 0)
    return fail("one-sided periodic face accepted");
  if (orc_lbm_step(0, ny, nz, faces[0], 1.0, pop.data(), tmp.data(), nullptr, nullptr, 1) == 0)
    return fail("empty lattice accepted");
  std::printf("oracle sanitizer run: ok\n");
  return 0;
}
