// Drives every entry point of the oracle on small geometries, for a build
// with AddressSanitizer and UndefinedBehaviorSanitizer (any report aborts the
// program).  Prints "oracle driver: all checks passed" when every call that
// should succeed did, every call that should fail was refused, and every
// result is finite.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cg_oracle.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s (%s)\n", what, orc_last_error());
    ++g_fail;
  }
}

bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// Small deterministic generator (64-bit LCG, top bits) for the geometries.
struct Lcg {
  uint64_t s;
  double uni() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

orc_params base(int dim, int nx, int ny, int nz) {
  orc_params p;
  std::memset(&p, 0, sizeof(p));
  p.dim = dim;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.collision = dim == 3 ? 1 : 0;
  p.tau_r = 1.0;
  p.tau_b = 0.7;
  p.sigma = 0.02;
  p.beta = 0.9;
  p.rho0 = 1.0;
  p.theta_deg = 60.0;
  p.rho_in = 1.0;
  p.rho_out = 1.0;
  p.eps_c = 1e-6;
  p.eps_f = 1e-12;
  p.eps_v = 1e-12;
  return p;
}

// A channel along z with solid x/y walls, random solid voxels inside the
// middle section, open (Zou-He) or periodic z.
std::vector<uint8_t> channel(int nx, int ny, int nz, double frac, uint64_t seed) {
  Lcg r{seed};
  std::vector<uint8_t> s((size_t)nx * ny * nz, 0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const bool wall = x == 0 || y == 0 || x == nx - 1 || y == ny - 1;
        const bool mid = z >= 3 && z < nz - 3;
        s[x + (size_t)nx * (y + (size_t)ny * z)] = wall || (mid && r.uni() < frac);
      }
  return s;
}

std::vector<double> slug_phase(int nx, int ny, int nz, int z0, int z1) {
  std::vector<double> p((size_t)nx * ny * nz);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) p[x + (size_t)nx * (y + (size_t)ny * z)] = (z >= z0 && z < z1) ? 1.0 : -1.0;
  return p;
}

void exercise(const char* name, const orc_params& p, const std::vector<uint8_t>& solid, const double* theta_field,
              const std::vector<double>& phi0, int steps) {
  std::printf("case %s\n", name);
  orc_sim* s = orc_create(&p, solid.data(), theta_field);
  check(s != nullptr, name);
  if (!s) return;
  const size_t V = (size_t)p.nx * p.ny * p.nz;
  const int Q = orc_q(s);
  check(orc_set_phase(s, phi0.data()) == 0, "set_phase");
  check(orc_step(s, steps) == 0, "step");
  std::vector<double> fr((size_t)Q * V), fb((size_t)Q * V);
  check(orc_get_state(s, fr.data(), fb.data()) == 0, "get_state");
  check(finite_all(fr) && finite_all(fb), "finite state");
  check(orc_set_state(s, fr.data(), fb.data()) == 0, "set_state");
  std::vector<double> rr(V), rb(V), ph(V), u(3 * V), n3(3 * V), c3(3 * V), k(V), f3(3 * V);
  check(orc_macro(s, rr.data(), rb.data(), ph.data(), u.data()) == 0, "macro");
  check(orc_macro(s, nullptr, nullptr, nullptr, nullptr) == 0, "macro without outputs");
  check(orc_stages(s, ph.data(), n3.data(), c3.data(), k.data(), f3.data()) == 0, "stages");
  check(finite_all(u) && finite_all(k) && finite_all(f3), "finite stages");
  orc_obs o;
  for (int axis = 0; axis < p.dim; ++axis) check(orc_observe(s, axis, 1, &o) == 0, "observe");
  check(orc_observe_slab(s, p.dim - 1, 1, 3, p.dim - 1, 2, &o) == 0, "observe_slab");
  check(std::isfinite(o.mass_r) && o.nan_count == 0, "finite observables");
  double J = 0.0;
  for (int obj = 0; obj < 3; ++obj) check(orc_objective(s, obj, p.dim - 1, 1, 3, &J) == 0 && std::isfinite(J), "objective");
  std::vector<uint8_t> cls(V);
  std::vector<double> g3(V), nw3(3 * V), ct(V), st(V);
  check(orc_setup_info(s, cls.data(), g3.data(), nw3.data(), ct.data(), st.data()) == 0, "setup_info");
  const double g[3] = {0.0, 0.0, 1e-5};
  check(orc_set_body_force(s, g) == 0, "set_body_force");
  std::vector<int64_t> perm(V);
  for (size_t v = 0; v < V; ++v) perm[v] = (int64_t)(V - 1 - v);
  check(orc_set_visit_order(s, perm.data()) == 0, "set_visit_order");
  perm[0] = perm[1];
  check(orc_set_visit_order(s, perm.data()) != 0, "set_visit_order refuses a repeated voxel");
  if (p.bc == 1) {
    check(orc_set_pressure(s, 1.02, 1.0) == 0, "set_pressure");
    check(orc_set_pressure(s, -1.0, 1.0) != 0, "set_pressure refuses a negative density");
    check(orc_switch_inlet(s, p.zeta_r >= 0.5 ? 0.0 : 1.0) == 0, "switch_inlet");
    check(orc_switch_inlet(s, 0.5) != 0, "switch_inlet refuses a mixed fluid");
  } else {
    check(orc_set_pressure(s, 1.02, 1.0) != 0, "set_pressure refuses a run without faces");
  }
  check(orc_step(s, 3) == 0, "step after changes");
  check(orc_get_state(s, fr.data(), fb.data()) == 0 && finite_all(fr) && finite_all(fb), "finite after changes");
  orc_destroy(s);
  // forward-mode derivative along theta (global) and g_z
  if (p.scheme == 1 || p.scheme == 2) {
    orc_tangent_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.objective = 1;
    sp.axis = p.dim - 1;
    sp.lo = 0;
    sp.hi = 1 << 30;
    sp.n_steps = 3;
    std::vector<double> dir(V, 0.0);
    for (size_t v = 0; v < V; ++v) dir[v] = solid[v] ? 1.0 : 0.0;
    for (int seed : {0, 1 + (p.dim - 1), 4}) {
      if (seed == 0 && theta_field) continue;
      if (seed == 4 && !theta_field) continue;
      sp.seed = seed;
      sp.theta_dir = seed == 4 ? dir.data() : nullptr;
      double Jt = 0.0, dJ = 0.0;
      check(orc_tangent(&p, solid.data(), theta_field, phi0.data(), &sp, &Jt, &dJ) == 0 && std::isfinite(dJ),
            "tangent");
    }
  }
}

void node_functions() {
  int e[19 * 3], opp[19];
  double w[19];
  check(orc_lattice(2, e, w, opp) == 9, "lattice 2");
  check(orc_lattice(3, e, w, opp) == 19, "lattice 3");
  check(orc_lattice(4, e, w, opp) < 0, "lattice refuses dim 4");
  double M[19 * 19], n2[19];
  check(orc_mrt_matrix(M, n2) == 0, "mrt matrix");
  const double u[3] = {0.01, -0.02, 0.005}, F[3] = {1e-4, 0.0, -2e-4};
  double meq[19], S[19], sf[19];
  check(orc_meq(1.01, 1.0, u, meq) == 0, "meq");
  double s_nu = 0.0, s_q = 0.0;
  check(orc_rates(0.3, 1.0, 0.6, &s_nu, &s_q) == 0, "rates");
  for (int i = 0; i < 19; ++i) S[i] = i % 3 ? s_nu : s_q;
  check(orc_forcing_moments(u, F, S, sf) == 0, "forcing moments");
  double ft[19], out[19], cr[19], cb[19];
  orc_lattice(3, e, w, opp);
  for (int i = 0; i < 19; ++i) ft[i] = w[i] * (1.0 + 0.01 * i);
  for (int coll = 0; coll < 2; ++coll)
    check(orc_collide_node(3, coll, ft, 1.03, 1.0, u, F, s_nu, s_q, nullptr, out) == 0, "collide node");
  check(orc_collide_node(3, 1, ft, 1.03, 1.0, u, F, s_nu, s_q, S, out) == 0, "collide node with rates");
  const double nrm[3] = {0.6, 0.0, 0.8};
  check(orc_recolor(3, out, 0.7, 0.33, 0.9, nrm, cr, cb) == 0, "recolor");
  const double nc[3] = {0.0, 0.6, 0.8}, nw[3] = {0.0, 0.0, 1.0};
  double r3[3];
  for (double th : {15.0, 60.0, 90.0, 135.0, 170.0}) {
    for (int line = 0; line < 2; ++line)
      check(orc_scheme1(3, nc, nw, th, line, 1e-12, 1e-12, r3) == 0 && std::isfinite(r3[0]), "scheme1");
    check(orc_scheme2(3, nc, nw, th, 1e-12, r3) == 0 && std::isfinite(r3[0]), "scheme2");
  }
  double a[19], b[19];
  for (int i = 0; i < 19; ++i) {
    a[i] = 0.4 * w[i];
    b[i] = 0.6 * w[i];
  }
  check(orc_zouhe_inlet(a, b, 1.02, 0.25) == 0, "zou-he inlet");
  check(orc_zouhe_outlet(a, b, 1.0, 0.2) == 0, "zou-he outlet");
}

}  // namespace

int main() {
  orc_set_threads(2);
  node_functions();
  {
    // 3D channel, Zou-He faces, Type-I, MRT, Scheme-I, mixed injection
    const int nx = 8, ny = 8, nz = 14;
    orc_params p = base(3, nx, ny, nz);
    p.bc = 1;
    p.rho_in = 1.02;
    p.zeta_r = 0.25;
    p.scheme = 1;
    const auto s = channel(nx, ny, nz, 0.15, 7);
    exercise("channel-mrt-scheme1-type1", p, s, nullptr, slug_phase(nx, ny, nz, 4, 9), 12);
    // the same with BGK, Scheme-II, a per-voxel angle field and a body force
    p.collision = 0;
    p.scheme = 2;
    p.rho_in = 1.0;
    p.zeta_r = 1.0;
    p.g[2] = 1e-5;
    std::vector<double> th((size_t)nx * ny * nz, 0.0);
    Lcg r{3};
    for (size_t v = 0; v < th.size(); ++v) th[v] = s[v] ? 20.0 + 140.0 * r.uni() : 0.0;
    exercise("channel-bgk-scheme2-field-type2", p, s, th.data(), slug_phase(nx, ny, nz, 4, 9), 12);
    // fictitious-density wetting, literal Scheme-I start on a periodic z
    p = base(3, nx, ny, nz);
    p.scheme = 3;
    p.theta_deg = 140.0;
    p.periodic[2] = 1;
    exercise("channel-fictitious-periodic", p, s, nullptr, slug_phase(nx, ny, nz, 2, 7), 10);
    p.scheme = 1;
    p.s1_line = 1;
    exercise("channel-scheme1-literal", p, s, nullptr, slug_phase(nx, ny, nz, 2, 7), 10);
  }
  {
    // 2D sessile drop on a wall, periodic x
    const int nx = 24, ny = 12;
    orc_params p = base(2, nx, ny, 1);
    p.periodic[0] = 1;
    p.scheme = 1;
    std::vector<uint8_t> s((size_t)nx * ny, 0);
    std::vector<double> ph((size_t)nx * ny, -1.0);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        s[x + nx * y] = y == 0 || y == ny - 1;
        const double dx = x - 12.0, dy = y - 1.0;
        if (dx * dx + dy * dy < 25.0 && !s[x + nx * y]) ph[x + nx * y] = 1.0;
      }
    exercise("sessile-2d-scheme1", p, s, nullptr, ph, 15);
    p.scheme = 2;
    exercise("sessile-2d-scheme2", p, s, nullptr, ph, 15);
  }
  {
    // 3D periodic drop, no solid
    const int n = 8;
    orc_params p = base(3, n, n, n);
    p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    std::vector<uint8_t> s((size_t)n * n * n, 0);
    std::vector<double> ph((size_t)n * n * n, -1.0);
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
          const double d2 = (x - 3.5) * (x - 3.5) + (y - 3.5) * (y - 3.5) + (z - 3.5) * (z - 3.5);
          if (d2 < 6.25) ph[x + n * (y + n * z)] = 1.0;
        }
    exercise("periodic-drop", p, s, nullptr, ph, 10);
  }
  {
    // refusals
    std::vector<uint8_t> s(4 * 4 * 4, 0);
    orc_params p = base(3, 4, 4, 4);
    check(orc_create(&p, s.data(), nullptr) == nullptr, "fluid on a wall face is refused");
    p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    p.tau_r = 0.4;
    check(orc_create(&p, s.data(), nullptr) == nullptr, "tau below 1/2 is refused");
    p.tau_r = 1.0;
    p.scheme = 7;
    check(orc_create(&p, s.data(), nullptr) == nullptr, "unknown scheme is refused");
    std::vector<uint8_t> all_solid(4 * 4 * 4, 1);
    p.scheme = 0;
    check(orc_create(&p, all_solid.data(), nullptr) == nullptr, "no fluid is refused");
  }
  if (g_fail) {
    std::printf("oracle driver: %d checks failed\n", g_fail);
    return 1;
  }
  std::printf("oracle driver: all checks passed\n");
  return 0;
}
