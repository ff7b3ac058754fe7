// Drives the library's host set-up code (voxel classes, boundary sets,
// smoothing, wall normals, contact angles, sparse index and pull tables) on
// small geometries, for a build of its host pass with AddressSanitizer and
// UndefinedBehaviorSanitizer.  Prints "setup driver: all checks passed" when
// every geometry that should be accepted was, every one that should be
// refused was, and the tables agree with a plain neighbour search.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "setup.hpp"
#include "step.hpp"

namespace {

int g_fail = 0;

void check(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what.c_str());
    ++g_fail;
  }
}

struct Lcg {
  uint64_t s;
  double uni() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

// Source of every pull link from a direct neighbour search over the voxels:
// the fluid node at x - e_i, kOpen across the open z faces, else kBounce.
int expected_source(const cg::HostSetup& S, const std::vector<uint8_t>& solid, const std::vector<int>& node_of,
                    int n, const int* e, bool open_z) {
  const int v = S.node_vox[n];
  int c[3] = {v % S.nx, (v / S.nx) % S.ny, v / (S.nx * S.ny)};
  const int dims[3] = {S.nx, S.ny, S.nz};
  for (int a = 0; a < 3; ++a) {
    c[a] -= e[a];
    if (c[a] < 0 || c[a] >= dims[a]) {
      if (open_z && a == 2) return cg::kOpen;
      if (!S.per[a]) return cg::kBounce;
      c[a] = (c[a] + dims[a]) % dims[a];
    }
  }
  const int u = c[0] + S.nx * (c[1] + S.ny * c[2]);
  return solid[u] ? cg::kBounce : node_of[u];
}

void run(const char* name, int dim, int nx, int ny, int nz, const uint8_t per[3], int bc,
         const std::vector<uint8_t>& solid, int scheme, const double* field, bool expect_ok) {
  cg_geometry g{};
  g.dim = dim;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.solid = solid.data();
  for (int a = 0; a < 3; ++a) g.periodic[a] = per[a];
  cg_wetting w{};
  w.scheme = scheme;
  w.theta_deg = 70.0;
  w.theta_field_deg = field;
  cg_bc b{};
  b.type = bc;
  b.rho_in = 1.01;
  b.rho_out = 1.0;
  b.zeta_r = 0.5;
  for (int table : {0, 16, 32}) {
    cg::HostSetup S;
    std::string err;
    const int rc = cg::build_setup(g, w, b, &S, &err, table);
    std::printf("case %s table %d: rc %d %s\n", name, table, rc, err.c_str());
    if (!expect_ok) {
      check(rc != 0, std::string(name) + ": refused");
      return;
    }
    check(rc == 0, std::string(name) + ": accepted");
    if (rc != 0) return;
    const int V = nx * ny * nz;
    int nfl = 0;
    std::vector<int> node_of(V, -1);
    for (int v = 0; v < V; ++v) nfl += solid[v] == 0;
    check(S.N == nfl, std::string(name) + ": fluid node count");
    for (int n = 0; n < S.N; ++n) node_of[S.node_vox[n]] = n;
    // the int32 table against the neighbour search
    int bad = 0;
    for (int n = 0; n < S.N; ++n)
      for (int i = 1; i < S.Q; ++i) {
        int e[3];
        for (int a = 0; a < 3; ++a) e[a] = dim == 3 ? cg::Lat<3>::e(i, a) : cg::Lat<2>::e(i, a);
        const int want = expected_source(S, solid, node_of, n, e, bc == 1);
        bad += S.nbr[(size_t)(i - 1) * S.Np + n] != want;
      }
    check(bad == 0, std::string(name) + ": pull table against the neighbour search");
    for (size_t k = 0; k < S.cos_t.size(); ++k)
      if (!std::isfinite(S.cos_t[k]) || !std::isfinite(S.sin_t[k])) {
        check(false, std::string(name) + ": finite angles");
        break;
      }
    for (double x : S.nw)
      if (!std::isfinite(x)) {
        check(false, std::string(name) + ": finite wall normals");
        break;
      }
    // the angles again from a field, as a separate call
    std::vector<double> ct, st, fd;
    std::vector<unsigned> fl = S.flags;
    std::string e2;
    check(cg::contact_angles(S, 35.0, field, &ct, &st, &fl, &fd, &e2) != 0,
          std::string(name) + ": contact_angles refuses unsized outputs");
    ct = S.cos_t;
    st = S.sin_t;
    fd = S.sb_fd;
    check(cg::contact_angles(S, 35.0, field, &ct, &st, &fl, &fd, &e2) == 0, std::string(name) + ": contact_angles");
  }
}

// The face kernel's launch covers whole 64-node tiles (the pull table
// decodes per tile): wave w takes the w-th tile holding inlet nodes, then the
// tiles holding outlet nodes.  Every face node must come up exactly once,
// and each wave's nodes must lie in one tile.
void face_tile_mapping() {
  Lcg r{99};
  for (int trial = 0; trial < 4000; ++trial) {
    cg::StepParams P{};
    P.N = 1 + (int)(r.uni() * 5000);
    P.n_in = (int)(r.uni() * (P.N + 1));
    if (P.n_in > P.N) P.n_in = P.N;
    P.n_out = (int)(r.uni() * (P.N - P.n_in + 1));
    if (P.n_out > P.N - P.n_in) P.n_out = P.N - P.n_in;
    std::vector<int> seen(P.N, 0);
    const int T = cg::face_tiles(P);
    bool ok = true;
    for (int w = 0; w < T; ++w) {
      int tile = -1;
      for (int lane = 0; lane < 64; ++lane) {
        const int n = cg::face_node(P, (w << 6) + lane);
        if (n < 0) continue;
        if (n < 0 || n >= P.N) ok = false;
        else seen[n] += 1;
        if (tile < 0) tile = n >> 6;
        if ((n >> 6) != tile) ok = false;
      }
    }
    for (int n = 0; n < P.N; ++n) {
      const bool want = n < P.n_in || n >= P.N - P.n_out;
      if (seen[n] != (want ? 1 : 0)) ok = false;
    }
    if (!ok) {
      check(false, "face tile mapping N=" + std::to_string(P.N) + " in=" + std::to_string(P.n_in) +
                       " out=" + std::to_string(P.n_out));
      return;
    }
  }
}

}  // namespace

int main() {
  face_tile_mapping();
  Lcg r{2407};
  {
    // 3D channel with random solids, Zou-He z, walls on x and y
    const int nx = 10, ny = 9, nz = 16;
    std::vector<uint8_t> s(nx * ny * nz, 0);
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const bool wall = x == 0 || y == 0 || x == nx - 1 || y == ny - 1;
          s[x + nx * (y + ny * z)] = wall || (z >= 3 && z < nz - 3 && r.uni() < 0.25);
        }
    const uint8_t per[3] = {0, 0, 0};
    std::vector<double> th(s.size(), 0.0);
    for (size_t v = 0; v < s.size(); ++v) th[v] = s[v] ? 15.0 + 150.0 * r.uni() : 0.0;
    run("channel-zouhe-scheme1", 3, nx, ny, nz, per, 1, s, 1, nullptr, true);
    run("channel-zouhe-scheme2-field", 3, nx, ny, nz, per, 1, s, 2, th.data(), true);
    run("channel-zouhe-fictitious", 3, nx, ny, nz, per, 1, s, 3, th.data(), true);
    const uint8_t perz[3] = {0, 0, 1};
    run("channel-periodic-z", 3, nx, ny, nz, perz, 0, s, 1, nullptr, true);
    // a fluid voxel on a wall face is refused
    std::vector<uint8_t> bad = s;
    bad[5 + nx * (0 + ny * 5)] = 0;
    run("fluid-on-wall", 3, nx, ny, nz, per, 1, bad, 1, nullptr, false);
  }
  {
    // fully periodic box with a few solid grains
    const int n = 12;
    std::vector<uint8_t> s(n * n * n, 0);
    for (size_t v = 0; v < s.size(); ++v) s[v] = r.uni() < 0.1;
    const uint8_t per[3] = {1, 1, 1};
    run("periodic-grains", 3, n, n, n, per, 0, s, 2, nullptr, true);
    std::vector<uint8_t> none(n * n * n, 0);
    run("periodic-empty", 3, n, n, n, per, 0, none, 0, nullptr, true);
    std::vector<uint8_t> all(n * n * n, 1);
    run("all-solid", 3, n, n, n, per, 0, all, 0, nullptr, false);
  }
  {
    // 2D strip between walls, periodic x
    const int nx = 30, ny = 12;
    std::vector<uint8_t> s(nx * ny, 0);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) s[x + nx * y] = y == 0 || y == ny - 1 || (y == 1 && x % 7 == 3);
    const uint8_t per[3] = {1, 0, 0};
    run("strip-2d", 2, nx, ny, 1, per, 0, s, 1, nullptr, true);
  }
  if (g_fail) {
    std::printf("setup driver: %d checks failed\n", g_fail);
    return 1;
  }
  std::printf("setup driver: all checks passed\n");
  return 0;
}
