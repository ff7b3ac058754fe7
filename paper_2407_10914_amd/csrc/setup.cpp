// Once-per-run host setup in FP64 (see setup.hpp).  Built without fused
// multiply-add so that the smoothed image and the wall normal are the exact
// IEEE results of the sums as written.
#include "setup.hpp"

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <thread>

#include "step.hpp"

namespace cg {
namespace {

struct Box {
  int dim, Q, nx, ny, nz;
  int per[3];
  bool open_z;
  int e(int i, int a) const { return dim == 3 ? Lat<3>::e(i, a) : Lat<2>::e(i, a); }
  double w(int i) const { return dim == 3 ? Lat<3>::w(i) : Lat<2>::w(i); }
  int opposite(int i) const { return dim == 3 ? opp<3>(i) : opp<2>(i); }
  int idx(int x, int y, int z) const { return x + nx * (y + ny * z); }
  void xyz(int v, int* c) const {
    c[0] = v % nx;
    c[1] = (v / nx) % ny;
    c[2] = v / (nx * ny);
  }
  // x + e_i along the lattice link: index, -1 past a wall face, -2 past an open face
  int link(int v, int i) const {
    int c[3];
    xyz(v, c);
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      c[a] += e(i, a);
      if (c[a] < 0 || c[a] >= n[a]) {
        if (per[a])
          c[a] = (c[a] + n[a]) % n[a];
        else if (a == 2 && open_z)
          return -2;
        else
          return -1;
      }
    }
    return idx(c[0], c[1], c[2]);
  }
  // image value with periodic wrap, zero-gradient extension past the open
  // faces and solid (0) past a wall face
  double img(const std::vector<double>& g, int x, int y, int z) const {
    int c[3] = {x, y, z};
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      if (c[a] < 0 || c[a] >= n[a]) {
        if (per[a])
          c[a] = (c[a] + n[a]) % n[a];
        else if (a == 2 && open_z)
          c[a] = c[a] < 0 ? 0 : n[a] - 1;
        else
          return 0.0;
      }
    }
    return g[idx(c[0], c[1], c[2])];
  }
};

// Eq. (25): 27-point (2D: 9-point) weighted sum over the neighbourhood,
// visited k (z) outermost and i (x) innermost.
void smooth_pass(const Box& b, const std::vector<double>& g, std::vector<double>& h) {
  const int kz0 = b.dim == 3 ? -1 : 0, kz1 = b.dim == 3 ? 1 : 0;
  auto work = [&](int z0, int z1) {
    for (int z = z0; z < z1; ++z)
      for (int y = 0; y < b.ny; ++y)
        for (int x = 0; x < b.nx; ++x) {
          double s = 0.0;
          for (int k = kz0; k <= kz1; ++k)
            for (int j = -1; j <= 1; ++j)
              for (int i = -1; i <= 1; ++i) {
                const int r2 = i * i + j * j + k * k;
                double ws;
                if (b.dim == 3)
                  ws = r2 == 0 ? 8.0 / 27.0 : (r2 == 1 ? 2.0 / 27.0 : (r2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
                else
                  ws = r2 == 0 ? 4.0 / 9.0 : (r2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
                s += ws * b.img(g, x + i, y + j, z + k);
              }
          h[b.idx(x, y, z)] = s;
        }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, (unsigned)b.nz);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    const int z0 = (int)((long)b.nz * t / nt), z1 = (int)((long)b.nz * (t + 1) / nt);
    th.emplace_back(work, z0, z1);
  }
  for (auto& t : th) t.join();
}

}  // namespace

int build_setup(const cg_geometry& g, const cg_wetting& wet, const cg_bc& bc, HostSetup* out, std::string* err,
                int pull_table) {
  HostSetup& S = *out;
  Box b;
  b.dim = g.dim;
  if (g.dim != 2 && g.dim != 3) {
    *err = "dim must be 2 or 3";
    return CG_EINVAL;
  }
  b.Q = g.dim == 3 ? 19 : 9;
  b.nx = g.nx;
  b.ny = g.ny;
  b.nz = g.nz;
  for (int a = 0; a < 3; ++a) b.per[a] = g.periodic[a] ? 1 : 0;
  b.open_z = bc.type == CG_BC_ZOUHE;
  if (b.nx < 1 || b.ny < 1 || b.nz < 1) {
    *err = "extents must be positive";
    return CG_EINVAL;
  }
  if (g.dim == 2 && b.nz != 1) {
    *err = "dim 2 needs nz == 1";
    return CG_EINVAL;
  }
  const long Vl = (long)b.nx * b.ny * b.nz;
  if (Vl > (long)kVoxMask + 1) {
    *err = "more than 2^27 voxels: the per-node word holds a 27-bit voxel index";
    return CG_EUNSUPPORTED;
  }
  if (b.open_z && (g.dim != 3 || b.per[2] || b.nz < 3)) {
    *err = "Zou-He faces need D3Q19, a non-periodic z axis and nz >= 3";
    return g.dim != 3 ? CG_EUNSUPPORTED : CG_EINVAL;
  }
  const int V = (int)Vl;
  const uint8_t* solid = g.solid;
  auto fluid = [&](int v) { return solid[v] == 0; };
  int N = 0;
  for (int v = 0; v < V; ++v) N += fluid(v);
  if (N == 0) {
    *err = "no fluid voxel";
    return CG_EINVAL;
  }
  for (int v = 0; v < V; ++v) {
    if (!fluid(v)) continue;
    int c[3];
    b.xyz(v, c);
    const int n[3] = {b.nx, b.ny, b.nz};
    for (int a = 0; a < g.dim; ++a) {
      if (b.per[a] || (a == 2 && b.open_z)) continue;
      if (c[a] == 0 || c[a] == n[a] - 1) {
        *err = "fluid voxel on a face that is neither periodic nor open";
        return CG_EINVAL;
      }
    }
    if (b.open_z && c[2] == b.nz - 1 && !fluid(b.idx(c[0], c[1], b.nz - 2))) {
      *err = "outlet fluid voxel without a fluid voxel upstream";
      return CG_EINVAL;
    }
  }
  const int Q = b.Q;
  S.dim = g.dim;
  S.Q = Q;
  S.nx = b.nx;
  S.ny = b.ny;
  S.nz = b.nz;
  S.V = V;
  for (int a = 0; a < 3; ++a) S.per[a] = b.per[a];
  S.bc = bc.type;
  S.N = N;
  S.Np = (N + 255) / 256 * 256;
  if ((long)S.Np * Q >= (1L << 31)) {
    *err = "fluid node count too large for 32-bit indexing";
    return CG_EUNSUPPORTED;
  }
  const int Np = S.Np;

  // sparse index in lexicographic voxel order
  std::vector<int> vox_node(V, -1);
  S.node_vox.resize(N);
  {
    int k = 0;
    for (int v = 0; v < V; ++v)
      if (fluid(v)) {
        vox_node[v] = k;
        S.node_vox[k++] = v;
      }
  }

  // boundary sets along lattice links
  std::vector<uint8_t> is_fb(V, 0);
  for (int v = 0; v < V; ++v) {
    bool sb = false;
    unsigned mask = 0;
    for (int i = 1; i < Q; ++i) {
      const int y = b.link(v, i);
      if (y < 0) continue;
      if (fluid(v) && !fluid(y)) is_fb[v] = 1;
      if (!fluid(v) && fluid(y)) {
        sb = true;
        mask |= 1u << i;
      }
    }
    if (sb) {
      // bit 0: the voxel lies on a domain face (its stencil needs wrap/clamp)
      int c[3];
      b.xyz(v, c);
      if (c[0] == 0 || c[0] == b.nx - 1 || c[1] == 0 || c[1] == b.ny - 1 ||
          (g.dim == 3 && (c[2] == 0 || c[2] == b.nz - 1)))
        mask |= 1u;
      S.sb_vox.push_back(v);
      S.sb_mask.push_back(mask);
    }
  }

  // smoothed image, three passes of Eq. (25) on g = 1 (fluid) / 0 (solid)
  std::vector<double> gi(V), h(V);
  for (int v = 0; v < V; ++v) gi[v] = fluid(v) ? 1.0 : 0.0;
  for (int it = 0; it < 3; ++it) {
    smooth_pass(b, gi, h);
    gi.swap(h);
  }
  S.g3 = gi;

  // contact angle per fluid boundary point
  const bool field = wet.theta_field_deg != nullptr;

  S.nbr.assign((size_t)(Q - 1) * Np, kBounce);
  S.flags.assign(Np, 0u);
  S.nw.assign((size_t)3 * Np, 0.0);
  S.cos_t.assign(Np, 0.0);
  S.sin_t.assign(Np, 0.0);
  S.n_fb = S.n_in = S.n_out = 0;
  for (int n = 0; n < N; ++n) {
    const int v = S.node_vox[n];
    int c[3];
    b.xyz(v, c);
    unsigned fl = 0;
    if (c[0] == 0 || c[0] == b.nx - 1 || c[1] == 0 || c[1] == b.ny - 1 ||
        (g.dim == 3 && (c[2] == 0 || c[2] == b.nz - 1)))
      fl |= FL_FACE;
    if (b.open_z && c[2] == 0) {
      fl |= FL_IN;
      S.n_in++;
    }
    if (b.open_z && c[2] == b.nz - 1) {
      fl |= FL_OUT;
      S.n_out++;
    }
    // pull sources: x - e_i
    for (int i = 1; i < Q; ++i) {
      const int s = b.link(v, b.opposite(i));
      int code;
      if (s >= 0 && fluid(s))
        code = vox_node[s];
      else if (s == -2)
        code = kOpen;
      else
        code = kBounce;
      S.nbr[(size_t)(i - 1) * Np + n] = code;
    }
    if (is_fb[v]) {
      S.n_fb++;
      // Eq. (26): isotropic gradient of the smoothed image, normalised
      double gr[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < g.dim; ++a) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i)
          s += b.w(i) * (double)b.e(i, a) * b.img(gi, c[0] + b.e(i, 0), c[1] + b.e(i, 1), c[2] + b.e(i, 2));
        gr[a] = 3.0 * s;
      }
      double m = 0.0;
      for (int a = 0; a < g.dim; ++a) m += gr[a] * gr[a];
      m = std::sqrt(m);
      if (m > 1e-12) {
        fl |= FL_WET;
        for (int a = 0; a < g.dim; ++a) S.nw[(size_t)a * Np + n] = gr[a] / m;
      }
      S.fb_node.push_back(n);
      S.fb_off.push_back((int)S.fb_vox.size());
      for (int i = 1; i < Q; ++i) {
        const int y = b.link(v, i);
        if (y < 0 || fluid(y)) continue;
        S.fb_vox.push_back(y);
        S.fb_w.push_back(b.w(i));
      }
    }
    S.flags[n] = fl;
  }
  S.fb_off.push_back((int)S.fb_vox.size());
  S.s1_line = wet.scheme1_line;

  // 16-bit pull table: per (direction, tile of 256 nodes) the smallest offset
  // s - n of a fluid source, per node the remainder
  S.ntiles = Np >> kTileShift;
  S.nbr16.assign((size_t)(Q - 1) * Np, (int16_t)kD16Bounce);
  S.nbr_base.assign((size_t)(Q - 1) * S.ntiles, 0);
  bool fits = pull_table != 32;
  for (int i = 1; i < Q && fits; ++i) {
    for (int t = 0; t < S.ntiles && fits; ++t) {
      const int n0 = t << kTileShift, n1 = std::min(N, (t + 1) << kTileShift);
      long lo = 0;
      bool any = false;
      for (int n = n0; n < n1; ++n) {
        const int c = S.nbr[(size_t)(i - 1) * Np + n];
        if (c >= 0) {
          lo = any ? std::min(lo, (long)c - n) : (long)c - n;
          any = true;
        }
      }
      S.nbr_base[(size_t)(i - 1) * S.ntiles + t] = (int)lo;
      for (int n = n0; n < n1; ++n) {
        const int c = S.nbr[(size_t)(i - 1) * Np + n];
        int16_t dd;
        if (c >= 0) {
          const long r = (long)c - n - lo;
          if (r > kD16Max) {
            fits = false;
            break;
          }
          dd = (int16_t)r;
        } else {
          dd = (int16_t)(c == kOpen ? kD16Open : kD16Bounce);
        }
        S.nbr16[nbr16_index(Q - 1, i, n)] = dd;
      }
    }
  }
  if (!fits) {
    S.nbr16.clear();
    S.nbr_base.clear();
  }

  // 8-bit pull table: per wave of 64 nodes and direction the smallest offset
  // s - n of a fluid source, per node the remainder in 0..252 (253: the wave
  // did not fit and reads the 16/32-bit table, 254 bounce-back, 255 open
  // face).  Every entry of a fitting wave is decoded here and checked against
  // the plain table; any mismatch drops the 8-bit table altogether.
  if (pull_table == 0 || pull_table == 8) {
    const int qm1 = Q - 1, W8 = (qm1 + 3) / 4, nt64 = Np / 64;
    S.nbr8.assign((size_t)nt64 * W8 * 64, 0xFDFDFDFDu);
    S.nbr8_head.assign((size_t)nt64 * qm1, 0);
    bool good = true;
    long fitting = 0;
    for (int t = 0; t < nt64 && good; ++t) {
      const int n0 = t * 64, n1 = std::min(N, n0 + 64);
      int* head = &S.nbr8_head[(size_t)t * qm1];
      bool ok = true;
      for (int i = 1; i < Q && ok; ++i) {
        long lo = 0, hi = 0;
        bool any = false;
        for (int n = n0; n < n1; ++n) {
          const int c = S.nbr[(size_t)(i - 1) * Np + n];
          if (c < 0) continue;
          const long d = (long)c - n;
          lo = any ? std::min(lo, d) : d;
          hi = any ? std::max(hi, d) : d;
          any = true;
        }
        if (any && hi - lo > 252) ok = false;
        head[i - 1] = (int)lo;
      }
      if (!ok) {
        for (int i = 0; i < qm1; ++i) head[i] = 0;
        continue;  // bytes stay 253: the whole wave takes the 16/32-bit table
      }
      ++fitting;
      for (int i = 1; i < Q; ++i) {
        for (int n = n0; n < n0 + 64; ++n) {
          const int c = n < n1 ? S.nbr[(size_t)(i - 1) * Np + n] : kBounce;
          const uint32_t byte = c >= 0 ? (uint32_t)((long)c - n - head[i - 1]) : (c == kOpen ? 255u : 254u);
          uint32_t& w = S.nbr8[((size_t)t * W8 + (size_t)((i - 1) >> 2)) * 64 + (size_t)(n & 63)];
          const int sh = 8 * ((i - 1) & 3);
          w = (w & ~(0xFFu << sh)) | (byte << sh);
        }
      }
      for (int i = 1; i < Q && good; ++i) {
        for (int n = n0; n < n1; ++n) {
          const uint32_t w = S.nbr8[((size_t)t * W8 + (size_t)((i - 1) >> 2)) * 64 + (size_t)(n & 63)];
          const int byte = (int)((w >> (8 * ((i - 1) & 3))) & 0xFFu);
          const long dec = byte < 253 ? (long)n + head[i - 1] + byte : (byte == 254 ? kBounce : (byte == 255 ? kOpen : -9));
          if (dec != S.nbr[(size_t)(i - 1) * Np + n] || dec >= N) {
            good = false;
            break;
          }
        }
      }
    }
    if (!good || fitting == 0) {
      S.nbr8.clear();
      S.nbr8_head.clear();
      fitting = 0;
    }
    S.n8_waves = fitting;
  }

  S.sb_fd.assign(S.sb_vox.size(), 0.0);
  return contact_angles(S, wet.theta_deg, field ? wet.theta_field_deg : nullptr, &S.cos_t, &S.sin_t, &S.flags,
                        &S.sb_fd, err);
}

int contact_angles(const HostSetup& S, double theta_deg, const double* theta_field_deg, std::vector<double>* cos_t,
                   std::vector<double>* sin_t, std::vector<unsigned>* flags, std::vector<double>* sb_fd,
                   std::string* err) {
  const size_t np = (size_t)S.Np;
  if (!cos_t || !sin_t || !flags || !sb_fd || cos_t->size() != np || sin_t->size() != np || flags->size() != np ||
      sb_fd->size() != S.sb_vox.size()) {
    *err = "contact_angles: output arrays must hold one entry per padded node (and per solid boundary point)";
    return CG_EINVAL;
  }
  const double deg = M_PI / 180.0;
  // Eq. (24) with the angle measured through fluid b: the fixed phase of a
  // solid boundary point is cos(180 deg - theta) = -cos(theta)
  for (size_t k = 0; k < S.sb_vox.size(); ++k) {
    const double th = theta_field_deg ? theta_field_deg[S.sb_vox[k]] : theta_deg;
    (*sb_fd)[k] = -std::cos(th * deg);
  }
  for (size_t k = 0; k < S.fb_node.size(); ++k) {
    const int n = S.fb_node[k];
    double th;
    if (!theta_field_deg) {
      th = theta_deg;
    } else {
      double num = 0.0, den = 0.0;
      for (int l = S.fb_off[k]; l < S.fb_off[k + 1]; ++l) {
        const double t = theta_field_deg[S.fb_vox[l]];
        if (!(t > 0.0 && t < 180.0)) {
          *err = "theta field must lie in (0, 180) degrees on solid voxels";
          return CG_EINVAL;
        }
        num += S.fb_w[l] * t;
        den += S.fb_w[l];
      }
      th = num / den;
    }
    // one libm call for both (GNU sincos, the routine compilers also emit
    // for a cos/sin pair of one argument; separate cos and sin calls can
    // differ from it in the last place)
    double sn, cs;
    sincos(th * deg, &sn, &cs);
    (*cos_t)[n] = cs;
    (*sin_t)[n] = sn;
    unsigned& fl = (*flags)[n];
    fl &= ~FL_S1POS;
    if (S.s1_line == CG_S1_LITERAL || th > 90.0) fl |= FL_S1POS;
  }
  return CG_OK;
}

}  // namespace cg
