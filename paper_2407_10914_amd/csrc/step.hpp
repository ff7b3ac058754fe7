// Device code of one colour-gradient time step (arXiv:2407.10914, Sec. II).
//
// One thread per fluid node.  Per step the kernels run in the order the
// method needs (the phase field of all nodes before any gradient, all normals
// before any curvature):
//   k_phase   densities and phase field, Eqs. (7)-(9), inlet phi (Sec. II.D.1)
//             and outlet phi (Eq. 39), written to a dense voxel grid;
//   k_sb_phi  phase field extrapolated to the solid boundary points, Eq. (34);
//   k_normal  colour gradient, Eq. (6), unit normal, Eq. (27), wetting
//             Scheme-I / Scheme-II at the fluid boundary points, Eqs. (28)-(33);
//   k_sb_n    normal extrapolated to the solid boundary points, Eq. (35);
//   k_main    pull streaming with halfway bounce-back, Zou-He faces
//             (Appendix B), curvature, Eq. (12), force, Eqs. (5) and (36),
//             velocity, Eq. (22), rates, Eqs. (13)-(16), BGK/MRT collision,
//             Eqs. (2)-(4) and (A.3)-(A.5), recolouring, Eqs. (20)-(21), store.
//
// Two state layouts:
//   double: canonical post-collision populations f^r', f^b' ([Q][Np] each);
//           every operation follows the order of the reference definition
//           (sums over i ascending, no fused multiply-add: the translation
//           unit is built with -ffp-contract=off).
//   float:  compact post-collision state: g''_i = f^t''_i - w_i rho0 ([Q][Np]),
//           a = rho^r/rho ([Np]) and c = beta rho^r rho^b / rho * n ([D][Np]).
//           The recoloured red population that a pull reads is rebuilt as
//           f^r_i = a (w_i rho0 + g''_i) + w_i c.e_i, which is Eq. (20); the
//           total is carried as a deviation from rest so that the momentum
//           is not lost to single-precision rounding of O(1) values.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

namespace cg {

enum : unsigned {
  FL_FACE = 1u,   // on a domain face: stencils need wrap / clamp
  FL_WET = 2u,    // fluid boundary point with a usable wall normal
  FL_IN = 4u,     // Zou-He inlet node (z = 0)
  FL_OUT = 8u,    // Zou-He outlet node (z = nz-1)
  FL_S1POS = 16u  // Scheme-I secant start uses s = +1
};
// per-node word: voxel index in the low kVoxBits bits, flags above
constexpr int kVoxBits = 27;
constexpr unsigned kVoxMask = (1u << kVoxBits) - 1u;

// number of observable accumulators (see k_main, MODE_OBS)
constexpr int kObsN = 15;

// Pull-table codes (entries >= 0 are source node indices).
constexpr int kBounce = -1;
constexpr int kOpen = -2;

struct StepParams {
  int nx, ny, nz;
  int N;     // fluid nodes
  int Np;    // stride of per-node arrays
  int nsb;   // solid boundary points
  int V;     // voxels
  int per[3];
  int bc;    // 0 none, 1 Zou-He z faces
  // Zou-He face nodes: in voxel order the inlet plane's nodes come first and
  // the outlet plane's last, so they are nodes [0, n_in) and [N - n_out, N)
  int n_in, n_out;
  int scheme;     // 0 none, 1 Scheme-I, 2 Scheme-II, 3 fictitious density (Eq. 24)
  int collision;  // 0 BGK, 1 MRT
  double half_sigma;  // 0.5 * sigma
  double beta, rho0;
  double nu_r, nu_b;  // (tau - 1/2)/3
  float hinv_nu_r, hinv_nu_b;  // 1/(2 nu_r), 1/(2 nu_b) for the single-precision rates
  double rg[3];       // rho0 * g, force density of Eq. (36)
  double rin_r, rin_b;  // rho_in * zeta^r, rho_in * zeta^b
  double rho_in, rho_out, phi_in, zeta_r;
  double eps_c, eps_f, eps_v;
  int flux_axis, flux_plane;
  // observables restricted to lo <= coordinate[slab_axis] < hi (axis < 0: all)
  int slab_axis, slab_lo, slab_hi;
};

template <class Real>
struct Vec4T;
template <>
struct Vec4T<float> {
  using type = float4;
};
template <>
struct Vec4T<double> {
  using type = double4;
};
template <class Real>
using Vec4 = typename Vec4T<Real>::type;

// Interface normal as the dense grid stores it: three components and no
// padding, so that a stencil gather of a wave touches a quarter fewer cache
// lines than with 16-byte vectors.
template <class Real>
struct Norm3 {
  Real x, y, z;
};
template <class Real>
__device__ __forceinline__ Vec4<Real> n_get(const Norm3<Real>* p, int i) {
  const Norm3<Real> t = p[i];
  Vec4<Real> o;
  o.x = t.x;
  o.y = t.y;
  o.z = t.z;
  o.w = Real(0);
  return o;
}
template <class Real>
__device__ __forceinline__ void n_put(Norm3<Real>* p, int i, const Vec4<Real>& v) {
  p[i] = Norm3<Real>{v.x, v.y, v.z};
}

// Pull table: the source node of direction i (i >= 1) of node n, or a code.
// Stored as 16-bit deltas against a per-tile base (a tile is 256 consecutive
// nodes; every wave lies inside one tile): s = n + base[i][tile] + d, with two
// reserved deltas for the bounce-back and open-face codes.  Geometries whose
// offsets do not fit use the 32-bit table instead (wide != nullptr).
constexpr int kTileShift = 8;
// the two codes decode by one add: kD16Bounce + kD16Code = kBounce,
// kD16Open + kD16Code = kOpen
constexpr int kD16Code = 32766;
constexpr int kD16Bounce = kBounce - kD16Code;  // -32767
constexpr int kD16Open = kOpen - kD16Code;      // -32768
constexpr int kD16Max = 32767;

// The deltas of the 64 nodes of one wave are stored together, two directions
// per 32-bit word ([Np/64][(Q-1)/2][64] words; direction 2k+1 in the low half,
// 2k+2 in the high half): a wave reads its whole table row with (Q-1)/2 loads
// from one contiguous block instead of Q-1 separate streams.
__host__ __device__ __forceinline__ size_t nbr16_index(int qm1, int i, int n) {
  const size_t word = ((size_t)(n >> 6) * (size_t)(qm1 / 2) + (size_t)((i - 1) >> 1)) * 64u + (size_t)(n & 63);
  return 2u * word + (size_t)((i - 1) & 1);
}

struct Nbr {
  const int16_t* d;  // [Np/64][(Q-1)/2][64][2], see nbr16_index
  const int* base;   // [Q-1][ntiles]
  const int* wide;   // [Q-1][Np] or nullptr
  int Np, ntiles, qm1;
  // 8-bit table (on the 256^3 rock 99.8 % of the waves fit): per wave of 64
  // nodes a base per direction, per node four directions to a 32-bit word,
  // the byte being s - n - base_i, or 254 (bounce-back) / 255 (open face); a
  // wave whose offsets do not fit holds 253 everywhere and reads the tables
  // above instead, as does every single entry (get).  Null when not built.
  const uint32_t* d8;  // [Np/64][(Q-1+3)/4][64]
  const int* h8;       // [Np/64][Q-1]
  // One entry (any node, any lane).
  template <int i>
  __device__ __forceinline__ int get(int n) const {
    if (wide) return wide[(i - 1) * Np + n];
    const int dd = d[nbr16_index(qm1, i, n)];
    const int b = base[(i - 1) * ntiles + (n >> kTileShift)];
    const int t = n + b + dd;
    return dd < kD16Bounce + 1 ? dd + kD16Code : t;
  }
  // All Q-1 entries of node n, src[i] for i = 1..Q-1.  Every lane of the
  // wave must ask for a node of the same tile (true for node_id() and the
  // batched tiles, which are aligned to 64 nodes): the bases are then read
  // once per wave, before any decode, and the decode is a select.
  template <int Q>
  __device__ __forceinline__ void all(int n, int* src) const {
    if (d8) {
      // words and bases are read unconditionally (no load waits on a flag),
      // the decode is a select; a wave that holds the escape byte 253 (all of
      // its bytes, set on the host) falls through to the 16/32-bit table
      const int t = __builtin_amdgcn_readfirstlane(n >> 6);
      constexpr int W8 = (Q - 1 + 3) / 4;
      uint32_t w[W8];
      unroll<W8>([&](auto K) {
        constexpr int k = K;
        w[k] = __builtin_nontemporal_load(&d8[(t * W8 + k) * 64 + (n & 63)]);
      });
      int b8[Q];
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        b8[i] = h8[t * (Q - 1) + (i - 1)];
      });
      bool esc = false;
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        const int byte = (int)((w[(i - 1) >> 2] >> (8 * ((i - 1) & 3))) & 0xFFu);
        int s = n + b8[i] + byte;
        // opaque: keeps the select from being turned into a branch with the
        // base's load inside it
        asm("" : "+v"(s));
        src[i] = byte < 253 ? s : (byte == 254 ? kBounce : kOpen);
        esc = esc || byte == 253;
      });
      if (__builtin_amdgcn_ballot_w64(esc) == 0) return;
    }
    if (wide) {
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        src[i] = wide[(i - 1) * Np + n];
      });
      return;
    }
    static_assert((Q - 1) % 2 == 0, "pull-table words hold two directions");
    const int tile = __builtin_amdgcn_readfirstlane(n >> kTileShift);
    int b[Q], dd[Q];
    const int* dw = reinterpret_cast<const int*>(d);
    unroll<(Q - 1) / 2>([&](auto K) {
      constexpr int k = K;
      const int wv = __builtin_nontemporal_load(&dw[((n >> 6) * ((Q - 1) / 2) + k) * 64 + (n & 63)]);
      dd[2 * k + 1] = (int)(int16_t)(wv & 0xffff);
      dd[2 * k + 2] = wv >> 16;
    });
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      b[i] = base[(i - 1) * ntiles + tile];
    });
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      const int t = n + b[i] + dd[i];
      src[i] = dd[i] < kD16Bounce + 1 ? dd[i] + kD16Code : t;
    });
  }
};

template <class Real>
struct Geo {
  Nbr nbr;                 // pull table
  const unsigned* vf;      // [Np] voxel index | flags << kVoxBits
  const int* sb_vox;       // [nsb]
  const unsigned* sb_mask; // [nsb] bit i: the link s + e_i ends on a fluid voxel in
                           // the domain; bit 0: the voxel lies on a domain face
  const Real* nw;          // [3][Np] wall normal (unit)
  const Real* cos_t;       // [Np]
  const Real* sin_t;       // [Np]
  const Real* sb_fd;       // [nsb] fixed phase of the fictitious-density model, Eq. (24)
};

// Storage of the phase-field grid.  Double precision stores phi itself.
// Single precision stores d = phi - 1 (phi >= 0) or d = phi + 1 (phi < 0)
// rounded to float, with the lowest mantissa bit replaced by the choice
// (1: phi < 0).  Near the bulk, where |C| is small and n = C/|C| would turn
// a rounding of phi near +-1 (6e-8 in float) into a direction error of up
// to ~1e-3 that the curvature of neighbouring interface nodes picks up, the
// stored value keeps relative precision in phi -+ 1 (at most one unit in the
// last place of d, also past +-1, where rounding can take phi).  Decoding is
// exact in double.
template <class Real>
struct PhiStore;
template <>
struct PhiStore<double> {
  using type = double;
};
template <>
struct PhiStore<float> {
  using type = float;
};
__device__ __forceinline__ double phi_dec(double s) { return s; }
__device__ __forceinline__ double phi_dec(float s) {
  return (__builtin_bit_cast(uint32_t, s) & 1u) ? (double)s - 1.0 : (double)s + 1.0;
}
template <class T>
__device__ __forceinline__ T phi_enc(double p);
template <>
__device__ __forceinline__ double phi_enc<double>(double p) {
  return p;
}
template <>
__device__ __forceinline__ float phi_enc<float>(double p) {
  const bool neg = p < 0.0;
  const float d = (float)(neg ? p + 1.0 : p - 1.0);
  return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, d) & ~1u) | (neg ? 1u : 0u));
}

template <class Real>
struct Grids {
  using PhiT = typename PhiStore<Real>::type;
  PhiT* phi;        // [V] phase field (fluid nodes and solid boundary points), see PhiStore
  Norm3<Real>* n;   // [V] interface normal after wetting, fluid and S_b
  Norm3<Real>* c;   // [Np] colour gradient after wetting
  Vec4<Real>* f;    // [Np] force (xyz) and curvature (w)
};

// ------------------------------------------------------------------- helpers

// Block index -> logical tile, so that each of the 8 XCDs (blocks are dealt
// round-robin) works on one contiguous range of nodes and keeps its stencil
// neighbours in its own L2.  With the plain mapping all XCDs work on the same
// planes and k_main's L2 fetches grow from 1.0 to 1.68 GB per launch on the
// 256^3 rock (the extra lines come from the other XCDs' working sets, which
// the memory-side cache serves, so its time barely changes).
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ int node_id() {
  return xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}
// Plain mapping, for k_normal (measured faster there: 70 -> 62 us on the
// 256^3 rock; the other step kernels were within 1 % either way) and for the
// adjoint kernels (reverse sweep 2.6 instead of 2.9 forward steps at 128^3).
__device__ __forceinline__ int node_id_plain() {
  return blockIdx.x * blockDim.x + threadIdx.x;
}

// A voxel and, when it lies on a domain face, its coordinates (decomposed once
// per node rather than once per neighbour).
struct Pos {
  int v, x, y, z;
  bool face;
};

__device__ __forceinline__ Pos make_pos(const StepParams& P, int v, bool face) {
  Pos p{v, 0, 0, 0, face};
  if (face) {
    const int nxy = P.nx * P.ny;
    p.z = v / nxy;
    const int r = v - p.z * nxy;
    p.y = r / P.nx;
    p.x = r - p.y * P.nx;
  }
  return p;
}

// Neighbour voxels for the gradient stencils: periodic axes wrap, other axes
// clamp (zero-gradient ghosts beyond the open faces; fluid nodes never reach
// past a wall face).  Branch-free: the wrapped/clamped index is formed for
// every node (from the zero coordinates of an interior node it is simply
// unused) and selected.
__device__ __forceinline__ int wrap_or_clamp(int x, int n, bool per) {
  const int w = x + (x < 0 ? n : 0) - (x >= n ? n : 0);
  const int c = min(max(x, 0), n - 1);
  return per ? w : c;
}

template <int D, int i>
__device__ __forceinline__ int nb_vox(const StepParams& P, const Pos& p) {
  constexpr int ex = Lat<D>::e(i, 0), ey = Lat<D>::e(i, 1), ez = Lat<D>::e(i, 2);
  const int fast = p.v + ex + P.nx * (ey + P.ny * ez);
  int x = p.x + ex, y = p.y + ey, z = p.z + ez;
  if constexpr (ex != 0) x = wrap_or_clamp(x, P.nx, P.per[0] != 0);
  if constexpr (ey != 0) y = wrap_or_clamp(y, P.ny, P.per[1] != 0);
  if constexpr (ez != 0) z = wrap_or_clamp(z, P.nz, P.per[2] != 0);
  const int slow = x + P.nx * (y + P.ny * z);
  return p.face ? slow : fast;
}

// Neighbour voxels of p along every direction, idx[i] for i = 1..Q-1.  A wave
// with no face node (almost all of them) takes a constant offset per direction
// (a uniform branch); otherwise nb_vox's wrap/clamp path serves every lane.
template <int D>
__device__ __forceinline__ void nb_all(const StepParams& P, const Pos& p, int* idx) {
  constexpr int Q = Lat<D>::Q;
  if (__builtin_amdgcn_ballot_w64(p.face) == 0) {
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      constexpr int ex = Lat<D>::e(i, 0), ey = Lat<D>::e(i, 1), ez = Lat<D>::e(i, 2);
      idx[i] = p.v + (ex + P.nx * (ey + P.ny * ez));
    });
  } else {
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      idx[i] = nb_vox<D, i>(P, p);
    });
  }
}

template <class Real, int D>
__device__ __forceinline__ Real dotv(const Real* a, const Real* b) {
  Real s = a[0] * b[0];
  s = s + a[1] * b[1];
  if constexpr (D == 3) s = s + a[2] * b[2];
  return s;
}

// ------------------------------------------------------------ state layouts

// Canonical post-collision populations (double path).
template <class Real, int D>
struct InCanon {
  static constexpr bool kPull = true;
  const Real* fr;
  const Real* fb;
  int Np;
  template <int i, class CT>
  __device__ __forceinline__ void get(int s, CT& r, CT& x) const {
    r = (CT)fr[i * Np + s];
    x = (CT)fb[i * Np + s];
  }
  // pulled direction i >= 1 of node n with pull-table entry s (see load_node)
  template <int i, class CT>
  __device__ __forceinline__ void get_pull(int s, int n, CT& r, CT& x) const {
    constexpr int o = opp<D>(i);
    const int idx = s >= 0 ? i * Np + s : o * Np + n;
    const CT a = (CT)fr[idx], b = (CT)fb[idx];
    const bool open = s < kBounce;
    r = open ? CT(0) : a;
    x = open ? CT(0) : b;
  }
};

// Compact post-collision state (float path); x = g = f^t - w rho0.
// AC[s] = (a, c_x, c_y, c_z) with a = rho^r/rho and c = beta rho^r rho^b/rho n.
template <int D>
struct InCompact {
  static constexpr bool kPull = true;
  static constexpr bool kSplitRest = true;
  const float* T;
  const float4* AC;
  int Np;
  float rho0;
  // Written by the phase stage, read by the step kernel of the same step:
  // RS[n] = red density pulled into node n, summed in double (after the
  // Zou-He faces at face nodes); FS[q * (n_in + n_out) + k] = the five
  // unknown totals g the faces set at face node k (inlet nodes first).  The
  // step kernel then needs no source's (a, c) record.
  double* RS;
  float* FS;
  // The rest population of node n (get<0>) split into its two loads and its
  // arithmetic, so that load_node can issue the loads ahead of the pull table.
  struct Rest {
    float t, a;
  };
  __device__ __forceinline__ Rest load_rest(int n) const { return Rest{T[n], AC[n].x}; }
  template <class CT>
  __device__ __forceinline__ void finish_rest(const Rest& q, CT& r, CT& x) const {
    const CT t = (CT)q.t;
    r = (CT)q.a * ((CT)Lat<D>::w(0) * (CT)rho0 + t);
    x = t;
  }
  template <int i, class CT>
  __device__ __forceinline__ void get(int s, CT& r, CT& x) const {
    constexpr double w = Lat<D>::w(i);
    const CT t = (CT)T[i * Np + s];
    const float4 ac = AC[s];
    CT r0 = (CT)ac.x * ((CT)w * (CT)rho0 + t);
    if constexpr (i != 0) {
      const CT cc[3] = {(CT)ac.y, (CT)ac.z, (CT)ac.w};
      CT ce = CT(0);
      unroll<D>([&](auto A_) {
        constexpr int d = A_;
        constexpr int e = Lat<D>::e(i, d);
        if constexpr (e == 1) ce = ce + cc[d];
        if constexpr (e == -1) ce = ce - cc[d];
      });
      r0 = r0 + (CT)w * ce;
    }
    r = r0;
    x = t;
  }
  // pulled direction i >= 1 of node n with pull-table entry s (see load_node):
  // the same value as get<i>(s) from a fluid source, get<opp(i)>(n) for a
  // bounce-back link (the rebuilt red term changes sign with e), 0 for an open
  // face, without a branch.  load_pull issues the two loads, finish_pull does
  // the arithmetic; get_pull is both.
  struct Raw {
    float t;
    float4 ac;
  };
  template <int i>
  __device__ __forceinline__ Raw load_pull(int s, int n) const {
    constexpr int o = opp<D>(i);
    const bool fl = s >= 0;
    int node = fl ? s : n;
    int row = fl ? i * Np : o * Np;
    // opaque to the optimiser: otherwise it turns the selects into branches
    // (reusing the node's own (a, c) on bounce-back lanes) that wait for
    // earlier loads before issuing the remaining gathers
    asm("" : "+v"(node), "+v"(row));
    return Raw{T[row + node], AC[node]};
  }
  template <int i, class CT>
  __device__ __forceinline__ void finish_pull(const Raw& q, int s, CT& r, CT& x) const {
    constexpr double w = Lat<D>::w(i);
    const bool fl = s >= 0;
    const CT t = (CT)q.t;
    const float4 ac = q.ac;
    // every component of c enters, the ones along which e_i is 0 with a zero
    // factor (which cannot be folded away): the record is then read by one
    // 16-byte load instead of two or three narrower ones, which keeps the
    // loads of a node within the hardware's count of loads in flight
    CT ce = (CT)(float)Lat<D>::e(i, 0) * (CT)ac.y + (CT)(float)Lat<D>::e(i, 1) * (CT)ac.z;
    if constexpr (D == 3) ce = ce + (CT)(float)Lat<D>::e(i, 2) * (CT)ac.w;
    const CT r0 = (CT)ac.x * ((CT)w * (CT)rho0 + t) + (CT)w * (fl ? ce : -ce);
    const bool open = s < kBounce;
    r = open ? CT(0) : r0;
    x = open ? CT(0) : t;
  }
  template <int i, class CT>
  __device__ __forceinline__ void get_pull(int s, int n, CT& r, CT& x) const {
    finish_pull<i>(load_pull<i>(s, n), s, r, x);
  }
  // the total alone (g of direction i as pulled; 0 on an open face)
  template <int i>
  __device__ __forceinline__ float load_pull_t(int s, int n) const {
    constexpr int o = opp<D>(i);
    const bool fl = s >= 0;
    int node = fl ? s : n;
    int row = fl ? i * Np : o * Np;
    asm("" : "+v"(node), "+v"(row));
    return T[row + node];
  }
};

// Leading components of a node's (a, c) record that direction i uses: a and
// c up to the last axis along which e_i is not zero (one load per
// direction, narrower where it can be).
template <int D, int i>
constexpr int ac_width() {
  return Lat<D>::e(i, 2) != 0 ? 4 : (Lat<D>::e(i, 1) != 0 ? 3 : (Lat<D>::e(i, 0) != 0 ? 2 : 1));
}
template <int W>
struct ACw;
template <>
struct alignas(8) ACw<2> {
  float a, c0;
};
template <>
struct ACw<3> {
  float a, c0, c1;
};
template <>
struct alignas(16) ACw<4> {
  float a, c0, c1, c2;
};

// Red and total density pulled into node n of the compact state, summed in
// double over i ascending as they are rebuilt (the rest population first):
// the same values and the same order of additions as rebuilding every pulled
// population with InCompact::finish_pull in double and summing afterwards,
// without keeping the rebuilt populations.  The loads are issued as in
// load_node; each direction reads only the components of (a, c) it uses.
template <int D>
__device__ __forceinline__ void pull_sums_compact(const InCompact<D>& in, const Nbr& nbr, int n, double rho0,
                                                  double& red, double& tot) {
  constexpr int Q = Lat<D>::Q;
  const float t0 = in.T[n];
  const float a0 = in.AC[n].x;
  __builtin_amdgcn_sched_barrier(0);
  int src[Q];
  nbr.template all<Q>(n, src);
  float tr[Q];
  float ra[Q], rc0[Q], rc1[Q], rc2[Q];
  // per direction, bit i: the source is a fluid node (else bounce-back from
  // the node itself), and the link crosses an open face (a zero); the table
  // entries themselves are not needed once the loads are issued
  uint32_t fluid_bits = 0u, open_bits = 0u;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    constexpr int o = opp<D>(i);
    constexpr int W = ac_width<D, i>();
    const bool fl = src[i] >= 0;
    fluid_bits |= fl ? (1u << i) : 0u;
    open_bits |= src[i] < kBounce ? (1u << i) : 0u;
    int node = fl ? src[i] : n;
    int row = fl ? i * in.Np : o * in.Np;
    asm("" : "+v"(node), "+v"(row));
    tr[i] = in.T[row + node];
    const ACw<W> q = *reinterpret_cast<const ACw<W>*>(&in.AC[node]);
    ra[i] = q.a;
    rc0[i] = q.c0;
    if constexpr (W >= 3) rc1[i] = q.c1;
    if constexpr (W >= 4) rc2[i] = q.c2;
  });
  __builtin_amdgcn_sched_barrier(0);
  const double w0 = Lat<D>::w(0);
  double r = (double)a0 * (w0 * (double)in.rho0 + (double)t0);
  double t = w0 * rho0 + (double)t0;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    constexpr int W = ac_width<D, i>();
    constexpr double w = Lat<D>::w(i);
    const bool fl = fluid_bits & (1u << i);
    const double g = (double)tr[i];
    double ce = (double)(float)Lat<D>::e(i, 0) * (double)rc0[i];
    if constexpr (W >= 3) ce = ce + (double)(float)Lat<D>::e(i, 1) * (double)rc1[i];
    if constexpr (W >= 4) ce = ce + (double)(float)Lat<D>::e(i, 2) * (double)rc2[i];
    const double r0 = (double)ra[i] * (w * (double)in.rho0 + g) + w * (fl ? ce : -ce);
    const bool open = open_bits & (1u << i);
    r = r + (open ? 0.0 : r0);
    t = t + (w * rho0 + (open ? 0.0 : g));
  });
  red = r;
  tot = t;
}

// Unknown directions of the inlet and of the outlet (Eqs. B.1-B.18): the
// populations that enter the domain through the face.
constexpr int kZhIn[5] = {5, 11, 12, 15, 16};
constexpr int kZhOut[5] = {6, 13, 14, 17, 18};

// Index of a Zou-He face node among the face nodes (inlet ones first).
__device__ __forceinline__ int face_slot(const StepParams& P, unsigned fl, int n) {
  return (fl & FL_IN) ? n : P.n_in + (n - (P.N - P.n_out));
}

// Pulled totals g_i of node n of the compact state (the step kernel's pull:
// no red share).  Same order of loads as load_node.
template <int D>
__device__ __forceinline__ void load_node_t(const InCompact<D>& in, const Nbr& nbr, int n, float* fx) {
  constexpr int Q = Lat<D>::Q;
  const float t0 = in.T[n];
  __builtin_amdgcn_sched_barrier(0);
  int src[Q];
  nbr.template all<Q>(n, src);
  float raw[Q];
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    raw[i] = in.template load_pull_t<i>(src[i], n);
  });
  __builtin_amdgcn_sched_barrier(0);
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    fx[i] = src[i] < kBounce ? 0.f : raw[i];
  });
  fx[0] = t0;
}

// Pre-collision populations stored at their own node (first step after the
// state was set from the host).
template <class Real, int D>
struct InPre {
  static constexpr bool kPull = false;
  const Real* r_;
  const Real* x_;
  int Np;
  template <int i, class CT>
  __device__ __forceinline__ void get(int s, CT& r, CT& x) const {
    r = (CT)r_[i * Np + s];
    x = (CT)x_[i * Np + s];
  }
};

template <class Real, int D>
struct OutCanon {
  Real* fr;
  Real* fb;
  int Np;
};

template <int D>
struct OutCompact {
  float* T;
  float4* AC;
  int Np;
};

template <class In>
constexpr auto requires_split_rest(int) -> decltype(In::kSplitRest, bool()) {
  return true;
}
template <class In>
constexpr bool requires_split_rest(long) {
  return false;
}
template <class In>
constexpr bool split_rest() {
  if constexpr (requires_split_rest<In>(0)) return In::kSplitRest;
  return false;
}

// Gather the pre-collision populations of node n (pull streaming with halfway
// bounce-back: f_i(x) = f'_i(x - e_i) from a fluid source, f'_opp(i)(x) when
// the source is solid; open-face unknowns are left 0 for the Zou-He step).
// The pulled loads carry no branch, so all of them are issued back to back.
template <int D, class In, class CT>
__device__ __forceinline__ void load_node(const In& in, const Nbr& nbr, int n, CT* fr, CT* fx) {
  constexpr int Q = Lat<D>::Q;
  if constexpr (In::kPull) {
    int src[Q];
    if constexpr (split_rest<In>()) {
      // the rest population's loads first, kept there by a scheduling
      // barrier (otherwise they sink below the gathers and add a round trip)
      const auto q = in.load_rest(n);
      __builtin_amdgcn_sched_barrier(0);
      nbr.template all<Q>(n, src);
      // all gathers issued before any is used (a use in between waits for
      // every older load, which splits the gather into several round trips)
      typename In::Raw raw[Q];
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        raw[i] = in.template load_pull<i>(src[i], n);
      });
      __builtin_amdgcn_sched_barrier(0);
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        in.template finish_pull<i>(raw[i], src[i], fr[i], fx[i]);
      });
      in.finish_rest(q, fr[0], fx[0]);
    } else {
      nbr.template all<Q>(n, src);
      in.template get<0>(n, fr[0], fx[0]);
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        in.template get_pull<i>(src[i], n, fr[i], fx[i]);
      });
    }
  } else {
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      in.template get<i>(n, fr[i], fx[i]);
    });
  }
}

// Populations of the node upstream of outlet node n (z = nz-2), entry by
// entry (that node may lie in another tile than the wave's other nodes):
// pulled for a post-streaming state, its own for a state set at the nodes.
template <int D, class In, class CT>
__device__ __forceinline__ void load_outlet_upstream(const In& in, const Nbr& nbr, int n, CT* fr, CT* fx) {
  constexpr int Q = Lat<D>::Q;
  if constexpr (D == 3) {
    const int u = nbr.template get<kDirZp>(n);
    if constexpr (In::kPull) {
      in.template get<0>(u, fr[0], fx[0]);
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        in.template get_pull<i>(nbr.template get<i>(u), u, fr[i], fx[i]);
      });
    } else {
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        in.template get<i>(u, fr[i], fx[i]);
      });
    }
  } else {
    load_node<D>(in, nbr, n, fr, fx);
  }
}

// -------------------------------------------------------------- Zou-He faces

// Inlet, one colour (or the total deviation), Eqs. (B.1)-(B.8).
template <class CT>
__device__ __forceinline__ void zh_in(CT* f, CT rho_s) {
  CT S = f[0] + f[1] + f[2] + f[3] + f[4] + f[7] + f[8] + f[9] + f[10];
  CT T = f[6] + f[13] + f[14] + f[17] + f[18];
  CT j = rho_s - (S + CT(2) * T);
  CT Nx = CT(0.5) * ((f[1] + f[7] + f[9]) - (f[2] + f[8] + f[10]));
  CT Ny = CT(0.5) * ((f[3] + f[7] + f[8]) - (f[4] + f[9] + f[10]));
  f[5] = f[6] + j / CT(3);
  f[11] = f[14] + j / CT(6) - Nx;
  f[12] = f[13] + j / CT(6) + Nx;
  f[15] = f[18] + j / CT(6) - Ny;
  f[16] = f[17] + j / CT(6) + Ny;
}

// Outlet unknowns for one colour given jc = jt * chi^s, Eqs. (B.10)-(B.18).
template <class CT>
__device__ __forceinline__ void zh_out_color(CT* f, CT jc) {
  CT Nx = CT(0.5) * ((f[1] + f[7] + f[9]) - (f[2] + f[8] + f[10]));
  CT Ny = CT(0.5) * ((f[3] + f[7] + f[8]) - (f[4] + f[9] + f[10]));
  f[6] = f[5] - jc / CT(3);
  f[13] = f[12] - jc / CT(6) - Nx;
  f[14] = f[11] - jc / CT(6) + Nx;
  f[17] = f[16] - jc / CT(6) - Ny;
  f[18] = f[15] - jc / CT(6) + Ny;
}

// Apply the faces to node populations.  Canonical layout: x = f^b, per-colour
// inlet and chi-weighted outlet exactly as written.  Deviation layout
// (x = f^t - w rho0): the red colour as written, the total with the deviation
// densities (the weights of the known directions sum to 1 for both faces).
// Both faces are evaluated on copies and merged by value selects: the inlet
// sets directions {5, 11, 12, 15, 16}, the outlet {6, 13, 14, 17, 18}, and a
// node is never both.  (Conditional stores into the node arrays would be
// merged by the compiler into stores through a selected pointer, which moves
// the arrays out of registers.)
template <bool kDev, class CT>
__device__ __forceinline__ void zou_he(const StepParams& P, unsigned fl, CT phi_up, CT* fr, CT* fx) {
  const bool in = fl & FL_IN;
  const bool out = fl & FL_OUT;
  CT ir[19], ix[19], orr[19], ox[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    ir[i] = fr[i];
    ix[i] = fx[i];
    orr[i] = fr[i];
    ox[i] = fx[i];
  }
  zh_in(ir, (CT)P.rin_r);
  if constexpr (kDev)
    zh_in(ix, (CT)(P.rho_in - P.rho0));
  else
    zh_in(ix, (CT)P.rin_b);
  if constexpr (kDev) {
    CT S = ox[0] + ox[1] + ox[2] + ox[3] + ox[4] + ox[7] + ox[8] + ox[9] + ox[10];
    CT T = ox[5] + ox[11] + ox[12] + ox[15] + ox[16];
    const CT jt = -(CT)(P.rho_out - P.rho0) + (S + CT(2) * T);
    zh_out_color(orr, jt * (CT(0.5) * (CT(1) + phi_up)));
    zh_out_color(ox, jt);
  } else {
    CT ft[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) ft[i] = orr[i] + ox[i];
    CT S = ft[0] + ft[1] + ft[2] + ft[3] + ft[4] + ft[7] + ft[8] + ft[9] + ft[10];
    CT T = ft[5] + ft[11] + ft[12] + ft[15] + ft[16];
    const CT jt = -(CT)P.rho_out + (S + CT(2) * T);
    const CT chr = CT(0.5) * (CT(1) + phi_up);
    const CT chb = CT(0.5) * (CT(1) - phi_up);
    zh_out_color(orr, jt * chr);
    zh_out_color(ox, jt * chb);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    fr[kZhIn[q]] = in ? ir[kZhIn[q]] : fr[kZhIn[q]];
    fx[kZhIn[q]] = in ? ix[kZhIn[q]] : fx[kZhIn[q]];
    fr[kZhOut[q]] = out ? orr[kZhOut[q]] : fr[kZhOut[q]];
    fx[kZhOut[q]] = out ? ox[kZhOut[q]] : fx[kZhOut[q]];
  }
}

// ------------------------------------------------------------------ moments

// Densities of the loaded node: rr = sum f^r, rb, rho (Eqs. 8-9), drho (the
// density handed to the equilibrium: rho itself, or the deviation sum of g
// that never rounds through rho), and the total populations ft used by the
// collision (canonical: f^r + f^b; deviation: g as loaded).
// Deviation layout: rho (used for phi, rho^b and the recolouring fractions)
// is the sum of the rebuilt totals w_i rho0 + g_i with the same single-
// precision weights the pull uses to rebuild f^r.  Those weights do not sum
// to exactly 1 (the excess is about 1.5e-8), and dividing rho^r by rho0 +
// sum g instead would grow the red mass by that excess every step.
template <int D, bool kDev, class CT>
__device__ __forceinline__ void node_moments(const CT* fr, CT* fx, CT rho0, CT& rr, CT& rb, CT& rho, CT& drho) {
  constexpr int Q = Lat<D>::Q;
  CT a = fr[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) a = a + fr[i];
  CT b = fx[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) b = b + fx[i];
  rr = a;
  if constexpr (kDev) {
    drho = b;
    CT t = (CT)Lat<D>::w(0) * rho0 + fx[0];
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      t = t + ((CT)Lat<D>::w(i) * rho0 + fx[i]);
    });
    rho = t;
    rb = t - a;
  } else {
    rb = b;
    rho = a + b;
    drho = rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) fx[i] = fr[i] + fx[i];  // fx becomes f^t
  }
}

// ------------------------------------------------------------------ wetting

// Scheme-I, Eqs. (28)-(31): secant on f(v) = v.n_w - |v| cos(theta) along the
// line through v0 = n_c and v1 = n_c - (n_c + s n_w)/2, three secant steps,
// guards on |f|, on the secant denominator, on |v| and on n_c || n_w.
template <class CT, int D>
__device__ __forceinline__ void scheme1(CT* n, const CT* nw, CT cos_t, CT sgn, CT eps_f, CT eps_v) {
  CT cr;
  if constexpr (D == 3) {
    CT c0 = n[1] * nw[2] - n[2] * nw[1];
    CT c1 = n[2] * nw[0] - n[0] * nw[2];
    CT c2 = n[0] * nw[1] - n[1] * nw[0];
    cr = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  } else {
    cr = fabs(n[0] * nw[1] - n[1] * nw[0]);
  }
  if (cr <= eps_v) return;
  CT v0[3], v1[3];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    v0[c] = n[c];
    v1[c] = n[c] - CT(0.5) * (n[c] + sgn * nw[c]);
  }
  CT f0 = dotv<CT, D>(v0, nw) - sqrt(dotv<CT, D>(v0, v0)) * cos_t;
  CT f1 = dotv<CT, D>(v1, nw) - sqrt(dotv<CT, D>(v1, v1)) * cos_t;
  for (int it = 2; it <= 4; ++it) {
    if (fabs(f1) <= eps_f || fabs(f1 - f0) <= eps_f) break;
    CT v2[3];
#pragma unroll
    for (int c = 0; c < D; ++c) v2[c] = (v0[c] * f1 - v1[c] * f0) / (f1 - f0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      v0[c] = v1[c];
      v1[c] = v2[c];
    }
    f0 = f1;
    if (it < 4) f1 = dotv<CT, D>(v1, nw) - sqrt(dotv<CT, D>(v1, v1)) * cos_t;
  }
  CT nv = sqrt(dotv<CT, D>(v1, v1));
  if (nv <= eps_v) return;
#pragma unroll
  for (int c = 0; c < D; ++c) n[c] = v1[c] / nv;
}

// Scheme-II, Eqs. (32)-(33), with cos(theta') = n_w.n_c and
// sin(theta') = |n_c - (n_w.n_c) n_w|; the candidate nearer to n_c is kept.
template <class CT, int D>
__device__ __forceinline__ void scheme2(CT* n, const CT* nw, CT cos_t, CT sin_t, CT eps_v) {
  CT ctp = dotv<CT, D>(nw, n);
  CT t[3];
#pragma unroll
  for (int c = 0; c < D; ++c) t[c] = n[c] - ctp * nw[c];
  CT stp = sqrt(dotv<CT, D>(t, t));
  if (stp <= eps_v) return;
  CT np[3], nm[3];
  {
    CT s = sin_t;
    CT A = cos_t - s * ctp / stp;
    CT B = s / stp;
#pragma unroll
    for (int c = 0; c < D; ++c) np[c] = A * nw[c] + B * n[c];
  }
  {
    CT s = -sin_t;
    CT A = cos_t - s * ctp / stp;
    CT B = s / stp;
#pragma unroll
    for (int c = 0; c < D; ++c) nm[c] = A * nw[c] + B * n[c];
  }
  CT dp = (np[0] - n[0]) * (np[0] - n[0]);
  CT dm = (nm[0] - n[0]) * (nm[0] - n[0]);
#pragma unroll
  for (int c = 1; c < D; ++c) {
    dp = dp + (np[c] - n[c]) * (np[c] - n[c]);
    dm = dm + (nm[c] - n[c]) * (nm[c] - n[c]);
  }
  if (dp <= dm) {
#pragma unroll
    for (int c = 0; c < D; ++c) n[c] = np[c];
  } else {
#pragma unroll
    for (int c = 0; c < D; ++c) n[c] = nm[c];
  }
}

// ---------------------------------------------------------------- collision

// Equilibrium (deviation from w_i rho0 when kDev) of the incompressible
// model: h_i = w_i [drho + rho0 (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)], with
// drho = rho (canonical) or rho - rho0 (deviation).
template <int D, int i, class CT>
__device__ __forceinline__ CT eq_i(CT drho, CT rho0, const CT* u, CT usq) {
  constexpr double w = Lat<D>::w(i);
  CT eu = CT(0);
  bool first = true;
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    constexpr int e = Lat<D>::e(i, a);
    if constexpr (e != 0) {
      const CT t = e == 1 ? u[a] : -u[a];
      eu = first ? t : eu + t;
      first = false;
    }
  });
  return (CT)w * (drho + rho0 * (CT(3) * eu + CT(4.5) * eu * eu - CT(1.5) * usq));
}

// Guo forcing population: w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)].
template <int D, int i, class CT>
__device__ __forceinline__ CT guo_i(const CT* u, const CT* F) {
  constexpr double w = Lat<D>::w(i);
  CT emuF = ((CT)Lat<D>::e(i, 0) - u[0]) * F[0];
  emuF = emuF + ((CT)Lat<D>::e(i, 1) - u[1]) * F[1];
  if constexpr (D == 3) emuF = emuF + ((CT)Lat<D>::e(i, 2) - u[2]) * F[2];
  CT eu = CT(0), eF = CT(0);
  bool first = true;
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    constexpr int e = Lat<D>::e(i, a);
    if constexpr (e != 0) {
      const CT tu = e == 1 ? u[a] : -u[a];
      const CT tF = e == 1 ? F[a] : -F[a];
      eu = first ? tu : eu + tu;
      eF = first ? tF : eF + tF;
      first = false;
    }
  });
  return (CT)w * (CT(3) * emuF + CT(9) * eu * eF);
}

// sum_j M_kj v_j over the non-zero entries in ascending j
template <int k, class CT>
__device__ __forceinline__ CT mrow(const CT* v) {
  CT s = CT(0);
  bool first = true;
  unroll<19>([&](auto J) {
    constexpr int j = J;
    constexpr int m = Mkj(k, j);
    if constexpr (m != 0) {
      CT t;
      if constexpr (m == 1)
        t = v[j];
      else if constexpr (m == -1)
        t = -v[j];
      else
        t = (CT)m * v[j];
      s = first ? t : s + t;
      first = false;
    }
  });
  return s;
}

// MRT collision on the total distribution:
// f'' = f - M^-1 [ S (m - m^eq) - (I - S/2) M Fbar ].
// kExact evaluates m and m^eq separately (reference order); otherwise
// M (f - f^eq) is formed in one product.
template <bool kExact, class CT>
__device__ __forceinline__ void collide_mrt(CT* ft, CT drho, CT rho0, const CT* u, const CT* F, CT s_nu, CT s_q) {
  constexpr int D = 3;
  CT usq = u[0] * u[0];
  usq = usq + u[1] * u[1];
  usq = usq + u[2] * u[2];
  CT fe[19], fb[19];
  unroll<19>([&](auto I) {
    constexpr int i = I;
    fe[i] = eq_i<D, i>(drho, rho0, u, usq);
    fb[i] = guo_i<D, i>(u, F);
  });
  CT corr[19];
  if constexpr (kExact) {
    unroll<19>([&](auto K) {
      constexpr int k = K;
      constexpr int rc = rate_class(k);
      const CT mm = mrow<k>(ft);
      const CT me = mrow<k>(fe);
      const CT mf = mrow<k>(fb);
      if constexpr (rc == 0) {
        corr[k] = -mf;
      } else {
        const CT S = rc == 1 ? s_nu : s_q;
        const CT sf = (CT(1) - CT(0.5) * S) * mf;
        corr[k] = S * (mm - me) - sf;
      }
    });
  } else {
    CT d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = ft[i] - fe[i];
    const CT hnu = CT(1) - CT(0.5) * s_nu, hq = CT(1) - CT(0.5) * s_q;
    unroll<19>([&](auto K) {
      constexpr int k = K;
      constexpr int rc = rate_class(k);
      const CT mf = mrow<k>(fb);
      if constexpr (rc == 0) {
        corr[k] = -mf;
      } else {
        const CT md = mrow<k>(d);
        corr[k] = rc == 1 ? (s_nu * md - hnu * mf) : (s_q * md - hq * mf);
      }
    });
  }
  unroll<19>([&](auto I) {
    constexpr int i = I;
    CT s = CT(0);
    bool first = true;
    unroll<19>([&](auto K) {
      constexpr int k = K;
      if constexpr (Mkj(k, i) != 0) {
        const CT t = (CT)Minv(i, k) * corr[k];
        s = first ? t : s + t;
        first = false;
      }
    });
    ft[i] = ft[i] - s;
  });
}

// Structure of the D3Q19 moment basis that collide_mrt_pairs relies on: the
// rows relaxed at S_nu are even in e (equal on i and opp(i)), the rows relaxed
// at S_q are odd, and the conserved rows are the density (all ones) and the
// three momentum components.  With orthogonal rows the ten even rows span the
// vectors that are even over the pairs (i, opp(i)) and the nine odd rows the
// odd ones.
constexpr bool mrt_pair_structure() {
  int n1 = 0, n2 = 0;
  for (int k = 0; k < 19; ++k) {
    const int rc = rate_class(k);
    n1 += rc == 1;
    n2 += rc == 2;
    for (int i = 1; i < 19; ++i) {
      const int a = Mkj(k, i), b = Mkj(k, opp<3>(i));
      if (rc == 1 && a != b) return false;
      if (rc == 2 && a != -b) return false;
    }
  }
  for (int i = 0; i < 19; ++i)
    if (Mkj(0, i) != 1 || Mkj(3, i) != Lat<3>::e(i, 0) || Mkj(5, i) != Lat<3>::e(i, 1) ||
        Mkj(7, i) != Lat<3>::e(i, 2))
      return false;
  return n1 == 9 && n2 == 6 && rate_class(0) == 0 && rate_class(3) == 0 && rate_class(5) == 0 &&
         rate_class(7) == 0 && Mnorm2(3) == 10;
}

// MRT collision, single-precision form.  With y = f - f^eq + Fbar/2 the
// operator of Eqs. (2)-(4) reads f'' = f + Fbar - M^-1 S M y.  Because of
// mrt_pair_structure(), M^-1 S M y = S_nu (y_even - mean(y)) +
// S_q (y_odd - P_j y_odd), where y_even / y_odd are the half-sums /
// half-differences over the pairs (i, opp(i)) and P_j projects on the three
// momentum rows (|row|^2 = 10).  That is the same linear map as the 19x19
// transform pair, at about a third of the operations.  Per pair the
// equilibrium and the Guo term split the same way:
//   f^eq even = w (drho + rho0 (4.5 (e.u)^2 - 1.5 u.u)), odd = 3 w rho0 e.u;
//   Fbar even = w (9 (e.u)(e.F) - 3 u.F),                odd = 3 w e.F.
template <class CT>
__device__ __forceinline__ void collide_mrt_pairs(CT* g, CT drho, CT rho0, const CT* u, const CT* F, CT s_nu,
                                                  CT s_q) {
  static_assert(mrt_pair_structure(), "D3Q19 moment basis lost its even/odd structure");
  CT usq = u[0] * u[0];
  usq = usq + u[1] * u[1];
  usq = usq + u[2] * u[2];
  CT uF = u[0] * F[0];
  uF = uF + u[1] * F[1];
  uF = uF + u[2] * F[2];
  const CT a0 = drho - CT(1.5) * rho0 * usq;  // f^eq even / w without the (e.u)^2 term
  const CT c0 = CT(-3) * uF;                  // Fbar even / w without the (e.F) term
  const CT r45 = CT(4.5) * rho0;
  constexpr double w0 = Lat<3>::w(0);
  const CT fb0 = (CT)w0 * c0;
  const CT y0 = g[0] - (CT)w0 * a0 + CT(0.5) * fb0;
  const CT hs_nu = CT(0.5) * s_nu, hs_q = CT(0.5) * s_q;
  // First pass, per pair leader i (i < opp(i) = o): Ye = y_i + y_o and
  // Yo = y_i - y_o; g_i and g_o take every term that needs neither mean(y)
  // nor the momentum of Yo, which the second pass adds.
  CT sum = y0;
  CT J[3] = {CT(0), CT(0), CT(0)};
  unroll<19>([&](auto I) {
    constexpr int i = I;
    constexpr int o = opp<3>(i);
    if constexpr (i > 0 && o > i) {
      constexpr double w = Lat<3>::w(i);
      CT eu = CT(0), eF = CT(0);
      bool first = true;
      unroll<3>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<3>::e(i, a);
        if constexpr (e != 0) {
          const CT tu = e == 1 ? u[a] : -u[a];
          const CT tF = e == 1 ? F[a] : -F[a];
          eu = first ? tu : eu + tu;
          eF = first ? tF : eF + tF;
          first = false;
        }
      });
      const CT eqe = (CT)w * (a0 + r45 * eu * eu);
      const CT eqo = (CT)(3.0 * w) * rho0 * eu;
      const CT Be = (CT)w * (c0 + CT(9) * eu * eF);
      const CT Bo = (CT)(3.0 * w) * eF;
      const CT gi = g[i], go = g[o];
      const CT Ye = (gi + go) - CT(2) * eqe + Be;
      const CT Yo = (gi - go) - CT(2) * eqo + Bo;
      sum = sum + Ye;
      unroll<3>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<3>::e(i, a);
        if constexpr (e == 1) J[a] = J[a] + Yo;
        if constexpr (e == -1) J[a] = J[a] - Yo;
      });
      const CT E = hs_nu * Ye, O = hs_q * Yo;
      g[i] = gi + (Be + Bo) - (E + O);
      g[o] = go + (Be - Bo) - (E - O);
    }
  });
  // Second pass: the density and momentum projections,
  // +S_nu mean(y) on every population, +-S_q (e_i.J)/10 on each pair.
  const CT ybar = sum * CT(1.0 / 19.0);
  const CT cn = s_nu * ybar;
  const CT Jq[3] = {J[0] * (CT(0.1) * s_q), J[1] * (CT(0.1) * s_q), J[2] * (CT(0.1) * s_q)};
  g[0] = g[0] + fb0 - s_nu * (y0 - ybar);
  unroll<19>([&](auto I) {
    constexpr int i = I;
    constexpr int o = opp<3>(i);
    if constexpr (i > 0 && o > i) {
      CT eJ = CT(0);
      bool first = true;
      unroll<3>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<3>::e(i, a);
        if constexpr (e != 0) {
          const CT t = e == 1 ? Jq[a] : -Jq[a];
          eJ = first ? t : eJ + t;
          first = false;
        }
      });
      g[i] = g[i] + (cn + eJ);
      g[o] = g[o] + (cn - eJ);
    }
  });
}

// Rates of Eqs. (13)-(16), single-precision path: the same expressions
// rearranged to two hardware reciprocals (about 1 ulp each),
// 1/nu = (1 + phi)/(2 nu_r) + (1 - phi)/(2 nu_b), S_nu = (1/nu) / (3 + (1/nu)/2).
__device__ __forceinline__ void rates_f32(const StepParams& P, float phi, float& s_nu, float& s_q) {
  const float inv_nu = (1.f + phi) * P.hinv_nu_r + (1.f - phi) * P.hinv_nu_b;
  s_nu = inv_nu * __builtin_amdgcn_rcpf(3.f + 0.5f * inv_nu);
  s_q = (8.f * (2.f - s_nu)) * __builtin_amdgcn_rcpf(8.f - s_nu);
}

// Single-relaxation-time collision with Guo forcing:
// f'' = f - S_nu (f - f^eq) + (1 - S_nu/2) Fbar.
template <int D, class CT>
__device__ __forceinline__ void collide_bgk(CT* ft, CT drho, CT rho0, const CT* u, const CT* F, CT s_nu) {
  CT usq = u[0] * u[0];
  usq = usq + u[1] * u[1];
  if constexpr (D == 3) usq = usq + u[2] * u[2];
  const CT h = CT(1) - CT(0.5) * s_nu;
  unroll<Lat<D>::Q>([&](auto I) {
    constexpr int i = I;
    const CT fe = eq_i<D, i>(drho, rho0, u, usq);
    const CT fb = guo_i<D, i>(u, F);
    ft[i] = ft[i] - s_nu * (ft[i] - fe) + h * fb;
  });
}

// Rates of Eqs. (13)-(16) from the local phase field.
template <class CT>
__device__ __forceinline__ void rates(const StepParams& P, CT phi, CT& s_nu, CT& s_q) {
  const CT nr = (CT)P.nu_r, nb = (CT)P.nu_b;
  CT inv_nu = (CT(1) + phi) / (CT(2) * nr) + (CT(1) - phi) / (CT(2) * nb);
  CT nu = CT(1) / inv_nu;
  s_nu = CT(1) / (CT(3) * nu + CT(0.5));
  s_q = (CT(8) * (CT(2) - s_nu)) / (CT(8) - s_nu);
}

}  // namespace cg
