// __global__ kernels of the time step, observables and state transfer.
// Instantiated per precision in kernels_f64.hip / kernels_f32.hip.
//
// Order within one step: k_phase -> k_sb_phi -> k_normal -> k_sb_n -> k_main
// (k_main evaluates the curvature and force of its node itself; k_curv stores
// them for the macroscopic fields, the observables and the adjoint).  Each
// kernel needs the previous one complete over the whole grid (stencils of
// radius 1 on the previous output).
#pragma once

#include "step.hpp"

namespace cg {

__device__ __forceinline__ int vox_of(unsigned vf) { return (int)(vf & kVoxMask); }

// Loads of per-node data that one thread reads once per kernel: marked
// non-temporal so that they do not push the stencil neighbours' lines, which
// several waves reuse, out of L2.
__device__ __forceinline__ unsigned ld_once(const unsigned* p) { return __builtin_nontemporal_load(p); }
template <class Real>
__device__ __forceinline__ Vec4<Real> ld_once3(const Norm3<Real>* p) {
  Vec4<Real> o;
  o.x = __builtin_nontemporal_load(&p->x);
  o.y = __builtin_nontemporal_load(&p->y);
  o.z = __builtin_nontemporal_load(&p->z);
  o.w = Real(0);
  return o;
}
__device__ __forceinline__ unsigned flags_of(unsigned vf) { return vf >> kVoxBits; }

// ------------------------------------------------------------------ k_phase
// Densities and phase field at every fluid node, Eqs. (7)-(9); inlet nodes take
// phi_in (Sec. II.D.1), outlet nodes the phase one node upstream (Eq. 39).
// The sums are taken in double for either state layout.
template <class Real, int D, class In>
__device__ __forceinline__ void d_phase(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, const In& in, int n) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  using CT = double;
  if (n >= P.N) return;
  const unsigned vf = ld_once(&G.vf[n]);
  const unsigned fl = flags_of(vf);
  CT phi;
  if (fl & FL_IN) {
    phi = P.phi_in;
  } else if (std::is_same_v<In, InCompact<D>>) {
    // the compact state: the two sums only, accumulated as the pulled
    // populations are rebuilt in double (see pull_sums_compact); an outlet
    // node's phase, the one of the node upstream (Eq. 39), is copied by
    // k_face once this stage has stored that node's
    if constexpr (std::is_same_v<In, InCompact<D>>) {
      if (fl & FL_OUT) return;
      CT rr, rho;
      pull_sums_compact<D>(in, G.nbr, n, P.rho0, rr, rho);
      phi = (rr - (rho - rr)) / rho;
      __builtin_nontemporal_store(rr, &in.RS[n]);
    }
  } else {
    // pulled populations rebuilt in double (for the compact float state the
    // red population is a (w rho0 + g) + w c.e of single-precision factors)
    CT fr[Q], fx[Q];
    if (fl & FL_OUT) {
      // an outlet node takes the phase of the node upstream; its populations
      // are pulled with that node's own (uniform) tile, by a whole-wave call
      // made only by waves that hold an outlet node
      load_outlet_upstream<D>(in, G.nbr, n, fr, fx);
    } else {
      load_node<D>(in, G.nbr, n, fr, fx);
    }
    CT rr, rb, rho;
    if constexpr (kDev) {
      CT a = fr[0], t = (CT)Lat<D>::w(0) * P.rho0 + fx[0];
      unroll<Q - 1>([&](auto I) {
        constexpr int i = I + 1;
        a = a + fr[i];
        t = t + ((CT)Lat<D>::w(i) * P.rho0 + fx[i]);
      });
      rr = a;
      rho = t;
      rb = t - a;
    } else {
      CT drho;
      node_moments<D, kDev>(fr, fx, (CT)P.rho0, rr, rb, rho, drho);
    }
    phi = (rr - rb) / rho;
  }
  R.phi[vox_of(vf)] = phi_enc<typename Grids<Real>::PhiT>(phi);
}

// Zou-He face node n of the compact single-precision state, after the phase
// stage: an outlet node first takes the stored phase of the node upstream
// (Eq. 39); then its pulled populations with the faces applied, Appendix B,
// in the step kernel's single-precision arithmetic.  The step kernel takes
// the red sum and the five unknowns from here.  A kernel of
// its own, so that the per-colour pull of these few nodes does not set the
// register count of the phase stage.
template <class Real, int D, class In>
__device__ __forceinline__ void d_face(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, const In& in,
                                       int n) {
  if constexpr (std::is_same_v<In, InCompact<D>> && D == 3) {
    constexpr int Q = Lat<D>::Q;
    const unsigned vf = ld_once(&G.vf[n]);
    const unsigned fl = flags_of(vf);
    const int v = vox_of(vf);
    auto enc = R.phi[v];
    if (fl & FL_OUT) {
      // Eq. (39): the phase of the node upstream, as the phase stage stored it
      enc = R.phi[v - P.nx * P.ny];
      R.phi[v] = enc;
    }
    float fr[Q], fx[Q];
    load_node<D>(in, G.nbr, n, fr, fx);
    zou_he<true>(P, fl, (float)phi_dec(enc), fr, fx);
    double rs = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) rs = rs + (double)fr[i];
    in.RS[n] = rs;
    const int k = face_slot(P, fl, n), nf = P.n_in + P.n_out;
    const bool fin = fl & FL_IN;
#pragma unroll
    for (int q = 0; q < 5; ++q) in.FS[q * nf + k] = fin ? fx[kZhIn[q]] : fx[kZhOut[q]];
  }
}

// Wave w of the launch covers one whole tile of 64 nodes (the pull table
// decodes per tile): first the tiles that hold inlet nodes, then those that
// hold outlet nodes; lanes on other nodes return.  face_tiles() gives the
// number of waves.
__host__ __device__ inline int face_tiles_in(const StepParams& P) { return (P.n_in + 63) >> 6; }
__host__ __device__ inline int face_tiles(const StepParams& P) {
  return P.n_out > 0 ? face_tiles_in(P) + ((P.N + 63) >> 6) - ((P.N - P.n_out) >> 6) : face_tiles_in(P);
}
// The face node thread t of the launch works on, or -1.
__host__ __device__ inline int face_node(const StepParams& P, int t) {
  const int w = t >> 6, lane = t & 63, tin = face_tiles_in(P);
  if (t < 0 || w >= face_tiles(P)) return -1;
  const int n = w < tin ? (w << 6) + lane : ((((P.N - P.n_out) >> 6) + w - tin) << 6) + lane;
  const bool face = w < tin ? n < P.n_in : (n >= P.N - P.n_out && n < P.N);
  return face ? n : -1;
}
template <class Real, int D, class In>
__global__ void k_face(StepParams P, Geo<Real> G, Grids<Real> R, In in) {
  const int n = face_node(P, node_id_plain());
  if (n >= 0) d_face<Real, D, In>(P, G, R, in, n);
}

template <class Real, int D, class In>
__global__ void k_phase(StepParams P, Geo<Real> G, Grids<Real> R, In in) {
  d_phase<Real, D, In>(P, G, R, in, node_id());
}

// ----------------------------------------------------------------- k_sb_phi
// Raw buffer loads whose out-of-range lanes return 0 without touching memory:
// a gather over a masked subset of links with no branch per link, so all the
// loads of a point are in flight together.  offset = kOffNone masks a lane;
// it stays out of range for every component offset added to it (the grids
// are below 2^32 - 256 bytes, checked when the run is created).  Vectors are
// read component by component (x, y, z; w is not needed there): a single
// 128-bit raw buffer load of a float4 was compiled into one dword load by the
// toolchain in use, the per-component form is merged into dwordx3 correctly.
constexpr uint32_t kOffNone = 0xFFFFFFC0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t grid_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(uint32_t)bytes, 0x00020000);
}

__device__ __forceinline__ float bload1(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double bload1(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <class Real>
__device__ __forceinline__ Vec4<Real> bload3(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  Vec4<Real> o;
  o.x = bload1(r, off, Real(0));
  o.y = bload1(r, off + (uint32_t)sizeof(Real), Real(0));
  o.z = bload1(r, off + 2u * (uint32_t)sizeof(Real), Real(0));
  o.w = Real(0);
  return o;
}

// Eq. (34): weighted mean of the fluid link neighbours, i ascending (links
// that do not end on a fluid voxel load nothing and add an exact zero).
template <class Real, int D>
__device__ __forceinline__ void d_sb_phi(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, int s) {
  constexpr int Q = Lat<D>::Q;
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  if (P.scheme == 3) {
    // fictitious-density wetting: a fixed phase per solid boundary point
    R.phi[v] = phi_enc<typename Grids<Real>::PhiT>((double)G.sb_fd[s]);
    return;
  }
  const unsigned m = G.sb_mask[s];
  const Pos ps = make_pos(P, v, m & 1u);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  using PhiT = typename Grids<Real>::PhiT;
  const auto rs = grid_rsrc(R.phi, sizeof(PhiT) * (size_t)P.V);
  // a fluid voxel of the outlet layer is an outlet node, whose phase is the
  // node upstream's (Eq. 39): read there, so this stage does not wait for the
  // copy the face stage makes (the two share a launch)
  if (P.n_out > 0) {
    const int first_out = P.V - P.nx * P.ny;
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      if constexpr (D == 3 && Lat<D>::e(i, 2) >= 0)
        nbi[i] = nbi[i] >= first_out ? nbi[i] - P.nx * P.ny : nbi[i];
    });
  }
  double ph[Q];
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    const bool on = m & (1u << i);
    const uint32_t off = on ? (uint32_t)nbi[i] * (uint32_t)sizeof(PhiT) : kOffNone;
    ph[i] = phi_dec(bload1(rs, off, PhiT(0)));
  });
  double num = 0.0, den = 0.0;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    constexpr double w = Lat<D>::w(i);
    const bool on = m & (1u << i);
    num = num + (on ? w * ph[i] : 0.0);
    den = den + (on ? w : 0.0);
  });
  R.phi[v] = phi_enc<PhiT>(num / den);
}

template <class Real, int D>
__global__ void k_sb_phi(StepParams P, Geo<Real> G, Grids<Real> R) {
  d_sb_phi<Real, D>(P, G, R, node_id());
}

// The face stage and the solid-boundary phase stage in one launch (both need
// only the phase stage): the first nfb blocks cover the face tiles, the rest
// the solid boundary points with the XCD-aware mapping of their own range
// (nfb is a multiple of 8, so block b of that range runs on XCD b mod 8).
template <class Real, int D, class In>
__global__ void k_face_sb_phi(StepParams P, Geo<Real> G, Grids<Real> R, In in, int nfb) {
  if ((int)blockIdx.x < nfb) {
    const int n = face_node(P, (int)(blockIdx.x * blockDim.x + threadIdx.x));
    if (n >= 0) d_face<Real, D, In>(P, G, R, in, n);
  } else {
    const int b = (int)blockIdx.x - nfb;
    d_sb_phi<Real, D>(P, G, R, xcd_tile(b, (int)gridDim.x - nfb) * (int)blockDim.x + (int)threadIdx.x);
  }
}

// ----------------------------------------------------------------- k_normal
// Colour gradient, Eq. (6), unit normal, Eq. (27), wetting at the fluid
// boundary points (Sec. II.B.3 step 3) keeping |C|.  Double arithmetic for
// either layout.
template <class Real, int D>
__device__ __forceinline__ void d_normal(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, int n) {
  constexpr int Q = Lat<D>::Q;
  using CT = double;
  if (n >= P.N) return;
  const unsigned vf = ld_once(&G.vf[n]);
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  const Pos ps = make_pos(P, v, fl & FL_FACE);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  double ph[Q];
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    if constexpr (i > 0) ph[i] = phi_dec(R.phi[nbi[i]]);
  });
  CT C[3] = {CT(0), CT(0), CT(0)};
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    CT s = CT(0);
    bool first = true;
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int e = Lat<D>::e(i, a);
      if constexpr (e != 0) {
        constexpr double we = Lat<D>::w(i) * e;
        const CT t = (CT)we * (CT)ph[i];
        s = first ? t : s + t;
        first = false;
      }
    });
    C[a] = CT(3) * s;
  });
  const CT cm = sqrt(dotv<CT, D>(C, C));
  CT nn[3] = {CT(0), CT(0), CT(0)};
  if (cm > (CT)P.eps_c) {
#pragma unroll
    for (int a = 0; a < D; ++a) nn[a] = C[a] / cm;
    if ((fl & FL_WET) && (P.scheme == 1 || P.scheme == 2)) {
      CT w3[3];
#pragma unroll
      for (int a = 0; a < D; ++a) w3[a] = (CT)G.nw[a * P.Np + n];
      if (P.scheme == 1)
        scheme1<CT, D>(nn, w3, (CT)G.cos_t[n], (fl & FL_S1POS) ? CT(1) : CT(-1), (CT)P.eps_f, (CT)P.eps_v);
      else
        scheme2<CT, D>(nn, w3, (CT)G.cos_t[n], (CT)G.sin_t[n], (CT)P.eps_v);
#pragma unroll
      for (int a = 0; a < D; ++a) C[a] = cm * nn[a];
    }
  }
  Vec4<Real> nv, cv;
  nv.x = (Real)nn[0];
  nv.y = (Real)nn[1];
  nv.z = (Real)nn[2];
  nv.w = Real(0);
  cv.x = (Real)C[0];
  cv.y = (Real)C[1];
  cv.z = (Real)C[2];
  cv.w = Real(0);
  n_put(R.n, v, nv);
  n_put(R.c, n, cv);
}

template <class Real, int D>
__global__ void k_normal(StepParams P, Geo<Real> G, Grids<Real> R) {
  d_normal<Real, D>(P, G, R, node_id_plain());
}

// ------------------------------------------------------------------- k_sb_n
// Eq. (35): normal extrapolated to the solid boundary points, not renormalised
// (masked buffer loads as in d_sb_phi).
template <class Real, int D>
__device__ __forceinline__ void d_sb_n(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, int s) {
  constexpr int Q = Lat<D>::Q;
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  const unsigned m = G.sb_mask[s];
  const Pos ps = make_pos(P, v, m & 1u);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  const auto rs = grid_rsrc(R.n, sizeof(Norm3<Real>) * (size_t)P.V);
  Vec4<Real> q[Q];
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    const bool on = m & (1u << i);
    const uint32_t off = on ? (uint32_t)nbi[i] * (uint32_t)sizeof(Norm3<Real>) : kOffNone;
    q[i] = bload3<Real>(rs, off);
  });
  Real num[3] = {Real(0), Real(0), Real(0)};
  Real den = Real(0);
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    constexpr double w = Lat<D>::w(i);
    const bool on = m & (1u << i);
    const Real qq[3] = {q[i].x, q[i].y, q[i].z};
#pragma unroll
    for (int a = 0; a < D; ++a) num[a] = num[a] + (on ? (Real)w * qq[a] : Real(0));
    den = den + (on ? (Real)w : Real(0));
  });
  Vec4<Real> o;
  o.x = num[0] / den;
  o.y = num[1] / den;
  o.z = D == 3 ? num[2] / den : Real(0);
  o.w = Real(0);
  n_put(R.n, v, o);
}

template <class Real, int D>
__global__ void k_sb_n(StepParams P, Geo<Real> G, Grids<Real> R) {
  d_sb_n<Real, D>(P, G, R, node_id());
}

// ------------------------------------------------------------------- k_curv
// Curvature, Eq. (12), from the isotropic derivatives of n (same stencil as
// Eq. 6), and the force F = 1/2 sigma kappa C (Eq. 5) + rho_o g (Eq. 36).
// The double layout evaluates it in the order of the definition; the float
// layout in single precision with the factor 3 folded into the stencil weights
// (the force is ~1e-5 of a population, so its rounding stays far below the
// single-precision tolerance).  The time step evaluates this inside k_main (the
// force of a node is used by that node only); k_curv stores it for the
// macroscopic fields, the observables and the adjoint.
// CT is the arithmetic type: the storage precision inside the time step, double
// where the macroscopic fields and the observables are read out.
template <class Real, int D, class CT = Real>
__device__ __forceinline__ void curv_force(const StepParams& P, const Grids<Real>& R, int n, int v, const Pos& ps,
                                           const Vec4<Real>& self, double* F, double& k) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  Vec4<Real> nb[Q];
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    if constexpr (i > 0) nb[i] = n_get(R.n, nbi[i]);
  });
  CT d[3][3];
  unroll<D>([&](auto B_) {
    constexpr int b = B_;
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      CT s = CT(0);
      bool first = true;
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        constexpr int e = Lat<D>::e(i, b);
        if constexpr (e != 0) {
          constexpr double we = (kDev ? 3.0 : 1.0) * Lat<D>::w(i) * e;
          const CT na = (CT)(a == 0 ? nb[i].x : (a == 1 ? nb[i].y : nb[i].z));
          const CT t = (CT)we * na;
          s = first ? t : s + t;
          first = false;
        }
      });
      d[b][a] = kDev ? s : CT(3) * s;
    });
  });
  const CT nx_ = (CT)self.x, ny_ = (CT)self.y, nz_ = (CT)self.z;
  CT kk;
  if constexpr (D == 3) {
    kk = (nx_ * nx_ - CT(1)) * d[0][0] + (ny_ * ny_ - CT(1)) * d[1][1] + (nz_ * nz_ - CT(1)) * d[2][2] +
         (d[1][0] + d[0][1]) * nx_ * ny_ + (d[2][0] + d[0][2]) * nx_ * nz_ + (d[1][2] + d[2][1]) * nz_ * ny_;
  } else {
    kk = (nx_ * nx_ - CT(1)) * d[0][0] + (ny_ * ny_ - CT(1)) * d[1][1] + (d[1][0] + d[0][1]) * nx_ * ny_;
  }
  k = (double)kk;
  // C as stored by k_normal: rebuilding it as |C| n in single precision
  // triples its rounding, which the force passes straight to the velocity
  const Vec4<Real> c = ld_once3<Real>(&R.c[n]);
  const CT C[3] = {(CT)c.x, (CT)c.y, (CT)c.z};
  F[0] = F[1] = F[2] = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) F[a] = (double)((CT)P.half_sigma * kk * C[a] + (CT)P.rg[a]);
}

template <class Real, int D>
__device__ __forceinline__ void d_curv(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, int n) {
  if (n >= P.N) return;
  const unsigned vf = ld_once(&G.vf[n]);
  const int v = vox_of(vf);
  const Pos ps = make_pos(P, v, flags_of(vf) & FL_FACE);
  double F[3], k;
  curv_force<Real, D>(P, R, n, v, ps, n_get(R.n, v), F, k);
  Vec4<Real> o;
  o.x = (Real)F[0];
  o.y = (Real)F[1];
  o.z = (Real)F[2];
  o.w = (Real)k;
  R.f[n] = o;
}

template <class Real, int D>
__global__ void k_curv(StepParams P, Geo<Real> G, Grids<Real> R) {
  d_curv<Real, D>(P, G, R, node_id());
}

// ------------------------------------------------------------------- k_main
enum { MODE_STEP = 0, MODE_MACRO = 1, MODE_OBS = 2 };

// Dense FP64 outputs of MODE_MACRO (any pointer may be null).
struct MacroOut {
  double* rho_r;
  double* rho_b;
  double* phi;
  double* u;      // [3][V]
  double* kappa;
  double* force;  // [3][V]
  double* cvec;   // [3][V]
  // MODE_STEP: when set, the node's force (xyz) and curvature (w) are also
  // stored here (Vec4<Real>[Np], the layout of Grids::f), for a consumer that
  // needs them after the step (the adjoint's kept front fields)
  void* fstore;
};

// partial sums per block: [gridDim][kObsN]
struct ObsOut {
  double* part;
};

template <int BS>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) t += sh[k];
  return t;
}

template <int BS>
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) t = fmax(t, sh[k]);
  return t;
}

// Pull, faces, velocity, rates, collision, recolouring, store (MODE_STEP);
// or the macroscopic fields (MODE_MACRO); or the observable reductions
// (MODE_OBS).
// Per-node part of the fused kernel (n < P.N).  MODE_OBS accumulates into o.
template <class Real, int D, int Mode, class In, class Out>
__device__ __forceinline__ void d_main(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R, const In& in,
                                       const Out& out, const MacroOut& mo, int n, double* o) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  using CT = double;
  const unsigned vf = ld_once(&G.vf[n]);
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  // the step computes in the storage precision; the read-out modes rebuild
  // the pulled populations and evaluate everything in double
  using VT = std::conditional_t<Mode == MODE_STEP, Real, CT>;
  // the single-precision step pulls the totals g only: the red density
  // pulled in (and at face nodes the unknowns the faces set) were summed by
  // the phase stage of this step
  constexpr bool kSums = Mode == MODE_STEP && std::is_same_v<In, InCompact<D>>;
  VT fr[Q], fx[Q];
  VT rr, rb, rho, drho;
  [[maybe_unused]] double rr_in = 0.0;
  if constexpr (kSums) {
    load_node_t<D>(in, G.nbr, n, fx);
    if constexpr (D == 3) {
      if (fl & (FL_IN | FL_OUT)) {
        const int k = face_slot(P, fl, n), nf = P.n_in + P.n_out;
        const bool fin = fl & FL_IN;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float g = in.FS[q * nf + k];
          fx[kZhIn[q]] = fin ? g : fx[kZhIn[q]];
          fx[kZhOut[q]] = fin ? fx[kZhOut[q]] : g;
        }
      }
    }
    rr_in = __builtin_nontemporal_load(&in.RS[n]);
    VT b = fx[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) b = b + fx[i];
    VT t = (VT)Lat<D>::w(0) * (VT)P.rho0 + fx[0];
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      t = t + ((VT)Lat<D>::w(i) * (VT)P.rho0 + fx[i]);
    });
    drho = b;
    rho = t;
    rr = (VT)rr_in;
    rb = t - rr;
  } else {
    load_node<D>(in, G.nbr, n, fr, fx);
    if constexpr (In::kPull) {
      if (D == 3 && (fl & (FL_IN | FL_OUT))) zou_he<kDev>(P, fl, (VT)phi_dec(R.phi[v]), fr, fx);
    }
    node_moments<D, kDev>(fr, fx, (VT)P.rho0, rr, rb, rho, drho);
  }
  // the phase of this node from the densities just pulled (k_phase stored
  // the same value, summed in double); Zou-He nodes keep the stored one,
  // which the boundary condition imposes
  VT phi;
  if constexpr (kDev && Mode == MODE_STEP)
    phi = (rr - rb) * __builtin_amdgcn_rcpf(rho);
  else
    phi = (rr - rb) / rho;
  if (fl & (FL_IN | FL_OUT)) phi = (VT)phi_dec(R.phi[v]);
  const Vec4<Real> n4 = n_get(R.n, v);
  // curvature and force of this node (what k_curv stores), in the arithmetic
  // of the mode
  double Fd[3], kd;
  curv_force<Real, D, VT>(P, R, n, v, make_pos(P, v, fl & FL_FACE), n4, Fd, kd);
  if constexpr (Mode == MODE_STEP) {
    Vec4<Real> f4;
    f4.x = (Real)Fd[0];
    f4.y = (Real)Fd[1];
    f4.z = (Real)Fd[2];
    f4.w = (Real)kd;
    if (mo.fstore) static_cast<Vec4<Real>*>(mo.fstore)[n] = f4;
  }
  // velocity, Eq. (22), in the storage precision for the collision and in
  // double for the reported fields; the deviation layout balances momentum
  // with rho0 + sum g
  using UT = VT;
  const UT F[3] = {(UT)Fd[0], (UT)Fd[1], (UT)Fd[2]};
  const UT rho_u = kDev ? (UT)P.rho0 + (UT)drho : (UT)rho;
  UT u[3] = {UT(0), UT(0), UT(0)};
  // single-precision step: one hardware reciprocal (about 1 ulp) for the three
  // velocity components
  [[maybe_unused]] UT inv_rho_u = UT(0);
  if constexpr (kDev && Mode == MODE_STEP) inv_rho_u = __builtin_amdgcn_rcpf(rho_u);
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    UT j = UT(0);
    bool first = true;
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int e = Lat<D>::e(i, a);
      if constexpr (e != 0) {
        const UT t = e == 1 ? (UT)fx[i] : -(UT)fx[i];
        j = first ? t : j + t;
        first = false;
      }
    });
    if constexpr (kDev && Mode == MODE_STEP)
      u[a] = (j + UT(0.5) * F[a]) * inv_rho_u;
    else
      u[a] = (j + UT(0.5) * F[a]) / rho_u;
  });
  if constexpr (Mode == MODE_STEP) {
    Real s_nu, s_q;
    if constexpr (kDev)
      rates_f32(P, phi, s_nu, s_q);
    else
      rates(P, phi, s_nu, s_q);
    Real ur[3], Fr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ur[a] = (Real)u[a];
      Fr[a] = (Real)F[a];
    }
    if constexpr (D == 3) {
      if (P.collision == 1) {
        if constexpr (kDev)
          collide_mrt_pairs(fx, drho, (Real)P.rho0, ur, Fr, s_nu, s_q);
        else
          collide_mrt<true>(fx, drho, (Real)P.rho0, ur, Fr, s_nu, s_q);
      } else
        collide_bgk<D>(fx, drho, (Real)P.rho0, ur, Fr, s_nu);
    } else {
      collide_bgk<D>(fx, drho, (Real)P.rho0, ur, Fr, s_nu);
    }
    // recolouring, Eqs. (20)-(21)
    const Real rsum = rr + rb;
    if constexpr (kDev) {
      // a is the red share of every population leaving the node: the red
      // density pulled in (summed in double) over the post-collision total
      // as the next phase stage rebuilds it from g'' (w rho0 + g'' in
      // double), correctly rounded, so the red mass leaving equals the red
      // mass that arrived up to the rounding of a (single-precision sums
      // drifted the colour masses by ~1e-9 per step while interfaces move).
      // b only scales the segregation term, whose weights cancel.
      double rrd = 0.0, td = 0.0;
      if constexpr (kSums) rrd = rr_in;
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (!kSums) rrd = rrd + (double)fr[i];
        td = td + ((double)Lat<D>::w(i) * (double)(float)P.rho0 + (double)fx[i]);
      });
      const Real a = (Real)(rrd / td);
      const Real b = rr * rb * __builtin_amdgcn_rcpf(rsum);
      const Real bb = (Real)P.beta * b;
      float4 ac;
      ac.x = a;
      ac.y = bb * n4.x;
      ac.z = bb * n4.y;
      ac.w = D == 3 ? bb * n4.z : 0.f;
      typedef float v4f __attribute__((ext_vector_type(4)));
      const v4f acv = {ac.x, ac.y, ac.z, ac.w};
      __builtin_nontemporal_store(acv, reinterpret_cast<v4f*>(&out.AC[n]));
#pragma unroll
      for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(fx[i], &out.T[i * out.Np + n]);
    } else {
      const Real a = rr / rsum;
      const Real b = rr * rb / rsum;
      const Real nvec[3] = {n4.x, n4.y, n4.z};
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        const Real fpp = fx[i];
        Real r;
        if constexpr (i == 0) {
          r = a * fpp;
        } else {
          Real edn = Real(0);
          bool first = true;
          unroll<D>([&](auto C_) {
            constexpr int c = C_;
            constexpr int e = Lat<D>::e(i, c);
            if constexpr (e != 0) {
              const Real t = e == 1 ? nvec[c] : -nvec[c];
              edn = first ? t : edn + t;
              first = false;
            }
          });
          constexpr double w = Lat<D>::w(i);
          r = a * fpp + (Real)P.beta * (Real)w * b * edn;
        }
        out.fr[i * out.Np + n] = r;
        out.fb[i * out.Np + n] = fpp - r;
      });
    }
  } else if constexpr (Mode == MODE_MACRO) {
    const Vec4<Real> c4 = n_get(R.c, n);
    if (mo.rho_r) mo.rho_r[v] = (double)rr;
    if (mo.rho_b) mo.rho_b[v] = (double)rb;
    if (mo.phi) mo.phi[v] = (double)phi;
    if (mo.kappa) mo.kappa[v] = kd;
    const double cc[3] = {(double)c4.x, (double)c4.y, (double)c4.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (mo.u) mo.u[(size_t)a * P.V + v] = (double)u[a];
      if (mo.force) mo.force[(size_t)a * P.V + v] = (double)F[a];
      if (mo.cvec) mo.cvec[(size_t)a * P.V + v] = cc[a];
    }
  } else {
    const double a = rr, b = rb, ph = phi;
    double u2 = 0.0;
    bool ok = isfinite(a) && isfinite(b);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      ok = ok && isfinite((double)u[c]);
      u2 += (double)u[c] * (double)u[c];
    }
    const int nxy = P.nx * P.ny;
    const int cz = v / nxy, cr = v - cz * nxy, cy = cr / P.nx, cx = cr - cy * P.nx;
    auto coord = [&](int axis) { return axis == 0 ? cx : (axis == 1 ? cy : cz); };
    // the plane flux over its whole plane, everything else over the slab
    if (ok && P.flux_axis >= 0 && P.flux_axis < D && coord(P.flux_axis) == P.flux_plane) {
      const double ua = (double)u[P.flux_axis];
      o[12] = (a + b) * ua;
      o[13] = a * ua;
      o[14] = b * ua;
    }
    const bool in_slab =
        P.slab_axis < 0 || (coord(P.slab_axis) >= P.slab_lo && coord(P.slab_axis) < P.slab_hi);
    if (!in_slab) {
    } else if (!ok) {
      o[11] = 1.0;
    } else {
      o[0] = a;
      o[1] = b;
      o[2] = 1.0;
      o[3] = ph < 0.0 ? 1.0 : 0.0;
      o[4] = (1.0 + ph) / 2.0;
      o[5] = (1.0 - ph) / 2.0;
      const double pr = (a + b) / 3.0;
      if (ph > 0.9) {
        o[6] = pr;
        o[7] = 1.0;
      }
      if (ph < -0.9) {
        o[8] = pr;
        o[9] = 1.0;
      }
      o[10] = sqrt(u2);
    }
  }
}

template <class Real, int D, int BS, int Mode, class In, class Out>
__global__ void __launch_bounds__(BS) k_main(StepParams P, Geo<Real> G, Grids<Real> R, In in, Out out,
                                             MacroOut mo, ObsOut oo) {
  const int n = node_id();
  double o[kObsN];
  if constexpr (Mode == MODE_OBS) {
#pragma unroll
    for (int k = 0; k < kObsN; ++k) o[k] = 0.0;
  }
  if (n < P.N) d_main<Real, D, Mode>(P, G, R, in, out, mo, n, o);
  if constexpr (Mode == MODE_OBS) {
    __shared__ double sh[BS / 64];
#pragma unroll
    for (int q = 0; q < kObsN; ++q) {
      const double t = (q == 10) ? block_max<BS>(o[q], sh) : block_sum<BS>(o[q], sh);
      if (threadIdx.x == 0) oo.part[blockIdx.x * kObsN + q] = t;
    }
  }
}

// Second pass of the observables: one block per accumulator; each thread
// reduces a fixed strided subset in order, then a fixed tree (deterministic).
template <class Real>
__global__ void k_obs_final(const double* part, int nblocks, double* out) {
  const int q = blockIdx.x;
  __shared__ double sh[256];
  double t = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const double x = part[b * kObsN + q];
    t = (q == 10) ? fmax(t, x) : t + x;
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      sh[threadIdx.x] = (q == 10) ? fmax(sh[threadIdx.x], sh[threadIdx.x + w]) : sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = sh[0];
}

// ------------------------------------------------------ interface points
// Interface points along one grid line of the phase-field grid (Sec. III.B:
// the drop's base and height are read where phi changes sign along a line;
// Sec. IV.A: the front on the tube axis).  The profile is
// p(k) = (1 - t) phi(v0 + k*stride) + t phi(v0 + shift + k*stride) for
// k = lo .. hi-1 (t = 0: one line; otherwise blended with the parallel line
// one voxel over, for an axis between two columns).  A crossing is k where
// p(k) == 0, or k + p(k) / (p(k) - p(k+1)) where p(k) p(k+1) < 0, plus hi-1
// when p(hi-1) == 0.  One wave scans the line in order and compacts the
// crossings with ballots, so they come out ascending; at most max_out are
// stored, out[0] receives their total count.  Evaluated without fused
// multiply-adds (the same roundings as the plain expression in double).
template <class T>
__global__ void __launch_bounds__(64) k_line_crossings(const T* phi, int v0, int stride, int shift, double t,
                                                       int lo, int hi, int max_out, double* out) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  int found = 0;
  for (int base = lo; base < hi; base += 64) {
    const int k = base + lane;
    double pos = 0.0;
    bool hit = false;
    if (k < hi) {
      auto prof = [&](int kk) {
        const double a = phi_dec(phi[v0 + kk * stride]);
        if (t == 0.0) return a;
        const double b = phi_dec(phi[v0 + shift + kk * stride]);
        return (1.0 - t) * a + t * b;
      };
      const double a = prof(k);
      if (a == 0.0) {
        hit = true;
        pos = (double)k;
      } else if (k + 1 < hi) {
        const double b = prof(k + 1);
        if (a * b < 0.0) {
          hit = true;
          pos = (double)k + ((double)(k + 1) - (double)k) * a / (a - b);
        }
      }
    }
    const unsigned long long m = __builtin_amdgcn_ballot_w64(hit);
    const int before = __builtin_popcountll(m & ((1ull << lane) - 1ull));
    if (hit && found + before < max_out) out[1 + found + before] = pos;
    found += __builtin_popcountll(m);
  }
  if (lane == 0) out[0] = (double)found;
}

// -------------------------------------------------------- state transfer
// Canonical pre-collision populations of the current state, as FP64 dense
// [Q][V] arrays (pull, bounce-back and faces applied; the compact layout is
// rebuilt in double).
template <class Real, int D, class In>
__global__ void k_export(StepParams P, Geo<Real> G, Grids<Real> R, In in, double* fr_out, double* fb_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const unsigned vf = ld_once(&G.vf[n]);
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  double fr[Q], fx[Q];
  load_node<D>(in, G.nbr, n, fr, fx);
  if constexpr (In::kPull) {
    if (D == 3 && (fl & (FL_IN | FL_OUT))) zou_he<kDev>(P, fl, phi_dec(R.phi[v]), fr, fx);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    fr_out[(size_t)i * P.V + v] = fr[i];
    fb_out[(size_t)i * P.V + v] = kDev ? ((Lat<D>::w(i) * P.rho0 + fx[i]) - fr[i]) : fx[i];
  }
}

// Pre-collision populations of the current state at their own nodes (pull,
// bounce-back and faces applied, as d_main sees them), in the staging layout
// of a state set from the host: (f^r, f^b) for double, (f^r, g) for float.
template <class Real, int D, class In>
__global__ void k_materialize(StepParams P, Geo<Real> G, Grids<Real> R, In in, Real* r_out, Real* x_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const unsigned vf = ld_once(&G.vf[n]);
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  // rebuilt and faced in double, stored in the staging precision
  double fr[Q], fx[Q];
  load_node<D>(in, G.nbr, n, fr, fx);
  if constexpr (In::kPull) {
    if (D == 3 && (fl & (FL_IN | FL_OUT))) zou_he<kDev>(P, fl, phi_dec(R.phi[v]), fr, fx);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    r_out[i * P.Np + n] = (Real)fr[i];
    x_out[i * P.Np + n] = (Real)fx[i];
  }
}

// Eqs. (37)-(38) on the staged pre-collision populations of the inlet nodes:
// the previously injected colour joins the newly injected one (to_red: red)
// and is cleared.  Float staging holds (f^r, g = f^t - w rho0): only f^r
// changes, to the total or to zero.
template <class Real, int D>
__global__ void k_switch_inlet(StepParams P, Geo<Real> G, Real* r, Real* x, int to_red) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  if (!(flags_of(G.vf[n]) & FL_IN)) return;
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    const int k = i * P.Np + n;
    if constexpr (kDev) {
      const Real tot = (Real)Lat<D>::w(i) * (Real)P.rho0 + x[k];
      r[k] = to_red ? tot : Real(0);
    } else {
      const Real a = r[k], b = x[k];
      r[k] = to_red ? a + b : Real(0);
      x[k] = to_red ? Real(0) : b + a;
    }
  });
}

// Dense FP64 canonical populations -> pre-collision staging at the nodes.
template <class Real, int D>
__global__ void k_import(StepParams P, Geo<Real> G, const double* fr, const double* fb, Real* r_out, Real* x_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const int v = vox_of(G.vf[n]);
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    const double a = fr[(size_t)i * P.V + v], b = fb[(size_t)i * P.V + v];
    r_out[i * P.Np + n] = (Real)a;
    x_out[i * P.Np + n] = kDev ? (Real)((a + b) - Lat<D>::w(i) * P.rho0) : (Real)b;
  });
}

// Rest state from a per-node phase: f^s_i = w_i rho^s, rho^r = rho0 (1 + phi)/2,
// rho^b = rho0 (1 - phi)/2.
template <class Real, int D>
__global__ void k_set_phase(StepParams P, const double* phi_nodes, Real* r_out, Real* x_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const double ph = phi_nodes[n];
  const double r = P.rho0 * (1.0 + ph) / 2.0;
  const double b = P.rho0 * (1.0 - ph) / 2.0;
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    constexpr double w = Lat<D>::w(i);
    const double fr = w * r, fb = w * b;
    r_out[i * P.Np + n] = (Real)fr;
    x_out[i * P.Np + n] = kDev ? (Real)((fr + fb) - w * P.rho0) : (Real)fb;
  });
}

// Phase-field grid (stored as PhiStore) -> dense FP64 array.
template <class T>
__global__ void k_grid_copy(int count, const T* grid, double* dst) {
  const int n = node_id();
  if (n >= count) return;
  dst[n] = phi_dec(grid[n]);
}

// Dense voxel grid of normals -> dense FP64 [3][V] array.
template <class Real>
__global__ void k_grid_copy3(int count, const Norm3<Real>* grid, double* dst) {
  const int n = node_id();
  if (n >= count) return;
  const Vec4<Real> q = n_get(grid, n);
  dst[n] = (double)q.x;
  dst[(size_t)count + n] = (double)q.y;
  dst[2 * (size_t)count + n] = (double)q.z;
}

}  // namespace cg
