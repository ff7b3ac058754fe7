// Device code of the discrete adjoint of one colour-gradient time step.
//
// The state at time t is the pair of pre-collision populations f^r_i, f^b_i at
// the fluid nodes; one step is the map t -> t+1 of Sec. II (phase field,
// extrapolations into the solid boundary points, wetting, curvature and force,
// velocity, collision, recolouring, pull streaming with halfway bounce-back).
// Given lambda_{t+1} = dJ/df_{t+1}, one reverse step forms
//   lambda_t = (d f_{t+1} / d f_t)^T lambda_{t+1}
// and accumulates the parameter adjoints (dF/dg)^T lambda, (dn/dtheta)^T lambda.
//
// The adjoint is kept in a compact form with the same structure as the
// forward map: lambda^r_i = L_i + R^r, lambda^b_i = L_i + R^b, where L_i is the
// adjoint of the total population (collision and streaming act on the total)
// and R^r, R^b collect everything that enters through the colour densities
// (phase field, recolouring fractions, rates).
//
// Every transposed stencil is written as a gather at the receiving node (no
// atomics; the result does not depend on thread order).  Reverse kernels of a
// step, after the forward stages of that step were recomputed from its state:
//   ka_node    reverse streaming (gather of lambda_{t+1} along the pull links,
//              bounce-back included), then the reverse of recolouring, of the
//              MRT/BGK collision with Guo forcing, of the velocity, of the
//              rates; writes L, the node-local density adjoints, lambda kappa,
//              lambda C from the force, lambda n from the recolouring
//   ka_curv    transpose of the curvature stencil (Eq. 12) into lambda n, at
//              fluid nodes and solid boundary points
//   ka_normal  transpose of the normal extrapolation (Eq. 35) into the fluid,
//              then the reverse of wetting (Scheme-I / Scheme-II, Jacobian from
//              a 4-lane forward-mode evaluation of the same code) and of
//              n = C/|C| (Eq. 27) into lambda C
//   ka_sb_phi  transpose of the colour-gradient stencil (Eq. 6) at the solid
//              boundary points
//   ka_phi     the same at fluid nodes, the transpose of the phase
//              extrapolation (Eq. 34), and phi = (rho^r - rho^b)/rho: writes R
//   ka_face    (Zou-He runs) the transpose of the faces of Appendix B at the
//              inlet and outlet nodes, which turns the adjoint of their
//              post-face populations into the adjoint of the pulled ones
//
// Zou-He faces.  The state at a face node is the pulled populations; the
// faces (Eqs. B.1-B.18) then set the unknown directions, so the node's own
// reverse (ka_face_node) runs on the post-face populations and ka_face maps
// the result back through the face.  At the inlet the face fixes both colour
// densities (rho_in zeta^s), so the adjoint of every known pulled population
// is the same for both colours and R is zero there.  At the outlet the
// adjoint of a pulled population along +z is L_i + 2 R^s (the direction and
// its reflected unknown both carry the node's density), in the plane L_i +
// R^s; the reverse streaming applies that factor 2.  The outlet's chi^s and
// its phase (Eq. 39) both come from the node upstream, whose density adjoint
// receives their share.  The gradient stencils clamp at the open faces (the
// face layer stands in for the missing one), so their transposes mirror e_z
// on the clamped links.
#pragma once

#include "kernels.hpp"

namespace cg {

// ------------------------------------------------------- forward-mode lanes
// A value with four directional derivatives.  Branches compare values only,
// so the lanes are the derivative of the branch the value takes.
template <class S>
struct Tan4 {
  S v;
  S d[4];
  __device__ __forceinline__ Tan4() : v(S(0)), d{S(0), S(0), S(0), S(0)} {}
  __device__ __forceinline__ Tan4(double a) : v(S(a)), d{S(0), S(0), S(0), S(0)} {}
};
template <class S>
__device__ __forceinline__ Tan4<S> operator+(const Tan4<S>& a, const Tan4<S>& b) {
  Tan4<S> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <class S>
__device__ __forceinline__ Tan4<S> operator-(const Tan4<S>& a, const Tan4<S>& b) {
  Tan4<S> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <class S>
__device__ __forceinline__ Tan4<S> operator-(const Tan4<S>& a) {
  Tan4<S> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = -a.d[k];
  return r;
}
template <class S>
__device__ __forceinline__ Tan4<S> operator*(const Tan4<S>& a, const Tan4<S>& b) {
  Tan4<S> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <class S>
__device__ __forceinline__ Tan4<S> operator/(const Tan4<S>& a, const Tan4<S>& b) {
  const S q = a.v / b.v;
  const S ib = S(1) / b.v;
  Tan4<S> r;
  r.v = q;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = (a.d[k] - q * b.d[k]) * ib;
  return r;
}
template <class S>
__device__ __forceinline__ bool operator<=(const Tan4<S>& a, const Tan4<S>& b) {
  return a.v <= b.v;
}
template <class S>
__device__ __forceinline__ bool operator<(const Tan4<S>& a, const Tan4<S>& b) {
  return a.v < b.v;
}
template <class S>
__device__ __forceinline__ Tan4<S> sqrt(const Tan4<S>& a) {
  const S s = ::sqrt(a.v);
  Tan4<S> r;
  r.v = s;
  const S h = s > S(0) ? S(0.5) / s : S(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * h;
  return r;
}
template <class S>
__device__ __forceinline__ Tan4<S> fabs(const Tan4<S>& a) {
  return a.v < S(0) ? -a : a;
}

// --------------------------------------------------------------- buffers
template <class Real>
struct Vec2T;
template <>
struct Vec2T<float> {
  using type = float2;
};
template <>
struct Vec2T<double> {
  using type = double2;
};
template <class Real>
using Vec2 = typename Vec2T<Real>::type;

struct AdjParams {
  double delta;  // floor of |C| in the Jacobian of C/|C| (0: exact)
  int objective; // 0 saturation, 1 red volume, 2 plane flux
  int axis, lo, hi;
};

template <class Real>
struct AdjBufs {
  const Real* lf_in;   // [Q][Np] L at t+1
  Real* lf_out;        // [Q][Np] L at t
  Vec2<Real>* lr;      // [Np] (R^r, R^b): read at t+1 by ka_node, rewritten at t by ka_phi
  Vec4<Real>* na;      // [Np] density adjoints of the node part, dphi/drho^r, dphi/drho^b
  Vec4<Real>* lcf;     // [Np] lambda C (after wetting) from the force
  Real* lk;            // [V] lambda kappa at fluid voxels, 0 elsewhere
  Vec4<Real>* ln;      // [V] lambda n at fluid voxels and solid boundary points
  Vec4<Real>* lc;      // [V] lambda C (before wetting) at fluid voxels, 0 elsewhere
  Real* lphi;          // [V] lambda phi / (sum of link weights) at solid boundary points, 0 elsewhere
  const Real* iden;    // [V] 1 / (sum of fluid-link weights) at solid boundary points, 0 elsewhere
  const double* idf;   // [Np] 1 / (sum of solid-link weights) at fluid boundary points, 0 elsewhere
  double* pacc;        // [blocks][kPaccCols] per-block sums over steps of lambda F (xyz), lambda theta
                       // (per degree), lambda rho_in, lambda rho_out
  double* lth;         // [V] sum over steps of lambda theta * idf at fluid boundary voxels
  Real* lpo;           // [n_out] lambda phi of each outlet node (its phase is the node's upstream, Eq. 39)
  Real* ljt;           // [n_out] j^t of each outlet node's face (Eq. B.9), for ka_face
  int face_pull;       // the state of this step is a pulled one (the faces were applied to it)
};

// j^t of an outlet node from its pulled totals (canonical totals, or the
// deviations g of the compact state, whose known weights sum to 1).
template <bool kDev, class CT>
__device__ __forceinline__ CT outlet_jt(const StepParams& P, const CT* ft) {
  const CT S = ft[0] + ft[1] + ft[2] + ft[3] + ft[4] + ft[7] + ft[8] + ft[9] + ft[10];
  const CT T = ft[5] + ft[11] + ft[12] + ft[15] + ft[16];
  return -(CT)(kDev ? P.rho_out - P.rho0 : P.rho_out) + (S + CT(2) * T);
}

// Columns of the per-block parameter sums.
constexpr int kPaccCols = 6;
constexpr int kColTheta = 3, kColRhoIn = 4, kColRhoOut = 5;

// A link of p whose z step is clamped at an open face: the forward gradient
// stencils read the face layer itself there (zero-gradient ghost), so in
// their transposes the relation runs within the layer, with e_z mirrored.
// Only the z faces can be open; walls bound the other axes (a fluid node
// never clamps there, and the solid voxels it would reach hold no adjoint).
template <int D, int j>
__device__ __forceinline__ bool clamped_z(const StepParams& P, const Pos& p) {
  if constexpr (D != 3) {
    return false;
  } else {
    constexpr int ez = Lat<D>::e(j, 2);
    if constexpr (ez == 0) {
      return false;
    } else {
      return p.face && P.per[2] == 0 && (ez < 0 ? p.z == 0 : p.z == P.nz - 1);
    }
  }
}

__device__ __forceinline__ int coord_of(const StepParams& P, int v, int axis) {
  const int nxy = P.nx * P.ny;
  const int z = v / nxy, r = v - z * nxy, y = r / P.nx, x = r - y * P.nx;
  return axis == 0 ? x : (axis == 1 ? y : z);
}

template <int D, class Real>
__device__ __forceinline__ void nbr_all(const Geo<Real>& G, int n, int* src) {
  G.nbr.template all<Lat<D>::Q>(n, src);
}

// Colour densities of populations fr (red) and fx (blue for the FP64 state;
// g = f^t - w rho0 for the compact FP32 state).
template <class Real, int D>
__device__ __forceinline__ void adj_sums(const StepParams& P, const Real* fr, const Real* fx, Real& rr, Real& rb,
                                         Real& rho) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  Real a = fr[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) a = a + fr[i];
  rr = a;
  if constexpr (kDev) {
    Real t = (Real)Lat<D>::w(0) * (Real)P.rho0 + fx[0];
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      t = t + ((Real)Lat<D>::w(i) * (Real)P.rho0 + fx[i]);
    });
    rho = t;
    rb = t - a;
  } else {
    Real b = fx[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) b = b + fx[i];
    rb = b;
    rho = a + b;
  }
}

// Pulled populations of node n of the state `in` and their colour densities.
template <class Real, int D, class In>
__device__ __forceinline__ void adj_load(const StepParams& P, const Geo<Real>& G, const In& in, int n, Real* fr,
                                         Real* fx, Real& rr, Real& rb, Real& rho) {
  load_node<D>(in, G.nbr, n, fr, fx);
  adj_sums<Real, D>(P, fr, fx, rr, rb, rho);
}

// The same with the Zou-He faces applied at a face node of a pulled state
// (Appendix B): the populations the collision of the next step takes, and
// the state as the oracle holds it.  The outlet's stored phase is the
// upstream node's (Eq. 39), set by the phase stages of this state.
template <class Real, int D, class In>
__device__ __forceinline__ void adj_load_faced(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R,
                                               const In& in, int n, Real* fr, Real* fx, Real& rr, Real& rb,
                                               Real& rho) {
  load_node<D>(in, G.nbr, n, fr, fx);
  if constexpr (D == 3 && In::kPull) {
    const unsigned vf = G.vf[n];
    const unsigned fl = flags_of(vf);
    if (fl & (FL_IN | FL_OUT))
      zou_he<sizeof(Real) == 4>(P, fl, (Real)phi_dec(R.phi[vox_of(vf)]), fr, fx);
  }
  adj_sums<Real, D>(P, fr, fx, rr, rb, rho);
}

// ------------------------------------------------------------------ ka_node
// Streaming form, three passes over the directions so that few per-direction
// values stay live:
//   pass 1  gather (delta_i, mu_i) = (lambda c^r_i - lambda c^b_i,
//           lambda c^b_i + a delta_i) of the post-collision populations, form
//           y_i = f_i - f^eq_i + Fbar_i/2 and accumulate the moments M y,
//           M delta, M mu and the recolouring adjoints;
//   between lambda a = sum_i f''_i delta_i with f'' = f + Fbar - M^-1 S M y
//           (BGK: M = I, S = S_nu), the rate adjoints lambda S_k = -(M mu)_k (M y)_k / |M_k|^2;
//   pass 2  lambda y_i = -(M^T S M^-T mu)_i, lambda f_i = mu_i + lambda y_i,
//           lambda f^eq_i = -lambda y_i, lambda Fbar_i = mu_i + lambda y_i / 2
//           and their contributions to lambda rho, lambda u, lambda F;
//   pass 3  lambda f_i += e_i . lambda j (velocity, Eq. 22), store L.
// kSeed: no lambda_{t+1}; the plane-flux objective J = sum (j + F/2)_axis is
// seeded at the plane nodes instead (terminal condition of objective 2).
// kFaceMode, runs with Zou-He faces: 1, the reverse streaming reads
// lambda_{t+1} in its face form (open links carry nothing, the outlet's +z
// populations weigh R twice); 2, the state at t is a pulled one as well: the
// face nodes are skipped here and done by the kFace instantiation, which
// runs on their post-face populations.
// lF receives this node's lambda F (summed per block by the caller).
template <class Real, int D, bool kSeed, bool kMrt, int kFaceMode, bool kFace, class In>
__device__ __forceinline__ void d_adj_node(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R,
                                           const In& in, const AdjBufs<Real>& A, const AdjParams& AP, int n,
                                           double* lFout) {
  static_assert(D == 3 || !kMrt, "MRT is defined for D3Q19");
  static_assert(kFaceMode == 0 || D == 3, "the faces are those of D3Q19 runs");
  static_assert(kFaceMode < 2 || In::kPull, "the faces act on pulled states");
  static_assert(kFaceMode == 2 || !kFace, "face nodes are handled apart for pulled states only");
  constexpr bool kFaces = kFaceMode >= 1;
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  using CT = Real;
  const unsigned vf = G.vf[n];
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  if constexpr (kFaceMode == 2 && !kFace) {
    if (fl & (FL_IN | FL_OUT)) return;
  }
  const CT rho0 = (CT)P.rho0;
  // pull-table entries of the node (the reverse streaming uses them too)
  int src[Q];
  nbr_all<D>(G, n, src);
  // state at t: x_i = f^t_i (canonical) or g_i = f^t_i - w_i rho0 (compact).
  // The compact state needs only the totals here: rho^r follows from the
  // phase field k_phase computed from the same state, rho^r = rho (1 + phi)/2.
  CT x[Q];
  CT rr, rb, rho, drho;
  if constexpr (kDev) {
    if constexpr (kFace) {
      // per-colour pull with the faces applied, as the step kernel takes
      // them; rho^r is the post-face red sum (the node's phase is not its own)
      Real fr[Q];
      load_node<D>(in, G.nbr, n, fr, x);
      if (fl & FL_OUT) A.ljt[n - (P.N - P.n_out)] = outlet_jt<true>(P, x);
      zou_he<true>(P, fl, (Real)phi_dec(R.phi[v]), fr, x);
      CT a = fr[0];
#pragma unroll
      for (int i = 1; i < Q; ++i) a = a + fr[i];
      rr = a;
    } else if constexpr (In::kPull) {
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (i == 0) {
          x[0] = (CT)in.T[n];
        } else {
          const int s = src[i];
          x[i] = (CT)(s >= 0 ? in.T[i * P.Np + s] : in.T[opp<D>(i) * P.Np + n]);
        }
      });
    } else {
      // a state set at the nodes holds the red populations themselves: rho^r
      // is their sum, as the step takes it (at the face nodes the stored
      // phase is not the node's own ratio)
      CT a = CT(0);
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        CT r, g;
        in.template get<i>(n, r, g);
        x[i] = g;
        a = a + r;
      });
      rr = a;
    }
    CT t = (CT)Lat<D>::w(0) * rho0 + x[0];
    CT sg = x[0];
    unroll<Q - 1>([&](auto I) {
      constexpr int i = I + 1;
      t = t + ((CT)Lat<D>::w(i) * rho0 + x[i]);
      sg = sg + x[i];
    });
    rho = t;
    drho = sg;
    if constexpr (!kFace && In::kPull) rr = rho * (CT(1) + (CT)phi_dec(R.phi[v])) * CT(0.5);
    rb = rho - rr;
  } else {
    Real fr[Q], fx[Q];
    load_node<D>(in, G.nbr, n, fr, fx);
    if constexpr (kFace) {
      if (fl & FL_OUT) {
        CT ft[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) ft[i] = fr[i] + fx[i];
        A.ljt[n - (P.N - P.n_out)] = outlet_jt<false>(P, ft);
      }
      zou_he<false>(P, fl, (Real)phi_dec(R.phi[v]), fr, fx);
    }
    CT a = fr[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) a = a + (CT)fr[i];
    CT b = fx[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) b = b + (CT)fx[i];
    rr = a;
    rb = b;
    rho = a + b;
    drho = rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = (CT)fr[i] + (CT)fx[i];
  }
  const CT rho_u = kDev ? rho0 + drho : rho;
  const Vec4<Real> f4 = R.f[n];
  const Vec4<Real> n4 = n_get(R.n, v);
  const CT F[3] = {(CT)f4.x, (CT)f4.y, (CT)f4.z};
  const CT kap = (CT)f4.w;
  const CT nv[3] = {(CT)n4.x, (CT)n4.y, (CT)n4.z};
  const CT phi = (CT)phi_dec(R.phi[v]);
  CT u[3] = {CT(0), CT(0), CT(0)};
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    CT j = CT(0);
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int e = Lat<D>::e(i, a);
      if constexpr (e == 1) j = j + x[i];
      if constexpr (e == -1) j = j - x[i];
    });
    u[a] = (j + CT(0.5) * F[a]) / rho_u;
  });
  CT usq = u[0] * u[0] + u[1] * u[1];
  if constexpr (D == 3) usq = usq + u[2] * u[2];
  CT s_nu, s_q;
  rates(P, phi, s_nu, s_q);
  const CT ra = rr / rho;
  const CT rbb = rr * rb / rho;

  // ---- y = f - f^eq + Fbar/2 per direction and, for MRT, its projections.
  // The relaxation part of the MRT operator is R = M^-1 S M =
  // S_nu P_e + S_q P_o (see collide_mrt_pairs): P_e takes the half-sum over a
  // pair (i, opp(i)) minus the mean over all 19, P_o the half-difference minus
  // the projection on the momentum rows.  Both are symmetric projections, so
  // R^T = R; the adjoint needs dl.R y (for lambda a), mu.P_e y and mu.P_o y
  // (the rates) and R mu (the adjoint of y).  Ey[L] / Oy[L] hold (P_e y) and
  // (P_o y) at the pair leader L = min(i, opp(i)); (P_o y) changes sign on the
  // partner.
  // bg_i = f_i + Fbar_i, the factor of the recolouring adjoint in lambda a
  CT yv[Q], bg[Q];
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    constexpr double w = Lat<D>::w(i);
    const CT gu = guo_i<D, i>(u, F);
    yv[i] = x[i] - eq_i<D, i>(drho, rho0, u, usq) + CT(0.5) * gu;
    bg[i] = (kDev ? (CT)w * rho0 + x[i] : x[i]) + gu;
  });
  CT Ey[kMrt ? Q : 1], Oy[kMrt ? Q : 1];
  if constexpr (kMrt) {
    static_assert(mrt_pair_structure(), "D3Q19 moment basis lost its even/odd structure");
    CT sy = yv[0];
    CT Jy[3] = {CT(0), CT(0), CT(0)};
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int o = opp<D>(i);
      if constexpr (i > 0 && o > i) {
        sy = sy + (yv[i] + yv[o]);
        unroll<3>([&](auto A_) {
          constexpr int a = A_;
          constexpr int e = Lat<D>::e(i, a);
          if constexpr (e == 1) Jy[a] = Jy[a] + (yv[i] - yv[o]);
          if constexpr (e == -1) Jy[a] = Jy[a] - (yv[i] - yv[o]);
        });
      }
    });
    const CT ybar = sy * CT(1.0 / 19.0);
    Ey[0] = yv[0] - ybar;
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int o = opp<D>(i);
      if constexpr (i > 0 && o > i) {
        CT eJ = CT(0);
        unroll<3>([&](auto A_) {
          constexpr int a = A_;
          constexpr int e = Lat<D>::e(i, a);
          if constexpr (e == 1) eJ = eJ + Jy[a];
          if constexpr (e == -1) eJ = eJ - Jy[a];
        });
        Ey[i] = CT(0.5) * (yv[i] + yv[o]) - ybar;
        Oy[i] = CT(0.5) * (yv[i] - yv[o]) - CT(0.1) * eJ;
      }
    });
  }
  // ---- pass 1: the adjoint arriving from t+1 along the reversed pull
  CT mu[Q];
  CT a1 = CT(0), lb = CT(0), lnr[3] = {CT(0), CT(0), CT(0)};
  CT dRy = CT(0), mPe = CT(0), mPo = CT(0);  // MRT: dl.R y, mu.P_e y, mu.P_o y
  CT my0 = CT(0), md0 = CT(0);               // BGK: mu.y, y.dl
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    constexpr double w = Lat<D>::w(i);
    // reverse streaming: c_i(x) became f_i(x + e_i) when that voxel is fluid,
    // else f_opp(i)(x) (halfway bounce-back)
    CT dl = CT(0), m = CT(0);
    if constexpr (!kSeed) {
      int li, ri;
      // zf, the weight of R at the target: 2 for a pulled +z population of an
      // outlet node, 0 for a -z one (an unknown of the face; the link it
      // stands for left through the open face), 1 elsewhere.  A link that
      // left through the inlet reads an unknown of the inlet node, whose L
      // and R the face transpose set to zero.
      CT zf = CT(1);
      if constexpr (i == 0) {
        li = n;
        ri = n;
      } else {
        constexpr int o = opp<D>(i);
        const int s = src[o];  // node at x - e_o = x + e_i
        ri = s >= 0 ? s : n;
        int row = s >= 0 ? i * P.Np : o * P.Np;
        // opaque to the optimiser, which would otherwise split the selects
        // into branches that wait for earlier loads
        asm("" : "+v"(ri), "+v"(row));
        li = row + ri;
        if constexpr (kFaces) {
          constexpr int ez = Lat<D>::e(i, 2);
          if constexpr (ez != 0) {
            const CT zo = s >= 0 ? CT(1 + ez) : CT(1 - ez);
            zf = ri >= P.N - P.n_out ? zo : CT(1);
          }
        }
      }
      const CT l = A.lf_in[li];
      const Vec2<Real> r = A.lr[ri];
      dl = zf * ((CT)r.x - (CT)r.y);
      m = l + zf * (CT)r.y + ra * dl;
    }
    a1 = a1 + bg[i] * dl;
    if constexpr (kMrt) {
      constexpr int L = i < opp<D>(i) ? i : opp<D>(i);
      const CT pe = Ey[L];
      if constexpr (i == 0) {
        dRy = dRy + s_nu * pe * dl;
        mPe = mPe + m * pe;
      } else {
        const CT po = i == L ? Oy[L] : -Oy[L];
        dRy = dRy + (s_nu * pe + s_q * po) * dl;
        mPe = mPe + m * pe;
        mPo = mPo + m * po;
      }
    } else {
      md0 = md0 + yv[i] * dl;
      my0 = my0 + m * yv[i];
    }
    mu[i] = m;
    if constexpr (i > 0) {
      CT en = CT(0);
      unroll<D>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<D>::e(i, a);
        if constexpr (e == 1) en = en + nv[a];
        if constexpr (e == -1) en = en - nv[a];
      });
      const CT q = (CT)(P.beta * w) * dl;
      lb = lb + q * en;
      unroll<D>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<D>::e(i, a);
        if constexpr (e == 1) lnr[a] = lnr[a] + q;
        if constexpr (e == -1) lnr[a] = lnr[a] - q;
      });
    }
  });
  // ---- lambda a, the rate adjoints and R mu
  CT la, lsnu, lsq = CT(0);
  CT lyv[kMrt ? Q : 1];
  if constexpr (kMrt) {
    la = a1 - dRy;
    lsnu = -mPe;
    lsq = -mPo;
    CT sm = mu[0];
    CT Jm[3] = {CT(0), CT(0), CT(0)};
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int o = opp<D>(i);
      if constexpr (i > 0 && o > i) {
        sm = sm + (mu[i] + mu[o]);
        unroll<3>([&](auto A_) {
          constexpr int a = A_;
          constexpr int e = Lat<D>::e(i, a);
          if constexpr (e == 1) Jm[a] = Jm[a] + (mu[i] - mu[o]);
          if constexpr (e == -1) Jm[a] = Jm[a] - (mu[i] - mu[o]);
        });
      }
    });
    const CT mbar = sm * CT(1.0 / 19.0);
    lyv[0] = -s_nu * (mu[0] - mbar);
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int o = opp<D>(i);
      if constexpr (i > 0 && o > i) {
        CT eJ = CT(0);
        unroll<3>([&](auto A_) {
          constexpr int a = A_;
          constexpr int e = Lat<D>::e(i, a);
          if constexpr (e == 1) eJ = eJ + Jm[a];
          if constexpr (e == -1) eJ = eJ - Jm[a];
        });
        const CT Em = CT(0.5) * (mu[i] + mu[o]) - mbar;
        const CT Om = CT(0.5) * (mu[i] - mu[o]) - CT(0.1) * eJ;
        lyv[i] = -(s_nu * Em + s_q * Om);
        lyv[o] = -(s_nu * Em - s_q * Om);
      }
    });
  } else {
    la = a1 - s_nu * md0;
    lsnu = -my0;
  }
  // ---- pass 2: adjoints of f^eq and Fbar with respect to rho, u and F.
  // With qe_i = w_i rho0 lambda_feq,i and qg_i = w_i lambda_Fbar,i,
  //   lambda u = sum_i e_i [3 qe_i + 9 (qe_i e_i.u + qg_i e_i.F)] - 3 u sum qe - 3 F sum qg,
  //   lambda F = sum_i e_i [3 qg_i + 9 qg_i e_i.u]                 - 3 u sum qg,
  // (f^eq_i = w [drho + rho0 (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)],
  //  Fbar_i = w [3 (e - u).F + 9 (e.u)(e.F)]), so each direction adds two
  // scalars along e_i.
  CT lrho = CT(0), lu[3] = {CT(0), CT(0), CT(0)}, lF[3] = {CT(0), CT(0), CT(0)};
  CT sqe = CT(0), sqg = CT(0);
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    constexpr double w = Lat<D>::w(i);
    CT ly;
    if constexpr (kMrt) {
      ly = lyv[i];
    } else {
      ly = -s_nu * mu[i];
    }
    const CT lfe = -ly;
    const CT lgu = mu[i] + CT(0.5) * ly;
    lrho = lrho + (CT)w * lfe;
    const CT qe = (CT)w * lfe * rho0;
    const CT qg = (CT)w * lgu;
    sqe = sqe + qe;
    sqg = sqg + qg;
    if constexpr (i > 0) {
      CT eu = CT(0), eF = CT(0);
      unroll<D>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<D>::e(i, a);
        if constexpr (e == 1) {
          eu = eu + u[a];
          eF = eF + F[a];
        }
        if constexpr (e == -1) {
          eu = eu - u[a];
          eF = eF - F[a];
        }
      });
      const CT Au = CT(3) * qe + CT(9) * (qe * eu + qg * eF);
      const CT AF = CT(3) * qg + CT(9) * qg * eu;
      unroll<D>([&](auto A_) {
        constexpr int a = A_;
        constexpr int e = Lat<D>::e(i, a);
        if constexpr (e == 1) {
          lu[a] = lu[a] + Au;
          lF[a] = lF[a] + AF;
        }
        if constexpr (e == -1) {
          lu[a] = lu[a] - Au;
          lF[a] = lF[a] - AF;
        }
      });
    }
    mu[i] = mu[i] + ly;  // lambda f_i (total) before the velocity term
  });
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lu[a] = lu[a] - CT(3) * (u[a] * sqe + F[a] * sqg);
    lF[a] = lF[a] - CT(3) * u[a] * sqg;
  }
  // rates, Eqs. (13)-(16): S_nu(phi), S_q(S_nu)
  {
    const CT inv_nu = (CT(1) + phi) / (CT(2) * (CT)P.nu_r) + (CT(1) - phi) / (CT(2) * (CT)P.nu_b);
    const CT nuv = CT(1) / inv_nu;
    const CT dinv = CT(1) / (CT(2) * (CT)P.nu_r) - CT(1) / (CT(2) * (CT)P.nu_b);
    const CT dsdphi = CT(3) * s_nu * s_nu * nuv * nuv * dinv;
    const CT dq = CT(-48) / ((CT(8) - s_nu) * (CT(8) - s_nu));
    lsnu = (lsnu + lsq * dq) * dsdphi;  // now lambda phi (node part)
  }
  // velocity, Eq. (22): u = (j + F/2) / rho
  CT lj[3] = {CT(0), CT(0), CT(0)};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lj[a] = lu[a] / rho_u;
    lF[a] = lF[a] + CT(0.5) * lj[a];
    lrho = lrho - lj[a] * u[a];
  }
  if constexpr (kSeed) {
    if (coord_of(P, v, AP.axis) == AP.lo) {
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (a == AP.axis) {
          lj[a] = lj[a] + CT(1);
          lF[a] = lF[a] + CT(0.5);
        }
    }
  }
  // ---- pass 3: store L
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    CT t = mu[i];
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      constexpr int e = Lat<D>::e(i, a);
      if constexpr (e == 1) t = t + lj[a];
      if constexpr (e == -1) t = t - lj[a];
    });
    A.lf_out[i * P.Np + n] = t;
  });
  // recolouring fractions a = rho^r/rho, b = rho^r rho^b / rho; rho = rho^r + rho^b
  const CT irho = CT(1) / rho;
  CT lrr = la * irho + lb * rb * irho;
  CT lrb = lb * rr * irho;
  lrho = lrho - (la * ra + lb * rbb) * irho;
  lrr = lrr + lrho;
  lrb = lrb + lrho;
  // phi = (rho^r - rho^b) / rho, except at an inlet node (phi_in) and an
  // outlet node (the upstream node's phase, Eq. 39): their lambda phi does
  // not reach their own densities; the outlet's goes to the node upstream
  // (ka_face; not needed for the first step of the call, whose adjoint is
  // not used)
  bool own = true;
  if constexpr (D == 3) own = !(fl & (FL_IN | FL_OUT));
  const CT dr = own ? CT(2) * rb * irho * irho : CT(0);
  const CT db = own ? CT(-2) * rr * irho * irho : CT(0);
  Vec4<Real> na;
  na.x = lrr + lsnu * dr;
  na.y = lrb + lsnu * db;
  na.z = dr;
  na.w = db;
  A.na[n] = na;
  if constexpr (kFace) {
    if (fl & FL_OUT) A.lpo[n - (P.N - P.n_out)] = lsnu;
  }
  // force F = sigma/2 kappa C + rho0 g
  const Vec4<Real> c4 = n_get(R.c, n);
  const CT Cv[3] = {(CT)c4.x, (CT)c4.y, (CT)c4.z};
  CT lkap = CT(0);
#pragma unroll
  for (int a = 0; a < D; ++a) lkap = lkap + lF[a] * Cv[a];
  A.lk[v] = lkap * (CT)P.half_sigma;
  const CT hk = (CT)P.half_sigma * kap;
  Vec4<Real> q;
  q.x = hk * lF[0];
  q.y = hk * lF[1];
  q.z = D == 3 ? hk * lF[2] : Real(0);
  q.w = Real(0);
  A.lcf[n] = q;
  Vec4<Real> l4;
  l4.x = lnr[0] * rbb;
  l4.y = lnr[1] * rbb;
  l4.z = D == 3 ? lnr[2] * rbb : Real(0);
  l4.w = Real(0);
  A.ln[v] = l4;
#pragma unroll
  for (int a = 0; a < D; ++a) lFout[a] = (double)lF[a];
}

// Per-block sums of this step's parameter adjoints, added to the block's own
// accumulator row (same block -> same tile every launch: deterministic).
template <int BS, int NC>
__device__ __forceinline__ void block_accumulate(const double* vals, int col0, double* pacc) {
  __shared__ double sh[BS / 64];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double t = block_sum<BS>(vals[c], sh);
    if (threadIdx.x == 0) pacc[blockIdx.x * kPaccCols + col0 + c] += t;
  }
}

// Three waves per SIMD: without the hint the compiler keeps every gather of
// the node in flight in 221 VGPRs (two waves); with it 158 VGPRs, no spills
// (four waves would spill).
template <class Real, int D, bool kSeed, bool kMrt, int kFaceMode, class In>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
ka_node(StepParams P, Geo<Real> G, Grids<Real> R, In in, AdjBufs<Real> A, AdjParams AP) {
  const int n = node_id_plain();
  double lF[3] = {0.0, 0.0, 0.0};
  if (n < P.N) d_adj_node<Real, D, kSeed, kMrt, kFaceMode, false, In>(P, G, R, in, A, AP, n, lF);
  block_accumulate<256, 3>(lF, 0, A.pacc);
}

// The same at the Zou-He face nodes of a pulled state, one wave per 64-node
// tile that holds face nodes (the pull table decodes per tile).
template <class Real, int D, bool kSeed, bool kMrt, class In>
__global__ void __launch_bounds__(256)
ka_face_node(StepParams P, Geo<Real> G, Grids<Real> R, In in, AdjBufs<Real> A, AdjParams AP) {
  const int n = face_node(P, node_id_plain());
  double lF[3] = {0.0, 0.0, 0.0};
  if (n >= 0) d_adj_node<Real, D, kSeed, kMrt, 2, true, In>(P, G, R, in, A, AP, n, lF);
  block_accumulate<256, 3>(lF, 0, A.pacc);
}

// ------------------------------------------------------------------ ka_curv
// kappa(x) = sum_ab (n_a n_b - delta_ab) d_b n_a with d_b n_a = 3 sum_i w_i e_ib n_a(x + e_i):
//   at y = x + e_i: lambda n_a(y) += 3 w_i lambda kappa(x) (n_a(x) (e_i.n(x)) - e_ia)
//   at x itself:    lambda n_a(x) += lambda kappa(x) sum_b (d_b n_a + d_a n_b) n_b
// Written as a gather at y over x = y + e_j (e_j = -e_i); on a link clamped
// at an open face x lies in y's layer and e_j enters mirrored in z (the own
// stencil d keeps e_j: it is y's forward stencil).
template <class Real, int D, bool kSb>
__device__ __forceinline__ void d_adj_curv(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R,
                                           const AdjBufs<Real>& A, int idx) {
  constexpr int Q = Lat<D>::Q;
  using CT = Real;
  int v;
  bool face;
  if constexpr (kSb) {
    if (idx >= P.nsb) return;
    v = G.sb_vox[idx];
    face = G.sb_mask[idx] & 1u;
  } else {
    if (idx >= P.N) return;
    const unsigned vf = G.vf[idx];
    v = vox_of(vf);
    face = flags_of(vf) & FL_FACE;
  }
  const Pos ps = make_pos(P, v, face);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  CT acc[3] = {CT(0), CT(0), CT(0)};
  CT d[3][3] = {{CT(0), CT(0), CT(0)}, {CT(0), CT(0), CT(0)}, {CT(0), CT(0), CT(0)}};
  // a solid boundary point gathers from its fluid links only (lambda kappa is
  // zero on every other voxel, so the skipped terms are exact zeros): masked
  // buffer loads, all in flight together
  [[maybe_unused]] unsigned msk = 0;
  [[maybe_unused]] __amdgpu_buffer_rsrc_t rn, rk;
  if constexpr (kSb) {
    msk = G.sb_mask[idx];
    rn = grid_rsrc(R.n, sizeof(Norm3<Real>) * (size_t)P.V);
    rk = grid_rsrc(A.lk, sizeof(Real) * (size_t)P.V);
  }
  unroll<Q - 1>([&](auto J) {
    constexpr int j = J + 1;
    constexpr double w = Lat<D>::w(j);
    const int x = nbi[j];
    const bool cl = clamped_z<D, j>(P, ps);
    Vec4<Real> q;
    CT lk;
    if constexpr (kSb) {
      const bool on = (msk & (1u << j)) || cl;
      q = bload3<Real>(rn, on ? (uint32_t)x * (uint32_t)sizeof(Norm3<Real>) : kOffNone);
      lk = bload1(rk, on ? (uint32_t)x * (uint32_t)sizeof(Real) : kOffNone, Real(0));
    } else {
      q = n_get(R.n, x);
      lk = (CT)A.lk[x];
    }
    const CT nq[3] = {(CT)q.x, (CT)q.y, (CT)q.z};
    // e_j, mirrored in z on a clamped link
    CT ej[3];
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      constexpr CT e = (CT)Lat<D>::e(j, a);
      ej[a] = (a == 2 && cl) ? -e : e;
    });
    CT en = CT(0);
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      en = en + ej[a] * nq[a];
    });
    const CT c = (CT)(3.0 * w) * lk;
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      acc[a] = acc[a] + c * (ej[a] - nq[a] * en);
    });
    if constexpr (!kSb) {
      unroll<D>([&](auto B_) {
        constexpr int b = B_;
        constexpr int e = Lat<D>::e(j, b);
        if constexpr (e != 0) {
          unroll<D>([&](auto A_) {
            constexpr int a = A_;
            d[b][a] = d[b][a] + (CT)(3.0 * w * e) * nq[a];
          });
        }
      });
    }
  });
  Vec4<Real> o;
  if constexpr (!kSb) {
    const Vec4<Real> s4 = n_get(R.n, v);
    const CT ns[3] = {(CT)s4.x, (CT)s4.y, (CT)s4.z};
    const CT lk = (CT)A.lk[v];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      CT t = CT(0);
#pragma unroll
      for (int b = 0; b < D; ++b) t = t + (d[b][a] + d[a][b]) * ns[b];
      acc[a] = acc[a] + lk * t;
    }
    o = A.ln[v];
    o.x = o.x + acc[0];
    o.y = o.y + acc[1];
    if constexpr (D == 3) o.z = o.z + acc[2];
  } else {
    o.x = acc[0];
    o.y = acc[1];
    o.z = D == 3 ? acc[2] : CT(0);
    o.w = Real(0);
  }
  A.ln[v] = o;
}

// The fluid nodes and the solid boundary points in one launch: the first nfb
// blocks take the fluid nodes, the others the solid boundary points, so each
// block runs one of the two code paths and the short solid-boundary part
// overlaps the tail of the fluid part (the two write disjoint voxels and
// read only what the node stage wrote).  A launch over both lists with the
// choice made per thread measured slower than two launches (56 against
// 28 + 17 us at 128^3); this split per block saves about 5 us per step.
template <class Real, int D>
__global__ void ka_curv(StepParams P, Geo<Real> G, Grids<Real> R, AdjBufs<Real> A, int nfb) {
  if ((int)blockIdx.x < nfb)
    d_adj_curv<Real, D, false>(P, G, R, A, node_id_plain());
  else
    d_adj_curv<Real, D, true>(P, G, R, A, ((int)blockIdx.x - nfb) * (int)blockDim.x + (int)threadIdx.x);
}

// ---------------------------------------------------------------- ka_normal
template <class Real, int D>
__device__ __forceinline__ void d_adj_normal(const StepParams& P, const Geo<Real>& G, const Grids<Real>& R,
                                             const AdjBufs<Real>& A, const AdjParams& AP, int n, double* lthout) {
  constexpr int Q = Lat<D>::Q;
  using CT = Real;
  using TT = Tan4<Real>;
  const unsigned vf = G.vf[n];
  const int v = vox_of(vf);
  const unsigned fl = flags_of(vf);
  const Pos ps = make_pos(P, v, fl & FL_FACE);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  const double idf = A.idf[n];
  // lambda n: own part plus the transpose of Eq. (35) from the solid boundary
  // points next to a fluid boundary point
  const Vec4<Real> l4 = A.ln[v];
  CT ln[3] = {(CT)l4.x, (CT)l4.y, (CT)l4.z};
  if (idf != 0.0) {
    // every neighbour is read (no branch per link, so the loads overlap); a
    // voxel that is not a solid boundary point has iden = 0 and a finite
    // lambda n, and adds an exact zero
    unroll<Q - 1>([&](auto J) {
      constexpr int j = J + 1;
      const int x = nbi[j];
      const Real id = A.iden[x];
      const Vec4<Real> q = A.ln[x];
      // (the points' links are unclamped)
      const CT c = clamped_z<D, j>(P, ps) ? CT(0) : (CT)Lat<D>::w(j) * (CT)id;
      ln[0] = ln[0] + c * (CT)q.x;
      ln[1] = ln[1] + c * (CT)q.y;
      if constexpr (D == 3) ln[2] = ln[2] + c * (CT)q.z;
    });
  }
  const Vec4<Real> f4 = A.lcf[n];
  const CT lco[3] = {(CT)f4.x, (CT)f4.y, (CT)f4.z};
  // colour gradient before wetting, Eq. (6)
  CT C[3] = {CT(0), CT(0), CT(0)};
  unroll<Q - 1>([&](auto J) {
    constexpr int j = J + 1;
    const CT ph = (CT)phi_dec(R.phi[nbi[j]]);
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      constexpr int e = Lat<D>::e(j, a);
      if constexpr (e != 0) C[a] = C[a] + (CT)(3.0 * Lat<D>::w(j) * e) * ph;
    });
  });
  const CT cm = ::sqrt(dotv<CT, D>(C, C));
  CT lci[3] = {lco[0], lco[1], lco[2]};
  CT lth = CT(0);
  if (cm > (CT)P.eps_c) {
    CT ch[3] = {C[0] / cm, C[1] / cm, D == 3 ? C[2] / cm : CT(0)};
    CT lch[3], lcm = CT(0);
    if ((fl & FL_WET) && (P.scheme == 1 || P.scheme == 2)) {
      TT nn[3], w3[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        nn[a].v = ch[a];
        if (a < D) nn[a].d[a] = CT(1);
        w3[a].v = a < D ? G.nw[a * P.Np + n] : Real(0);
      }
      constexpr CT deg = (CT)(3.14159265358979323846 / 180.0);
      const CT ctv = G.cos_t[n], stv = G.sin_t[n];
      TT ct, st;
      ct.v = ctv;
      st.v = stv;
      ct.d[3] = -stv * deg;
      st.d[3] = ctv * deg;
      if (P.scheme == 1)
        scheme1<TT, D>(nn, w3, ct, TT((fl & FL_S1POS) ? 1.0 : -1.0), TT(P.eps_f), TT(P.eps_v));
      else
        scheme2<TT, D>(nn, w3, ct, st, TT(P.eps_v));
      // C_out = |C| n_wet
      CT lnt[3];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        lnt[b] = ln[b] + cm * lco[b];
        lcm = lcm + nn[b].v * lco[b];
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        CT s = CT(0);
#pragma unroll
        for (int b = 0; b < D; ++b) s = s + nn[b].d[a] * lnt[b];
        lch[a] = s;
      }
#pragma unroll
      for (int b = 0; b < D; ++b) lth += nn[b].d[3] * lnt[b];
#pragma unroll
      for (int a = 0; a < D; ++a) lci[a] = CT(0);
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) lch[a] = ln[a];
    }
    // n = C / |C|: (I - n n^T) / |C|
    const CT cd = cm > (CT)AP.delta ? cm : (CT)AP.delta;
    CT dp = CT(0);
#pragma unroll
    for (int a = 0; a < D; ++a) dp = dp + ch[a] * lch[a];
#pragma unroll
    for (int a = 0; a < D; ++a) lci[a] = lci[a] + lcm * ch[a] + (lch[a] - ch[a] * dp) / cd;
  }
  Vec4<Real> o;
  o.x = (Real)lci[0];
  o.y = (Real)lci[1];
  o.z = D == 3 ? (Real)lci[2] : Real(0);
  o.w = Real(0);
  A.lc[v] = o;
  if (lth != CT(0)) A.lth[v] += (double)lth * idf;
  *lthout = (double)lth;
}

template <class Real, int D>
__global__ void __launch_bounds__(256) ka_normal(StepParams P, Geo<Real> G, Grids<Real> R, AdjBufs<Real> A, AdjParams AP) {
  const int n = node_id_plain();
  double lth = 0.0;
  if (n < P.N) d_adj_normal<Real, D>(P, G, R, A, AP, n, &lth);
  block_accumulate<256, 1>(&lth, kColTheta, A.pacc);
}

// ------------------------------------------------------- ka_sb_phi, ka_phi
// C(x) = 3 sum_i w_i e_i phi(x + e_i)  =>  lambda phi(y) = -3 sum_j w_j e_j . lambda C(y + e_j)
// On a link clamped at an open face the node x = y + (e_j with no z step)
// reads y along the direction e_j mirrored in z, so e_z changes sign there.
template <int D, int j, class Real>
__device__ __forceinline__ Real grad_t_term(const Real* qq, bool mirror) {
  Real t = Real(0);
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    constexpr int e = Lat<D>::e(j, a);
    if constexpr (a < 2) {
      if constexpr (e == 1) t = t + qq[a];
      if constexpr (e == -1) t = t - qq[a];
    } else if constexpr (e != 0) {
      const Real z = e == 1 ? qq[2] : -qq[2];
      t = t + (mirror ? -z : z);
    }
  });
  return t;
}

template <class Real, int D>
__device__ __forceinline__ Real adj_grad_t(const StepParams& P, const AdjBufs<Real>& A, const Pos& ps,
                                           const int* nbi) {
  constexpr int Q = Lat<D>::Q;
  Real acc = Real(0);
  unroll<Q - 1>([&](auto J) {
    constexpr int j = J + 1;
    const Vec4<Real> q = A.lc[nbi[j]];
    const Real qq[3] = {q.x, q.y, q.z};
    const Real t = grad_t_term<D, j>(qq, clamped_z<D, j>(P, ps));
    acc = acc + (Real)(-3.0 * Lat<D>::w(j)) * t;
  });
  return acc;
}

// The same at a solid boundary point, over its fluid links only: lambda C is
// written on fluid voxels alone (zero elsewhere), so the skipped terms are
// exact zeros; masked buffer loads keep every gather in flight together.
// (The links of a point's mask are unclamped; in a face layer the fluid
// nodes of the layer that read the point through a clamped link are
// gathered as well.)
template <class Real, int D>
__device__ __forceinline__ Real adj_grad_t_sb(const StepParams& P, const AdjBufs<Real>& A, const Pos& ps,
                                              const int* nbi, unsigned msk) {
  constexpr int Q = Lat<D>::Q;
  const auto rc = grid_rsrc(A.lc, sizeof(Vec4<Real>) * (size_t)P.V);
  Real acc = Real(0);
  unroll<Q - 1>([&](auto J) {
    constexpr int j = J + 1;
    const bool cl = clamped_z<D, j>(P, ps);
    const bool on = (msk & (1u << j)) || cl;
    const Vec4<Real> q =
        bload3<Real>(rc, on ? (uint32_t)nbi[j] * (uint32_t)sizeof(Vec4<Real>) : kOffNone);
    const Real qq[3] = {q.x, q.y, q.z};
    const Real t = grad_t_term<D, j>(qq, cl);
    acc = acc + (Real)(-3.0 * Lat<D>::w(j)) * t;
  });
  return acc;
}

template <class Real, int D>
__global__ void ka_sb_phi(StepParams P, Geo<Real> G, AdjBufs<Real> A) {
  const int s = node_id_plain();
  if (P.scheme == 3) {
    // fictitious density, Eq. (24): phi(x_s) = -cos(theta(x_s)) is a
    // parameter, not a mean of the fluid neighbours, so its adjoint goes to
    // the contact angle, d phi / d theta = sin(theta) pi/180 per degree
    // (sin >= 0 on (0, 180) deg), and nothing flows back to the fluid phase
    double lth = 0.0;
    if (s < P.nsb) {
      const int v = G.sb_vox[s];
      const unsigned m = G.sb_mask[s];
      const Pos ps = make_pos(P, v, m & 1u);
      int nbi[Lat<D>::Q];
      nb_all<D>(P, ps, nbi);
      const double lp = (double)adj_grad_t_sb<Real, D>(P, A, ps, nbi, m);
      const double c = (double)G.sb_fd[s];
      lth = lp * ::sqrt(::fmax(0.0, 1.0 - c * c)) * (M_PI / 180.0);
      A.lphi[v] = Real(0);
      A.lth[v] += lth;
    }
    block_accumulate<256, 1>(&lth, kColTheta, A.pacc);
    return;
  }
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  const unsigned m = G.sb_mask[s];
  const Pos ps = make_pos(P, v, m & 1u);
  int nbi[Lat<D>::Q];
  nb_all<D>(P, ps, nbi);
  A.lphi[v] = adj_grad_t_sb<Real, D>(P, A, ps, nbi, m) * A.iden[v];
}

template <class Real, int D>
__global__ void ka_phi(StepParams P, Geo<Real> G, AdjBufs<Real> A) {
  constexpr int Q = Lat<D>::Q;
  const int n = node_id_plain();
  if (n >= P.N) return;
  const unsigned vf = G.vf[n];
  const int v = vox_of(vf);
  const Pos ps = make_pos(P, v, flags_of(vf) & FL_FACE);
  int nbi[Q];
  nb_all<D>(P, ps, nbi);
  Real lp = adj_grad_t<Real, D>(P, A, ps, nbi);
  if (A.idf[n] != 0.0) {
    // transpose of Eq. (34): phi(s) = sum_i w_i phi(s + e_i) / sum_i w_i
    // over the point's (unclamped) links
    unroll<Q - 1>([&](auto J) {
      constexpr int j = J + 1;
      const Real w = clamped_z<D, j>(P, ps) ? Real(0) : (Real)Lat<D>::w(j);
      lp = lp + w * A.lphi[nbi[j]];
    });
  }
  const Vec4<Real> na = A.na[n];
  Vec2<Real> r;
  r.x = na.x + lp * na.z;
  r.y = na.y + lp * na.w;
  A.lr[n] = r;
  // the phase of an outlet node of a pulled state is the upstream node's
  // (Eq. 39): its lambda phi is handed on by ka_face
  if (A.face_pull && (flags_of(vf) & FL_OUT)) A.lpo[n - (P.N - P.n_out)] += lp;
}

// -------------------------------------------------------- objective, seeds
// Per-block partial sums over the objective's slab (or plane): rho^r, rho^b,
// (1 + phi)/2, and the plane flux (j + F/2)_axis.
constexpr int kObjN = 4;

template <class Real, int D, int BS, class In>
__global__ void __launch_bounds__(BS) ka_obj(StepParams P, Geo<Real> G, Grids<Real> R, In in, AdjParams AP,
                                             double* part) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id_plain();
  double o[kObjN] = {0.0, 0.0, 0.0, 0.0};
  if (n < P.N) {
    const int v = vox_of(G.vf[n]);
    const int c = coord_of(P, v, AP.axis);
    Real fr[Q], fx[Q], rr, rb, rho;
    adj_load_faced<Real, D>(P, G, R, in, n, fr, fx, rr, rb, rho);
    if (c >= AP.lo && c < AP.hi) {
      o[0] = (double)rr;
      o[1] = (double)rb;
      o[2] = (1.0 + ((double)rr - (double)rb) / (double)rho) / 2.0;
    }
    if (c == AP.lo && AP.objective == 2) {
      double j = 0.0;
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        const double ft = kDev ? (double)fx[i] : (double)fr[i] + (double)fx[i];
        constexpr int e0 = Lat<D>::e(i, 0), e1 = Lat<D>::e(i, 1), e2 = Lat<D>::e(i, 2);
        const int e = AP.axis == 0 ? e0 : (AP.axis == 1 ? e1 : e2);
        j += (double)e * ft;
      });
      const Vec4<Real> f4 = R.f[n];
      const double Fa = AP.axis == 0 ? (double)f4.x : (AP.axis == 1 ? (double)f4.y : (double)f4.z);
      o[3] = j + 0.5 * Fa;
    }
  }
  __shared__ double sh[BS / 64];
#pragma unroll
  for (int q = 0; q < kObjN; ++q) {
    const double t = block_sum<BS>(o[q], sh);
    if (threadIdx.x == 0) part[blockIdx.x * kObjN + q] = t;
  }
}

// Fixed-order reduction of [nb][nq] partials: one block per quantity.
// (Templated on the precision only so that each precision's translation unit
// owns its own instance.)
template <class Real>
__global__ void ka_reduce(const double* part, int nb, int nq, double* out) {
  const int q = blockIdx.x;
  __shared__ double sh[256];
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) t += part[(size_t)b * nq + q];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = sh[0];
}

// Terminal adjoint of objectives 0 and 1 (node-local in the densities):
// saturation J = S_r / (S_r + S_b): dJ/drho^r = S_b / S^2, dJ/drho^b = -S_r / S^2;
// red volume J = sum (1 + phi)/2: dJ/drho^r = rho^b / rho^2, dJ/drho^b = -rho^r / rho^2.
template <class Real, int D, class In>
__global__ void ka_seed_local(StepParams P, Geo<Real> G, Grids<Real> R, In in, AdjParams AP, const double* sums,
                              Real* lf, Vec2<Real>* lr) {
  constexpr int Q = Lat<D>::Q;
  const int n = node_id_plain();
  if (n >= P.N) return;
  const int v = vox_of(G.vf[n]);
  const int c = coord_of(P, v, AP.axis);
  double gr = 0.0, gb = 0.0;
  if (c >= AP.lo && c < AP.hi) {
    if (AP.objective == 0) {
      const double S = sums[0] + sums[1];
      gr = sums[1] / (S * S);
      gb = -sums[0] / (S * S);
    } else {
      Real fr[Q], fx[Q], rr, rb, rho;
      adj_load_faced<Real, D>(P, G, R, in, n, fr, fx, rr, rb, rho);
      const double ir = 1.0 / (double)rho;
      gr = (double)rb * ir * ir;
      gb = -(double)rr * ir * ir;
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) lf[i * P.Np + n] = Real(0);
  Vec2<Real> r;
  r.x = (Real)gr;
  r.y = (Real)gb;
  lr[n] = r;
}

// ------------------------------------------------------------------ ka_face
// Transpose of the Zou-He faces (Appendix B) at each face node x of a pulled
// state.  On entry L (the total part) and R = (R^r, R^b) are the adjoint of
// x's post-face populations, lambda^s_i = L_i + R^s; on exit L holds the
// known pulled directions, with R as the reverse streaming reads it (inlet:
// R = 0; outlet: weight 2 along +z).  With the per-colour unknowns of the
// faces written as f_u = f_k(u) + c_u j^s +- N^s (B.4-B.8, B.14-B.18):
//   inlet,  j^s = rho_in zeta^s - (S^s + 2 T^s):  lambda_j^s = lambda_j^L + R^s
//           (the five unknowns carry weights 1/3 + 4/6 = 1), the R^s
//           cancel on every known direction;
//   outlet, j^s = chi^s j^t, j^t = (S^t + 2 T^t) - rho_out:
//           lambda_j^s = lambda_j^L - R^s, lambda j^t = lambda_j^L - sum_s chi^s R^s,
//           lambda phi_up += j^t (R^b - R^r) / 2 from chi^s = (1 +- phi_up)/2,
//           and phi_up (with the outlet node's own lambda phi, Eq. 39)
//           passes to the upstream node's densities.
// The node also adds its shares of dJ/drho_in and dJ/drho_out.
// kStep: after a node stage, which left j^t of the outlet faces in ljt and the
// upstream nodes' d phi / d rho^s in na; otherwise (the terminal condition of
// a node-local objective) both are formed from the state's populations.
template <class Real, int D, bool kStep, class In>
__global__ void __launch_bounds__(256) ka_face(StepParams P, Geo<Real> G, Grids<Real> R, In in, Real* L,
                                               Vec2<Real>* lr, const Real* lpo, const Real* ljt,
                                               const Vec4<Real>* na, double* pacc) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  using CT = Real;
  const int n = face_node(P, node_id_plain());
  double g[2] = {0.0, 0.0};
  if constexpr (D == 3) {
    if (n >= 0) {
      const unsigned vf = G.vf[n];
      const unsigned fl = flags_of(vf);
      const bool inl = fl & FL_IN;
      CT l[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) l[i] = L[i * P.Np + n];
      const Vec2<Real> r = lr[n];
      const CT Rr = (CT)r.x, Rb = (CT)r.y;
      // sums over the known directions: S in the plane, T the directions
      // leaving through the face (their unknowns are their reflections)
      constexpr int kS[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};
      CT o[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) o[i] = CT(0);
      CT lj, lnx, lny, lam = CT(0);
      if (inl) {
        lj = l[5] / CT(3) + (l[11] + l[12] + l[15] + l[16]) / CT(6);
        lnx = l[12] - l[11];
        lny = l[16] - l[15];
        lam = -lj;  // d j / d f_k = -1 (S), -2 (T)
      } else {
        lj = -l[6] / CT(3) - (l[13] + l[14] + l[17] + l[18]) / CT(6);
        lnx = l[14] - l[13];
        lny = l[18] - l[17];
        const CT phu = (CT)phi_dec(R.phi[vox_of(vf)]);
        const CT chr = CT(0.5) * (CT(1) + phu), chb = CT(0.5) * (CT(1) - phu);
        lam = lj - (chr * Rr + chb * Rb);  // lambda j^t; d j^t / d f_k = +1 (S), +2 (T)
        g[1] = -(double)lam;               // d j^t / d rho_out = -1
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) o[kS[k]] = l[kS[k]] + lam;
      // Nx = (f1 + f7 + f9 - f2 - f8 - f10)/2, Ny = (f3 + f7 + f8 - f4 - f9 - f10)/2
      const CT hx = CT(0.5) * lnx, hy = CT(0.5) * lny;
      o[1] = o[1] + hx;
      o[2] = o[2] - hx;
      o[3] = o[3] + hy;
      o[4] = o[4] - hy;
      o[7] = o[7] + hx + hy;
      o[8] = o[8] - hx + hy;
      o[9] = o[9] + hx - hy;
      o[10] = o[10] - hx - hy;
      if (inl) {
        // known T = {6, 13, 14, 17, 18}; unknowns 5 <- 6, 11 <- 14, 12 <- 13, 15 <- 18, 16 <- 17
        o[6] = l[6] + CT(2) * lam + l[5];
        o[13] = l[13] + CT(2) * lam + l[12];
        o[14] = l[14] + CT(2) * lam + l[11];
        o[17] = l[17] + CT(2) * lam + l[16];
        o[18] = l[18] + CT(2) * lam + l[15];
        const double zr = P.zeta_r;
        g[0] = (double)lj + zr * (double)Rr + (1.0 - zr) * (double)Rb;
        Vec2<Real> z0;
        z0.x = Real(0);
        z0.y = Real(0);
        lr[n] = z0;
      } else {
        // known T = {5, 11, 12, 15, 16}; unknowns 6 <- 5, 13 <- 12, 14 <- 11, 17 <- 16, 18 <- 15
        o[5] = l[5] + CT(2) * lam + l[6];
        o[12] = l[12] + CT(2) * lam + l[13];
        o[11] = l[11] + CT(2) * lam + l[14];
        o[16] = l[16] + CT(2) * lam + l[17];
        o[15] = l[15] + CT(2) * lam + l[18];
        // j^t of the face, and d phi / d rho^s of the upstream node u
        const int slot = n - (P.N - P.n_out);
        const int u = G.nbr.template get<kDirZp>(n);
        CT jt, dru, dbu;
        if constexpr (kStep) {
          jt = ljt[slot];
          const Vec4<Real> nu = na[u];
          dru = nu.z;
          dbu = nu.w;
        } else {
          Real fr[Q], fx[Q], rr, rb, rho;
          adj_load<Real, D>(P, G, in, n, fr, fx, rr, rb, rho);
          CT ft[Q];
#pragma unroll
          for (int i = 0; i < Q; ++i) ft[i] = kDev ? fx[i] : fr[i] + fx[i];
          jt = outlet_jt<kDev>(P, ft);
          load_outlet_upstream<D>(in, G.nbr, n, fr, fx);
          adj_sums<Real, D>(P, fr, fx, rr, rb, rho);
          const CT ir = CT(1) / rho;
          dru = CT(2) * rb * ir * ir;
          dbu = CT(-2) * rr * ir * ir;
        }
        const CT lphu = lpo[slot] + CT(0.5) * jt * (Rb - Rr);
        Vec2<Real> ru = lr[u];
        ru.x = ru.x + lphu * dru;
        ru.y = ru.y + lphu * dbu;
        lr[u] = ru;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) L[i * P.Np + n] = o[i];
    }
  }
  block_accumulate<256, 2>(g, kColRhoIn, pacc);
}

// ------------------------------------------------------------ setup, output
// 1 / (sum of the weights of the fluid links) at each solid boundary point.
template <class Real, int D>
__global__ void ka_iden(StepParams P, Geo<Real> G, Real* iden) {
  constexpr int Q = Lat<D>::Q;
  const int s = node_id_plain();
  if (s >= P.nsb) return;
  const unsigned m = G.sb_mask[s];
  double den = 0.0;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    if (m & (1u << i)) den += Lat<D>::w(i);
  });
  iden[G.sb_vox[s]] = (Real)(1.0 / den);
}

// 1 / (sum of the weights of the solid links) at each fluid boundary point
// (links whose pull source is a solid voxel; the lattice is symmetric).
template <class Real, int D>
__global__ void ka_idf(StepParams P, Geo<Real> G, double* idf) {
  constexpr int Q = Lat<D>::Q;
  const int n = node_id_plain();
  if (n >= P.N) return;
  double den = 0.0;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    if (G.nbr.template get<i>(n) == kBounce) den += Lat<D>::w(i);
  });
  idf[n] = den > 0.0 ? 1.0 / den : 0.0;
}

// dJ/dtheta(s) at each solid boundary point: the transpose of the weighted
// mean that gives a fluid boundary point its angle (w_i over its solid links).
template <class Real, int D>
__global__ void ka_theta_field(StepParams P, Geo<Real> G, const double* lth, double* out) {
  constexpr int Q = Lat<D>::Q;
  const int s = node_id_plain();
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  if (P.scheme == 3) {
    out[v] = lth[v];  // the point's own angle (fictitious density)
    return;
  }
  const unsigned m = G.sb_mask[s];
  const Pos ps = make_pos(P, v, m & 1u);
  double acc = 0.0;
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    if (m & (1u << i)) acc += Lat<D>::w(i) * lth[nb_vox<D, i>(P, ps)];
  });
  out[v] = acc;
}

template <class Real, class T>
__global__ void ka_fill(size_t count, T* p, T value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

}  // namespace cg
