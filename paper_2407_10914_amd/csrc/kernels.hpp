// __global__ kernels of the time step, observables and state transfer.
// Instantiated per precision in kernels_f64.hip / kernels_f32.hip.
#pragma once

#include "step.hpp"

namespace cg {

// ------------------------------------------------------------------ k_phase
// Densities and phase field at every fluid node, Eqs. (7)-(9); inlet nodes take
// phi_in (Sec. II.D.1), outlet nodes the phase one node upstream (Eq. 39).
template <class Real, int D, class In>
__global__ void k_phase(StepParams P, Geo<Real> G, Grids<Real> R, In in) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const unsigned fl = G.flags[n];
  Real phi;
  if (fl & FL_IN) {
    phi = (Real)P.phi_in;
  } else {
    const int src = (fl & FL_OUT) ? G.nbr[(kDirZp - 1) * P.Np + n] : n;
    Real fr[Q], fx[Q];
    load_node<D>(in, G.nbr, P.Np, src, fr, fx);
    Real rr, rb, rho, drho;
    node_moments<D, kDev>(fr, fx, (Real)P.rho0, rr, rb, rho, drho);
    phi = (rr - rb) / rho;
  }
  R.phi[G.vox[n]] = phi;
}

// ----------------------------------------------------------------- k_sb_phi
// Eq. (34): weighted mean of the fluid link neighbours, i ascending.
template <class Real, int D>
__global__ void k_sb_phi(StepParams P, Geo<Real> G, Grids<Real> R) {
  constexpr int Q = Lat<D>::Q;
  const int s = node_id();
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  const unsigned m = G.sb_mask[s];
  Real num = Real(0), den = Real(0);
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    if (m & (1u << i)) {
      constexpr double w = Lat<D>::w(i);
      const int y = nb_slow(P, v, Lat<D>::e(i, 0), Lat<D>::e(i, 1), Lat<D>::e(i, 2));
      num = num + (Real)w * R.phi[y];
      den = den + (Real)w;
    }
  });
  R.phi[v] = num / den;
}

// ----------------------------------------------------------------- k_normal
// Colour gradient, Eq. (6), unit normal, Eq. (27), wetting at the fluid
// boundary points (Sec. II.B.3 step 3) keeping |C|.
template <class Real, int D>
__global__ void k_normal(StepParams P, Geo<Real> G, Grids<Real> R) {
  constexpr int Q = Lat<D>::Q;
  const int n = node_id();
  if (n >= P.N) return;
  const int v = G.vox[n];
  const unsigned fl = G.flags[n];
  const bool face = fl & FL_FACE;
  Real ph[Q];
  unroll<Q>([&](auto I) {
    constexpr int i = I;
    if constexpr (i > 0) ph[i] = R.phi[nb_vox<D, i>(P, v, face)];
  });
  Real C[3] = {Real(0), Real(0), Real(0)};
  unroll<D>([&](auto A_) {
    constexpr int a = A_;
    Real s = Real(0);
    bool first = true;
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      constexpr int e = Lat<D>::e(i, a);
      if constexpr (e != 0) {
        constexpr double we = Lat<D>::w(i) * e;
        const Real t = (Real)we * ph[i];
        s = first ? t : s + t;
        first = false;
      }
    });
    C[a] = Real(3) * s;
  });
  const Real cm = sqrt(dotv<Real, D>(C, C));
  Real nn[3] = {Real(0), Real(0), Real(0)};
  if (cm > (Real)P.eps_c) {
#pragma unroll
    for (int a = 0; a < D; ++a) nn[a] = C[a] / cm;
    if ((fl & FL_WET) && P.scheme != 0) {
      Real w3[3];
#pragma unroll
      for (int a = 0; a < D; ++a) w3[a] = G.nw[a * P.Np + n];
      if (P.scheme == 1)
        scheme1<Real, D>(nn, w3, G.cos_t[n], (fl & FL_S1POS) ? Real(1) : Real(-1), (Real)P.eps_f, (Real)P.eps_v);
      else
        scheme2<Real, D>(nn, w3, G.cos_t[n], G.sin_t[n], (Real)P.eps_v);
#pragma unroll
      for (int a = 0; a < D; ++a) C[a] = cm * nn[a];
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R.n[a * P.V + v] = nn[a];
    R.c[a * P.Np + n] = C[a];
  }
}

// ------------------------------------------------------------------- k_sb_n
// Eq. (35): normal extrapolated to the solid boundary points, not renormalised.
template <class Real, int D>
__global__ void k_sb_n(StepParams P, Geo<Real> G, Grids<Real> R) {
  constexpr int Q = Lat<D>::Q;
  const int s = node_id();
  if (s >= P.nsb) return;
  const int v = G.sb_vox[s];
  const unsigned m = G.sb_mask[s];
  Real num[3] = {Real(0), Real(0), Real(0)};
  Real den = Real(0);
  unroll<Q - 1>([&](auto I) {
    constexpr int i = I + 1;
    if (m & (1u << i)) {
      constexpr double w = Lat<D>::w(i);
      const int y = nb_slow(P, v, Lat<D>::e(i, 0), Lat<D>::e(i, 1), Lat<D>::e(i, 2));
#pragma unroll
      for (int a = 0; a < D; ++a) num[a] = num[a] + (Real)w * R.n[a * P.V + y];
      den = den + (Real)w;
    }
  });
#pragma unroll
  for (int a = 0; a < D; ++a) R.n[a * P.V + v] = num[a] / den;
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

// Pull, faces, curvature, force, velocity, rates, collision, recolouring,
// store (MODE_STEP); or the macroscopic fields (MODE_MACRO); or the
// observable reductions (MODE_OBS).
template <class Real, int D, int BS, int Mode, class In, class Out>
__global__ void __launch_bounds__(BS) k_main(StepParams P, Geo<Real> G, Grids<Real> R, In in, Out out,
                                             MacroOut mo, ObsOut oo) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  const bool active = n < P.N;
  double o[kObsN];
  if constexpr (Mode == MODE_OBS) {
#pragma unroll
    for (int k = 0; k < kObsN; ++k) o[k] = 0.0;
  }
  if (active) {
    const int v = G.vox[n];
    const unsigned fl = G.flags[n];
    const bool face = fl & FL_FACE;
    Real fr[Q], fx[Q];
    load_node<D>(in, G.nbr, P.Np, n, fr, fx);
    if constexpr (In::kPull) {
      if (D == 3 && (fl & (FL_IN | FL_OUT))) zou_he<kDev>(P, fl, R.phi[v], fr, fx);
    }
    Real rr, rb, rho, drho;
    node_moments<D, kDev>(fr, fx, (Real)P.rho0, rr, rb, rho, drho);
    const Real phi = R.phi[v];
    // curvature, Eq. (12), from the isotropic derivatives of n
    Real nb[D][Q];
    unroll<Q>([&](auto I) {
      constexpr int i = I;
      if constexpr (i > 0) {
        const int y = nb_vox<D, i>(P, v, face);
#pragma unroll
        for (int a = 0; a < D; ++a) nb[a][i] = R.n[a * P.V + y];
      }
    });
    Real d[3][3];
    unroll<D>([&](auto B_) {
      constexpr int b = B_;
      unroll<D>([&](auto A_) {
        constexpr int a = A_;
        Real s = Real(0);
        bool first = true;
        unroll<Q>([&](auto I) {
          constexpr int i = I;
          constexpr int e = Lat<D>::e(i, b);
          if constexpr (e != 0) {
            constexpr double we = Lat<D>::w(i) * e;
            const Real t = (Real)we * nb[a][i];
            s = first ? t : s + t;
            first = false;
          }
        });
        d[b][a] = Real(3) * s;
      });
    });
    Real nx_ = R.n[v], ny_ = R.n[P.V + v], nz_ = Real(0);
    if constexpr (D == 3) nz_ = R.n[2 * P.V + v];
    Real k;
    if constexpr (D == 3) {
      k = (nx_ * nx_ - Real(1)) * d[0][0] + (ny_ * ny_ - Real(1)) * d[1][1] + (nz_ * nz_ - Real(1)) * d[2][2] +
          (d[1][0] + d[0][1]) * nx_ * ny_ + (d[2][0] + d[0][2]) * nx_ * nz_ + (d[1][2] + d[2][1]) * nz_ * ny_;
    } else {
      k = (nx_ * nx_ - Real(1)) * d[0][0] + (ny_ * ny_ - Real(1)) * d[1][1] + (d[1][0] + d[0][1]) * nx_ * ny_;
    }
    // force, Eq. (5) + rho_o g (Eq. 36); velocity, Eq. (22) (deviation layout:
    // the density of the momentum balance is rho0 + sum g)
    const Real rho_u = kDev ? (Real)P.rho0 + drho : rho;
    Real C[3] = {Real(0), Real(0), Real(0)}, F[3] = {Real(0), Real(0), Real(0)}, u[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      C[a] = R.c[a * P.Np + n];
      F[a] = (Real)P.half_sigma * k * C[a] + (Real)P.rg[a];
    }
    unroll<D>([&](auto A_) {
      constexpr int a = A_;
      Real j = Real(0);
      bool first = true;
      unroll<Q>([&](auto I) {
        constexpr int i = I;
        constexpr int e = Lat<D>::e(i, a);
        if constexpr (e != 0) {
          const Real t = e == 1 ? fx[i] : -fx[i];
          j = first ? t : j + t;
          first = false;
        }
      });
      u[a] = (j + Real(0.5) * F[a]) / rho_u;
    });
    if constexpr (Mode == MODE_STEP) {
      Real s_nu, s_q;
      rates(P, phi, s_nu, s_q);
      if constexpr (D == 3) {
        if (P.collision == 1)
          collide_mrt<!kDev>(fx, drho, (Real)P.rho0, u, F, s_nu, s_q);
        else
          collide_bgk<D>(fx, drho, (Real)P.rho0, u, F, s_nu);
      } else {
        collide_bgk<D>(fx, drho, (Real)P.rho0, u, F, s_nu);
      }
      // recolouring, Eqs. (20)-(21)
      const Real rsum = rr + rb;
      const Real a = rr / rsum;
      const Real b = rr * rb / rsum;
      if constexpr (kDev) {
        out.A[n] = a;
        const Real bb = (Real)P.beta * b;
        out.Cc[n] = bb * nx_;
        out.Cc[out.Np + n] = bb * ny_;
        if constexpr (D == 3) out.Cc[2 * out.Np + n] = bb * nz_;
#pragma unroll
        for (int i = 0; i < Q; ++i) out.T[i * out.Np + n] = fx[i];
      } else {
        const Real nvec[3] = {nx_, ny_, nz_};
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
      if (mo.rho_r) mo.rho_r[v] = (double)rr;
      if (mo.rho_b) mo.rho_b[v] = (double)rb;
      if (mo.phi) mo.phi[v] = (double)phi;
      if (mo.kappa) mo.kappa[v] = (double)k;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (mo.u) mo.u[a * P.V + v] = (double)u[a];
        if (mo.force) mo.force[a * P.V + v] = (double)F[a];
        if (mo.cvec) mo.cvec[a * P.V + v] = (double)C[a];
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
      if (!ok) {
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
        if (P.flux_axis >= 0 && P.flux_axis < D) {
          const int nxy = P.nx * P.ny;
          const int z = v / nxy, r = v - z * nxy, y = r / P.nx, x = r - y * P.nx;
          const int c = P.flux_axis == 0 ? x : (P.flux_axis == 1 ? y : z);
          if (c == P.flux_plane) {
            const double ua = (double)u[P.flux_axis];
            o[12] = (a + b) * ua;
            o[13] = a * ua;
            o[14] = b * ua;
          }
        }
      }
    }
  }
  if constexpr (Mode == MODE_OBS) {
    __shared__ double sh[BS / 64];
#pragma unroll
    for (int q = 0; q < kObsN; ++q) {
      const double t = (q == 10) ? block_max<BS>(o[q], sh) : block_sum<BS>(o[q], sh);
      if (threadIdx.x == 0) oo.part[blockIdx.x * kObsN + q] = t;
    }
  }
}

// Second pass of the observables: partial sums in block order (deterministic).
// (templated only so that each precision's unit owns its instance)
template <class Real>
__global__ void k_obs_final(const double* part, int nblocks, double* out) {
  const int q = threadIdx.x;
  if (q >= kObsN) return;
  double t = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double x = part[b * kObsN + q];
    t = (q == 10) ? fmax(t, x) : t + x;
  }
  out[q] = t;
}

// -------------------------------------------------------- state transfer
// Canonical pre-collision populations of the current state, as FP64 dense
// [Q][V] arrays (pull, bounce-back and faces applied).
template <class Real, int D, class In>
__global__ void k_export(StepParams P, Geo<Real> G, Grids<Real> R, In in, double* fr_out, double* fb_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const int v = G.vox[n];
  const unsigned fl = G.flags[n];
  double fr[Q], fx[Q];
  load_node<D>(in, G.nbr, P.Np, n, fr, fx);
  if constexpr (In::kPull) {
    if (D == 3 && (fl & (FL_IN | FL_OUT))) zou_he<kDev>(P, fl, (double)R.phi[v], fr, fx);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    fr_out[(size_t)i * P.V + v] = fr[i];
    fb_out[(size_t)i * P.V + v] = kDev ? ((Lat<D>::w(i) * P.rho0 + fx[i]) - fr[i]) : fx[i];
  }
}

// Dense FP64 canonical populations -> pre-collision staging at the nodes.
template <class Real, int D>
__global__ void k_import(StepParams P, Geo<Real> G, const double* fr, const double* fb, Real* r_out, Real* x_out) {
  constexpr int Q = Lat<D>::Q;
  constexpr bool kDev = sizeof(Real) == 4;
  const int n = node_id();
  if (n >= P.N) return;
  const int v = G.vox[n];
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

// Scatter a per-node array into a dense FP64 voxel array (dense must be zeroed).
template <class Real>
__global__ void k_scatter(int N, int Np, int comps, int V, const int* vox, const Real* src, double* dst) {
  const int n = node_id();
  if (n >= N) return;
  for (int c = 0; c < comps; ++c) dst[(size_t)c * V + vox[n]] = (double)src[c * Np + n];
}

// Copy a dense voxel grid at the listed voxels to a dense FP64 array.
template <class Real>
__global__ void k_grid_copy(int count, const int* list, int comps, int V, const Real* grid, double* dst) {
  const int n = node_id();
  if (n >= count) return;
  const int v = list ? list[n] : n;
  for (int c = 0; c < comps; ++c) dst[(size_t)c * V + v] = (double)grid[(size_t)c * V + v];
}

}  // namespace cg
