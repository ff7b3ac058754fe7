/*
 * Plain FP64 CPU oracle of the colour-gradient lattice Boltzmann time step of
 * Sedahmed & Coelho, arXiv:2407.10914 (model of Chen et al., their Ref. [20]).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg are its only users.  It shares no code with the GPU path.
 *
 * It is deliberately plain: dense arrays over the whole voxel box, one loop per
 * stage in the order the paper gives, every lattice sum taken over i = 0..Q-1
 * in index order, matrix products written out as loops over the full matrix.
 * Readings of the paper where it is silent or garbled are marked "reading:".
 *
 * The whole file is generic over the scalar type R so that the same code also
 * runs on forward-mode dual numbers (value + one directional derivative).
 * That gives the exact discrete derivative of the step with respect to the
 * contact angle and the body force, used to check the GPU adjoint.
 */
#include "cg_oracle.h"

#include <cmath>
#include <cstdio>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;
int fail(const std::string& m) {
  g_err = m;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Forward-mode dual number: value v and derivative d along one direction.  */
/* Branches compare values only.                                            */
/* ------------------------------------------------------------------------ */
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
inline double der(double) { return 0.0; }
inline double der(Dual a) { return a.d; }
inline bool finite(double a) { return std::isfinite(a); }
inline bool finite(Dual a) { return std::isfinite(a.v); }

using std::cos;
using std::fabs;
using std::sin;
using std::sqrt;

/* ------------------------------------------------------------------------ */
/* Lattices                                                                  */
/* ------------------------------------------------------------------------ */
struct Lattice {
  int dim, q;
  int e[19][3];
  double w[19];
  int opp[19];
};

/* D3Q19 velocities and weights exactly as tabulated in Appendix A, Eq. (A.1)
 * (columns of the 3x19 matrix) and Eq. (A.2). */
const int kE19[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                         {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, 1, 0}, {1, -1, 0},
                         {-1, -1, 0}, {1, 0, 1},  {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1},
                         {0, 1, 1},  {0, -1, 1},  {0, 1, -1}, {0, -1, -1}};

Lattice make_lattice(int dim) {
  Lattice L;
  std::memset(&L, 0, sizeof(L));
  L.dim = dim;
  if (dim == 3) {
    L.q = 19;
    for (int i = 0; i < 19; ++i) {
      for (int a = 0; a < 3; ++a) L.e[i][a] = kE19[i][a];
      L.w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  } else {
    /* reading: the paper has no 2D lattice; D2Q9 is taken as the in-plane
     * subset of the D3Q19 set above, kept in the same order, with the usual
     * D2Q9 weights 4/9, 1/9, 1/36. */
    const int sub[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};
    L.q = 9;
    for (int i = 0; i < 9; ++i) {
      for (int a = 0; a < 3; ++a) L.e[i][a] = kE19[sub[i]][a];
      L.w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  }
  for (int i = 0; i < L.q; ++i)
    for (int j = 0; j < L.q; ++j)
      if (L.e[j][0] == -L.e[i][0] && L.e[j][1] == -L.e[i][1] && L.e[j][2] == -L.e[i][2])
        L.opp[i] = j;
  return L;
}

/* ------------------------------------------------------------------------ */
/* MRT transformation matrix, Appendix A, Eq. (A.3).                         */
/* reading: two printed rows (the p_xy and p_yz rows) are garbled, so M is   */
/* built from the polynomial definition of each moment in the order of       */
/* Eq. (3); the pin tests check it against every printed row that is intact. */
/* ------------------------------------------------------------------------ */
struct Mrt {
  double M[19][19];
  double Minv[19][19];
  double norm2[19];
};

int moment_poly(int k, int ex, int ey, int ez) {
  const int e2 = ex * ex + ey * ey + ez * ez;
  switch (k) {
    case 0: return 1;                                   /* rho */
    case 1: return 19 * e2 - 30;                        /* e */
    case 2: return (21 * e2 * e2 - 53 * e2 + 24) / 2;   /* epsilon */
    case 3: return ex;                                  /* j_x */
    case 4: return (5 * e2 - 9) * ex;                   /* q_x */
    case 5: return ey;                                  /* j_y */
    case 6: return (5 * e2 - 9) * ey;                   /* q_y */
    case 7: return ez;                                  /* j_z */
    case 8: return (5 * e2 - 9) * ez;                   /* q_z */
    case 9: return 3 * ex * ex - e2;                    /* 3 p_xx */
    case 10: return (3 * e2 - 5) * (3 * ex * ex - e2);  /* 3 pi_xx */
    case 11: return ey * ey - ez * ez;                  /* p_ww */
    case 12: return (3 * e2 - 5) * (ey * ey - ez * ez); /* pi_ww */
    case 13: return ex * ey;                            /* p_xy */
    case 14: return ey * ez;                            /* p_yz */
    case 15: return ex * ez;                            /* p_xz */
    case 16: return ex * (ey * ey - ez * ez);           /* m_x */
    case 17: return ey * (ez * ez - ex * ex);           /* m_y */
    case 18: return ez * (ex * ex - ey * ey);           /* m_z */
  }
  return 0;
}

Mrt make_mrt() {
  Mrt m;
  for (int k = 0; k < 19; ++k)
    for (int i = 0; i < 19; ++i) m.M[k][i] = (double)moment_poly(k, kE19[i][0], kE19[i][1], kE19[i][2]);
  /* rows are orthogonal, so M^-1 = M^T diag(1/|row|^2) */
  for (int k = 0; k < 19; ++k) {
    double s = 0.0;
    for (int i = 0; i < 19; ++i) s += m.M[k][i] * m.M[k][i];
    m.norm2[k] = s;
  }
  for (int i = 0; i < 19; ++i)
    for (int k = 0; k < 19; ++k) m.Minv[i][k] = m.M[k][i] / m.norm2[k];
  return m;
}

const Mrt& mrt() {
  static const Mrt m = make_mrt();
  return m;
}

/* ------------------------------------------------------------------------ */
/* Node-level pieces                                                         */
/* ------------------------------------------------------------------------ */

/* Relaxation rates, Eqs. (13)-(16): harmonic-mean viscosity of the mixture,
 * S_nu from Eq. (13) with c = dt = 1, S_q = S_m = 8(2 - S_nu)/(8 - S_nu). */
template <class R>
void rates(R phi, double tau_r, double tau_b, R* s_nu, R* s_q) {
  const double nu_r = (tau_r - 0.5) / 3.0;
  const double nu_b = (tau_b - 0.5) / 3.0;
  R inv_nu = (1.0 + phi) / (2.0 * nu_r) + (1.0 - phi) / (2.0 * nu_b);
  R nu = 1.0 / inv_nu;
  *s_nu = 1.0 / (3.0 * nu + 0.5);
  *s_q = (8.0 * (2.0 - *s_nu)) / (8.0 - *s_nu);
}

/* Equilibrium populations of the incompressible model (the density
 * fluctuation rho is decoupled from j = rho_o u, Sec. II.A):
 * f^eq_i = w_i [rho + rho_o (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)].
 * reading: m^eq = M f^eq as stated in Sec. II.A; the printed m_10^eq of
 * Eq. (A.4) contradicts that and its own "-3/2 p_xx" label, and is not used. */
template <class R>
void feq(const Lattice& L, R rho, double rho0, const R* u, R* out) {
  R usq = 0.0;
  for (int a = 0; a < L.dim; ++a) usq += u[a] * u[a];
  for (int i = 0; i < L.q; ++i) {
    R eu = 0.0;
    for (int a = 0; a < L.dim; ++a) eu += (double)L.e[i][a] * u[a];
    out[i] = L.w[i] * (rho + rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
  }
}

/* Guo forcing in velocity space: Fbar_i = w_i [3 (e_i - u) + 9 (e_i.u) e_i] . F
 * (Sec. II.A, the force of Eq. (5) enters through Guo's scheme). */
template <class R>
void guo(const Lattice& L, const R* u, const R* F, R* out) {
  for (int i = 0; i < L.q; ++i) {
    R emuF = 0.0, eu = 0.0, eF = 0.0;
    for (int a = 0; a < L.dim; ++a) {
      emuF += ((double)L.e[i][a] - u[a]) * F[a];
      eu += (double)L.e[i][a] * u[a];
      eF += (double)L.e[i][a] * F[a];
    }
    out[i] = L.w[i] * (3.0 * emuF + 9.0 * eu * eF);
  }
}

/* MRT collision on the total distribution, Eq. (2) with Eq. (4) and (A.3)-(A.5).
 * reading: the force enters as f'' = f - M^-1 [ S (m - m^eq) - S^F ]; Eq. (2)
 * prints S^F inside S(.) with a plus sign, which (S_j = 0) would cancel the
 * force on the momentum.  S^F = (I - S/2) M Fbar, which reproduces every
 * row of Eq. (A.5).  The diagonal of S follows the moment order of Eq. (3);
 * Eq. (4) prints a spurious extra 0 at position 9. */
template <class R>
void collide_mrt(const Lattice& L, const R* ft, R rho, double rho0, const R* u, const R* F,
                 const R* S, R* out) {
  const Mrt& m = mrt();
  R fe[19], fb[19], mm[19], me[19], mf[19], corr[19];
  feq(L, rho, rho0, u, fe);
  guo(L, u, F, fb);
  for (int k = 0; k < 19; ++k) {
    R a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < 19; ++i) {
      a += m.M[k][i] * ft[i];
      b += m.M[k][i] * fe[i];
      c += m.M[k][i] * fb[i];
    }
    mm[k] = a;
    me[k] = b;
    mf[k] = c;
  }
  for (int k = 0; k < 19; ++k) {
    R sf = (1.0 - 0.5 * S[k]) * mf[k];
    corr[k] = S[k] * (mm[k] - me[k]) - sf;
  }
  for (int i = 0; i < 19; ++i) {
    R s = 0.0;
    for (int k = 0; k < 19; ++k) s += m.Minv[i][k] * corr[k];
    out[i] = ft[i] - s;
  }
}

/* Relaxation vector of Eq. (4) in the moment order of Eq. (3), with
 * S_e = S_eps = S_pi = S_nu (Eq. 15) and S_q = S_m (Eq. 16). */
template <class R>
void mrt_rates(R s_nu, R s_q, R* S) {
  const R z = 0.0;
  R v[19] = {z, s_nu, s_nu, z, s_q, z, s_q, z, s_q, s_nu, s_nu, s_nu, s_nu, s_nu, s_nu, s_nu, s_q, s_q, s_q};
  for (int k = 0; k < 19; ++k) S[k] = v[k];
}

/* Single-relaxation-time (BGK) collision with Guo forcing, used for the 2D
 * lattice (the paper gives MRT for D3Q19 only):
 * f'' = f - S_nu (f - f^eq) + (1 - S_nu/2) Fbar. */
template <class R>
void collide_bgk(const Lattice& L, const R* ft, R rho, double rho0, const R* u, const R* F, R s_nu,
                 R* out) {
  R fe[19], fb[19];
  feq(L, rho, rho0, u, fe);
  guo(L, u, F, fb);
  for (int i = 0; i < L.q; ++i) out[i] = ft[i] - s_nu * (ft[i] - fe[i]) + (1.0 - 0.5 * s_nu) * fb[i];
}

/* Latva-Kokko recolouring, Eqs. (20)-(21); the i = 0 population gets only
 * the first term. */
template <class R>
void recolor(const Lattice& L, const R* fpp, R rr, R rb, double beta, const R* n, R* fr, R* fb) {
  R rho = rr + rb;
  R a = rr / rho;
  R b = rr * rb / rho;
  for (int i = 0; i < L.q; ++i) {
    if (i == 0) {
      fr[i] = a * fpp[i];
    } else {
      R edn = 0.0;
      for (int c = 0; c < L.dim; ++c) edn += (double)L.e[i][c] * n[c];
      fr[i] = a * fpp[i] + beta * L.w[i] * b * edn;
    }
    fb[i] = fpp[i] - fr[i];
  }
}

template <class R>
R dotv(int dim, const R* a, const R* b) {
  R s = 0.0;
  for (int c = 0; c < dim; ++c) s += a[c] * b[c];
  return s;
}

/* Scheme-I (Leclaire et al.), Eqs. (28)-(31): secant iteration on
 * f(v) = v.n_w - |v| cos(theta) starting from v0 = n_c, v1 = n_c - lambda (n_c + s n_w),
 * lambda = 1/2, stopping at n = 4, then normalising.
 * reading (line): with n_w pointing into the fluid, the printed v1 (s = +1) only
 * reaches angles above theta'/2; for theta <= 90 deg the paper obtains the angle by
 * exchanging the fluids, which is the same as taking s = -1.  line = 1 keeps s = +1.
 * reading (guards): the iteration stops and keeps the latest iterate when |f| or the
 * secant denominator drops to eps_f; n_c is kept when it is parallel to n_w or the
 * final vector is shorter than eps_v. */
template <class R>
void scheme1(int dim, R* n, const double* nw, R cos_t, int sgn, double eps_f, double eps_v) {
  R cr;
  if (dim == 3) {
    R c0 = n[1] * nw[2] - n[2] * nw[1];
    R c1 = n[2] * nw[0] - n[0] * nw[2];
    R c2 = n[0] * nw[1] - n[1] * nw[0];
    cr = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  } else {
    cr = fabs(n[0] * nw[1] - n[1] * nw[0]);
  }
  if (cr <= eps_v) return;
  R nwr[3] = {nw[0], nw[1], nw[2]};
  R v0[3], v1[3];
  for (int c = 0; c < dim; ++c) {
    v0[c] = n[c];
    v1[c] = n[c] - 0.5 * (n[c] + (double)sgn * nw[c]);
  }
  R f0 = dotv(dim, v0, nwr) - sqrt(dotv(dim, v0, v0)) * cos_t;
  R f1 = dotv(dim, v1, nwr) - sqrt(dotv(dim, v1, v1)) * cos_t;
  for (int it = 2; it <= 4; ++it) {
    if (fabs(f1) <= eps_f || fabs(f1 - f0) <= eps_f) break;
    R v2[3];
    for (int c = 0; c < dim; ++c) v2[c] = (v0[c] * f1 - v1[c] * f0) / (f1 - f0);
    for (int c = 0; c < dim; ++c) {
      v0[c] = v1[c];
      v1[c] = v2[c];
    }
    f0 = f1;
    if (it < 4) f1 = dotv(dim, v1, nwr) - sqrt(dotv(dim, v1, v1)) * cos_t;
  }
  R nv = sqrt(dotv(dim, v1, v1));
  if (nv <= eps_v) return;
  for (int c = 0; c < dim; ++c) n[c] = v1[c] / nv;
}

/* Scheme-II (Akai et al.), Eqs. (32)-(33): the two unit vectors n_+/- at angle
 * theta from n_w in the plane of n_w and n_c; keep the one nearer to n_c.
 * reading: cos(theta') = n_w.n_c and sin(theta') = |n_c - (n_w.n_c) n_w|, which
 * equal cos/sin of arccos(n_w.n_c) for unit vectors; n_c is kept when
 * sin(theta') <= eps_v (n_c parallel to n_w); ties go to n_+. */
template <class R>
void scheme2(int dim, R* n, const double* nw, R cos_t, R sin_t, double eps_v) {
  R nwr[3] = {nw[0], nw[1], nw[2]};
  R ctp = dotv(dim, nwr, n);
  R t[3];
  for (int c = 0; c < dim; ++c) t[c] = n[c] - ctp * nw[c];
  R stp = sqrt(dotv(dim, t, t));
  if (stp <= eps_v) return;
  R np[3], nm[3];
  for (int pm = 0; pm < 2; ++pm) {
    R s = pm == 0 ? sin_t : -sin_t; /* sin(+theta), sin(-theta); cos is even */
    R A = cos_t - s * ctp / stp;
    R B = s / stp;
    R* o = pm == 0 ? np : nm;
    for (int c = 0; c < dim; ++c) o[c] = A * nw[c] + B * n[c];
  }
  R dp = 0.0, dm = 0.0;
  for (int c = 0; c < dim; ++c) {
    dp += (np[c] - n[c]) * (np[c] - n[c]);
    dm += (nm[c] - n[c]) * (nm[c] - n[c]);
  }
  const R* o = (dp <= dm) ? np : nm;
  for (int c = 0; c < dim; ++c) n[c] = o[c];
}

/* Zou-He (non-equilibrium bounce-back) pressure inlet at z = 0 for one colour,
 * Eqs. (B.1)-(B.8); rho_s = rho_in * zeta^s. Unknowns: 5, 11, 12, 15, 16. */
template <class R>
void zouhe_in_color(R* f, R rho_s) {
  R S = f[0] + f[1] + f[2] + f[3] + f[4] + f[7] + f[8] + f[9] + f[10];
  R T = f[6] + f[13] + f[14] + f[17] + f[18];
  R j = rho_s - (S + 2.0 * T);
  R Nx = 0.5 * ((f[1] + f[7] + f[9]) - (f[2] + f[8] + f[10]));
  R Ny = 0.5 * ((f[3] + f[7] + f[8]) - (f[4] + f[9] + f[10]));
  f[5] = f[6] + j / 3.0;
  f[11] = f[14] + j / 6.0 - Nx;
  f[12] = f[13] + j / 6.0 + Nx;
  f[15] = f[18] + j / 6.0 - Ny;
  f[16] = f[17] + j / 6.0 + Ny;
}

/* Zou-He pressure outlet at z = nz-1, Eqs. (B.9)-(B.18): total normal momentum
 * from the total populations, shared between colours by chi^s(phi) with phi
 * taken one node upstream (Eq. 39). Unknowns: 6, 13, 14, 17, 18. */
template <class R>
void zouhe_out(R* fr, R* fb, R rho_out, R phi_up) {
  R ft[19];
  for (int i = 0; i < 19; ++i) ft[i] = fr[i] + fb[i];
  R S = ft[0] + ft[1] + ft[2] + ft[3] + ft[4] + ft[7] + ft[8] + ft[9] + ft[10];
  R T = ft[5] + ft[11] + ft[12] + ft[15] + ft[16];
  R jt = -rho_out + (S + 2.0 * T);
  R chi[2] = {0.5 * (1.0 + phi_up), 0.5 * (1.0 - phi_up)};
  R* fs[2] = {fr, fb};
  for (int s = 0; s < 2; ++s) {
    R* f = fs[s];
    R Nx = 0.5 * ((f[1] + f[7] + f[9]) - (f[2] + f[8] + f[10]));
    R Ny = 0.5 * ((f[3] + f[7] + f[8]) - (f[4] + f[9] + f[10]));
    R jc = jt * chi[s];
    f[6] = f[5] - jc / 3.0;
    f[13] = f[12] - jc / 6.0 - Nx;
    f[14] = f[11] - jc / 6.0 + Nx;
    f[17] = f[16] - jc / 6.0 - Ny;
    f[18] = f[15] - jc / 6.0 + Ny;
  }
}

/* ------------------------------------------------------------------------ */
/* The simulation                                                            */
/* ------------------------------------------------------------------------ */
template <class R>
struct Sim {
  orc_params p;
  Lattice L;
  int D, Q;
  long nx, ny, nz, V;
  std::vector<uint8_t> solid, is_fb, is_sb;
  std::vector<double> g3, nw;          /* smoothed image, wall normal [3][V] */
  std::vector<uint8_t> nw_ok;
  std::vector<double> theta_vox;        /* per-voxel contact angle (deg), solids */
  std::vector<R> theta_fb, cos_t, sin_t;/* at F_b nodes */
  std::vector<int> s1_sign;
  R theta_global;
  R gforce[3];
  R rho_in_v, rho_out_v; /* Zou-He densities (parameters of the derivative) */
  std::vector<R> fr, fb, pr, pb;        /* state [Q][V] and post-collision */
  std::vector<R> rr, rb, rho, phi, kap; /* [V] */
  std::vector<R> cvec, nvec, frc, uvel; /* [3][V] */
  /* Order in which the per-voxel loops of a step visit the voxels (and the
   * face loops the (x, y) positions): the identity unless a caller sets a
   * permutation.  Every stage reads only what an earlier stage wrote, so the
   * order changes no result; a test runs both. */
  std::vector<long> visit, plane_visit;

  long idx(long x, long y, long z) const { return x + nx * (y + ny * z); }
  void coords(long v, long* c) const {
    c[0] = v % nx;
    c[1] = (v / nx) % ny;
    c[2] = v / (nx * ny);
  }
  bool open_axis(int a) const { return a == 2 && p.bc == 1; }

  /* Link neighbour x + e_i: index, or -1 outside across a wall face, -2
   * outside across an open face.  Periodic axes wrap. */
  long link(long v, int i) const {
    long c[3];
    coords(v, c);
    const long n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      c[a] += L.e[i][a];
      if (c[a] < 0 || c[a] >= n[a]) {
        if (p.periodic[a]) {
          c[a] = (c[a] + n[a]) % n[a];
        } else if (open_axis(a)) {
          return -2;
        } else {
          return -1;
        }
      }
    }
    return idx(c[0], c[1], c[2]);
  }

  /* Stencil neighbour for the gradient stencils (Eqs. 6, 12).
   * reading: beyond an open face the fields are extended with zero gradient
   * (the ghost takes the value of the nearest in-domain plane). */
  long stencil(long v, int i) const {
    long c[3];
    coords(v, c);
    const long n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      c[a] += L.e[i][a];
      if (c[a] < 0 || c[a] >= n[a]) {
        if (p.periodic[a]) {
          c[a] = (c[a] + n[a]) % n[a];
        } else if (open_axis(a)) {
          c[a] = c[a] < 0 ? 0 : n[a] - 1;
        } else {
          return -1;
        }
      }
    }
    return idx(c[0], c[1], c[2]);
  }

  /* Image value for the smoothing of Eq. (25) and the gradient of Eq. (26).
   * reading: periodic axes wrap, open faces extend the boundary plane, and
   * beyond a wall face the image is solid (0). */
  double img(const std::vector<double>& g, long x, long y, long z) const {
    long c[3] = {x, y, z};
    const long n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      if (c[a] < 0 || c[a] >= n[a]) {
        if (p.periodic[a])
          c[a] = (c[a] + n[a]) % n[a];
        else if (open_axis(a))
          c[a] = c[a] < 0 ? 0 : n[a] - 1;
        else
          return 0.0;
      }
    }
    return g[idx(c[0], c[1], c[2])];
  }

  bool fluid(long v) const { return solid[v] == 0; }

  int init(const orc_params* prm, const uint8_t* sol, const double* theta_field) {
    p = *prm;
    D = p.dim;
    if (D != 2 && D != 3) return fail("dim must be 2 or 3");
    L = make_lattice(D);
    Q = L.q;
    nx = p.nx;
    ny = p.ny;
    nz = p.nz;
    if (nx < 1 || ny < 1 || nz < 1) return fail("bad extents");
    if (D == 2 && nz != 1) return fail("dim 2 needs nz == 1");
    if (D == 2 && p.collision != 0) return fail("MRT is defined for D3Q19 only");
    if (D == 2 && p.bc != 0) return fail("Zou-He faces are defined for D3Q19 only");
    if (p.bc == 1 && (p.periodic[2] || nz < 3)) return fail("Zou-He needs a non-periodic z with nz >= 3");
    if (!(p.tau_r > 0.5) || !(p.tau_b > 0.5)) return fail("tau must exceed 1/2");
    if (p.beta < 0.0 || p.beta > 1.0) return fail("beta must lie in [0,1]");
    if (p.scheme < 0 || p.scheme > 3) return fail("scheme must be 0, 1, 2 or 3");
    if (p.scheme != 0 && !(p.theta_deg > 0.0 && p.theta_deg < 180.0) && !theta_field)
      return fail("theta must lie in (0,180)");
    V = nx * ny * nz;
    solid.assign(sol, sol + V);
    visit.resize(V);
    for (long v = 0; v < V; ++v) visit[v] = v;
    plane_visit.resize(nx * ny);
    for (long k = 0; k < nx * ny; ++k) plane_visit[k] = k;
    long nfl = 0;
    for (long v = 0; v < V; ++v) nfl += fluid(v);
    if (nfl == 0) return fail("no fluid voxel");
    /* fluid voxels may not touch a face that is neither periodic nor open */
    for (long v = 0; v < V; ++v) {
      if (!fluid(v)) continue;
      long c[3];
      coords(v, c);
      const long n[3] = {nx, ny, nz};
      for (int a = 0; a < D; ++a) {
        if (p.periodic[a] || open_axis(a)) continue;
        if (c[a] == 0 || c[a] == n[a] - 1) return fail("fluid voxel on a wall face");
      }
      if (p.bc == 1 && c[2] == nz - 1 && !fluid(idx(c[0], c[1], nz - 2)))
        return fail("outlet fluid voxel without fluid upstream");
    }
    /* boundary sets along the lattice links */
    is_fb.assign(V, 0);
    is_sb.assign(V, 0);
    for (long v = 0; v < V; ++v) {
      for (int i = 1; i < Q; ++i) {
        long y = link(v, i);
        if (y < 0) continue;
        if (fluid(v) && !fluid(y)) is_fb[v] = 1;
        if (!fluid(v) && fluid(y)) is_sb[v] = 1;
      }
    }
    theta_global = p.theta_deg;
    theta_vox.assign(V, p.theta_deg);
    has_field = theta_field != nullptr;
    if (theta_field)
      for (long v = 0; v < V; ++v) theta_vox[v] = theta_field[v];
    for (int a = 0; a < 3; ++a) gforce[a] = p.g[a];
    rho_in_v = p.rho_in;
    rho_out_v = p.rho_out;
    setup_wall_normal();
    map_contact_angle();
    const size_t n = (size_t)Q * V;
    fr.assign(n, 0.0);
    fb.assign(n, 0.0);
    pr.assign(n, 0.0);
    pb.assign(n, 0.0);
    rr.assign(V, 0.0);
    rb.assign(V, 0.0);
    rho.assign(V, 0.0);
    phi.assign(V, 0.0);
    kap.assign(V, 0.0);
    cvec.assign(3 * V, 0.0);
    nvec.assign(3 * V, 0.0);
    frc.assign(3 * V, 0.0);
    uvel.assign(3 * V, 0.0);
    return 0;
  }

  /* Wall normal, Eqs. (25)-(26): three passes of the 27-point (2D: 9-point)
   * smoothing of the binary image g (1 = fluid, 0 = solid), then the
   * isotropic gradient of g^(3) at the fluid boundary nodes.
   * reading: g = 1 in the fluid so n_w points into the fluid; n_w is
   * normalised (Eqs. 28, 32 need a unit vector) and no wetting is applied
   * where |grad g^(3)| <= 1e-12. */
  void setup_wall_normal() {
    std::vector<double> g(V), h(V);
    for (long v = 0; v < V; ++v) g[v] = fluid(v) ? 1.0 : 0.0;
    for (int it = 0; it < 3; ++it) {
      for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
          for (long x = 0; x < nx; ++x) {
            double s = 0.0;
            const int kz0 = D == 3 ? -1 : 0, kz1 = D == 3 ? 1 : 0;
            for (int k = kz0; k <= kz1; ++k)
              for (int j = -1; j <= 1; ++j)
                for (int i = -1; i <= 1; ++i) {
                  const int r2 = i * i + j * j + k * k;
                  double ws;
                  if (D == 3) {
                    ws = r2 == 0 ? 8.0 / 27.0 : r2 == 1 ? 2.0 / 27.0 : r2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
                  } else {
                    /* reading: 2D uses the 9-point [1,4,1]/6 (x) [1,4,1]/6 kernel */
                    ws = r2 == 0 ? 4.0 / 9.0 : r2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0;
                  }
                  s += ws * img(g, x + i, y + j, z + k);
                }
            h[idx(x, y, z)] = s;
          }
      g.swap(h);
    }
    g3 = g;
    nw.assign(3 * V, 0.0);
    nw_ok.assign(V, 0);
    for (long v = 0; v < V; ++v) {
      if (!is_fb[v]) continue;
      long c[3];
      coords(v, c);
      double gr[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i)
          s += L.w[i] * (double)L.e[i][a] * img(g3, c[0] + L.e[i][0], c[1] + L.e[i][1], c[2] + L.e[i][2]);
        gr[a] = 3.0 * s;
      }
      double m = 0.0;
      for (int a = 0; a < D; ++a) m += gr[a] * gr[a];
      m = std::sqrt(m);
      if (m > 1e-12) {
        nw_ok[v] = 1;
        for (int a = 0; a < D; ++a) nw[a * V + v] = gr[a] / m;
      }
    }
  }

  /* Contact angle at a fluid boundary node.
   * reading: with a per-voxel angle on the solid, a fluid boundary node takes
   * the w_i-weighted mean of its solid link neighbours, mirroring Eq. (34);
   * without a field every boundary node takes the global angle. */
  bool has_field = false;
  std::vector<R> theta_vox_r; /* per-voxel angle as R (the dual run seeds it) */
  void map_contact_angle() {
    theta_fb.assign(V, 0.0);
    cos_t.assign(V, 0.0);
    sin_t.assign(V, 0.0);
    s1_sign.assign(V, 0);
    if (theta_vox_r.empty()) {
      theta_vox_r.assign(V, 0.0);
      for (long v = 0; v < V; ++v) theta_vox_r[v] = theta_vox[v];
    }
    for (long v = 0; v < V; ++v) {
      if (!is_fb[v]) continue;
      if (!has_field) {
        theta_fb[v] = theta_global;
        continue;
      }
      R num = 0.0;
      double den = 0.0;
      for (int i = 1; i < Q; ++i) {
        long y = link(v, i);
        if (y < 0 || fluid(y)) continue;
        num += L.w[i] * theta_vox_r[y];
        den += L.w[i];
      }
      theta_fb[v] = num / den;
    }
    update_angle_trig();
  }

  void update_angle_trig() {
    const double deg = M_PI / 180.0;
    for (long v = 0; v < V; ++v) {
      if (!is_fb[v]) continue;
      R th = theta_fb[v];
      cos_t[v] = cos(th * deg);
      sin_t[v] = sin(th * deg);
      s1_sign[v] = (p.s1_line == 1 || val(th) > 90.0) ? 1 : -1;
    }
  }

  void set_phase(const double* phi0) {
    for (long v = 0; v < V; ++v) {
      if (!fluid(v)) continue;
      /* reading: initial state at rest, f^s_i = w_i rho^s with
       * rho^r = rho_o (1 + phi)/2, rho^b = rho_o (1 - phi)/2 */
      const double r = p.rho0 * (1.0 + phi0[v]) / 2.0;
      const double b = p.rho0 * (1.0 - phi0[v]) / 2.0;
      for (int i = 0; i < Q; ++i) {
        fr[(size_t)i * V + v] = L.w[i] * r;
        fb[(size_t)i * V + v] = L.w[i] * b;
      }
    }
  }

  /* Replacing the injected fluid in a restart, Eqs. (37)-(38) (Sec. II.D.1):
   * at every inlet node the populations of the previously injected colour are
   * added to those of the newly injected one and then cleared; later steps
   * inject the new fluid (zeta^r = 1 for red, 0 for blue). */
  int switch_inlet(double zeta_new) {
    if (p.bc != 1) return fail("the injected fluid needs Zou-He faces");
    if (zeta_new != 0.0 && zeta_new != 1.0) return fail("the new injected fluid must be pure (zeta_r 0 or 1)");
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        const long v = idx(x, y, 0);
        if (!fluid(v)) continue;
        for (int i = 0; i < Q; ++i) {
          R& a = fr[(size_t)i * V + v];
          R& b = fb[(size_t)i * V + v];
          if (zeta_new == 1.0) {
            a = a + b; /* Eq. (37), s = r */
            b = 0.0;   /* Eq. (38) */
          } else {
            b = b + a; /* Eq. (37), s = b */
            a = 0.0;   /* Eq. (38) */
          }
        }
      }
    p.zeta_r = zeta_new;
    return 0;
  }

  /* Visiting order of the step's loops: perm is a permutation of the V voxel
   * indices; the face loops take the (x, y) positions in the order in which
   * perm lists the voxels of the plane z = 0. */
  int set_visit_order(const int64_t* perm) {
    std::vector<uint8_t> seen(V, 0);
    for (long k = 0; k < V; ++k) {
      if (perm[k] < 0 || perm[k] >= V || seen[perm[k]]) return fail("not a permutation of the voxels");
      seen[perm[k]] = 1;
    }
    visit.assign(perm, perm + V);
    long j = 0;
    for (long k = 0; k < V; ++k)
      if (visit[k] < nx * ny) plane_visit[j++] = visit[k];
    return 0;
  }

  /* New Zou-He densities (Appendix B) for the next steps. */
  int set_pressure(double rho_in, double rho_out) {
    if (p.bc != 1) return fail("inlet/outlet densities need Zou-He faces");
    if (!(rho_in > 0.0) || !(rho_out > 0.0)) return fail("densities must be positive");
    p.rho_in = rho_in;
    p.rho_out = rho_out;
    rho_in_v = rho_in;
    rho_out_v = rho_out;
    return 0;
  }

  /* Steps S1-S8 of one time step: densities and phase field, wetting
   * treatment, curvature, force, velocity.  Fills the macroscopic arrays. */
  void macro() {
    const R phi_in = p.zeta_r - (1.0 - p.zeta_r);
    /* S1: Eqs. (7)-(9) */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V; ++k) {
      const long v = visit[k];
      if (!fluid(v)) continue;
      R a = 0.0, b = 0.0;
      for (int i = 0; i < Q; ++i) a += fr[(size_t)i * V + v];
      for (int i = 0; i < Q; ++i) b += fb[(size_t)i * V + v];
      rr[v] = a;
      rb[v] = b;
      rho[v] = a + b;
      phi[v] = (a - b) / rho[v];
    }
    if (p.bc == 1) {
      /* injected fluid at the inlet (Sec. II.D.1): phi(x_in) = zeta^r - zeta^b;
       * zero-gradient phase field at the outlet, Eq. (39) */
      for (long k = 0; k < nx * ny; ++k) {
          const long x = plane_visit[k] % nx, y = plane_visit[k] / nx;
          long vi = idx(x, y, 0);
          if (fluid(vi)) phi[vi] = phi_in;
          long vo = idx(x, y, nz - 1);
          if (fluid(vo)) phi[vo] = phi[idx(x, y, nz - 2)];
        }
    }
    /* S2: phase field extrapolated to the solid boundary points, Eq. (34);
     * with the fictitious-density model the solid boundary points carry a
     * fixed phase instead, Eq. (24).
     * reading: Eq. (24) sets phi(x_s) = cos(theta) with theta measured through
     * the red fluid; the angle here is measured through fluid b, as for the
     * other schemes, so phi(x_s) = cos(180 deg - theta) = -cos(theta). */
    for (long k = 0; k < V; ++k) {
      const long s = visit[k];
      if (!is_sb[s]) continue;
      if (p.scheme == 3) {
        const R th = has_field ? theta_vox_r[s] : theta_global;
        phi[s] = -cos(th * (M_PI / 180.0));
        continue;
      }
      R num = 0.0;
      double den = 0.0;
      for (int i = 1; i < Q; ++i) {
        long y = link(s, i);
        if (y < 0 || !fluid(y)) continue;
        num += L.w[i] * phi[y];
        den += L.w[i];
      }
      phi[s] = num / den;
    }
    /* S3: colour gradient, Eq. (6), and its unit vector, Eq. (27) */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V; ++k) {
      const long v = visit[k];
      if (!fluid(v)) continue;
      R C[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) {
        R s = 0.0;
        for (int i = 0; i < Q; ++i) s += L.w[i] * (double)L.e[i][a] * phi[stencil(v, i)];
        C[a] = 3.0 * s;
      }
      R cm = sqrt(dotv(D, C, C));
      R n[3] = {0.0, 0.0, 0.0};
      if (cm > p.eps_c)
        for (int a = 0; a < D; ++a) n[a] = C[a] / cm;
      /* S4: wetting at the fluid boundary points (Sec. II.B, steps 2-3);
       * the norm |C| is kept and only the direction changes */
      if (is_fb[v] && nw_ok[v] && cm > p.eps_c && (p.scheme == 1 || p.scheme == 2)) {
        double w3[3] = {nw[v], nw[V + v], nw[2 * V + v]};
        if (p.scheme == 1)
          scheme1(D, n, w3, cos_t[v], s1_sign[v], p.eps_f, p.eps_v);
        else
          scheme2(D, n, w3, cos_t[v], sin_t[v], p.eps_v);
        for (int a = 0; a < D; ++a) C[a] = cm * n[a];
      }
      for (int a = 0; a < 3; ++a) {
        cvec[a * V + v] = C[a];
        nvec[a * V + v] = n[a];
      }
    }
    /* S5: zero-interfacial-force extrapolation of n_c to the solid boundary
     * points, Eq. (35); not renormalised */
    for (long k = 0; k < V; ++k) {
      const long s = visit[k];
      if (!is_sb[s]) continue;
      R num[3] = {0.0, 0.0, 0.0};
      double den = 0.0;
      for (int i = 1; i < Q; ++i) {
        long y = link(s, i);
        if (y < 0 || !fluid(y)) continue;
        for (int a = 0; a < D; ++a) num[a] += L.w[i] * nvec[a * V + y];
        den += L.w[i];
      }
      for (int a = 0; a < D; ++a) nvec[a * V + s] = num[a] / den;
    }
    /* S6-S8: curvature, Eq. (12); CSF force, Eq. (5) plus the body force of
     * Eq. (36) as force density rho_o g; velocity, Eq. (22) */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V; ++k) {
      const long v = visit[k];
      if (!fluid(v)) continue;
      R d[3][3];  /* d[b][a] = d n_a / d x_b, same isotropic stencil as Eq. (6) */
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) d[b][a] = 0.0;
      for (int b = 0; b < D; ++b)
        for (int a = 0; a < D; ++a) {
          R s = 0.0;
          for (int i = 0; i < Q; ++i) s += L.w[i] * (double)L.e[i][b] * nvec[a * V + stencil(v, i)];
          d[b][a] = 3.0 * s;
        }
      const R nx_ = nvec[v], ny_ = nvec[V + v], nz_ = nvec[2 * V + v];
      R k;
      /* reading: Eq. (12) (kappa = -(I - nn):grad n) is used; Eq. (10) as printed
       * has the opposite sign.  2D keeps its x-y terms. */
      if (D == 3) {
        k = (nx_ * nx_ - 1.0) * d[0][0] + (ny_ * ny_ - 1.0) * d[1][1] + (nz_ * nz_ - 1.0) * d[2][2] +
            (d[1][0] + d[0][1]) * nx_ * ny_ + (d[2][0] + d[0][2]) * nx_ * nz_ +
            (d[1][2] + d[2][1]) * nz_ * ny_;
      } else {
        k = (nx_ * nx_ - 1.0) * d[0][0] + (ny_ * ny_ - 1.0) * d[1][1] + (d[1][0] + d[0][1]) * nx_ * ny_;
      }
      kap[v] = k;
      R F[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) F[a] = 0.5 * p.sigma * k * cvec[a * V + v] + p.rho0 * gforce[a];
      for (int a = 0; a < 3; ++a) frc[a * V + v] = F[a];
      for (int a = 0; a < D; ++a) {
        R j = 0.0;
        for (int i = 0; i < Q; ++i) j += (double)L.e[i][a] * (fr[(size_t)i * V + v] + fb[(size_t)i * V + v]);
        uvel[a * V + v] = (j + 0.5 * F[a]) / rho[v];
      }
    }
  }

  /* One full step: S1-S8 (macro), S9 collision, S10 recolouring, S11 pull
   * streaming with halfway bounce-back, S12 Zou-He faces. */
  void step() {
    macro();
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V; ++k) {
      const long v = visit[k];
      if (!fluid(v)) continue;
      R ft[19], out[19], cr[19], cb[19];
      for (int i = 0; i < Q; ++i) ft[i] = fr[(size_t)i * V + v] + fb[(size_t)i * V + v];
      R s_nu, s_q;
      rates(phi[v], p.tau_r, p.tau_b, &s_nu, &s_q);
      R u[3] = {uvel[v], uvel[V + v], uvel[2 * V + v]};
      R F[3] = {frc[v], frc[V + v], frc[2 * V + v]};
      if (p.collision == 1) {
        R S[19];
        mrt_rates(s_nu, s_q, S);
        collide_mrt(L, ft, rho[v], p.rho0, u, F, S, out);
      } else {
        collide_bgk(L, ft, rho[v], p.rho0, u, F, s_nu, out);
      }
      R n[3] = {nvec[v], nvec[V + v], nvec[2 * V + v]};
      recolor(L, out, rr[v], rb[v], p.beta, n, cr, cb);
      for (int i = 0; i < Q; ++i) {
        pr[(size_t)i * V + v] = cr[i];
        pb[(size_t)i * V + v] = cb[i];
      }
    }
    /* S11: pull streaming, Eq. (1); halfway bounce-back at solid links (P: no-slip
     * bounce-back; reading: halfway placement) */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V; ++k) {
      const long v = visit[k];
      if (!fluid(v)) continue;
      for (int i = 0; i < Q; ++i) {
        long src = link(v, L.opp[i]); /* x - e_i */
        R a, b;
        if (src >= 0 && fluid(src)) {
          a = pr[(size_t)i * V + src];
          b = pb[(size_t)i * V + src];
        } else if (src == -2) {
          a = 0.0; /* unknown, set by Zou-He below */
          b = 0.0;
        } else {
          a = pr[(size_t)L.opp[i] * V + v];
          b = pb[(size_t)L.opp[i] * V + v];
        }
        fr[(size_t)i * V + v] = a;
        fb[(size_t)i * V + v] = b;
      }
    }
    /* S12: Zou-He faces (Appendix B) right after streaming */
    if (p.bc == 1) {
      const double zr = p.zeta_r, zb = 1.0 - p.zeta_r;
      for (long k = 0; k < nx * ny; ++k) {
          const long x = plane_visit[k] % nx, y = plane_visit[k] / nx;
          long vi = idx(x, y, 0);
          if (fluid(vi)) {
            R a[19], b[19];
            for (int i = 0; i < 19; ++i) {
              a[i] = fr[(size_t)i * V + vi];
              b[i] = fb[(size_t)i * V + vi];
            }
            zouhe_in_color(a, rho_in_v * zr);
            zouhe_in_color(b, rho_in_v * zb);
            for (int i = 0; i < 19; ++i) {
              fr[(size_t)i * V + vi] = a[i];
              fb[(size_t)i * V + vi] = b[i];
            }
          }
          long vo = idx(x, y, nz - 1);
          if (fluid(vo)) {
            /* reading: chi^s uses phi one node upstream (Eq. 39), computed from
             * that node's populations after streaming */
            long vu = idx(x, y, nz - 2);
            R ra = 0.0, rbb = 0.0;
            for (int i = 0; i < 19; ++i) ra += fr[(size_t)i * V + vu];
            for (int i = 0; i < 19; ++i) rbb += fb[(size_t)i * V + vu];
            R phi_up = (ra - rbb) / (ra + rbb);
            R a[19], b[19];
            for (int i = 0; i < 19; ++i) {
              a[i] = fr[(size_t)i * V + vo];
              b[i] = fb[(size_t)i * V + vo];
            }
            zouhe_out(a, b, rho_out_v, phi_up);
            for (int i = 0; i < 19; ++i) {
              fr[(size_t)i * V + vo] = a[i];
              fb[(size_t)i * V + vo] = b[i];
            }
          }
        }
    }
  }

  /* Objectives of the adjoint checks, from the current state, over the
   * fluid nodes with lo <= coordinate[axis] < hi: 0: sum rho^r / sum rho;
   * 1: sum (1 + phi)/2; 2: sum of rho u_axis over the plane coordinate == lo. */
  R objective(int which, int axis, long lo, long hi) {
    if (which == 2) {
      macro();
      R q = 0.0;
      for (long v = 0; v < V; ++v) {
        if (!fluid(v)) continue;
        long c[3];
        coords(v, c);
        if (c[axis] != lo) continue;
        q += rho[v] * uvel[axis * V + v];
      }
      return q;
    }
    R sr = 0.0, st = 0.0, vr = 0.0;
    for (long v = 0; v < V; ++v) {
      if (!fluid(v)) continue;
      long c[3];
      coords(v, c);
      if (c[axis] < lo || c[axis] >= hi) continue;
      R a = 0.0, b = 0.0;
      for (int i = 0; i < Q; ++i) a += fr[(size_t)i * V + v];
      for (int i = 0; i < Q; ++i) b += fb[(size_t)i * V + v];
      sr += a;
      st += a + b;
      vr += (1.0 + (a - b) / (a + b)) / 2.0;
    }
    return which == 0 ? sr / st : vr;
  }

  /* Observables over the fluid nodes with slab_lo <= coordinate[slab_axis] <
   * slab_hi (slab_axis < 0: all fluid nodes); the plane flux is taken over
   * its whole plane. */
  void observe(int axis, int plane, orc_obs* o, int slab_axis = -1, long slab_lo = 0, long slab_hi = 0) {
    macro();
    std::memset(o, 0, sizeof(*o));
    double sr = 0, sb = 0, nfl = 0, nw = 0, vr = 0, vb = 0, pin = 0, pout = 0, nin = 0, nout = 0, umax = 0,
           nan = 0, ft = 0, fr_ = 0, fb_ = 0;
    for (long v = 0; v < V; ++v) {
      if (!fluid(v)) continue;
      const double a = val(rr[v]), b = val(rb[v]), ph = val(phi[v]);
      double u2 = 0.0;
      bool ok = finite(rr[v]) && finite(rb[v]);
      for (int c = 0; c < D; ++c) {
        double uc = val(uvel[c * V + v]);
        ok = ok && std::isfinite(uc);
        u2 += uc * uc;
      }
      long c[3];
      coords(v, c);
      const bool in_slab = slab_axis < 0 || (c[slab_axis] >= slab_lo && c[slab_axis] < slab_hi);
      if (!ok) {
        if (in_slab) nan += 1;
        continue;
      }
      if (axis >= 0 && axis < D && c[axis] == plane) {
        const double ua = val(uvel[axis * V + v]);
        ft += (a + b) * ua;
        fr_ += a * ua;
        fb_ += b * ua;
      }
      if (!in_slab) continue;
      nfl += 1;
      sr += a;
      sb += b;
      if (ph < 0.0) nw += 1;
      vr += (1.0 + ph) / 2.0;
      vb += (1.0 - ph) / 2.0;
      const double pr_ = (a + b) / 3.0;
      if (ph > 0.9) {
        pin += pr_;
        nin += 1;
      }
      if (ph < -0.9) {
        pout += pr_;
        nout += 1;
      }
      const double um = std::sqrt(u2);
      if (um > umax) umax = um;
    }
    o->mass_r = sr;
    o->mass_b = sb;
    o->n_fluid = nfl;
    o->sat_w = nfl > 0 ? nw / nfl : 0.0;
    o->sat_nw_mass = (sr + sb) > 0 ? sr / (sr + sb) : 0.0;
    o->flux_t = ft;
    o->flux_r = fr_;
    o->flux_b = fb_;
    o->vol_r = vr;
    o->vol_b = vb;
    o->p_in = nin > 0 ? pin / nin : 0.0;
    o->p_out = nout > 0 ? pout / nout : 0.0;
    o->n_in = nin;
    o->n_out = nout;
    o->u_max = umax;
    o->nan_count = nan;
  }
};

}  // namespace

/* ------------------------------------------------------------------------ */
/* C API                                                                      */
/* ------------------------------------------------------------------------ */
struct orc_sim {
  Sim<double> s;
};

extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

orc_sim* orc_create(const orc_params* p, const uint8_t* solid, const double* theta_field_deg) {
  if (!p || !solid) {
    fail("null argument");
    return nullptr;
  }
  orc_sim* h = new orc_sim();
  if (h->s.init(p, solid, theta_field_deg) != 0) {
    delete h;
    return nullptr;
  }
  return h;
}

void orc_destroy(orc_sim* s) { delete s; }
int orc_q(const orc_sim* s) { return s->s.Q; }

int orc_set_phase(orc_sim* s, const double* phi0) {
  if (!s || !phi0) return fail("null argument");
  s->s.set_phase(phi0);
  return 0;
}

int orc_set_state(orc_sim* s, const double* fr, const double* fb) {
  if (!s || !fr || !fb) return fail("null argument");
  const size_t n = (size_t)s->s.Q * s->s.V;
  std::memcpy(s->s.fr.data(), fr, n * sizeof(double));
  std::memcpy(s->s.fb.data(), fb, n * sizeof(double));
  return 0;
}

int orc_get_state(const orc_sim* s, double* fr, double* fb) {
  if (!s || !fr || !fb) return fail("null argument");
  const size_t n = (size_t)s->s.Q * s->s.V;
  std::memcpy(fr, s->s.fr.data(), n * sizeof(double));
  std::memcpy(fb, s->s.fb.data(), n * sizeof(double));
  return 0;
}

int orc_step(orc_sim* s, int n) {
  if (!s || n < 0) return fail("bad argument");
  for (int k = 0; k < n; ++k) s->s.step();
  return 0;
}

int orc_macro(orc_sim* s, double* rho_r, double* rho_b, double* phi, double* u3) {
  if (!s) return fail("null argument");
  Sim<double>& m = s->s;
  m.macro();
  for (long v = 0; v < m.V; ++v) {
    const bool f = m.fluid(v);
    if (rho_r) rho_r[v] = f ? m.rr[v] : 0.0;
    if (rho_b) rho_b[v] = f ? m.rb[v] : 0.0;
    if (phi) phi[v] = f ? m.phi[v] : 0.0;
    if (u3)
      for (int a = 0; a < 3; ++a) u3[a * m.V + v] = f ? m.uvel[a * m.V + v] : 0.0;
  }
  return 0;
}

int orc_stages(orc_sim* s, double* phi, double* n3, double* c3, double* kappa, double* f3) {
  if (!s) return fail("null argument");
  Sim<double>& m = s->s;
  m.macro();
  for (long v = 0; v < m.V; ++v) {
    const bool f = m.fluid(v);
    const bool keep = f || m.is_sb[v];
    if (phi) phi[v] = keep ? m.phi[v] : 0.0;
    if (kappa) kappa[v] = f ? m.kap[v] : 0.0;
    for (int a = 0; a < 3; ++a) {
      if (n3) n3[a * m.V + v] = keep ? m.nvec[a * m.V + v] : 0.0;
      if (c3) c3[a * m.V + v] = f ? m.cvec[a * m.V + v] : 0.0;
      if (f3) f3[a * m.V + v] = f ? m.frc[a * m.V + v] : 0.0;
    }
  }
  return 0;
}

/* OpenMP threads of the node loops (timing only: results do not depend on it). */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_switch_inlet(orc_sim* s, double zeta_r_new) {
  if (!s) return fail("null argument");
  return s->s.switch_inlet(zeta_r_new);
}

int orc_set_visit_order(orc_sim* s, const int64_t* perm) {
  if (!s || !perm) return fail("null argument");
  return s->s.set_visit_order(perm);
}
int orc_set_pressure(orc_sim* s, double rho_in, double rho_out) {
  if (!s) return fail("null argument");
  return s->s.set_pressure(rho_in, rho_out);
}

int orc_set_body_force(orc_sim* s, const double* g3) {
  if (!s || !g3) return fail("null argument");
  for (int a = 0; a < 3; ++a) s->s.gforce[a] = a < s->s.D ? g3[a] : 0.0;
  return 0;
}

int orc_observe(orc_sim* s, int axis, int plane, orc_obs* out) {
  if (!s || !out) return fail("null argument");
  s->s.observe(axis, plane, out);
  return 0;
}

int orc_observe_slab(orc_sim* s, int slab_axis, int lo, int hi, int axis, int plane, orc_obs* out) {
  if (!s || !out) return fail("null argument");
  if (slab_axis < 0 || slab_axis >= s->s.D) return fail("bad slab axis");
  s->s.observe(axis, plane, out, slab_axis, lo, hi);
  return 0;
}

int orc_setup_info(const orc_sim* s, uint8_t* cls, double* g3, double* nw3, double* cos_t, double* sin_t) {
  if (!s) return fail("null argument");
  const Sim<double>& m = s->s;
  for (long v = 0; v < m.V; ++v) {
    if (cls) cls[v] = m.fluid(v) ? (m.is_fb[v] ? 3 : 2) : (m.is_sb[v] ? 1 : 0);
    if (g3) g3[v] = m.g3[v];
    if (nw3)
      for (int a = 0; a < 3; ++a) nw3[a * m.V + v] = m.nw[a * m.V + v];
    if (cos_t) cos_t[v] = m.cos_t[v];
    if (sin_t) sin_t[v] = m.sin_t[v];
  }
  return 0;
}

int orc_objective(orc_sim* s, int objective, int axis, int lo, int hi, double* J) {
  if (!s || !J) return fail("null argument");
  if (objective < 0 || objective > 2 || axis < 0 || axis >= s->s.D) return fail("bad objective");
  *J = s->s.objective(objective, axis, lo, hi);
  return 0;
}

int orc_tangent(const orc_params* p, const uint8_t* solid, const double* theta_field_deg, const double* phi0,
                const orc_tangent_spec* spec, double* J, double* dJ) {
  if (!p || !solid || !phi0 || !spec || !J || !dJ) return fail("null argument");
  Sim<Dual> m;
  if (m.init(p, solid, theta_field_deg) != 0) return -1;
  if (spec->seed == 0) {
    if (theta_field_deg) return fail("seed 0 needs a global contact angle");
    m.theta_global = Dual(p->theta_deg, 1.0);
  } else if (spec->seed >= 1 && spec->seed <= 3) {
    m.gforce[spec->seed - 1] = Dual(p->g[spec->seed - 1], 1.0);
  } else if (spec->seed == 5 || spec->seed == 6) {
    if (p->bc != 1) return fail("seeds 5 and 6 need Zou-He faces");
    if (spec->seed == 5)
      m.rho_in_v = Dual(p->rho_in, 1.0);
    else
      m.rho_out_v = Dual(p->rho_out, 1.0);
  } else if (spec->seed == 4) {
    if (!theta_field_deg || !spec->theta_dir) return fail("seed 4 needs a theta field and a direction");
    m.theta_vox_r.assign(m.V, 0.0);
    for (long v = 0; v < m.V; ++v) m.theta_vox_r[v] = Dual(theta_field_deg[v], spec->theta_dir[v]);
  } else {
    return fail("unknown seed");
  }
  m.map_contact_angle();
  m.set_phase(phi0);
  for (int k = 0; k < spec->n_steps; ++k) m.step();
  if (spec->objective < 0 || spec->objective > 2 || spec->axis < 0 || spec->axis >= m.D)
    return fail("bad objective");
  Dual j = m.objective(spec->objective, spec->axis, spec->lo, spec->hi);
  *J = j.v;
  *dJ = j.d;
  return 0;
}

int orc_lattice(int dim, int* e, double* w, int* opp) {
  if (dim != 2 && dim != 3) return fail("dim must be 2 or 3");
  Lattice L = make_lattice(dim);
  for (int i = 0; i < L.q; ++i) {
    for (int a = 0; a < 3; ++a) e[i * 3 + a] = L.e[i][a];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return L.q;
}

int orc_mrt_matrix(double* M, double* norm2) {
  const Mrt& m = mrt();
  for (int k = 0; k < 19; ++k) {
    for (int i = 0; i < 19; ++i) M[k * 19 + i] = m.M[k][i];
    norm2[k] = m.norm2[k];
  }
  return 0;
}

int orc_meq(double rho, double rho0, const double* u3, double* meq19) {
  Lattice L = make_lattice(3);
  double fe[19];
  feq(L, rho, rho0, u3, fe);
  const Mrt& m = mrt();
  for (int k = 0; k < 19; ++k) {
    double s = 0.0;
    for (int i = 0; i < 19; ++i) s += m.M[k][i] * fe[i];
    meq19[k] = s;
  }
  return 0;
}

int orc_forcing_moments(const double* u3, const double* F3, const double* S19, double* sf19) {
  Lattice L = make_lattice(3);
  double fb[19];
  guo(L, u3, F3, fb);
  const Mrt& m = mrt();
  for (int k = 0; k < 19; ++k) {
    double s = 0.0;
    for (int i = 0; i < 19; ++i) s += m.M[k][i] * fb[i];
    sf19[k] = (1.0 - 0.5 * S19[k]) * s;
  }
  return 0;
}

int orc_rates(double phi, double tau_r, double tau_b, double* s_nu, double* s_q) {
  rates(phi, tau_r, tau_b, s_nu, s_q);
  return 0;
}

int orc_collide_node(int dim, int collision, const double* ft, double rho, double rho0, const double* u3,
                     const double* F3, double s_nu, double s_q, const double* S19, double* out) {
  Lattice L = make_lattice(dim);
  if (collision == 1) {
    if (dim != 3) return fail("MRT is D3Q19 only");
    double S[19];
    if (S19)
      for (int k = 0; k < 19; ++k) S[k] = S19[k];
    else
      mrt_rates(s_nu, s_q, S);
    collide_mrt(L, ft, rho, rho0, u3, F3, S, out);
  } else {
    collide_bgk(L, ft, rho, rho0, u3, F3, s_nu, out);
  }
  return 0;
}

int orc_recolor(int dim, const double* fpp, double rho_r, double rho_b, double beta, const double* n3,
                double* fr_out, double* fb_out) {
  Lattice L = make_lattice(dim);
  recolor(L, fpp, rho_r, rho_b, beta, n3, fr_out, fb_out);
  return 0;
}

int orc_scheme1(int dim, const double* nc3, const double* nw3, double theta_deg, int line, double eps_f,
                double eps_v, double* out3) {
  double n[3] = {nc3[0], nc3[1], dim == 3 ? nc3[2] : 0.0};
  const double deg = M_PI / 180.0;
  int sgn = (line == 1 || theta_deg > 90.0) ? 1 : -1;
  scheme1(dim, n, nw3, std::cos(theta_deg * deg), sgn, eps_f, eps_v);
  for (int a = 0; a < 3; ++a) out3[a] = n[a];
  return 0;
}

int orc_scheme2(int dim, const double* nc3, const double* nw3, double theta_deg, double eps_v, double* out3) {
  double n[3] = {nc3[0], nc3[1], dim == 3 ? nc3[2] : 0.0};
  const double deg = M_PI / 180.0;
  scheme2(dim, n, nw3, std::cos(theta_deg * deg), std::sin(theta_deg * deg), eps_v);
  for (int a = 0; a < 3; ++a) out3[a] = n[a];
  return 0;
}

int orc_zouhe_inlet(double* fr, double* fb, double rho_in, double zeta_r) {
  zouhe_in_color(fr, rho_in * zeta_r);
  zouhe_in_color(fb, rho_in * (1.0 - zeta_r));
  return 0;
}

int orc_zouhe_outlet(double* fr, double* fb, double rho_out, double phi_up) {
  zouhe_out(fr, fb, rho_out, phi_up);
  return 0;
}

}  // extern "C"
