/*
 * Plain FP64 CPU oracle of the colour-gradient lattice Boltzmann time step
 * (Sedahmed & Coelho, "Wetting and pressure gradient performance in lattice
 * Boltzmann color gradient model", arXiv:2407.10914).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this library; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * Every array is dense over the nx*ny*nz voxel box, x fastest:
 *   v = x + nx*(y + ny*z).  Population arrays are [Q][V].
 */
#ifndef CG_ORACLE_H
#define CG_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;               /* 2 (D2Q9) or 3 (D3Q19) */
  int nx, ny, nz;        /* nz = 1 for dim 2 */
  int periodic[3];       /* per axis */
  int collision;         /* 0 = BGK (Guo forcing), 1 = MRT (Sec. II.A) */
  int scheme;            /* 0 = none, 1 = Scheme-I, 2 = Scheme-II (Sec. II.B), 3 = fictitious density (Eq. 24) */
  int s1_line;           /* Scheme-I secant start: 0 = sign rule, 1 = literal Eq. (30) */
  int bc;                /* 0 = closed/periodic, 1 = Zou-He inlet z=0 / outlet z=nz-1 */
  double tau_r, tau_b;   /* relaxation times of the two fluids, Eq. (13) */
  double sigma;          /* interfacial tension gamma, Eq. (5) */
  double beta;           /* segregation parameter, Eq. (17) */
  double rho0;           /* reference density rho_o */
  double theta_deg;      /* contact angle measured through fluid b */
  double rho_in, rho_out;/* Zou-He densities, Appendix B */
  double zeta_r;         /* injected red fraction at the inlet, Eq. (B.1) */
  double g[3];           /* body-force acceleration, Eq. (36); force density rho_o*g */
  double eps_c;          /* |C| below which n = 0 (Eq. 27 guard) */
  double eps_f;          /* Scheme-I secant guards on |f| */
  double eps_v;          /* guards on |v|, |n_c x n_w| and sin(theta') */
} orc_params;

typedef struct {
  double mass_r, mass_b; /* sum of rho^r, rho^b over fluid nodes */
  double n_fluid;
  double sat_w;          /* #{phi < 0} / #fluid (Sec. IV.B) */
  double sat_nw_mass;    /* sum rho^r / sum rho */
  double flux_t, flux_r, flux_b; /* sum of rho*u_a, rho^r*u_a, rho^b*u_a on the flux plane */
  double vol_r, vol_b;   /* sum (1+phi)/2, sum (1-phi)/2 */
  double p_in, p_out;    /* mean rho/3 over phi>0.9 and phi<-0.9 */
  double n_in, n_out;
  double u_max;
  double nan_count;
} orc_obs;

typedef struct orc_sim orc_sim;

const char* orc_last_error(void);

orc_sim* orc_create(const orc_params* p, const uint8_t* solid, const double* theta_field_deg);
void orc_destroy(orc_sim* s);
int orc_q(const orc_sim* s);
int orc_set_phase(orc_sim* s, const double* phi0);
int orc_set_state(orc_sim* s, const double* fr, const double* fb);
int orc_get_state(const orc_sim* s, double* fr, double* fb);
int orc_step(orc_sim* s, int n);
/* Macroscopic fields of the current state (steps S1..S8 without collision).
 * Any output pointer may be NULL.  u3 is [3][V]. */
int orc_macro(orc_sim* s, double* rho_r, double* rho_b, double* phi, double* u3);
/* Stage dump of the current state: phi (fluid + S_b), n after wetting (fluid + S_b),
 * C after wetting, kappa, F; any pointer may be NULL. Vectors are [3][V]. */
int orc_stages(orc_sim* s, double* phi, double* n3, double* c3, double* kappa, double* f3);
/* Replace the injected fluid, Eqs. (37)-(38): at the inlet nodes the old
 * colour's populations move to the new colour (zeta_r_new: 1 = red, 0 = blue),
 * and later steps inject the new fluid.  Zou-He runs only. */
int orc_switch_inlet(orc_sim* s, double zeta_r_new);
/* OpenMP threads of the node loops (n > 0 sets them); returns the count in use.
 * Results do not depend on it: no loop reduces across nodes. */
int orc_set_threads(int n);
/* Order in which the step's per-voxel loops visit the voxels: perm holds a
 * permutation of the V voxel indices (x fastest); the face loops follow the
 * order of the z = 0 voxels in it.  Results do not depend on it (each stage
 * reads only earlier stages' outputs); it exists so that a test can show
 * that.  Returns -1 unless perm is a permutation. */
int orc_set_visit_order(orc_sim* s, const int64_t* perm);
/* New Zou-He inlet/outlet densities for the following steps. */
int orc_set_pressure(orc_sim* s, double rho_in, double rho_out);
/* New body-force acceleration g (Eq. 36) for the following steps. */
int orc_set_body_force(orc_sim* s, const double* g3);
/* axis: 0/1/2; plane: index on that axis */
int orc_observe(orc_sim* s, int axis, int plane, orc_obs* out);
/* The same over the fluid nodes with lo <= coordinate[slab_axis] < hi (the
 * plane flux still over its whole plane). */
int orc_observe_slab(orc_sim* s, int slab_axis, int lo, int hi, int axis, int plane, orc_obs* out);
/* cls: 0 interior solid, 1 S_b, 2 fluid, 3 F_b.  g3: smoothed image; nw3: [3][V];
 * cos_t/sin_t: contact angle at F_b nodes. */
int orc_setup_info(const orc_sim* s, uint8_t* cls, double* g3, double* nw3,
                   double* cos_t, double* sin_t);

/* ---- discrete derivative of an objective (forward mode, dual numbers) ----
 * Runs n_steps from the rest state of phi0 with every quantity carrying one
 * directional derivative and returns J and dJ along the seeded parameter:
 * seed 0: theta (global, degrees; requires no theta field), seed 1..3: the
 * x/y/z component of the body-force acceleration g, seed 4: the per-voxel
 * contact-angle field along theta_dir (V entries, degrees), seeds 5 and 6:
 * the Zou-He inlet and outlet densities rho_in, rho_out (Appendix B).
 * The objectives are taken over the fluid nodes of the slab
 * lo <= coordinate[axis] < hi of the final state:
 * objective 0: non-wetting mass saturation sum rho^r / sum rho;
 * objective 1: red volume sum (1 + phi)/2;
 * objective 2: total momentum flux sum rho u_axis over the plane
 *              coordinate[axis] == lo (u of Eq. 22; hi unused). */
typedef struct {
  int objective;
  int axis, lo, hi;
  int n_steps;
  int seed;
  const double* theta_dir;
} orc_tangent_spec;
int orc_tangent(const orc_params* p, const uint8_t* solid, const double* theta_field_deg, const double* phi0,
                const orc_tangent_spec* spec, double* J, double* dJ);
/* The objective of the current state of a plain run (same definitions). */
int orc_objective(orc_sim* s, int objective, int axis, int lo, int hi, double* J);

/* ---- single-node building blocks, exposed for the pin tests ---- */
int orc_lattice(int dim, int* e /*[Q][3]*/, double* w, int* opp);
int orc_mrt_matrix(double* M /*[19][19]*/, double* norm2 /*[19]*/);
int orc_meq(double rho, double rho0, const double* u3, double* meq19);
int orc_forcing_moments(const double* u3, const double* F3, const double* S19, double* sf19);
int orc_rates(double phi, double tau_r, double tau_b, double* s_nu, double* s_q);
/* Collide one node: ft[Q] pre-collision total populations -> out[Q].
 * S19 overrides the MRT rates when non-NULL (MRT only). */
int orc_collide_node(int dim, int collision, const double* ft, double rho, double rho0,
                     const double* u3, const double* F3, double s_nu, double s_q,
                     const double* S19, double* out);
int orc_recolor(int dim, const double* fpp, double rho_r, double rho_b, double beta,
                const double* n3, double* fr_out, double* fb_out);
int orc_scheme1(int dim, const double* nc3, const double* nw3, double theta_deg, int line,
                double eps_f, double eps_v, double* out3);
int orc_scheme2(int dim, const double* nc3, const double* nw3, double theta_deg,
                double eps_v, double* out3);
/* Zou-He on one D3Q19 node: fr/fb [19] in/out (unknown slots overwritten). */
int orc_zouhe_inlet(double* fr, double* fb, double rho_in, double zeta_r);
int orc_zouhe_outlet(double* fr, double* fb, double rho_out, double phi_up);

#ifdef __cplusplus
}
#endif
#endif
