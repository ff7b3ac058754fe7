/*
 * cg_lbm.h - C ABI of the MI355X (gfx950) colour-gradient lattice Boltzmann
 * library libcglbm.so.
 *
 * The library advances the two-colour lattice Boltzmann model of Sedahmed &
 * Coelho, arXiv:2407.10914 (Sec. II; the model of their Ref. [20]):
 *   - lattices: D3Q19 (Appendix A, Eqs. A.1-A.2) and D2Q9 (the in-plane
 *     subset of D3Q19, same order);
 *   - collision on the total distribution: MRT (Eqs. 2-4, A.3-A.5, D3Q19) or
 *     single-relaxation-time BGK, both with Guo forcing, local rates from the
 *     harmonic-mean viscosity (Eqs. 13-16);
 *   - continuum-surface-force tension F = 1/2 sigma kappa C (Eq. 5) with the
 *     isotropic colour gradient (Eq. 6) and curvature (Eq. 12);
 *   - Latva-Kokko recolouring (Eqs. 20-21);
 *   - wetting Scheme-I (secant, Eqs. 28-31) or Scheme-II (Eqs. 32-33) with the
 *     wall normal from the smoothed image (Eqs. 25-26), the phase field and
 *     the normal extrapolated into the solid boundary points (Eqs. 34-35),
 *     applied in the order of Sec. II.B.3;
 *   - pull streaming with halfway bounce-back at solid links;
 *   - Type-I Zou-He pressure inlet (z = 0) / outlet (z = nz-1) faces
 *     (Appendix B, with the injected fluid of Sec. II.D.1 and the outlet rule
 *     of Eq. 39) and/or a Type-II uniform body force (Eq. 36).
 *
 * Conventions shared by every call:
 *   - lattice units: dx = dt = c = 1, c_s^2 = 1/3;
 *   - voxel arrays are dense over nx*ny*nz, x fastest: v = x + nx*(y + ny*z);
 *     population arrays are [Q][V]; vector fields are [3][V];
 *   - the state at time t is the set of pre-collision populations f^r_i, f^b_i
 *     at the fluid voxels (left-hand side of Eq. 1 after streaming and the
 *     Zou-He faces);
 *   - every pointer argument is owned by the caller; the library copies what it
 *     needs before returning, except where a call says otherwise;
 *   - calls return CG_OK (0) or a negative cg_status; cg_last_error() returns a
 *     thread-local message for the last failure on the calling thread;
 *   - a handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef CG_LBM_H
#define CG_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CG_OK = 0,
  CG_EINVAL = -1,       /* bad argument or inconsistent geometry */
  CG_ENOMEM = -2,       /* device or host allocation failed */
  CG_EHIP = -3,         /* a HIP runtime call failed */
  CG_EUNSTABLE = -4,    /* NaN/Inf found in the state */
  CG_EUNSUPPORTED = -5, /* valid but not implemented combination */
  CG_ESTATE = -6        /* call not valid in the handle's current state */
} cg_status;

/* Geometry: solid[v] = 1 for a solid voxel, 0 for fluid (the binary matrix of
 * Sec. II.B.1).  dim = 2 requires nz = 1.  An axis is periodic or, when the
 * boundary type is CG_BC_ZOUHE, the z axis is open; on every other axis the
 * first and last layers must be solid. */
typedef struct {
  int dim;
  int nx, ny, nz;
  const uint8_t* solid;
  uint8_t periodic[3];
} cg_geometry;

/* Wetting models (Sec. II.B): Scheme-I (Eqs. 28-31) and Scheme-II
 * (Eqs. 32-33) change the interface normal at the fluid boundary points; the
 * fictitious-density model (Eq. 24) instead fixes the phase of every solid
 * boundary point to -cos(theta) (Eq. 24 written for an angle measured
 * through fluid b: cos of the angle through fluid r) and leaves the normals
 * as the colour gradient gives them.  The adjoint covers all three. */
enum { CG_WET_NONE = 0, CG_WET_SCHEME1 = 1, CG_WET_SCHEME2 = 2, CG_WET_FICTITIOUS = 3 };
/* Scheme-I secant start: SIGN_RULE takes v1 = n_c - (n_c + s n_w)/2 with
 * s = +1 for theta > 90 deg and s = -1 otherwise; LITERAL keeps s = +1 (Eq. 30
 * as printed). */
enum { CG_S1_SIGN_RULE = 0, CG_S1_LITERAL = 1 };

/* Wetting (Sec. II.B).  theta_deg is the contact angle measured through fluid
 * b.  theta_field_deg, when not NULL, gives a per-voxel angle on the solid
 * voxels (dense, V entries; fluid entries ignored); a fluid boundary node then
 * takes the w_i-weighted mean over its solid link neighbours. */
typedef struct {
  int scheme;
  double theta_deg;
  const double* theta_field_deg;
  int scheme1_line;
} cg_wetting;

enum { CG_BC_NONE = 0, CG_BC_ZOUHE = 1 };
/* Driving (Sec. II.C).  CG_BC_ZOUHE opens the z faces: a per-colour Zou-He
 * inlet at z = 0 with density rho_in and red fraction zeta_r (Eqs. B.1-B.8;
 * the injected phase is phi_in = zeta_r - (1 - zeta_r)) and a Zou-He outlet at
 * z = nz-1 with density rho_out (Eqs. B.9-B.18, phi of Eq. 39).  g is the
 * body-force acceleration of Eq. (36), applied as force density rho_o g at
 * every fluid node; it may be combined with either type.  Type-I driving is
 * CG_BC_ZOUHE with rho_in > rho_out and g = 0; Type-II is a g along z with
 * rho_in = rho_out (or a periodic z axis). */
typedef struct {
  int type;
  double rho_in, rho_out, zeta_r;
  double g[3];
} cg_bc;

enum { CG_FP32 = 0, CG_FP64 = 1 };
enum { CG_BGK = 0, CG_MRT = 1 };

typedef void* (*cg_alloc_fn)(size_t bytes, void* ctx);
typedef void (*cg_free_fn)(void* ptr, void* ctx);

/* Options.  precision: CG_FP64 evaluates every operation in the order of the
 * reference definition without fused multiply-adds; CG_FP32 stores a compact
 * post-collision state (total populations as deviations from w_i rho0, plus
 * the recolouring coefficients) and computes in single precision.  eps_c: |C| below which
 * the interface normal is zero (Eq. 27 guard); eps_f, eps_v: Scheme-I/II
 * guards.  stream: a hipStream_t (NULL = the default stream).  alloc/free: an
 * optional device allocator (for example the PyTorch caching allocator); NULL
 * uses hipMalloc/hipFree.  block: threads per block for the node kernels
 * (0 = default).  pull_table: the narrowest neighbour table the run may use,
 * 0 or 8 = one byte per link and node with a base per wave of 64 nodes
 * (default; waves whose offsets do not fit read the next table), 16 = two
 * bytes per link with a base per tile of 256 nodes, 32 = one int32 node
 * index per link; a narrower table is used only where its offsets fit, so
 * results never depend on this choice (other values: CG_EINVAL). */
typedef struct {
  int precision;
  int collision;
  double rho0;
  double eps_c, eps_f, eps_v;
  int device;
  void* stream;
  cg_alloc_fn alloc;
  cg_free_fn free;
  void* alloc_ctx;
  int block;
  int pull_table;
} cg_options;

/* Fill *opt with the defaults for the given precision: MRT, rho0 = 1,
 * eps_c = 1e-6, eps_f = eps_v = 1e-12 (FP64) or 1e-6 (FP32), device 0,
 * default stream, hipMalloc, default block. */
void cg_options_default(cg_options* opt, int precision);

typedef struct cg_lbm cg_lbm;

/* Create a run.  tau_r, tau_b > 1/2 (Eq. 13), 0 <= beta <= 1 (Eq. 17),
 * 0 < theta < 180 when a scheme is set.  Performs the once-per-run setup on
 * the host (voxel classes, boundary sets F_b and S_b along lattice links,
 * three smoothing passes and the wall normal of Eqs. 25-26 in FP64, the
 * sparse fluid-node index and pull table), uploads it, and leaves the state
 * at rest with phi = -1 (all fluid b).  Errors: CG_EINVAL, CG_EUNSUPPORTED
 * (MRT or Zou-He with dim = 2; more than 2^27 voxels; fluid nodes, rounded up
 * to 256, times Q reaching 2^31; a 16-byte-per-voxel grid reaching 2^32
 * bytes), CG_ENOMEM, CG_EHIP.  *out receives the handle. */
cg_status cg_lbm_create(const cg_geometry* geom, double tau_r, double tau_b, double sigma, double beta,
                        const cg_wetting* wet, const cg_bc* bc, const cg_options* opt, cg_lbm** out);

/* Free everything the handle owns (synchronises its stream first). */
void cg_lbm_destroy(cg_lbm* h);

/* Thread-local message of the last failure. */
const char* cg_last_error(void);

/* Initial state at rest: f^s_i = w_i rho^s with rho^r = rho0 (1 + phi)/2 and
 * rho^b = rho0 (1 - phi)/2 at every fluid voxel.  phi0: host, V doubles. */
cg_status cg_lbm_set_phase(cg_lbm* h, const double* phi0);

/* Set the state: canonical pre-collision populations fr, fb ([Q][V] doubles,
 * solid entries ignored), host or device memory. */
cg_status cg_lbm_set_state(cg_lbm* h, const double* fr, const double* fb, int src_is_device);

/* Enqueue n time steps on the handle's stream; returns without waiting. */
cg_status cg_lbm_step(cg_lbm* h, int64_t n);

/* Wait for the handle's stream. */
cg_status cg_lbm_sync(cg_lbm* h);

/* Number of completed steps. */
int64_t cg_lbm_time(const cg_lbm* h);

typedef struct {
  int64_t step;
  double mass_r, mass_b;        /* sum of rho^r, rho^b over fluid nodes (FP64 accumulation) */
  double n_fluid;               /* fluid nodes counted (finite ones) */
  double sat_w;                 /* #{phi < 0} / #fluid (Sec. IV.B) */
  double sat_nw_mass;           /* sum rho^r / sum rho */
  double flux_t, flux_r, flux_b;/* sum of rho u_a, rho^r u_a, rho^b u_a over the plane */
  double vol_r, vol_b;          /* sum (1 + phi)/2, sum (1 - phi)/2 */
  double p_in, p_out;           /* mean rho/3 (Eq. 23) over phi > 0.9 / phi < -0.9 */
  double n_in, n_out;
  double u_max;                 /* max |u| (Eq. 22) */
  double nan_count;             /* fluid nodes with a non-finite density or velocity */
} cg_observables;

/* Reductions over the current state (wavefront shuffles, then a fixed-order
 * second pass); axis/plane choose the flux plane (axis < 0: no flux).
 * Synchronises the stream.  Returns CG_EUNSTABLE if nan_count > 0 (out is
 * still filled). */
cg_status cg_lbm_observe(cg_lbm* h, int axis, int plane, cg_observables* out);

/* The reductions of cg_lbm_observe restricted to the fluid nodes with
 * lo <= coordinate[slab_axis] < hi (for example the porous sample between
 * the inlet and outlet buffer layers, over which Sec. IV.B counts the
 * wetting saturation); the plane flux (axis, plane) is still summed over its
 * whole plane.  CG_EINVAL for an empty or out-of-box slab; CG_EUNSTABLE if a
 * node of the slab is not finite.  Synchronises the stream. */
cg_status cg_lbm_observe_slab(cg_lbm* h, int slab_axis, int lo, int hi, int axis, int plane, cg_observables* out);

/* cg_lbm_observe for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same reductions and results, with the per-block partial sums and the
 * final sums kept in a 4 MiB array that the library holds in static device
 * memory on every device it runs on (until the process ends), instead of
 * memory the run allocated.  The call allocates nothing (no hipMalloc, no
 * allocator callback).  Limit: runs of at most 8,947,456 fluid nodes (one
 * partial record of 15 doubles per block of 256 nodes must fit); larger runs
 * get CG_EINVAL and a message.  All calls on one device share that device's
 * array, so calls that overlap on one device (other threads, other handles)
 * race; calls on one handle are serialised anyway.  Synchronises the stream.
 * Returns CG_EUNSTABLE if nan_count > 0 (out is still filled). */
cg_status cg_lbm_observe_noalloc(cg_lbm* h, int axis, int plane, cg_observables* out);

enum {
  CG_FIELD_RHO_R = 0, /* [V] */
  CG_FIELD_RHO_B = 1, /* [V] */
  CG_FIELD_PHI = 2,   /* [V] phase field at fluid nodes and solid boundary points */
  CG_FIELD_U = 3,     /* [3][V] velocity, Eq. (22) */
  CG_FIELD_F_R = 4,   /* [Q][V] canonical pre-collision red populations */
  CG_FIELD_F_B = 5,   /* [Q][V] canonical pre-collision blue populations */
  CG_FIELD_N = 6,     /* [3][V] interface normal after wetting, fluid and S_b */
  CG_FIELD_C = 7,     /* [3][V] colour gradient after wetting, fluid */
  CG_FIELD_KAPPA = 8, /* [V] curvature, Eq. (12) */
  CG_FIELD_FORCE = 9  /* [3][V] total force, Eq. (5) plus rho_o g */
};

/* Copy a field of the current state into dst (doubles, dense; entries where
 * the field is undefined are 0).  dst_is_device: dst is device memory on the
 * handle's device.  Synchronises the stream. */
cg_status cg_lbm_get_field(cg_lbm* h, int which, double* dst, int dst_is_device);

typedef struct {
  int dim, q, nx, ny, nz, precision, collision;
  int64_t voxels, fluid, fluid_boundary, solid_boundary, inlet, outlet;
  int64_t state_bytes;   /* bytes of one state copy on the device */
  int64_t device_bytes;  /* all device memory owned by the handle */
  int pull_bits;         /* narrowest neighbour table built: 8, 16 or 32 */
  int pull_fallback_bits;  /* the table that waves not fitting the 8-bit one
                              read: 16 or 32 (0 when pull_bits is 16 or 32) */
  int64_t pull_waves;      /* waves of 64 nodes */
  int64_t pull_waves_8bit; /* waves that read the 8-bit table */
} cg_info;

cg_status cg_lbm_info(const cg_lbm* h, cg_info* out);

/* Opaque device-state snapshot (checkpoint / resume, bitwise).  dst/src are
 * caller-owned host buffers of cg_lbm_snapshot_bytes() bytes: a 64-byte header
 * (time step, a fingerprint of precision, lattice, box and fluid node list)
 * and the state.  Loading restores the state and the time step, not the
 * parameters (angles, body force), and continues bit for bit as the run that
 * saved it.  cg_lbm_load returns CG_EINVAL when the snapshot comes from a run
 * of another geometry, lattice or precision.  Both calls synchronise the
 * handle's stream. */
int64_t cg_lbm_snapshot_bytes(const cg_lbm* h);
cg_status cg_lbm_save(cg_lbm* h, void* dst);
cg_status cg_lbm_load(cg_lbm* h, const void* src);

/* Kernel timing: mask selects the kernels whose every launch carries HIP
 * events on the handle's stream, attached to the dispatch (hipExtLaunchKernel),
 * so that they time the kernel's own start and end (bit k = k-th kernel in the order
 * cg_lbm_kernel_times reports: k_phase, k_sb_phi, k_normal, k_sb_n, k_curv,
 * k_main, k_face; -1 = all, 0 = off).  A time step runs k_phase, k_sb_phi,
 * k_normal, k_sb_n and k_main (which evaluates the curvature and force of its
 * node); in a single-precision run with Zou-He faces the face stage (the
 * outlet's upstream phase, the faces' unknowns at the face nodes) shares the
 * k_sb_phi launch and is timed with it; k_face counts its launches of its
 * own (state export and staging); k_curv stores the curvature and force for
 * the reverse steps of the adjoint.
 * cg_lbm_kernel_times synchronises, then reports for each kernel its name,
 * launch count and total milliseconds since the last reset (n: in =
 * capacity, out = count). */
cg_status cg_lbm_set_timing(cg_lbm* h, int mask);
/* Step replay from HIP graphs (on != 0): each step's launches are captured
 * once per ping-pong parity (on a stream of the handle's own) and replayed
 * on the handle's stream; a graph is captured again when the run's
 * parameters (cg_lbm_set_wetting, _set_body_force, _set_pressure,
 * _switch_inlet) or block sizes (cg_lbm_tune) have changed since.  Results
 * are those of the plain launches, bit for bit.  Steps with kernel timing on
 * and the first step after a state set from the host run as plain launches.
 * on = 0 releases the graphs.  Saves the launch overhead of small runs. */
cg_status cg_lbm_set_graph(cg_lbm* h, int on);
/* Number of step graphs the handle has captured so far (-1: NULL handle). */
int64_t cg_lbm_graph_captures(const cg_lbm* h);
cg_status cg_lbm_kernel_times(cg_lbm* h, char (*names)[32], int64_t* counts, double* total_ms, int* n);
cg_status cg_lbm_reset_timing(cg_lbm* h);

/* Block-size autotuner of one run: times reps steps with every kernel at 64,
 * then 128, then 256 threads per block (the kernel timers' events) and
 * keeps the fastest size per kernel for the run's later steps.  Advances the
 * run by 3 * reps steps (tune before taking the steps that matter).  report
 * (may be NULL) receives the choice and the times. */
cg_status cg_lbm_tune(cg_lbm* h, int reps, char* report, size_t report_len);

/* ---------------------------------------------------------------------- */
/* Parameters that can change between calls. */

/* New contact angles: the global angle (theta_field_deg NULL) or a per-voxel
 * field on the solid voxels (dense, V entries, host memory; a fluid boundary
 * point takes the w_i-weighted mean over its solid link neighbours, as at
 * creation).  Every angle must lie in (0, 180) degrees.  The Scheme-I secant
 * start sign follows the new angle.  Synchronises the stream.  A batch that
 * holds this run sees the new angles (it references the run's arrays). */
cg_status cg_lbm_set_wetting(cg_lbm* h, double theta_deg, const double* theta_field_deg);

/* New body-force acceleration g (Eq. 36; force density rho_o g) for the
 * following steps.  Synchronises the stream.  A batch that holds this run
 * picks up the new value at its next step. */
cg_status cg_lbm_set_body_force(cg_lbm* h, const double g[3]);

/* New Zou-He inlet and outlet densities (Appendix B, Eqs. B.1 and B.9) for
 * the following steps, e.g. the pressure stages of a drainage or imbibition
 * protocol (Sec. IV.B).  rho_in, rho_out > 0.  CG_EINVAL unless the run has
 * CG_BC_ZOUHE faces.  Synchronises the stream; a batch that holds the run
 * picks up the new values at its next step. */
cg_status cg_lbm_set_pressure(cg_lbm* h, double rho_in, double rho_out);

/* Replace the fluid injected at the inlet in a running simulation (Sec.
 * II.D.1, Eqs. 37-38): at every inlet node the pre-collision populations of
 * the previously injected colour are added to those of the new colour and
 * then cleared, and the following steps inject the new fluid (zeta_r = 1:
 * red, 0: blue; the inlet phase becomes +1 or -1).  The state is first
 * written out as pre-collision populations at their own nodes (what the
 * next step would pull), so the totals at every node are unchanged.
 * CG_EINVAL unless the run has CG_BC_ZOUHE faces and zeta_r is 0 or 1.
 * Synchronises the stream. */
cg_status cg_lbm_switch_inlet(cg_lbm* h, double zeta_r);

/* ---------------------------------------------------------------------- */
/* Geometric observables of the phase field (on the device). */

/* One grid line of the voxel box: the voxels with coordinate at[a] on every
 * axis a != axis, and lo <= coordinate[axis] < hi.  blend in [0, 1): the
 * profile is (1 - blend) phi(line) + blend phi(line shifted by one voxel
 * along blend_axis), for a line that lies between two grid lines (blend = 0:
 * the line itself; blend_axis is then ignored). */
typedef struct {
  int axis;
  int at[3];
  int lo, hi;
  int blend_axis;
  double blend;
} cg_line;

/* Interface points along a line: the positions (in voxel coordinates along
 * the axis) where the linearly interpolated phase field of the current state
 * (fluid nodes and solid boundary points) is zero, ascending.  points: host,
 * max_points (<= 256) entries; *n_points receives the total count (more than
 * max_points when there are more crossings; only max_points are written).
 * The phase field is computed on the device and read along the line by one
 * wavefront; nothing else crosses to the host.  CG_EINVAL for a line outside
 * the box.  Synchronises the stream. */
cg_status cg_lbm_line_crossings(cg_lbm* h, const cg_line* line, double* points, int max_points, int* n_points);

/* Sessile drop on a flat wall (Sec. III.B, Eqs. 45-46), from the phase field
 * in the plane spanned by base_axis and wall_axis (3D: at coordinate `slice`
 * on the third axis).  The base b is the distance between the first and last
 * interface points on the fluid row `row` next to the wall; the height h is
 * the first interface point above `row` on the drop's axis (the base's
 * midpoint, interpolated between the two nearest grid lines), measured from
 * the wall position `wall` (0.5 for a halfway bounce-back wall whose first
 * fluid row is 1).  radius = (4 h^2 + b^2) / (8 h) (Eq. 46); theta_deg =
 * atan2(b/2, radius - h) in degrees (Eq. 45 extended past 90 degrees): the
 * angle through the drop's own fluid.  CG_EINVAL when the row has fewer than
 * two interface points or the axis none above the row.  Synchronises the
 * stream. */
typedef struct {
  double base, height, radius, theta_deg;
  int n_base_points;
} cg_drop;

cg_status cg_lbm_drop_shape(cg_lbm* h, int base_axis, int wall_axis, int slice, double wall, int row, cg_drop* out);

/* ---------------------------------------------------------------------- */
/* Discrete adjoint (reverse mode) of n_steps time steps from the current
 * state.  J is an objective of the state after n_steps:
 *   CG_OBJ_SATURATION  sum rho^r / sum rho over the fluid nodes of the slab
 *                      lo <= coordinate[axis] < hi (the non-wetting mass
 *                      saturation of Sec. IV.B restricted to a region);
 *   CG_OBJ_RED_VOLUME  sum (1 + phi)/2 over the same slab (divided by the
 *                      slab's cross-section it is the volume-based interface
 *                      position of a displacement along axis);
 *   CG_OBJ_FLUX        sum rho u_axis (Eq. 22) over the fluid nodes of the
 *                      plane coordinate[axis] == lo.
 * The call returns J and its exact discrete derivative (every branch of the
 * step is held fixed: thresholds, the Scheme-I secant iterations and the
 * Scheme-II candidate choice) with respect to the global contact angle (per
 * degree; with a per-voxel field it is the derivative along a uniform shift
 * of the field), the per-voxel field, and the body-force acceleration g.
 * With the fictitious-density model the angle enters through the fixed phase
 * -cos(theta) of each solid boundary point (Eq. 24), so the field gradient
 * sits on those points' own voxels.
 * The forward sweep stores the state every checkpoint_every = K steps (the
 * segments counted from the end, the first one holding the remainder) and
 * keeps the last K states; the reverse sweep recomputes the states of each
 * earlier segment into a ring of K state buffers, so the first n_steps - K
 * states are computed twice (none with K >= n_steps) and the device memory
 * held during the call is about (n_steps/K + K + 2) state copies
 * (cg_info.state_bytes each, plus the front fields of K states) plus the adjoint
 * fields.  delta > 0 replaces |C| by max(|C|, delta) in the Jacobian of
 * n = C/|C| (Eq. 27) only; the forward arithmetic is unchanged; 0 keeps the
 * exact derivative.  Every boundary of the step is covered: closed and
 * periodic axes, the body force, and the Zou-He faces (Appendix B), whose
 * runs also return the derivatives with respect to the inlet and outlet
 * densities; an objective slab or plane may include the face layers (J then
 * reads the face nodes' populations after the faces, as the next collision
 * does).  The handle's state and step counter are left as they were.
 * Synchronises the stream. */
enum { CG_OBJ_SATURATION = 0, CG_OBJ_RED_VOLUME = 1, CG_OBJ_FLUX = 2 };

typedef struct {
  int objective;
  int axis;                  /* 0, 1 or 2 (< dim) */
  int lo, hi;                /* slab bounds (objectives 0, 1) or the plane (lo, objective 2) */
  int64_t n_steps;           /* >= 1 */
  int64_t checkpoint_every;  /* K >= 1 (values above n_steps act as n_steps) */
  double delta;              /* >= 0 */
} cg_adjoint_spec;

typedef struct {
  double J;                  /* out */
  double dJ_dtheta;          /* out: per degree */
  double dJ_dg[3];           /* out: per unit of acceleration */
  double* dJ_dtheta_field;   /* in: NULL or a device buffer of V doubles on the handle's device;
                                out: dJ/dtheta(x) (per degree) at the solid voxels next to the fluid,
                                0 elsewhere */
  double ms_forward;         /* out: GPU time of the forward sweep */
  double ms_reverse;         /* out: GPU time of the reverse sweep, recomputation included */
  int64_t work_bytes;        /* out: device memory the call allocated */
  double dJ_drho_in;         /* out: per unit of the Zou-He inlet density rho_in (0 without the faces) */
  double dJ_drho_out;        /* out: per unit of the Zou-He outlet density rho_out (0 without the faces) */
} cg_gradients;

cg_status cg_lbm_adjoint(cg_lbm* h, const cg_adjoint_spec* spec, cg_gradients* out);

/* ---------------------------------------------------------------------- */
/* Batched runs.  Many runs of one precision, one lattice and one stream
 * advance together: each stage of the step is one persistent launch over a
 * table of (run, tile) pairs for all runs, and the step loop is replayed from
 * a captured hipGraph.  The batch references the runs' device state and does
 * not own the runs: they must outlive it.  A run of a batch can still be
 * observed, read or stepped on its own through its cg_lbm handle (call
 * cg_batch_sync first); its step counter and buffers stay consistent. */
typedef struct cg_batch cg_batch;

/* runs: n >= 1 handles (caller-owned array, copied).  Errors: CG_EINVAL when
 * precision, lattice or stream differ. */
cg_status cg_batch_create(cg_lbm* const* runs, int n, cg_batch** out);
void cg_batch_destroy(cg_batch* b);
/* Enqueue n steps of every run (asynchronous). */
cg_status cg_batch_step(cg_batch* b, int64_t n);
cg_status cg_batch_sync(cg_batch* b);
/* Observables of run i (0 <= i < n, the order given to cg_batch_create) after
 * the batch's queued steps: waits for them, then does what cg_lbm_observe does
 * on that run's handle (same axis/plane arguments and errors). */
cg_status cg_batch_observe(cg_batch* b, int i, int axis, int plane, cg_observables* out);
/* on = 0: enqueue the stage launches directly instead of replaying a graph. */
cg_status cg_batch_set_graph(cg_batch* b, int on);
/* Autotuner: for every stage, time each block size in {64, 128, 256} and
 * persistent grid size in {one block per tile, 4, 8, 16, 32 blocks per CU}
 * over reps launches on the batch's own data, keep the fastest, and cache the
 * choice in $CGLBM_TUNE_CACHE (default ~/.cache/cglbm_autotune.txt) keyed by
 * architecture, lattice, precision and batch size class.  Takes one step
 * first when a run's state was just set.  report (may be NULL) receives a
 * summary. */
cg_status cg_batch_tune(cg_batch* b, int reps, char* report, size_t report_len);
/* total fluid nodes; chosen block and grid per stage (6 entries each, stages
 * in step order: phase, face (the Zou-He face nodes of single-precision
 * runs), sb_phi, normal, sb_n, main; grid 0 = one block per tile) */
cg_status cg_batch_info(const cg_batch* b, int64_t* total_nodes, int* block, int* grid);
/* Number of step graphs the batch has captured: one per starting ping-pong
 * parity, so at most 2 until the configuration changes (cg_batch_tune,
 * cg_batch_set_graph); -1 for a NULL batch. */
int64_t cg_batch_graph_captures(const cg_batch* b);

/* ---------------------------------------------------------------------- */
/* Measurement: streaming reference kernels for the HBM roofline. */

/* Time `reps` launches (after one untimed launch) of a plain streaming kernel
 * over `bytes` bytes of device memory on `stream` (a hipStream_t, NULL = the
 * default stream) and store the mean milliseconds per launch.  kind 0 reads
 * src (dst: 16 writable bytes that are written only in a case that cannot
 * occur), 1 writes dst, 2 copies src to dst.  The kernels move float4
 * elements with a grid-stride loop of grid blocks of `block` threads (64 to
 * 1024, a multiple of 64), four elements in flight per thread;
 * nontemporal != 0 marks every access as streaming.  Bytes moved per launch:
 * bytes (read, write) or 2 * bytes (copy).  src/dst: device pointers aligned
 * to 16 bytes; bytes a multiple of 16.  Errors: CG_EINVAL, CG_EHIP.
 * Synchronises the stream. */
cg_status cg_stream_probe(int kind, const void* src, void* dst, size_t bytes, int grid, int block,
                          int nontemporal, void* stream, int reps, float* ms_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* CG_LBM_H */
