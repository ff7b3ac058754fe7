// C ABI of libcglbm.so (declarations and contracts in include/cg_lbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cg_lbm.h"
#include "batch_base.hpp"
#include "engine_base.hpp"
#include "handle.hpp"
#include "setup.hpp"

namespace {
thread_local std::string g_err;
cg_status fail(cg_status s, const std::string& m) {
  g_err = m;
  return s;
}
}  // namespace

cg_status cg::set_error(cg_status s, const std::string& msg) { return fail(s, msg); }

namespace {

cg_status engine_status(cg_lbm* h, int rc) {
  if (rc == CG_OK) return CG_OK;
  return fail((cg_status)rc, h->eng->err_.empty() ? std::string("device engine error") : h->eng->err_);
}

struct DevTemp {
  cg_lbm* h;
  double* p = nullptr;
  size_t bytes = 0;
  DevTemp(cg_lbm* h_, size_t b) : h(h_), bytes(b) { p = (double*)h->al.get(b); }
  ~DevTemp() {
    if (p) {
      (void)hipStreamSynchronize(h->stream);
      h->al.put(p);
    }
  }
};

}  // namespace

extern "C" {

const char* cg_last_error(void) { return g_err.c_str(); }

void cg_options_default(cg_options* opt, int precision) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = precision;
  opt->collision = CG_MRT;
  opt->rho0 = 1.0;
  opt->eps_c = 1e-6;
  opt->eps_f = precision == CG_FP64 ? 1e-12 : 1e-6;
  opt->eps_v = precision == CG_FP64 ? 1e-12 : 1e-6;
  opt->device = 0;
  opt->block = 0;
}

cg_status cg_lbm_create(const cg_geometry* geom, double tau_r, double tau_b, double sigma, double beta,
                        const cg_wetting* wet, const cg_bc* bc, const cg_options* opt, cg_lbm** out) {
  if (!out) return fail(CG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!geom || !geom->solid) return fail(CG_EINVAL, "geometry or solid mask is NULL");
  cg_wetting w{};
  if (wet) w = *wet;
  cg_bc b{};
  if (bc) b = *bc;
  cg_options o;
  if (opt)
    o = *opt;
  else
    cg_options_default(&o, CG_FP32);
  if (!(tau_r > 0.5) || !(tau_b > 0.5)) return fail(CG_EINVAL, "tau_r and tau_b must exceed 1/2");
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(CG_EINVAL, "beta must lie in [0, 1]");
  if (!std::isfinite(sigma)) return fail(CG_EINVAL, "sigma must be finite");
  if (w.scheme < 0 || w.scheme > 3) return fail(CG_EINVAL, "unknown wetting scheme");
  if (w.scheme != 0 && !w.theta_field_deg && !(w.theta_deg > 0.0 && w.theta_deg < 180.0))
    return fail(CG_EINVAL, "theta must lie in (0, 180) degrees");
  if (b.type != CG_BC_NONE && b.type != CG_BC_ZOUHE) return fail(CG_EINVAL, "unknown boundary type");
  if (b.type == CG_BC_ZOUHE && !(b.zeta_r >= 0.0 && b.zeta_r <= 1.0))
    return fail(CG_EINVAL, "zeta_r must lie in [0, 1]");
  if (o.precision != CG_FP32 && o.precision != CG_FP64) return fail(CG_EINVAL, "unknown precision");
  if (o.collision != CG_BGK && o.collision != CG_MRT) return fail(CG_EINVAL, "unknown collision");
  if (geom->dim == 2 && o.collision == CG_MRT) return fail(CG_EUNSUPPORTED, "MRT is defined for D3Q19 only");
  if (geom->dim == 2 && b.type == CG_BC_ZOUHE) return fail(CG_EUNSUPPORTED, "Zou-He faces are defined for D3Q19");
  if (!(o.rho0 > 0.0)) return fail(CG_EINVAL, "rho0 must be positive");
  if (o.pull_table != 0 && o.pull_table != 8 && o.pull_table != 16 && o.pull_table != 32)
    return fail(CG_EINVAL, "pull_table must be 0, 8, 16 or 32");
  if (w.theta_field_deg) {
    const long V = (long)geom->nx * geom->ny * geom->nz;
    for (long v = 0; v < V; ++v)
      if (geom->solid[v] && !(w.theta_field_deg[v] > 0.0 && w.theta_field_deg[v] < 180.0))
        return fail(CG_EINVAL, "theta field must lie in (0, 180) degrees on solid voxels");
  }

  std::unique_ptr<cg_lbm> h(new cg_lbm());
  h->device = o.device;
  h->precision = o.precision;
  h->collision = o.collision;
  if (hipSetDevice(o.device) != hipSuccess) return fail(CG_EHIP, "hipSetDevice failed");
  h->stream = (hipStream_t)o.stream;
  h->al.fn = o.alloc;
  h->al.fr = o.free;
  h->al.ctx = o.alloc_ctx;
  std::string err;
  int rc = cg::build_setup(*geom, w, b, &h->S, &err, o.pull_table);
  if (rc != CG_OK) return fail((cg_status)rc, err);
  const cg::HostSetup& S = h->S;
  cg::StepParams& P = h->P;
  P.nx = S.nx;
  P.ny = S.ny;
  P.nz = S.nz;
  P.N = S.N;
  P.Np = S.Np;
  P.nsb = (int)S.sb_vox.size();
  P.V = S.V;
  for (int a = 0; a < 3; ++a) P.per[a] = S.per[a];
  P.bc = b.type;
  P.n_in = b.type == CG_BC_ZOUHE ? S.n_in : 0;
  P.n_out = b.type == CG_BC_ZOUHE ? S.n_out : 0;
  P.scheme = w.scheme;
  P.collision = o.collision;
  P.half_sigma = 0.5 * sigma;
  P.beta = beta;
  P.rho0 = o.rho0;
  P.nu_r = (tau_r - 0.5) / 3.0;
  P.nu_b = (tau_b - 0.5) / 3.0;
  P.hinv_nu_r = (float)(0.5 / P.nu_r);
  P.hinv_nu_b = (float)(0.5 / P.nu_b);
  for (int a = 0; a < 3; ++a) P.rg[a] = o.rho0 * b.g[a];
  if (geom->dim == 2) P.rg[2] = 0.0;
  P.rin_r = b.rho_in * b.zeta_r;
  P.rin_b = b.rho_in * (1.0 - b.zeta_r);
  P.rho_in = b.rho_in;
  P.rho_out = b.rho_out;
  P.phi_in = b.zeta_r - (1.0 - b.zeta_r);
  P.zeta_r = b.zeta_r;
  P.eps_c = o.eps_c;
  P.eps_f = o.eps_f;
  P.eps_v = o.eps_v;
  P.flux_axis = -1;
  P.flux_plane = 0;
  P.slab_axis = -1;
  P.slab_lo = P.slab_hi = 0;
  h->eng.reset(o.precision == CG_FP64 ? cg::make_engine_f64() : cg::make_engine_f32());
  rc = h->eng->init(S, P, o.block, &h->al, h->stream, &err);
  if (rc != CG_OK) {
    if (err.empty()) return engine_status(h.get(), rc);
    return fail((cg_status)rc, err);
  }
  *out = h.release();
  return CG_OK;
}

void cg_lbm_destroy(cg_lbm* h) { delete h; }

cg_status cg_lbm_set_phase(cg_lbm* h, const double* phi0) {
  if (!h || !phi0) return fail(CG_EINVAL, "NULL argument");
  std::vector<double> pn(h->S.N);
  for (int n = 0; n < h->S.N; ++n) pn[n] = phi0[h->S.node_vox[n]];
  h->eng->t = 0;
  return engine_status(h, h->eng->set_phase_nodes(pn.data()));
}

cg_status cg_lbm_set_state(cg_lbm* h, const double* fr, const double* fb, int src_is_device) {
  if (!h || !fr || !fb) return fail(CG_EINVAL, "NULL argument");
  return engine_status(h, h->eng->set_state_dense(fr, fb, src_is_device != 0));
}

cg_status cg_lbm_step(cg_lbm* h, int64_t n) {
  if (!h || n < 0) return fail(CG_EINVAL, "bad argument");
  return engine_status(h, h->eng->step(n));
}

cg_status cg_lbm_sync(cg_lbm* h) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(CG_EHIP, hipGetErrorString(hipGetLastError()));
  return CG_OK;
}

int64_t cg_lbm_time(const cg_lbm* h) { return h ? h->eng->t : -1; }

cg_status cg_lbm_observe(cg_lbm* h, int axis, int plane, cg_observables* out) {
  if (!h || !out) return fail(CG_EINVAL, "NULL argument");
  double o[cg::kObsN];
  int rc = h->eng->observe(axis, plane, o);
  if (rc != CG_OK) return engine_status(h, rc);
  if (cg::fill_observables(o, h->eng->t, out) > 0)
    return fail(CG_EUNSTABLE, "non-finite density or velocity in the state");
  return CG_OK;
}

cg_status cg_lbm_observe_slab(cg_lbm* h, int slab_axis, int lo, int hi, int axis, int plane, cg_observables* out) {
  if (!h || !out) return fail(CG_EINVAL, "NULL argument");
  const int n[3] = {h->S.nx, h->S.ny, h->S.nz};
  if (slab_axis < 0 || slab_axis >= h->S.dim || lo < 0 || hi <= lo || hi > n[slab_axis])
    return fail(CG_EINVAL, "bad slab");
  double o[cg::kObsN];
  int rc = h->eng->observe_slab(axis, plane, slab_axis, lo, hi, o);
  if (rc != CG_OK) return engine_status(h, rc);
  if (cg::fill_observables(o, h->eng->t, out) > 0)
    return fail(CG_EUNSTABLE, "non-finite density or velocity in the slab");
  return CG_OK;
}

cg_status cg_lbm_get_field(cg_lbm* h, int which, double* dst, int dst_is_device) {
  if (!h || !dst) return fail(CG_EINVAL, "NULL argument");
  const size_t V = (size_t)h->S.V, Q = (size_t)h->S.Q;
  size_t comps;
  switch (which) {
    case CG_FIELD_RHO_R:
    case CG_FIELD_RHO_B:
    case CG_FIELD_PHI:
    case CG_FIELD_KAPPA:
      comps = 1;
      break;
    case CG_FIELD_U:
    case CG_FIELD_N:
    case CG_FIELD_C:
    case CG_FIELD_FORCE:
      comps = 3;
      break;
    case CG_FIELD_F_R:
    case CG_FIELD_F_B:
      comps = Q;
      break;
    default:
      return fail(CG_EINVAL, "unknown field");
  }
  const size_t bytes = sizeof(double) * comps * V;
  std::unique_ptr<DevTemp> tmp;
  double* d = dst;
  if (!dst_is_device) {
    tmp.reset(new DevTemp(h, bytes));
    if (!tmp->p) return fail(CG_ENOMEM, "device temporary");
    d = tmp->p;
  }
  if (hipMemsetAsync(d, 0, bytes, h->stream) != hipSuccess) return fail(CG_EHIP, "memset");
  int rc = CG_OK;
  switch (which) {
    case CG_FIELD_RHO_R: rc = h->eng->macro(d, nullptr, nullptr, nullptr, nullptr, nullptr); break;
    case CG_FIELD_RHO_B: rc = h->eng->macro(nullptr, d, nullptr, nullptr, nullptr, nullptr); break;
    case CG_FIELD_U: rc = h->eng->macro(nullptr, nullptr, d, nullptr, nullptr, nullptr); break;
    case CG_FIELD_KAPPA: rc = h->eng->macro(nullptr, nullptr, nullptr, d, nullptr, nullptr); break;
    case CG_FIELD_FORCE: rc = h->eng->macro(nullptr, nullptr, nullptr, nullptr, d, nullptr); break;
    case CG_FIELD_C: rc = h->eng->macro(nullptr, nullptr, nullptr, nullptr, nullptr, d); break;
    case CG_FIELD_PHI: rc = h->eng->phi_grid(d); break;
    case CG_FIELD_N: rc = h->eng->n_grid(d); break;
    case CG_FIELD_F_R:
    case CG_FIELD_F_B: {
      DevTemp other(h, bytes);
      if (!other.p) return fail(CG_ENOMEM, "device temporary");
      rc = which == CG_FIELD_F_R ? h->eng->export_pops(d, other.p) : h->eng->export_pops(other.p, d);
      break;
    }
  }
  if (rc != CG_OK) return engine_status(h, rc);
  if (!dst_is_device) {
    if (hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
      return fail(CG_EHIP, "copy to host");
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(CG_EHIP, "stream sync");
  return CG_OK;
}

cg_status cg_lbm_info(const cg_lbm* h, cg_info* out) {
  if (!h || !out) return fail(CG_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->dim = h->S.dim;
  out->q = h->S.Q;
  out->nx = h->S.nx;
  out->ny = h->S.ny;
  out->nz = h->S.nz;
  out->precision = h->precision;
  out->collision = h->collision;
  out->voxels = h->S.V;
  out->fluid = h->S.N;
  out->fluid_boundary = h->S.n_fb;
  out->solid_boundary = (int64_t)h->S.sb_vox.size();
  out->inlet = h->S.n_in;
  out->outlet = h->S.n_out;
  out->state_bytes = (int64_t)h->eng->state_bytes();
  out->device_bytes = (int64_t)h->eng->device_bytes();
  const bool t16 = !h->S.nbr16.empty();
  out->pull_bits = !h->S.nbr8.empty() ? 8 : (t16 ? 16 : 32);
  out->pull_fallback_bits = out->pull_bits != 8 ? 0 : (t16 ? 16 : 32);
  out->pull_waves = (int64_t)h->S.Np / 64;
  out->pull_waves_8bit = (int64_t)h->S.n8_waves;
  return CG_OK;
}

int64_t cg_lbm_snapshot_bytes(const cg_lbm* h) { return h ? (int64_t)h->eng->snapshot_bytes() : -1; }

cg_status cg_lbm_save(cg_lbm* h, void* dst) {
  if (!h || !dst) return fail(CG_EINVAL, "NULL argument");
  return engine_status(h, h->eng->save(dst));
}

cg_status cg_lbm_load(cg_lbm* h, const void* src) {
  if (!h || !src) return fail(CG_EINVAL, "NULL argument");
  int rc = h->eng->load(src);
  if (rc == CG_EINVAL) return fail(CG_EINVAL, "snapshot does not match this run");
  return engine_status(h, rc);
}

cg_status cg_lbm_set_timing(cg_lbm* h, int mask) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  h->eng->set_timing(mask);
  return CG_OK;
}

cg_status cg_lbm_set_graph(cg_lbm* h, int on) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  h->eng->set_graph(on != 0);
  return CG_OK;
}

int64_t cg_lbm_graph_captures(const cg_lbm* h) { return h ? h->eng->graph_captures() : -1; }

cg_status cg_lbm_set_wetting(cg_lbm* h, double theta_deg, const double* theta_field_deg) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  if (!theta_field_deg && !(theta_deg > 0.0 && theta_deg < 180.0))
    return fail(CG_EINVAL, "theta must lie in (0, 180) degrees");
  std::vector<double> ct = h->S.cos_t, st = h->S.sin_t, fd = h->S.sb_fd;
  std::vector<unsigned> fl = h->S.flags;
  std::string err;
  int rc = cg::contact_angles(h->S, theta_deg, theta_field_deg, &ct, &st, &fl, &fd, &err);
  if (rc != CG_OK) return fail((cg_status)rc, err);
  rc = h->eng->set_angles(ct.data(), st.data(), fl.data(), fd.data());
  if (rc != CG_OK) return engine_status(h, rc);
  h->S.cos_t.swap(ct);
  h->S.sin_t.swap(st);
  h->S.flags.swap(fl);
  h->S.sb_fd.swap(fd);
  return CG_OK;
}

cg_status cg_lbm_set_body_force(cg_lbm* h, const double g[3]) {
  if (!h || !g) return fail(CG_EINVAL, "NULL argument");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g[a])) return fail(CG_EINVAL, "g must be finite");
  return engine_status(h, h->eng->set_body_force(g));
}

cg_status cg_lbm_set_pressure(cg_lbm* h, double rho_in, double rho_out) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  if (h->P.bc != CG_BC_ZOUHE) return fail(CG_EINVAL, "inlet/outlet densities need Zou-He faces");
  if (!(rho_in > 0.0 && std::isfinite(rho_in)) || !(rho_out > 0.0 && std::isfinite(rho_out)))
    return fail(CG_EINVAL, "densities must be positive and finite");
  return engine_status(h, h->eng->set_pressure(rho_in, rho_out));
}

cg_status cg_lbm_switch_inlet(cg_lbm* h, double zeta_r) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  if (h->P.bc != CG_BC_ZOUHE) return fail(CG_EINVAL, "the injected fluid needs Zou-He faces");
  if (zeta_r != 0.0 && zeta_r != 1.0) return fail(CG_EINVAL, "the new injected fluid must be pure (zeta_r 0 or 1)");
  return engine_status(h, h->eng->switch_inlet(zeta_r));
}

cg_status cg_lbm_line_crossings(cg_lbm* h, const cg_line* line, double* points, int max_points, int* n_points) {
  if (!h || !line || !n_points || (max_points > 0 && !points)) return fail(CG_EINVAL, "NULL argument");
  if (max_points < 0 || max_points > cg::kLineMax) return fail(CG_EINVAL, "max_points must lie in [0, 256]");
  const int dim = h->S.dim;
  const int n[3] = {h->S.nx, h->S.ny, h->S.nz};
  const int st[3] = {1, h->S.nx, h->S.nx * h->S.ny};
  const int a = line->axis;
  if (a < 0 || a >= dim) return fail(CG_EINVAL, "axis outside the lattice's dimensions");
  if (!(line->lo >= 0 && line->lo < line->hi && line->hi <= n[a])) return fail(CG_EINVAL, "bad lo/hi");
  int at[3] = {line->at[0], line->at[1], dim == 3 ? line->at[2] : 0};
  at[a] = 0;
  for (int k = 0; k < 3; ++k)
    if (at[k] < 0 || at[k] >= n[k]) return fail(CG_EINVAL, "line outside the box");
  int shift = 0;
  const double t = line->blend;
  if (!(t >= 0.0 && t < 1.0)) return fail(CG_EINVAL, "blend must lie in [0, 1)");
  if (t > 0.0) {
    const int b = line->blend_axis;
    if (b < 0 || b >= dim || b == a) return fail(CG_EINVAL, "bad blend_axis");
    if (at[b] + 1 >= n[b]) return fail(CG_EINVAL, "blended line outside the box");
    shift = st[b];
  }
  const int v0 = at[0] + n[0] * (at[1] + n[1] * at[2]);
  return engine_status(h, h->eng->line_crossings(v0, st[a], shift, t, line->lo, line->hi, max_points, points,
                                                 n_points));
}

cg_status cg_lbm_drop_shape(cg_lbm* h, int base_axis, int wall_axis, int slice, double wall, int row, cg_drop* out) {
  if (!h || !out) return fail(CG_EINVAL, "NULL argument");
  const int dim = h->S.dim;
  if (base_axis < 0 || base_axis >= dim || wall_axis < 0 || wall_axis >= dim || base_axis == wall_axis)
    return fail(CG_EINVAL, "bad axes");
  const int n[3] = {h->S.nx, h->S.ny, h->S.nz};
  if (row < 0 || row >= n[wall_axis]) return fail(CG_EINVAL, "row outside the box");
  std::memset(out, 0, sizeof(*out));
  const int third = 3 - base_axis - wall_axis;
  cg_line ln{};
  ln.axis = base_axis;
  ln.at[wall_axis] = row;
  if (dim == 3) ln.at[third] = slice;
  ln.lo = 0;
  ln.hi = n[base_axis];
  double xs[cg::kLineMax];
  int nx = 0;
  cg_status rc = cg_lbm_line_crossings(h, &ln, xs, cg::kLineMax, &nx);
  if (rc != CG_OK) return rc;
  out->n_base_points = nx;
  if (nx < 2) return fail(CG_EINVAL, "fewer than two interface points on the row next to the wall");
  const int last = (nx < cg::kLineMax ? nx : cg::kLineMax) - 1;
  const double base = xs[last] - xs[0];
  const double axis = 0.5 * (xs[0] + xs[last]);
  const int x0 = (int)std::floor(axis);
  cg_line up{};
  up.axis = wall_axis;
  up.at[base_axis] = x0;
  if (dim == 3) up.at[third] = slice;
  up.lo = row;
  up.hi = n[wall_axis];
  up.blend = axis - x0;
  up.blend_axis = base_axis;
  if (up.blend > 0.0 && x0 + 1 >= n[base_axis]) up.blend = 0.0;
  double ys[cg::kLineMax];
  int ny = 0;
  rc = cg_lbm_line_crossings(h, &up, ys, cg::kLineMax, &ny);
  if (rc != CG_OK) return rc;
  double y = -1.0;
  for (int k = 0; k < ny && k < cg::kLineMax; ++k)
    if (ys[k] > row) {
      y = ys[k];
      break;
    }
  if (y < 0.0) return fail(CG_EINVAL, "no interface point above the wall on the drop axis");
  const double hgt = y - wall;
  out->base = base;
  out->height = hgt;
  out->radius = (4.0 * hgt * hgt + base * base) / (8.0 * hgt);
  out->theta_deg = std::atan2(base / 2.0, out->radius - hgt) * (180.0 / M_PI);
  return CG_OK;
}

cg_status cg_lbm_adjoint(cg_lbm* h, const cg_adjoint_spec* spec, cg_gradients* out) {
  if (!h || !spec || !out) return fail(CG_EINVAL, "NULL argument");
  return engine_status(h, h->eng->adjoint(*spec, out));
}

cg_status cg_lbm_kernel_times(cg_lbm* h, char (*names)[32], int64_t* counts, double* total_ms, int* n) {
  if (!h || !names || !counts || !total_ms || !n) return fail(CG_EINVAL, "NULL argument");
  int64_t c[cg::K_COUNT];
  double ms[cg::K_COUNT];
  int rc = h->eng->kernel_times(c, ms);
  if (rc != CG_OK) return engine_status(h, rc);
  const int m = *n < cg::K_COUNT ? *n : cg::K_COUNT;
  for (int k = 0; k < m; ++k) {
    std::strncpy(names[k], cg::kKernelNames[k], 31);
    names[k][31] = 0;
    counts[k] = c[k];
    total_ms[k] = ms[k];
  }
  *n = m;
  return CG_OK;
}

cg_status cg_lbm_tune(cg_lbm* h, int reps, char* report, size_t report_len) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  std::string rep;
  int rc = h->eng->tune(reps, &rep);
  if (rc != CG_OK) return engine_status(h, rc);
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return CG_OK;
}

cg_status cg_lbm_reset_timing(cg_lbm* h) {
  if (!h) return fail(CG_EINVAL, "NULL handle");
  h->eng->reset_timing();
  return CG_OK;
}

struct cg_batch {
  std::unique_ptr<cg::BatchBase> impl;
  std::vector<cg_lbm*> runs;
};

cg_status cg_batch_create(cg_lbm* const* runs, int n, cg_batch** out) {
  if (!out) return fail(CG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!runs || n < 1) return fail(CG_EINVAL, "need at least one run");
  std::vector<cg::EngineBase*> engs;
  for (int i = 0; i < n; ++i) {
    if (!runs[i]) return fail(CG_EINVAL, "NULL run handle");
    if (runs[i]->precision != runs[0]->precision) return fail(CG_EINVAL, "runs differ in precision");
    engs.push_back(runs[i]->eng.get());
  }
  std::unique_ptr<cg_batch> b(new cg_batch());
  b->runs.assign(runs, runs + n);
  b->impl.reset(runs[0]->precision == CG_FP64 ? cg::make_batch_f64() : cg::make_batch_f32());
  std::string err;
  int rc = b->impl->init(engs, &runs[0]->al, &err);
  if (rc != CG_OK) return fail((cg_status)rc, err.empty() ? b->impl->err_ : err);
  *out = b.release();
  return CG_OK;
}

void cg_batch_destroy(cg_batch* b) {
  if (!b) return;
  (void)b->impl->sync();
  delete b;
}

cg_status cg_batch_step(cg_batch* b, int64_t n) {
  if (!b || n < 0) return fail(CG_EINVAL, "bad argument");
  int rc = b->impl->step(n);
  return rc == CG_OK ? CG_OK : fail((cg_status)rc, b->impl->err_);
}

cg_status cg_batch_sync(cg_batch* b) {
  if (!b) return fail(CG_EINVAL, "NULL batch");
  int rc = b->impl->sync();
  return rc == CG_OK ? CG_OK : fail((cg_status)rc, b->impl->err_);
}

cg_status cg_batch_observe(cg_batch* b, int i, int axis, int plane, cg_observables* out) {
  if (!b) return fail(CG_EINVAL, "NULL batch");
  if (i < 0 || i >= (int)b->runs.size()) return fail(CG_EINVAL, "run index out of range");
  const cg_status rc = cg_batch_sync(b);
  if (rc != CG_OK) return rc;
  return cg_lbm_observe(b->runs[i], axis, plane, out);
}

cg_status cg_batch_set_graph(cg_batch* b, int on) {
  if (!b) return fail(CG_EINVAL, "NULL batch");
  b->impl->set_graph(on != 0);
  return CG_OK;
}

cg_status cg_batch_tune(cg_batch* b, int reps, char* report, size_t report_len) {
  if (!b || reps < 1) return fail(CG_EINVAL, "bad argument");
  std::string rep;
  int rc = b->impl->tune(reps, &rep);
  if (rc != CG_OK) return fail((cg_status)rc, b->impl->err_);
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return CG_OK;
}

int64_t cg_batch_graph_captures(const cg_batch* b) { return b ? b->impl->captures() : -1; }

cg_status cg_batch_info(const cg_batch* b, int64_t* total_nodes, int* block, int* grid) {
  if (!b) return fail(CG_EINVAL, "NULL batch");
  if (total_nodes) *total_nodes = b->impl->total_nodes();
  int bs[8], gr[8];
  b->impl->get_config(bs, gr);
  for (int k = 0; k < 6; ++k) {
    if (block) block[k] = bs[k];
    if (grid) grid[k] = gr[k];
  }
  return CG_OK;
}

}  // extern "C"
