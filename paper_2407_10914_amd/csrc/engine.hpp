// Per-run device engine: owns the device arrays of one run and enqueues the
// kernels of the time step, the observables and the state transfers on the
// run's stream.  Engine<double> and Engine<float> are instantiated in their
// own translation units (different floating-point contraction flags).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "engine_base.hpp"
#include "kernels.hpp"

namespace cg {

#define CG_HIP(x)                        \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) {              \
      err_ = hipGetErrorString(e_);      \
      return CG_EHIP;                    \
    }                                    \
  } while (0)

template <class Real>
class AdjointRun;

template <class Real>
class Engine final : public EngineBase {
  template <class>
  friend class AdjointRun;

  static constexpr bool kF32 = sizeof(Real) == 4;
  static constexpr int BS = 256;
  using V4 = Vec4<Real>;

 public:
  ~Engine() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    drop_step_graphs();
    if (g_stream_) (void)hipStreamDestroy(g_stream_);
    for (void* p : owned_) al_->put(p);
    for (auto& ev : ev_pool_) (void)hipEventDestroy(ev);
  }

  int init(const HostSetup& S, const StepParams& P, int block, Alloc* al, hipStream_t st,
           std::string* err) override {
    if ((double)sizeof(V4) * (double)S.V > 4294967040.0) {  // the widest dense grid (adjoint fields)
      *err = "voxel grid too large for 32-bit offsets in this precision";
      return CG_EUNSUPPORTED;
    }
    if (block != 0) {
      if (block != 64 && block != 128 && block != 256) {
        *err = "block must be 64, 128 or 256";
        return CG_EINVAL;
      }
      for (int k = 0; k < K_COUNT; ++k) bs_[k] = block;
    }
    al_ = al;
    stream_ = st;
    P_ = P;
    // the phase stage hands the step kernel the face nodes' values by their
    // rank among the face nodes, which needs the inlet nodes first and the
    // outlet nodes last (voxel order with z slowest)
    for (int n = 0; n < S.N; ++n) {
      const unsigned f = S.flags[n] & (FL_IN | FL_OUT);
      const unsigned want = n < P.n_in ? FL_IN : (n >= S.N - P.n_out ? FL_OUT : 0u);
      if (f != want) {
        *err = "Zou-He face nodes are not the first and last nodes";
        return CG_EINVAL;
      }
    }
    dim_ = S.dim;
    Q_ = S.Q;
    const size_t Np = (size_t)S.Np, V = (size_t)S.V;
    const size_t Q = (size_t)S.Q;
    // fingerprint of what a snapshot's bytes mean: precision, lattice,
    // box and the fluid node list (FNV-1a, 64 bit)
    {
      uint64_t h = 1469598103934665603ull;
      auto mix = [&](int64_t x) {
        for (int k = 0; k < 8; ++k) {
          h ^= (uint64_t)((x >> (8 * k)) & 0xff);
          h *= 1099511628211ull;
        }
      };
      mix((int64_t)sizeof(Real));
      mix(S.dim);
      mix(S.Q);
      mix(S.nx);
      mix(S.ny);
      mix(S.nz);
      mix(S.N);
      for (int v : S.node_vox) mix(v);
      fingerprint_ = (int64_t)h;
    }
    bool alloc_failed = false;
    auto dev = [&](size_t bytes) -> void* {
      void* p = al_->get(bytes);
      if (p)
        owned_.push_back(p);
      else
        alloc_failed = true;
      return p;
    };
    const bool narrow = !S.nbr16.empty();
    int* nbr = narrow ? nullptr : (int*)dev(sizeof(int) * (Q - 1) * Np);
    int16_t* nbr16 = narrow ? (int16_t*)dev(sizeof(int16_t) * (Q - 1) * Np) : nullptr;
    int* nbase = narrow ? (int*)dev(sizeof(int) * (Q - 1) * (size_t)S.ntiles) : nullptr;
    const bool tab8 = !S.nbr8.empty();
    uint32_t* nbr8 = tab8 ? (uint32_t*)dev(sizeof(uint32_t) * S.nbr8.size()) : nullptr;
    int* head8 = tab8 ? (int*)dev(sizeof(int) * S.nbr8_head.size()) : nullptr;
    unsigned* vf = (unsigned*)dev(sizeof(unsigned) * Np);
    const size_t nsb = S.sb_vox.size();
    int* sbv = (int*)dev(sizeof(int) * (nsb ? nsb : 1));
    unsigned* sbm = (unsigned*)dev(sizeof(unsigned) * (nsb ? nsb : 1));
    Real* nw = (Real*)dev(sizeof(Real) * 3 * Np);
    Real* ct = (Real*)dev(sizeof(Real) * Np);
    Real* stt = (Real*)dev(sizeof(Real) * Np);
    Real* sbfd = (Real*)dev(sizeof(Real) * (nsb ? nsb : 1));
    using PhiT = typename Grids<Real>::PhiT;
    PhiT* phi = (PhiT*)dev(sizeof(PhiT) * V);
    Norm3<Real>* ng = (Norm3<Real>*)dev(sizeof(Norm3<Real>) * V);
    Norm3<Real>* cv = (Norm3<Real>*)dev(sizeof(Norm3<Real>) * Np);
    V4* fv = (V4*)dev(sizeof(V4) * Np);
    const int nb = (S.N + BS - 1) / BS;
    obs_part_ = (double*)dev(sizeof(double) * (size_t)kObsN * (nb + 1));
    obs_out_ = (double*)dev(sizeof(double) * kObsN);
    line_buf_ = (double*)dev(sizeof(double) * (kLineMax + 1));
    if (kF32) {
      for (int k = 0; k < 2; ++k) {
        T_[k] = (float*)dev(sizeof(float) * Q * Np);
        AC_[k] = (float4*)dev(sizeof(float4) * Np);
      }
      rs_ = (double*)dev(sizeof(double) * Np);
      fs_ = (float*)dev(sizeof(float) * 5 * (size_t)(P.n_in + P.n_out > 0 ? P.n_in + P.n_out : 1));
      pre_r_ = (Real*)dev(sizeof(Real) * Q * Np);
      pre_x_ = (Real*)dev(sizeof(Real) * Q * Np);
      state_bytes_ = sizeof(float) * Q * Np + sizeof(float4) * Np;
    } else {
      for (int k = 0; k < 2; ++k) {
        fr_[k] = (Real*)dev(sizeof(Real) * Q * Np);
        fb_[k] = (Real*)dev(sizeof(Real) * Q * Np);
      }
      state_bytes_ = sizeof(Real) * 2 * Q * Np;
    }
    if (alloc_failed) {
      *err = "device allocation failed";
      return CG_ENOMEM;
    }
    // upload
    std::vector<unsigned> vfp(Np, 0u);
    for (int n = 0; n < S.N; ++n) vfp[n] = (unsigned)S.node_vox[n] | (S.flags[n] << kVoxBits);
    std::vector<Real> nwr(3 * Np), ctr(Np), str(Np), fdr(nsb);
    for (size_t i = 0; i < 3 * Np; ++i) nwr[i] = (Real)S.nw[i];
    for (size_t i = 0; i < nsb; ++i) fdr[i] = (Real)S.sb_fd[i];
    for (size_t i = 0; i < Np; ++i) {
      ctr[i] = (Real)S.cos_t[i];
      str[i] = (Real)S.sin_t[i];
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* d, const void* h, size_t bytes) {
      if (e == hipSuccess && bytes) e = hipMemcpy(d, h, bytes, hipMemcpyHostToDevice);
    };
    if (narrow) {
      up(nbr16, S.nbr16.data(), sizeof(int16_t) * (Q - 1) * Np);
      up(nbase, S.nbr_base.data(), sizeof(int) * (Q - 1) * (size_t)S.ntiles);
    } else {
      up(nbr, S.nbr.data(), sizeof(int) * (Q - 1) * Np);
    }
    if (tab8) {
      up(nbr8, S.nbr8.data(), sizeof(uint32_t) * S.nbr8.size());
      up(head8, S.nbr8_head.data(), sizeof(int) * S.nbr8_head.size());
    }
    up(vf, vfp.data(), sizeof(unsigned) * Np);
    up(sbv, S.sb_vox.data(), sizeof(int) * nsb);
    up(sbm, S.sb_mask.data(), sizeof(unsigned) * nsb);
    up(nw, nwr.data(), sizeof(Real) * 3 * Np);
    up(ct, ctr.data(), sizeof(Real) * Np);
    up(stt, str.data(), sizeof(Real) * Np);
    up(sbfd, fdr.data(), sizeof(Real) * nsb);
    // voxels that no stage writes (interior solid) hold phi = 0
    if (e == hipSuccess) e = fill_phi_zero(phi, V, nullptr);
    if (e == hipSuccess) e = hipMemset(ng, 0, sizeof(Norm3<Real>) * V);
    if (e == hipSuccess) e = hipMemset(cv, 0, sizeof(Norm3<Real>) * Np);
    if (e == hipSuccess) e = hipMemset(fv, 0, sizeof(V4) * Np);
    if (e != hipSuccess) {
      *err = std::string("upload failed: ") + hipGetErrorString(e);
      return CG_EHIP;
    }
    G_ = Geo<Real>{Nbr{nbr16, nbase, nbr, (int)Np, S.ntiles, (int)Q - 1, nbr8, head8}, vf, sbv, sbm, nw, ct, stt,
                   sbfd};
    R_ = Grids<Real>{phi, ng, cv, fv};
    nsb_ = (int)nsb;
    dev_bytes_ = al_->total;
    // rest state, all fluid b
    std::vector<double> phi0(S.N, -1.0);
    return set_phase_nodes(phi0.data());
  }

  int set_phase_nodes(const double* phi_nodes_host) override {
    double* d = (double*)al_->get(sizeof(double) * P_.N);
    if (!d) return CG_ENOMEM;
    hipError_t e = hipMemcpyAsync(d, phi_nodes_host, sizeof(double) * P_.N, hipMemcpyHostToDevice, stream_);
    Real* r = pre_r();
    Real* x = pre_x();
    if (e == hipSuccess) {
      if (dim_ == 3)
        launch(-1, k_set_phase<Real, 3>, P_.N, P_, (const double*)d, r, x);
      else
        launch(-1, k_set_phase<Real, 2>, P_.N, P_, (const double*)d, r, x);
      e = hipStreamSynchronize(stream_);
    }
    al_->put(d);
    CG_HIP(e);
    CG_HIP(hipGetLastError());
    pre_ = true;
    return CG_OK;
  }

  int set_state_dense(const double* fr, const double* fb, bool devsrc) override {
    const size_t bytes = sizeof(double) * (size_t)Q_ * P_.V;
    const double *a = fr, *b = fb;
    double *ta = nullptr, *tb = nullptr;
    if (!devsrc) {
      ta = (double*)al_->get(bytes);
      tb = (double*)al_->get(bytes);
      if (!ta || !tb) {
        al_->put(ta);
        al_->put(tb);
        return CG_ENOMEM;
      }
      CG_HIP(hipMemcpyAsync(ta, fr, bytes, hipMemcpyHostToDevice, stream_));
      CG_HIP(hipMemcpyAsync(tb, fb, bytes, hipMemcpyHostToDevice, stream_));
      a = ta;
      b = tb;
    }
    if (dim_ == 3)
      launch(-1, k_import<Real, 3>, P_.N, P_, G_, a, b, pre_r(), pre_x());
    else
      launch(-1, k_import<Real, 2>, P_.N, P_, G_, a, b, pre_r(), pre_x());
    hipError_t e = hipStreamSynchronize(stream_);
    al_->put(ta);
    al_->put(tb);
    CG_HIP(e);
    CG_HIP(hipGetLastError());
    pre_ = true;
    return CG_OK;
  }

  int step(int64_t n) override {
    for (int64_t k = 0; k < n; ++k) {
      if (graph_on_ && !pre_ && timing_ == 0) {
        const int rc = graph_step();
        if (rc != CG_OK) return rc;
      } else if (dim_ == 3) {
        one_step<3>();
      } else {
        one_step<2>();
      }
      ++t;
    }
    CG_HIP(hipGetLastError());
    return CG_OK;
  }

  // Steps replayed from captured graphs: one graph per ping-pong parity (the
  // launches of one step from the state in buffer c), captured on the run's
  // stream the first time it is needed and again whenever the parameters the
  // kernels take by value or the block sizes have changed since.  The graphs
  // hold kernel launches only.
  void set_graph(bool on) override {
    graph_on_ = on;
    if (!on) drop_step_graphs();
  }
  int64_t graph_captures() const override { return g_captures_; }

  int macro(double* rr, double* rb, double* u, double* kap, double* F, double* C) override {
    MacroOut mo{rr, rb, nullptr, u, kap, F, C};
    if (dim_ == 3)
      run_macro<3>(mo);
    else
      run_macro<2>(mo);
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    return CG_OK;
  }

  int phi_grid(double* dst) override {
    if (dim_ == 3)
      front<3>(2);
    else
      front<2>(2);
    using PhiT = typename Grids<Real>::PhiT;
    launch(-1, k_grid_copy<PhiT>, P_.V, P_.V, (const PhiT*)R_.phi, dst);
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    return CG_OK;
  }

  int n_grid(double* dst) override {
    if (dim_ == 3)
      front<3>(4);
    else
      front<2>(4);
    launch(-1, k_grid_copy3<Real>, P_.V, P_.V, (const Norm3<Real>*)R_.n, dst);
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    return CG_OK;
  }

  int line_crossings(int v0, int stride, int shift, double t, int lo, int hi, int max_out, double* out,
                     int* count) override {
    if (dim_ == 3)
      front<3>(2);
    else
      front<2>(2);
    using PhiT = typename Grids<Real>::PhiT;
    hipLaunchKernelGGL(k_line_crossings<PhiT>, dim3(1), dim3(64), 0, stream_, (const PhiT*)R_.phi, v0, stride, shift,
                       t, lo, hi, max_out, line_buf_);
    CG_HIP(hipGetLastError());
    double h[kLineMax + 1];
    CG_HIP(hipMemcpyAsync(h, line_buf_, sizeof(double) * (1 + max_out), hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    *count = (int)h[0];
    for (int k = 0; k < max_out && k < *count; ++k) out[k] = h[1 + k];
    return CG_OK;
  }

  int export_pops(double* fr, double* fb) override {
    if (dim_ == 3)
      run_export<3>(fr, fb);
    else
      run_export<2>(fr, fb);
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    return CG_OK;
  }

  int observe(int axis, int plane, double* out) override {
    return observe_into(axis, plane, -1, 0, 0, obs_part_, obs_out_, out);
  }
  int observe_slab(int axis, int plane, int slab_axis, int lo, int hi, double* out) override {
    return observe_into(axis, plane, slab_axis, lo, hi, obs_part_, obs_out_, out);
  }

  // The observables, restricted to lo <= coordinate[slab_axis] < hi when
  // slab_axis >= 0, with caller-given device buffers for the per-block
  // partial sums (obs_partials() doubles) and the kObsN final sums.
  int observe_into(int axis, int plane, int slab_axis, int lo, int hi, double* part, double* sums,
                   double* out) override {
    P_.flux_axis = axis;
    P_.flux_plane = plane;
    P_.slab_axis = slab_axis;
    P_.slab_lo = lo;
    P_.slab_hi = hi;
    if (dim_ == 3)
      run_obs<3>(part, sums);
    else
      run_obs<2>(part, sums);
    CG_HIP(hipGetLastError());
    CG_HIP(hipMemcpyAsync(out, sums, sizeof(double) * kObsN, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    return CG_OK;
  }
  size_t obs_partials() const override { return (size_t)kObsN * (size_t)((P_.N + BS - 1) / BS); }

  // snapshot: header (time, pre flag, cur) + the live state buffers
  size_t snapshot_bytes() const override { return 64 + state_bytes_ + pre_bytes(); }
  int save(void* dst) override {
    CG_HIP(hipStreamSynchronize(stream_));
    char* p = (char*)dst;
    int64_t hdr[8] = {t, pre_ ? 1 : 0, cur_, (int64_t)state_bytes_, (int64_t)pre_bytes(), fingerprint_, 0, 0};
    std::memcpy(p, hdr, 64);
    p += 64;
    for (auto& s : state_segments(cur_)) {
      CG_HIP(hipMemcpy(p, s.first, s.second, hipMemcpyDeviceToHost));
      p += s.second;
    }
    if (kF32) {
      const size_t b = pre_bytes() / 2;
      CG_HIP(hipMemcpy(p, pre_r_, b, hipMemcpyDeviceToHost));
      CG_HIP(hipMemcpy(p + b, pre_x_, b, hipMemcpyDeviceToHost));
    }
    return CG_OK;
  }
  int load(const void* src) override {
    CG_HIP(hipStreamSynchronize(stream_));
    const char* p = (const char*)src;
    int64_t hdr[8];
    std::memcpy(hdr, p, 64);
    if (hdr[3] != (int64_t)state_bytes_ || hdr[4] != (int64_t)pre_bytes() || hdr[5] != fingerprint_) {
      err_ = "snapshot taken from a run of another geometry, lattice or precision";
      return CG_EINVAL;
    }
    p += 64;
    t = hdr[0];
    pre_ = hdr[1] != 0;
    cur_ = (int)hdr[2];
    for (auto& s : state_segments(cur_)) {
      CG_HIP(hipMemcpy(s.first, p, s.second, hipMemcpyHostToDevice));
      p += s.second;
    }
    if (kF32) {
      const size_t b = pre_bytes() / 2;
      CG_HIP(hipMemcpy(pre_r_, p, b, hipMemcpyHostToDevice));
      CG_HIP(hipMemcpy(pre_x_, p + b, b, hipMemcpyHostToDevice));
    }
    return CG_OK;
  }

  int adjoint(const cg_adjoint_spec& sp, cg_gradients* g) override;

  int set_angles(const double* cos_t, const double* sin_t, const unsigned* flags, const double* sb_fd) override {
    const size_t Np = P_.Np;
    std::vector<Real> c(Np), s(Np), fd(nsb_);
    for (int k = 0; k < nsb_; ++k) fd[k] = (Real)sb_fd[k];
    std::vector<unsigned> vfp(Np);
    CG_HIP(hipStreamSynchronize(stream_));
    CG_HIP(hipMemcpy(vfp.data(), G_.vf, sizeof(unsigned) * Np, hipMemcpyDeviceToHost));
    for (size_t n = 0; n < Np; ++n) {
      c[n] = (Real)cos_t[n];
      s[n] = (Real)sin_t[n];
      vfp[n] = (vfp[n] & kVoxMask) | (flags[n] << kVoxBits);
    }
    CG_HIP(hipMemcpy(const_cast<Real*>(G_.cos_t), c.data(), sizeof(Real) * Np, hipMemcpyHostToDevice));
    CG_HIP(hipMemcpy(const_cast<Real*>(G_.sin_t), s.data(), sizeof(Real) * Np, hipMemcpyHostToDevice));
    CG_HIP(hipMemcpy(const_cast<unsigned*>(G_.vf), vfp.data(), sizeof(unsigned) * Np, hipMemcpyHostToDevice));
    if (nsb_)
      CG_HIP(hipMemcpy(const_cast<Real*>(G_.sb_fd), fd.data(), sizeof(Real) * nsb_, hipMemcpyHostToDevice));
    ++params_version;
    return CG_OK;
  }

  int set_body_force(const double* g) override {
    CG_HIP(hipStreamSynchronize(stream_));
    for (int a = 0; a < 3; ++a) P_.rg[a] = a < dim_ ? P_.rho0 * g[a] : 0.0;
    ++params_version;
    return CG_OK;
  }

  // New Zou-He densities (Appendix B) for the following steps.  The faces of
  // the current state were applied with the old densities: the state is
  // written out as pre-collision populations first (the step kernels apply
  // the faces when they pull the stored post-collision state, which would
  // otherwise use the new densities on the current state).
  int set_pressure(double rho_in, double rho_out) override {
    if (dim_ == 3)
      materialize<3>();
    else
      materialize<2>();
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    P_.rho_in = rho_in;
    P_.rho_out = rho_out;
    P_.rin_r = rho_in * P_.zeta_r;
    P_.rin_b = rho_in * (1.0 - P_.zeta_r);
    ++params_version;
    return CG_OK;
  }

  // Replace the injected fluid, Eqs. (37)-(38): the state is first written
  // out as pre-collision populations at their own nodes (pull, bounce-back
  // and faces applied, as the next step would see them), then at the inlet
  // nodes the old colour's populations join the new colour's and are
  // cleared; the following steps inject the new fluid.
  int switch_inlet(double zeta_r) override {
    if (dim_ == 3)
      materialize<3>();
    else
      materialize<2>();
    if (dim_ == 3)
      launch(-1, k_switch_inlet<Real, 3>, P_.N, P_, G_, pre_r(), pre_x(), zeta_r == 1.0 ? 1 : 0);
    else
      launch(-1, k_switch_inlet<Real, 2>, P_.N, P_, G_, pre_r(), pre_x(), zeta_r == 1.0 ? 1 : 0);
    CG_HIP(hipGetLastError());
    CG_HIP(hipStreamSynchronize(stream_));
    P_.zeta_r = zeta_r;
    P_.rin_r = P_.rho_in * zeta_r;
    P_.rin_b = P_.rho_in * (1.0 - zeta_r);
    P_.phi_in = zeta_r - (1.0 - zeta_r);
    ++params_version;
    return CG_OK;
  }

  // Block size per kernel: time `reps` steps at each of 64, 128 and 256
  // threads (HIP events around every launch) and keep the fastest per
  // kernel.  Advances the run by 3 * reps steps.
  int tune(int reps, std::string* report) override {
    if (reps < 1) reps = 1;
    const int sizes[3] = {64, 128, 256};
    double best[K_COUNT];
    int pick[K_COUNT];
    for (int k = 0; k < K_COUNT; ++k) {
      best[k] = 1e300;
      pick[k] = bs_[k];
    }
    const int saved_mask = timing_;
    CG_HIP(hipStreamSynchronize(stream_));
    collect();
    int64_t c0[K_COUNT];
    double m0[K_COUNT];
    for (int k = 0; k < K_COUNT; ++k) {
      c0[k] = tcount_[k];
      m0[k] = tms_[k];
    }
    std::ostringstream os;
    for (int b : sizes) {
      for (int k = 0; k < K_COUNT; ++k) bs_[k] = b;
      timing_ = -1;
      int rc = step(reps);
      if (rc != CG_OK) return rc;
      CG_HIP(hipStreamSynchronize(stream_));
      collect();
      for (int k = 0; k < K_COUNT; ++k) {
        const int64_t n = tcount_[k] - c0[k];
        if (n > 0) {
          const double avg = (tms_[k] - m0[k]) / (double)n;
          if (avg < best[k]) {
            best[k] = avg;
            pick[k] = b;
          }
        }
        c0[k] = tcount_[k];
        m0[k] = tms_[k];
      }
    }
    timing_ = saved_mask;
    for (int k = 0; k < K_COUNT; ++k) {
      bs_[k] = pick[k];
      if (best[k] < 1e300) os << kKernelNames[k] << ": block " << pick[k] << " " << best[k] * 1e3 << " us; ";
    }
    if (report) *report = os.str();
    return CG_OK;
  }
  void blocks(int* out) const override {
    for (int k = 0; k < K_COUNT; ++k) out[k] = bs_[k];
  }

  void set_timing(int mask) override { timing_ = mask; }
  int kernel_times(int64_t* counts, double* ms) override {
    CG_HIP(hipStreamSynchronize(stream_));
    collect();
    for (int k = 0; k < K_COUNT; ++k) {
      counts[k] = tcount_[k];
      ms[k] = tms_[k];
    }
    return CG_OK;
  }
  void reset_timing() override {
    (void)hipStreamSynchronize(stream_);
    collect();
    for (int k = 0; k < K_COUNT; ++k) {
      tcount_[k] = 0;
      tms_[k] = 0.0;
    }
  }
  size_t state_bytes() const override { return state_bytes_; }
  size_t device_bytes() const override { return al_ ? al_->total : dev_bytes_; }

  // ---- access for the batch engine (same precision, same translation unit)
  const StepParams& params() const { return P_; }
  const Geo<Real>& geo() const { return G_; }
  const Grids<Real>& grids() const { return R_; }
  int dim() const { return dim_; }
  int cur() const { return cur_; }
  bool pre() const { return pre_; }
  hipStream_t stream() const { return stream_; }
  // post-collision state held in buffer c, and the writer into buffer c ^ 1
  template <int D>
  auto in_at(int c) const {
    if constexpr (kF32)
      return InCompact<D>{T_[c], AC_[c], P_.Np, (float)P_.rho0, rs_, fs_};
    else
      return InCanon<Real, D>{fr_[c], fb_[c], P_.Np};
  }
  template <int D>
  auto out_at(int c) const {
    if constexpr (kF32)
      return OutCompact<D>{T_[c ^ 1], AC_[c ^ 1], P_.Np};
    else
      return OutCanon<Real, D>{fr_[c ^ 1], fb_[c ^ 1], P_.Np};
  }
  uint64_t graph_key() const {
    uint64_t h = params_version * 1000003ull;
    for (int k = 0; k < K_COUNT; ++k) h = h * 31ull + (uint64_t)bs_[k];
    return h;
  }
  void drop_step_graphs() {
    // replays still queued on the run's stream finish before their graph goes
    if (g_exec_[0] || g_exec_[1]) (void)hipStreamSynchronize(stream_);
    for (int p = 0; p < 2; ++p) {
      if (g_exec_[p]) (void)hipGraphExecDestroy(g_exec_[p]);
      if (g_graph_[p]) (void)hipGraphDestroy(g_graph_[p]);
      g_exec_[p] = nullptr;
      g_graph_[p] = nullptr;
    }
  }
  int graph_step() {
    const int p = cur_;
    const uint64_t key = graph_key();
    if (g_exec_[p] && g_key_[p] != key) drop_step_graphs();
    if (!g_exec_[p]) {
      // captured on a private stream (the run's stream may be the null
      // stream, which cannot be captured); replayed on the run's stream
      if (!g_stream_ && hipStreamCreateWithFlags(&g_stream_, hipStreamNonBlocking) != hipSuccess) {
        g_stream_ = nullptr;
        err_ = "hipStreamCreateWithFlags failed";
        return CG_EHIP;
      }
      if (hipStreamBeginCapture(g_stream_, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        err_ = "hipStreamBeginCapture failed";
        return CG_EHIP;
      }
      hipStream_t run_stream = stream_;
      stream_ = g_stream_;
      if (dim_ == 3)
        step_with<3>(in_post<3>());
      else
        step_with<2>(in_post<2>());
      stream_ = run_stream;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(g_stream_, &g);
      if (e != hipSuccess || !g) {
        err_ = std::string("step graph capture: ") + hipGetErrorString(e);
        return CG_EHIP;
      }
      if (hipGraphInstantiate(&g_exec_[p], g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        g_exec_[p] = nullptr;
        err_ = "hipGraphInstantiate failed";
        return CG_EHIP;
      }
      g_graph_[p] = g;
      g_key_[p] = key;
      ++g_captures_;
    }
    CG_HIP(hipGraphLaunch(g_exec_[p], stream_));
    cur_ ^= 1;
    return CG_OK;
  }

  // account for n steps taken by a batch launch
  void advance(int64_t n) {
    if (n & 1) cur_ ^= 1;
    t += n;
    if (n) pre_ = false;
  }

  // phase-field grid set to phi = 0 (the encoded zero in single precision);
  // synchronous when s is null
  static hipError_t fill_phi_zero(typename Grids<Real>::PhiT* p, size_t count, hipStream_t s) {
    if constexpr (kF32) {
      // phi = 0: d = -1.0f, choice bit 0
      const auto d = reinterpret_cast<hipDeviceptr_t>(p);
      return s ? hipMemsetD32Async(d, 0xBF800000u, count, s) : hipMemsetD32(d, 0xBF800000u, count);
    } else {
      return s ? hipMemsetAsync(p, 0, sizeof(double) * count, s) : hipMemset(p, 0, sizeof(double) * count);
    }
  }

 private:
  StepParams P_{};
  Geo<Real> G_{};
  Grids<Real> R_{};
  Alloc* al_ = nullptr;
  hipStream_t stream_ = nullptr;
  int dim_ = 3, Q_ = 19, nsb_ = 0, cur_ = 0;
  static_assert(K_COUNT == 7, "one default block size per kernel");
  int bs_[K_COUNT] = {256, 256, 256, 256, 256, 256, 256};
  bool pre_ = true;
  bool graph_on_ = false;
  hipGraph_t g_graph_[2] = {nullptr, nullptr};
  hipGraphExec_t g_exec_[2] = {nullptr, nullptr};
  uint64_t g_key_[2] = {0, 0};
  hipStream_t g_stream_ = nullptr;
  int64_t g_captures_ = 0;
  Real* fr_[2] = {nullptr, nullptr};
  Real* fb_[2] = {nullptr, nullptr};
  float* T_[2] = {nullptr, nullptr};
  float4* AC_[2] = {nullptr, nullptr};
  double* rs_ = nullptr;  // phase stage -> step kernel: red density pulled in (FP32)
  float* fs_ = nullptr;   // phase stage -> step kernel: Zou-He unknowns of the face nodes
  Real* pre_r_ = nullptr;
  Real* pre_x_ = nullptr;
  double* obs_part_ = nullptr;
  double* obs_out_ = nullptr;
  double* line_buf_ = nullptr;
  size_t state_bytes_ = 0, dev_bytes_ = 0;
  int64_t fingerprint_ = 0;
  std::vector<void*> owned_;
  // timing
  int timing_ = 0;
  std::vector<hipEvent_t> ev_pool_;
  struct Rec {
    int k;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs_;
  int64_t tcount_[K_COUNT] = {0};
  double tms_[K_COUNT] = {0};

  size_t pre_bytes() const { return kF32 ? sizeof(Real) * 2 * (size_t)Q_ * P_.Np : 0; }
  // the canonical double state uses the current ping-pong buffers as staging
  Real* pre_r() { return kF32 ? pre_r_ : fr_[cur_]; }
  Real* pre_x() { return kF32 ? pre_x_ : fb_[cur_]; }

  std::vector<std::pair<void*, size_t>> state_segments(int c) {
    const size_t Np = P_.Np, Q = Q_;
    if (kF32) return {{T_[c], sizeof(float) * Q * Np}, {AC_[c], sizeof(float4) * Np}};
    return {{fr_[c], sizeof(Real) * Q * Np}, {fb_[c], sizeof(Real) * Q * Np}};
  }

  hipEvent_t get_event() {
    if (!ev_pool_.empty()) {
      hipEvent_t e = ev_pool_.back();
      ev_pool_.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  void collect() {
    for (auto& r : recs_) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        tcount_[r.k] += 1;
        tms_[r.k] += ms;
      }
      ev_pool_.push_back(r.a);
      ev_pool_.push_back(r.b);
    }
    recs_.clear();
  }

  template <class K, class... Args>
  void launch(int kid, K kern, int nthreads, Args... args) {
    launch_bs(kid, kid >= 0 ? bs_[kid] : BS, kern, nthreads, args...);
  }
  template <class K, class... Args>
  void launch_bs(int kid, int bs, K kern, int nthreads, Args... args) {
    if (nthreads <= 0) return;
    const int nb = (nthreads + bs - 1) / bs;
    const bool tm = kid >= 0 && (timing_ & (1 << kid));
    if (!tm) {
      hipLaunchKernelGGL(kern, dim3(nb), dim3(bs), 0, stream_, args...);
    } else {
      // events attached to the dispatch itself (its start and end), not
      // recorded as commands of their own around it, which would add the
      // queue's few microseconds between commands to every launch
      hipEvent_t a = get_event(), b = get_event();
      hipExtLaunchKernelGGL(kern, dim3(nb), dim3(bs), 0, stream_, a, b, 0u, args...);
      recs_.push_back({kid, a, b});
      if (recs_.size() > 4096) {
        (void)hipStreamSynchronize(stream_);
        collect();
      }
    }
  }

  template <int D>
  auto in_post() const {
    if constexpr (kF32)
      return InCompact<D>{T_[cur_], AC_[cur_], P_.Np, (float)P_.rho0, rs_, fs_};
    else
      return InCanon<Real, D>{fr_[cur_], fb_[cur_], P_.Np};
  }
  template <int D>
  auto in_pre() const {
    if constexpr (kF32)
      return InPre<Real, D>{pre_r_, pre_x_, P_.Np};
    else
      return InPre<Real, D>{fr_[cur_], fb_[cur_], P_.Np};
  }
  template <int D>
  auto out_next() const {
    const int nx = cur_ ^ 1;
    if constexpr (kF32)
      return OutCompact<D>{T_[nx], AC_[nx], P_.Np};
    else
      return OutCanon<Real, D>{fr_[nx], fb_[nx], P_.Np};
  }

  // stages 1..upto of the step before the fused kernel: phase field (1),
  // phase into the solid (2), normals with wetting (3), normals into the
  // solid (4), curvature and force (5)
  template <int D, class In>
  void front_with(const In& in, int upto) {
    if constexpr (std::is_same_v<In, InCompact<D>>) {
      if (upto >= 2 && nsb_ && P_.n_in + P_.n_out > 0) {
        // the face stage rides in the solid-boundary phase launch
        launch(K_PHASE, k_phase<Real, D, In>, P_.N, P_, G_, R_, in);
        const int bs = bs_[K_SB_PHI];
        const int nfb = ((64 * face_tiles(P_) + bs - 1) / bs + 7) / 8 * 8;
        const int nsbb = (nsb_ + bs - 1) / bs;
        launch_bs(K_SB_PHI, bs, k_face_sb_phi<Real, D, In>, (nfb + nsbb) * bs, P_, G_, R_, in, nfb);
      } else {
        phase_with<D>(in, true);
        if (upto >= 2 && nsb_) launch(K_SB_PHI, k_sb_phi<Real, D>, nsb_, P_, G_, R_);
      }
    } else {
      phase_with<D>(in, true);
      if (upto >= 2 && nsb_) launch(K_SB_PHI, k_sb_phi<Real, D>, nsb_, P_, G_, R_);
    }
    if (upto >= 3) launch(K_NORMAL, k_normal<Real, D>, P_.N, P_, G_, R_);
    if (upto >= 4 && nsb_) launch(K_SB_N, k_sb_n<Real, D>, nsb_, P_, G_, R_);
    if (upto >= 5) launch(K_CURV, k_curv<Real, D>, P_.N, P_, G_, R_);
  }
  template <int D>
  void front(int upto) {
    if (pre_)
      front_with<D>(in_pre<D>(), upto);
    else
      front_with<D>(in_post<D>(), upto);
  }

  // the step kernel at the tuned block size (its launch bounds follow it)
  template <int D, class In, class Out>
  void launch_main(const In& in, const Out& out, void* fstore = nullptr) {
    MacroOut mo{};
    mo.fstore = fstore;
    switch (bs_[K_MAIN]) {
      case 64:
        launch_bs(K_MAIN, 64, k_main<Real, D, 64, MODE_STEP, In, Out>, P_.N, P_, G_, R_, in, out, mo, ObsOut{});
        break;
      case 128:
        launch_bs(K_MAIN, 128, k_main<Real, D, 128, MODE_STEP, In, Out>, P_.N, P_, G_, R_, in, out, mo, ObsOut{});
        break;
      default:
        launch_bs(K_MAIN, 256, k_main<Real, D, 256, MODE_STEP, In, Out>, P_.N, P_, G_, R_, in, out, mo, ObsOut{});
    }
  }

  template <int D, class In>
  void step_with(const In& in) {
    auto out = out_next<D>();
    front_with<D>(in, 4);
    launch_main<D>(in, out);
  }
  template <int D>
  void one_step() {
    if (pre_)
      step_with<D>(in_pre<D>());
    else
      step_with<D>(in_post<D>());
    cur_ ^= 1;
    pre_ = false;
  }

  template <int D, class In>
  void macro_with(const In& in, MacroOut mo) {
    front_with<D>(in, 4);
    auto out = out_next<D>();
    launch(-1, k_main<Real, D, BS, MODE_MACRO, In, decltype(out)>, P_.N, P_, G_, R_, in, out, mo, ObsOut{});
  }
  template <int D>
  void run_macro(MacroOut mo) {
    if (pre_)
      macro_with<D>(in_pre<D>(), mo);
    else
      macro_with<D>(in_post<D>(), mo);
  }

  template <int D, class In>
  void obs_with(const In& in, double* part, double* sums) {
    front_with<D>(in, 4);
    auto out = out_next<D>();
    const int nb = (P_.N + BS - 1) / BS;
    launch(-1, k_main<Real, D, BS, MODE_OBS, In, decltype(out)>, P_.N, P_, G_, R_, in, out, MacroOut{},
           ObsOut{part});
    hipLaunchKernelGGL(k_obs_final<Real>, dim3(kObsN), dim3(256), 0, stream_, (const double*)part, nb, sums);
  }
  template <int D>
  void run_obs(double* part, double* sums) {
    if (pre_)
      obs_with<D>(in_pre<D>(), part, sums);
    else
      obs_with<D>(in_post<D>(), part, sums);
  }

  template <int D, class In>
  void export_with(const In& in, double* fr, double* fb) {
    phase_with<D>(in, false);
    launch(-1, k_export<Real, D, In>, P_.N, P_, G_, R_, in, fr, fb);
  }
  // The phase field of the state `in`; for the compact state the face kernel
  // gives the outlet nodes the upstream phase (Eq. 39) and stores the faces'
  // sums.  timed: under the phase and face stages' kernel timers.
  template <int D, class In>
  void phase_with(const In& in, bool timed) {
    launch(timed ? K_PHASE : -1, k_phase<Real, D, In>, P_.N, P_, G_, R_, in);
    if constexpr (std::is_same_v<In, InCompact<D>>) {
      if (P_.n_in + P_.n_out > 0)
        launch(timed ? K_FACE : -1, k_face<Real, D, In>, 64 * face_tiles(P_), P_, G_, R_, in);
    }
  }
  // Pre-collision populations of the current state at their own nodes
  // (the staging that a state set from the host uses).  The double layout
  // writes them into the other ping-pong buffer, which becomes current.
  template <int D>
  void materialize() {
    if (pre_) return;
    auto in = in_post<D>();
    phase_with<D>(in, false);
    if constexpr (kF32) {
      launch(-1, k_materialize<Real, D, decltype(in)>, P_.N, P_, G_, R_, in, pre_r_, pre_x_);
    } else {
      launch(-1, k_materialize<Real, D, decltype(in)>, P_.N, P_, G_, R_, in, fr_[cur_ ^ 1], fb_[cur_ ^ 1]);
      cur_ ^= 1;
    }
    pre_ = true;
  }

  template <int D>
  void run_export(double* fr, double* fb) {
    if (pre_)
      export_with<D>(in_pre<D>(), fr, fb);
    else
      export_with<D>(in_post<D>(), fr, fb);
  }
};

}  // namespace cg

#include "adjoint_run.hpp"
