// Host side of the discrete adjoint: forward sweep with checkpoints every K
// steps, then segment by segment (last first) the K states of the segment are
// recomputed from its checkpoint into a ring of state buffers and the reverse
// steps run from the last state of the segment down to its checkpoint.  The
// segments are counted from the end (the first one holds the remainder), so
// the last segment, whose states and front fields the forward sweep keeps
// and which is not recomputed, is always a full one: with memory for K near
// n_steps almost nothing is recomputed.
// Included at the end of engine.hpp (needs the complete Engine).
#pragma once

#include <algorithm>
#include <vector>

#include "adjoint.hpp"

namespace cg {

template <class Real>
class AdjointRun {
  using V4 = Vec4<Real>;
  using V2 = Vec2<Real>;
  static constexpr bool kF32 = sizeof(Real) == 4;
  static constexpr int BS = Engine<Real>::BS;

 public:
  explicit AdjointRun(Engine<Real>& e) : E(e) {}
  ~AdjointRun() {
    (void)hipStreamSynchronize(E.stream_);
    for (void* p : mem_) E.al_->put(p);
    for (hipEvent_t ev : ev_) (void)hipEventDestroy(ev);
  }

  int run(const cg_adjoint_spec& sp, cg_gradients* g) {
    if (sp.n_steps < 1 || sp.checkpoint_every < 1) {
      E.err_ = "n_steps and checkpoint_every must be >= 1";
      return CG_EINVAL;
    }
    if (sp.objective < 0 || sp.objective > 2 || sp.axis < 0 || sp.axis >= E.dim_ || !(sp.delta >= 0.0)) {
      E.err_ = "bad objective, axis or delta";
      return CG_EINVAL;
    }
    AP_.delta = sp.delta;
    AP_.objective = sp.objective;
    AP_.axis = sp.axis;
    AP_.lo = sp.lo;
    AP_.hi = sp.hi;
    return E.dim_ == 3 ? run_d<3>(sp, g) : run_d<2>(sp, g);
  }

 private:
  Engine<Real>& E;
  AdjParams AP_{};
  std::vector<void*> mem_;
  std::vector<hipEvent_t> ev_;
  size_t bytes_ = 0;
  struct Slot {
    void* a = nullptr;
    void* b = nullptr;
  };
  // adjoint buffers
  Real* lf_[2] = {nullptr, nullptr};
  V2* lr_ = nullptr;
  V4 *na_ = nullptr, *lcf_ = nullptr, *ln_ = nullptr, *lc_ = nullptr;
  Real *lk_ = nullptr, *lphi_ = nullptr, *iden_ = nullptr;
  double *idf_ = nullptr, *lth_ = nullptr, *part_ = nullptr, *sums_ = nullptr;
  double* pacc_ = nullptr;
  int npacc_ = 0;  // rows of pacc_
  Real* lpo_ = nullptr;  // lambda phi of the outlet nodes (Zou-He runs)
  Real* ljt_ = nullptr;  // j^t of the outlet faces (Zou-He runs)
  int face_pull_ = 0;    // the state of the current step is pulled and has face nodes
  // front fields (phase, normal, colour gradient, force) of the state at
  // t0 + k for each ring index k, kept from the recomputation so the reverse
  // step does not evaluate the front stages again; empty when the memory was
  // not available (the reverse step then recomputes them)
  std::vector<Grids<Real>> fg_;
  int p_ = 0;  // the current adjoint lives in lf_[p_], lr_

  void* get(size_t b) {
    void* p = E.al_->get(b);
    if (p) {
      mem_.push_back(p);
      bytes_ += b;
    }
    return p;
  }
  bool new_slot(Slot* s) {
    const size_t Q = E.Q_, Np = E.P_.Np;
    if (kF32) {
      s->a = get(sizeof(float) * Q * Np);
      s->b = get(sizeof(float4) * Np);
    } else {
      s->a = get(sizeof(Real) * Q * Np);
      s->b = get(sizeof(Real) * Q * Np);
    }
    return s->a && s->b;
  }
  template <int D>
  auto in_of(const Slot& s) const {
    if constexpr (kF32)
      return InCompact<D>{(const float*)s.a, (const float4*)s.b, E.P_.Np, (float)E.P_.rho0, E.rs_, E.fs_};
    else
      return InCanon<Real, D>{(const Real*)s.a, (const Real*)s.b, E.P_.Np};
  }
  template <int D>
  auto out_of(const Slot& s) const {
    if constexpr (kF32)
      return OutCompact<D>{(float*)s.a, (float4*)s.b, E.P_.Np};
    else
      return OutCanon<Real, D>{(Real*)s.a, (Real*)s.b, E.P_.Np};
  }
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) == hipSuccess) ev_.push_back(e);
    return e;
  }
  AdjBufs<Real> bufs() const {
    return AdjBufs<Real>{lf_[p_], lf_[p_ ^ 1], lr_,   na_,  lcf_,  lk_,  ln_,
                         lc_,     lphi_,       iden_, idf_, pacc_, lth_, lpo_, ljt_, face_pull_};
  }

  // one forward step from `in` into slot `out`; the front fields go to the
  // ring index k's grids when they are kept (k < 0: the engine's grids)
  template <int D, class In>
  void fstep(const In& in, const Slot& out, int64_t k = -1) {
    auto o = out_of<D>(out);
    const Grids<Real> saved = E.R_;
    const bool keep = k >= 0 && !fg_.empty();
    if (keep) E.R_ = fg_[(size_t)k];
    // k_main evaluates the force and curvature itself; a kept front also
    // gets them stored, for the reverse step
    E.template front_with<D>(in, 4);
    E.template launch_main<D>(in, o, keep ? (void*)E.R_.f : nullptr);
    E.R_ = saved;
  }

  // the reverse stages after the node stage (shared by the steps and the
  // flux terminal condition)
  template <int D>
  void reverse_tail(const Grids<Real>& R) {
    const StepParams& P = E.P_;
    const AdjBufs<Real> A = bufs();
    const int nfb = (P.N + BS - 1) / BS, nsbb = (P.nsb + BS - 1) / BS;
    E.launch_bs(-1, BS, ka_curv<Real, D>, (nfb + nsbb) * BS, P, E.G_, R, A, nfb);
    E.launch(-1, ka_normal<Real, D>, P.N, P, E.G_, R, A, AP_);
    if (P.nsb) E.launch(-1, ka_sb_phi<Real, D>, P.nsb, P, E.G_, A);
    E.launch(-1, ka_phi<Real, D>, P.N, P, E.G_, A);
    p_ ^= 1;
  }

  // Zou-He runs: whether the state `in` is a pulled one (the faces act on it)
  template <int D, class In>
  bool faces_of(const In&) const {
    return D == 3 && In::kPull && E.P_.n_in + E.P_.n_out > 0;
  }
  // the node stage; with Zou-He faces the reverse streaming reads the face
  // form of lambda_{t+1}, and the face nodes of a pulled state go apart
  template <int D, bool kSeed, class In>
  void node_stage(const In& in, const Grids<Real>& R) {
    const StepParams& P = E.P_;
    if constexpr (D == 3) {
      if (P.n_in + P.n_out > 0) {
        constexpr int kMode = In::kPull ? 2 : 1;
        if (P.collision == 1)
          E.launch(-1, ka_node<Real, D, kSeed, true, kMode, In>, P.N, P, E.G_, R, in, bufs(), AP_);
        else
          E.launch(-1, ka_node<Real, D, kSeed, false, kMode, In>, P.N, P, E.G_, R, in, bufs(), AP_);
        if constexpr (In::kPull) face_nodes<D, kSeed>(in, R);
        return;
      }
      if (P.collision == 1)
        E.launch(-1, ka_node<Real, D, kSeed, true, 0, In>, P.N, P, E.G_, R, in, bufs(), AP_);
      else
        E.launch(-1, ka_node<Real, D, kSeed, false, 0, In>, P.N, P, E.G_, R, in, bufs(), AP_);
    } else {
      E.launch(-1, ka_node<Real, D, kSeed, false, 0, In>, P.N, P, E.G_, R, in, bufs(), AP_);
    }
  }
  // the node stage at the face nodes of a pulled state (after ka_node,
  // which skips them)
  template <int D, bool kSeed, class In>
  void face_nodes(const In& in, const Grids<Real>& R) {
    const StepParams& P = E.P_;
    if constexpr (D == 3 && In::kPull) {
      const int nt = 64 * face_tiles(P);
      if (P.collision == 1)
        E.launch(-1, ka_face_node<Real, D, kSeed, true, In>, nt, P, E.G_, R, in, bufs(), AP_);
      else
        E.launch(-1, ka_face_node<Real, D, kSeed, false, In>, nt, P, E.G_, R, in, bufs(), AP_);
    }
  }
  // the transpose of the faces on the adjoint just formed (lf_[p_], lr_);
  // after_node: a node stage of this state ran (ljt_ and na_ are its)
  template <int D, class In>
  void face_transpose(const In& in, const Grids<Real>& R, bool after_node) {
    const StepParams& P = E.P_;
    if constexpr (D == 3 && In::kPull) {
      const int nt = 64 * face_tiles(P);
      if (after_node)
        E.launch(-1, ka_face<Real, D, true, In>, nt, P, E.G_, R, in, lf_[p_], lr_, (const Real*)lpo_,
                 (const Real*)ljt_, (const V4*)na_, pacc_);
      else
        E.launch(-1, ka_face<Real, D, false, In>, nt, P, E.G_, R, in, lf_[p_], lr_, (const Real*)lpo_,
                 (const Real*)ljt_, (const V4*)na_, pacc_);
    }
  }

  // lambda_{t} from lambda_{t+1}, the state at t being `in` (ring index k).
  // first: t is the first step of the call, whose state is held fixed as
  // it stands (after the faces, as the oracle holds a state): the faces that
  // made it are not part of the map, and lambda_0 itself is not needed.
  template <int D, class In>
  void rstep(const In& in, int64_t k, bool first) {
    const StepParams& P = E.P_;
    Grids<Real> R = E.R_;
    if (!fg_.empty()) {
      R = fg_[(size_t)k];
    } else {
      E.template front_with<D>(in, 5);
    }
    face_pull_ = faces_of<D>(in) ? 1 : 0;
    node_stage<D, false>(in, R);
    reverse_tail<D>(R);
    if (face_pull_ && !first) face_transpose<D>(in, R, true);
  }

  // objective of the state `in` (into sums_) and the terminal adjoint
  template <int D, class In>
  void terminal(const In& in) {
    const StepParams& P = E.P_;
    E.template front_with<D>(in, 5);
    const int nb = (P.N + BS - 1) / BS;
    face_pull_ = faces_of<D>(in) ? 1 : 0;
    E.launch(-1, ka_obj<Real, D, BS, In>, P.N, P, E.G_, E.R_, in, AP_, part_);
    hipLaunchKernelGGL(ka_reduce<Real>, dim3(kObjN), dim3(256), 0, E.stream_, (const double*)part_, nb, kObjN, sums_);
    if (AP_.objective == 2) {
      node_stage<D, true>(in, E.R_);
      reverse_tail<D>(E.R_);
    } else {
      E.launch(-1, ka_seed_local<Real, D, In>, P.N, P, E.G_, E.R_, in, AP_, (const double*)sums_, lf_[p_], lr_);
      // the objective does not read the outlet phase (Eq. 39): no lambda phi there
      if (face_pull_ && P.n_out > 0)
        E.launch(-1, ka_fill<Real, Real>, P.n_out, (size_t)P.n_out, lpo_, Real(0));
    }
    if (face_pull_) face_transpose<D>(in, E.R_, AP_.objective == 2);
  }

  template <int D>
  int run_d(const cg_adjoint_spec& sp, cg_gradients* g) {
    const StepParams& P = E.P_;
    const size_t Np = P.Np, V = P.V, Q = E.Q_;
    const int64_t T = sp.n_steps;
    const int64_t K = std::min<int64_t>(sp.checkpoint_every, T);
    const int64_t nseg = (T + K - 1) / K;
    // segment 0 holds the remainder L0 (1..K), every later one K steps;
    // checkpoint c (c >= 1) is the state at the start of segment c
    const int64_t L0 = T - (nseg - 1) * K;
    auto seg_len = [&](int64_t c) { return c == 0 ? L0 : K; };
    const int64_t t_last = nseg > 1 ? L0 + (nseg - 2) * K : 0;  // start of the last segment
    const int64_t Llast = seg_len(nseg - 1);
    auto is_ck = [&](int64_t t) { return t >= L0 && t <= t_last && t > 0 && (t - L0) % K == 0; };
    auto ck_of = [&](int64_t t) { return (size_t)((t - L0) / K); };
    // state buffers: checkpoints 1..nseg-1, two temporaries, the ring of K
    std::vector<Slot> ck((size_t)(nseg - 1)), tmp(2), ring((size_t)K);
    bool ok = true;
    for (auto& s : ck) ok = ok && new_slot(&s);
    for (auto& s : tmp) ok = ok && new_slot(&s);
    for (auto& s : ring) ok = ok && new_slot(&s);
    // front fields per ring index (optional: skipped when memory is short)
    {
      std::vector<Grids<Real>> g((size_t)K);
      bool gok = true;
      const size_t m0 = mem_.size(), b0 = bytes_;
      for (auto& x : g) {
        x.phi = (typename Grids<Real>::PhiT*)get(sizeof(typename Grids<Real>::PhiT) * V);
        x.n = (Norm3<Real>*)get(sizeof(Norm3<Real>) * V);
        x.c = (Norm3<Real>*)get(sizeof(Norm3<Real>) * Np);
        x.f = (V4*)get(sizeof(V4) * Np);
        gok = gok && x.phi && x.n && x.c && x.f;
        if (!gok) break;
      }
      if (gok) {
        fg_ = g;
      } else {
        while (mem_.size() > m0) {
          E.al_->put(mem_.back());
          mem_.pop_back();
        }
        bytes_ = b0;
      }
    }
    for (int k = 0; k < 2; ++k) lf_[k] = (Real*)get(sizeof(Real) * Q * Np);
    lr_ = (V2*)get(sizeof(V2) * Np);
    na_ = (V4*)get(sizeof(V4) * Np);
    lcf_ = (V4*)get(sizeof(V4) * Np);
    lk_ = (Real*)get(sizeof(Real) * V);
    ln_ = (V4*)get(sizeof(V4) * V);
    lc_ = (V4*)get(sizeof(V4) * V);
    lphi_ = (Real*)get(sizeof(Real) * V);
    iden_ = (Real*)get(sizeof(Real) * V);
    idf_ = (double*)get(sizeof(double) * Np);
    lth_ = (double*)get(sizeof(double) * V);
    const int nb = (P.N + BS - 1) / BS;
    // parameter rows: one per block of the node kernels, of the solid
    // boundary kernel (the fictitious-density angle adjoint) and of the face
    // kernels (whole 64-node tiles: at most N + 128 threads)
    npacc_ = std::max(nb + 1, (P.nsb + BS - 1) / BS);
    pacc_ = (double*)get(sizeof(double) * kPaccCols * (size_t)npacc_);
    part_ = (double*)get(sizeof(double) * 4 * (size_t)(nb + 1));
    sums_ = (double*)get(sizeof(double) * (kObjN + kPaccCols));
    lpo_ = (Real*)get(sizeof(Real) * (size_t)std::max(1, P.n_out));
    ljt_ = (Real*)get(sizeof(Real) * (size_t)std::max(1, P.n_out));
    ok = ok && lf_[0] && lf_[1] && lr_ && na_ && lcf_ && lk_ && ln_ && lc_ && lphi_ && iden_ && idf_ && lth_ &&
         pacc_ && part_ && sums_ && lpo_ && ljt_;
    if (!ok) {
      E.err_ = "device allocation for the adjoint failed";
      return CG_ENOMEM;
    }
    hipStream_t st = E.stream_;
    hipError_t e = hipSuccess;
    auto zero = [&](void* p, size_t b) {
      if (e == hipSuccess) e = hipMemsetAsync(p, 0, b, st);
    };
    zero(lk_, sizeof(Real) * V);
    zero(ln_, sizeof(V4) * V);
    zero(lc_, sizeof(V4) * V);
    zero(lphi_, sizeof(Real) * V);
    zero(iden_, sizeof(Real) * V);
    zero(lth_, sizeof(double) * V);
    zero(pacc_, sizeof(double) * kPaccCols * (size_t)npacc_);
    zero(lr_, sizeof(V2) * Np);
    zero(sums_, sizeof(double) * (kObjN + kPaccCols));
    zero(lpo_, sizeof(Real) * (size_t)std::max(1, P.n_out));
    zero(ljt_, sizeof(Real) * (size_t)std::max(1, P.n_out));
    // grid voxels that no stage writes (interior solid) are read as zeros
    for (auto& x : fg_) {
      if (e == hipSuccess) e = Engine<Real>::fill_phi_zero(x.phi, V, st);
      zero(x.n, sizeof(Norm3<Real>) * V);
    }
    if (e != hipSuccess) {
      E.err_ = hipGetErrorString(e);
      return CG_EHIP;
    }
    if (P.nsb) E.launch(-1, ka_iden<Real, D>, P.nsb, P, E.G_, iden_);
    E.launch(-1, ka_idf<Real, D>, P.N, P, E.G_, idf_);

    hipEvent_t e0 = event(), e1 = event(), e2 = event();
    if (!e0 || !e1 || !e2) {
      E.err_ = "hipEventCreate failed";
      return CG_EHIP;
    }
    (void)hipEventRecord(e0, st);
    // the state at t = 0 is the engine's own, left untouched
    Slot cur0;
    if (kF32) {
      cur0.a = E.T_[E.cur_];
      cur0.b = E.AC_[E.cur_];
    } else {
      cur0.a = E.fr_[E.cur_];
      cur0.b = E.fb_[E.cur_];
    }
    const bool pre0 = E.pre_;
    // f(In) on the state at t = cK (c = 0: the engine's state)
    auto with_ck = [&](int64_t c, auto&& f) {
      if (c == 0) {
        if (pre0)
          f(E.template in_pre<D>());
        else
          f(in_of<D>(cur0));
      } else {
        f(in_of<D>(ck[(size_t)(c - 1)]));
      }
    };
    // state at t0 + k of the current segment (k = 0: its checkpoint)
    auto with_seg = [&](int64_t c, int64_t k, auto&& f) {
      if (k == 0)
        with_ck(c, f);
      else
        f(in_of<D>(ring[(size_t)(k - 1)]));
    };

    // forward sweep: the checkpoints at the segment starts; the last
    // segment's states (and front fields) go to the ring
    for (int64_t t = 0; t < T; ++t) {
      const int64_t t1 = t + 1;
      Slot out;
      if (t1 > t_last)
        out = ring[(size_t)(t1 - t_last - 1)];
      else if (is_ck(t1))
        out = ck[ck_of(t1)];
      else
        out = tmp[(size_t)(t1 & 1)];
      const int64_t kg = t >= t_last ? t - t_last : -1;
      if (t == 0) {
        with_ck(0, [&](const auto& in) { fstep<D>(in, out, kg); });
      } else if (t > t_last) {
        fstep<D>(in_of<D>(ring[(size_t)(t - t_last - 1)]), out, kg);
      } else if (is_ck(t)) {
        fstep<D>(in_of<D>(ck[ck_of(t)]), out, kg);
      } else {
        fstep<D>(in_of<D>(tmp[(size_t)(t & 1)]), out);
      }
    }
    (void)hipEventRecord(e1, st);

    // terminal condition at t = T
    with_seg(nseg - 1, Llast, [&](const auto& in) { terminal<D>(in); });
    // reverse sweep
    for (int64_t c = nseg - 1; c >= 0; --c) {
      const int64_t L = seg_len(c);
      if (c != nseg - 1) {
        for (int64_t k = 0; k < L; ++k)
          with_seg(c, k, [&](const auto& in) { fstep<D>(in, ring[(size_t)k], k); });
      }
      for (int64_t k = L - 1; k >= 0; --k)
        with_seg(c, k, [&](const auto& in) { rstep<D>(in, k, c == 0 && k == 0); });
    }
    (void)hipEventRecord(e2, st);

    // parameter gradients
    hipLaunchKernelGGL(ka_reduce<Real>, dim3(kPaccCols), dim3(256), 0, st, (const double*)pacc_, npacc_, kPaccCols,
                       sums_ + kObjN);
    if (g->dJ_dtheta_field) {
      const size_t nbv = (V + 255) / 256;
      hipLaunchKernelGGL((ka_fill<Real, double>), dim3((unsigned)nbv), dim3(256), 0, st, V, g->dJ_dtheta_field, 0.0);
      if (P.nsb) E.launch(-1, ka_theta_field<Real, D>, P.nsb, P, E.G_, (const double*)lth_, g->dJ_dtheta_field);
    }
    double h[kObjN + kPaccCols];
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, sums_, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      E.err_ = hipGetErrorString(e);
      return CG_EHIP;
    }
    float ms1 = 0.f, ms2 = 0.f;
    (void)hipEventElapsedTime(&ms1, e0, e1);
    (void)hipEventElapsedTime(&ms2, e1, e2);
    if (AP_.objective == 0)
      g->J = h[0] / (h[0] + h[1]);
    else if (AP_.objective == 1)
      g->J = h[2];
    else
      g->J = h[3];
    g->dJ_dtheta = h[kObjN + kColTheta];
    for (int a = 0; a < 3; ++a) g->dJ_dg[a] = a < E.dim_ ? P.rho0 * h[kObjN + a] : 0.0;
    g->dJ_drho_in = P.bc == 1 ? h[kObjN + kColRhoIn] : 0.0;
    g->dJ_drho_out = P.bc == 1 ? h[kObjN + kColRhoOut] : 0.0;
    g->ms_forward = ms1;
    g->ms_reverse = ms2;
    g->work_bytes = (int64_t)bytes_;
    bool finite = std::isfinite(g->J) && std::isfinite(g->dJ_dtheta) && std::isfinite(g->dJ_drho_in) &&
                  std::isfinite(g->dJ_drho_out);
    for (int a = 0; a < 3; ++a) finite = finite && std::isfinite(g->dJ_dg[a]);
    if (!finite) {
      E.err_ = "non-finite objective or gradient";
      return CG_EUNSTABLE;
    }
    return CG_OK;
  }
};

template <class Real>
int Engine<Real>::adjoint(const cg_adjoint_spec& sp, cg_gradients* g) {
  AdjointRun<Real> run(*this);
  return run.run(sp, g);
}

}  // namespace cg
