// Precision-independent interface of the per-run device engine, so that the
// C ABI layer does not instantiate any kernel itself.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "setup.hpp"
#include "step.hpp"

namespace cg {

struct Alloc {
  cg_alloc_fn fn = nullptr;
  cg_free_fn fr = nullptr;
  void* ctx = nullptr;
  size_t total = 0;
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (fn) {
      p = fn(bytes, ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) total += bytes;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    if (fr)
      fr(p, ctx);
    else
      (void)hipFree(p);
  }
};

// most interface points one line query returns
constexpr int kLineMax = 256;

enum { K_PHASE = 0, K_SB_PHI, K_NORMAL, K_SB_N, K_CURV, K_MAIN, K_FACE, K_COUNT };
static const char* const kKernelNames[K_COUNT] = {"k_phase", "k_sb_phi", "k_normal", "k_sb_n",
                                                  "k_curv",  "k_main",   "k_face"};

struct EngineBase {
  virtual ~EngineBase() = default;
  virtual int init(const HostSetup& S, const StepParams& P, int block, Alloc* al, hipStream_t st,
                   std::string* err) = 0;
  virtual int set_phase_nodes(const double* phi_nodes_host) = 0;
  virtual int set_state_dense(const double* fr, const double* fb, bool dev) = 0;
  virtual int step(int64_t n) = 0;
  virtual int macro(double* rr, double* rb, double* u, double* kap, double* F, double* C) = 0;
  virtual int phi_grid(double* dst) = 0;
  virtual int n_grid(double* dst) = 0;
  virtual int export_pops(double* fr, double* fb) = 0;
  virtual int observe(int axis, int plane, double* out) = 0;
  virtual int observe_into(int axis, int plane, int slab_axis, int lo, int hi, double* part, double* sums,
                           double* out) = 0;
  // observables over a slab, with the run's own buffers
  virtual int observe_slab(int axis, int plane, int slab_axis, int lo, int hi, double* out) = 0;
  // doubles of per-block partial sums that observe_into needs
  virtual size_t obs_partials() const = 0;
  virtual size_t snapshot_bytes() const = 0;
  virtual int save(void* dst) = 0;
  virtual int load(const void* src) = 0;
  virtual int adjoint(const cg_adjoint_spec& sp, cg_gradients* g) = 0;
  virtual int set_angles(const double* cos_t, const double* sin_t, const unsigned* flags, const double* sb_fd) = 0;
  virtual int set_body_force(const double* g) = 0;
  virtual int set_pressure(double rho_in, double rho_out) = 0;
  // phi = 0 crossings along a line of the phase-field grid (see
  // k_line_crossings); out receives min(count, max_out) positions
  virtual int line_crossings(int v0, int stride, int shift, double t, int lo, int hi, int max_out, double* out,
                             int* count) = 0;
  virtual int switch_inlet(double zeta_r) = 0;
  virtual int tune(int reps, std::string* report) = 0;
  virtual void blocks(int* out) const = 0;
  virtual void set_timing(int mask) = 0;
  virtual void set_graph(bool on) = 0;
  virtual int64_t graph_captures() const = 0;
  virtual int kernel_times(int64_t* counts, double* ms) = 0;
  virtual void reset_timing() = 0;
  virtual size_t state_bytes() const = 0;
  virtual size_t device_bytes() const = 0;
  int64_t t = 0;
  // bumped whenever a parameter that the step kernels read changes (angles,
  // body force, Zou-He densities, injected fluid): a batch holding the run
  // re-reads its parameters then
  uint64_t params_version = 0;
  std::string err_;
};

EngineBase* make_engine_f64();
EngineBase* make_engine_f32();

}  // namespace cg
