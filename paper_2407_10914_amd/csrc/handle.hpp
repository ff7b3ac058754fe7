// The run handle behind the C ABI (shared by the translation units that
// implement cg_lbm.h) and the conversion of the observable sums.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>

#include "../../include/cg_lbm.h"
#include "engine_base.hpp"
#include "setup.hpp"

struct cg_lbm {
  cg::HostSetup S;
  cg::StepParams P{};
  cg::Alloc al;
  std::unique_ptr<cg::EngineBase> eng;
  hipStream_t stream = nullptr;
  int device = 0, precision = CG_FP32, collision = CG_MRT;
};

namespace cg {

// Sets the thread-local message that cg_last_error() returns; returns s.
cg_status set_error(cg_status s, const std::string& msg);

// The kObsN sums of the observable reduction (see d_main, MODE_OBS) as the
// public record; returns the count of non-finite nodes.
inline double fill_observables(const double* o, int64_t step, cg_observables* out) {
  std::memset(out, 0, sizeof(*out));
  out->step = step;
  out->mass_r = o[0];
  out->mass_b = o[1];
  out->n_fluid = o[2];
  out->sat_w = o[2] > 0 ? o[3] / o[2] : 0.0;
  out->sat_nw_mass = (o[0] + o[1]) > 0 ? o[0] / (o[0] + o[1]) : 0.0;
  out->vol_r = o[4];
  out->vol_b = o[5];
  out->p_in = o[7] > 0 ? o[6] / o[7] : 0.0;
  out->n_in = o[7];
  out->p_out = o[9] > 0 ? o[8] / o[9] : 0.0;
  out->n_out = o[9];
  out->u_max = o[10];
  out->nan_count = o[11];
  out->flux_t = o[12];
  out->flux_r = o[13];
  out->flux_b = o[14];
  return o[11];
}

}  // namespace cg
