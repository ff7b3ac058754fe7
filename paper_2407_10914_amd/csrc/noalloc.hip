// cg_lbm_observe_noalloc: the observable reductions of cg_lbm_observe with
// their scratch (the per-block partial sums and the final sums) in a
// file-scope device array instead of memory the run allocated, for callers
// that cannot allocate device memory.
//
// Host code never passes the array's name to a kernel or a copy: on the host
// it only stands for the symbol.  The array's device address is looked up once
// per device with hipGetSymbolAddress (that device current) and kept; the
// kernels receive that address.  Every call on one device shares that device's
// array; calls that overlap on one device race (a handle is not thread-safe
// either).  Nothing in the array has to start at zero: every block of the
// reduction writes all of its partial sums and the final pass writes every
// output before anything reads them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/cg_lbm.h"
#include "handle.hpp"

namespace {

// 4 MiB of doubles: the final sums followed by the partial sums of at most
// (kScratchDoubles - kObsN) / kObsN blocks of 256 fluid nodes, i.e. runs of up
// to 8,947,456 fluid nodes.
constexpr size_t kScratchDoubles = size_t(1) << 19;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mtx;
double* g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's copy of the array: looked up on the first
// call on the device, with that device current (the caller's current device
// is restored afterwards).
cg_status scratch_ptr(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return cg::set_error(CG_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mtx);
  if (!g_ptr[device]) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return cg::set_error(CG_EHIP, "hipGetDevice failed");
    if (prev != device && hipSetDevice(device) != hipSuccess) return cg::set_error(CG_EHIP, "hipSetDevice failed");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p)
      return cg::set_error(CG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = static_cast<double*>(p);
  }
  *out = g_ptr[device];
  return CG_OK;
}

}  // namespace

extern "C" cg_status cg_lbm_observe_noalloc(cg_lbm* h, int axis, int plane, cg_observables* out) {
  if (!h || !out) return cg::set_error(CG_EINVAL, "NULL argument");
  const size_t need = h->eng->obs_partials() + (size_t)cg::kObsN;
  if (need > kScratchDoubles)
    return cg::set_error(CG_EINVAL, "too many fluid nodes for the allocation-free observables (at most 8947456; "
                                    "this run has " + std::to_string(h->S.N) + ")");
  double* base = nullptr;
  cg_status rc = scratch_ptr(h->device, &base);
  if (rc != CG_OK) return rc;
  double o[cg::kObsN];
  const int erc = h->eng->observe_into(axis, plane, -1, 0, 0, base + cg::kObsN, base, o);
  if (erc != CG_OK)
    return cg::set_error((cg_status)erc, h->eng->err_.empty() ? std::string("device engine error") : h->eng->err_);
  if (cg::fill_observables(o, h->eng->t, out) > 0)
    return cg::set_error(CG_EUNSTABLE, "non-finite density or velocity in the state");
  return CG_OK;
}
