// Batched persistent launches: many runs of one precision and lattice advance
// together, one launch per stage of the step for all runs.
//
// Each stage kernel walks a flat table of (run, tile) pairs; a tile is one
// block's worth of consecutive nodes (or solid boundary points) of one run.
// The grid is persistent: every block takes one contiguous chunk of the
// table (the chunks are dealt so that each XCD gets contiguous work), and
// each tile reads its run's parameters and array pointers from a descriptor
// table in device memory.  Two descriptor tables (one per ping-pong parity)
// let a two-step sequence be captured once in a hipGraph and replayed; one
// graph per starting parity, both captured once and kept while the tables'
// addresses and the stage configuration stay the same (rewriting the tables'
// contents does not invalidate them).
// Block size and grid size per stage come from the autotuner below.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <sys/stat.h>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "batch_base.hpp"
#include "engine.hpp"

namespace cg {

template <class Real, int D>
using PostIn = std::conditional_t<sizeof(Real) == 4, InCompact<D>, InCanon<Real, D>>;
template <class Real, int D>
using PostOut = std::conditional_t<sizeof(Real) == 4, OutCompact<D>, OutCanon<Real, D>>;

template <class Real, int D>
struct RunDesc {
  StepParams P;
  Geo<Real> G;
  Grids<Real> R;
  PostIn<Real, D> in;
  PostOut<Real, D> out;
};

// Stages of one step (the main stage evaluates the curvature and force of its
// node itself).
enum { ST_PHASE = 0, ST_FACE, ST_SB_PHI, ST_NORMAL, ST_SB_N, ST_MAIN, ST_COUNT };
static const char* const kStageNames[ST_COUNT] = {"phase", "face", "sb_phi", "normal", "sb_n", "main"};
constexpr bool stage_on_sb(int st) { return st == ST_SB_PHI || st == ST_SB_N; }

template <class Real, int D, int BS, int St>
__global__ void __launch_bounds__(BS) kb_stage(const RunDesc<Real, D>* __restrict__ descs,
                                               const int2* __restrict__ tiles, int ntiles, int per_block) {
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int t0 = L * per_block;
  const int t1 = min(t0 + per_block, ntiles);
  for (int t = t0; t < t1; ++t) {
    const int2 tl = tiles[t];
    const RunDesc<Real, D>& d = descs[tl.x];
    const int n = tl.y + (int)threadIdx.x;
    if constexpr (St == ST_PHASE) {
      d_phase<Real, D>(d.P, d.G, d.R, d.in, n);
    } else if constexpr (St == ST_FACE) {
      // the node tiles of every run; only the Zou-He face nodes do work
      if (n < d.P.n_in || (n >= d.P.N - d.P.n_out && n < d.P.N)) d_face<Real, D>(d.P, d.G, d.R, d.in, n);
    } else if constexpr (St == ST_SB_PHI) {
      d_sb_phi<Real, D>(d.P, d.G, d.R, n);
    } else if constexpr (St == ST_NORMAL) {
      d_normal<Real, D>(d.P, d.G, d.R, n);
    } else if constexpr (St == ST_SB_N) {
      d_sb_n<Real, D>(d.P, d.G, d.R, n);
    } else {
      if (n < d.P.N) d_main<Real, D, MODE_STEP>(d.P, d.G, d.R, d.in, d.out, MacroOut{}, n, nullptr);
    }
  }
}

struct StageCfg {
  int bs = 256;
  int grid = 0;  // 0: one block per tile
};

template <class Real>
class Batch final : public BatchBase {
  using Eng = Engine<Real>;

 public:
  ~Batch() override {
    if (cap_stream_) (void)hipStreamSynchronize(cap_stream_);
    if (stream_) (void)hipStreamSynchronize(stream_);
    drop_graphs();
    for (void* p : owned_) al_->put(p);
    if (ev_in_) (void)hipEventDestroy(ev_in_);
    if (ev_out_) (void)hipEventDestroy(ev_out_);
    if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
  }

  int init(const std::vector<EngineBase*>& runs, Alloc* al, std::string* err) override {
    al_ = al;
    for (EngineBase* e : runs) {
      Eng* r = dynamic_cast<Eng*>(e);
      if (!r) {
        *err = "all runs of a batch must share one precision";
        return CG_EINVAL;
      }
      runs_.push_back(r);
    }
    dim_ = runs_[0]->dim();
    stream_ = runs_[0]->stream();
    for (Eng* r : runs_) {
      if (r->dim() != dim_) {
        *err = "all runs of a batch must share one lattice";
        return CG_EINVAL;
      }
      if (r->stream() != stream_) {
        *err = "all runs of a batch must share one stream";
        return CG_EINVAL;
      }
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
      *err = "hipGetDeviceProperties failed";
      return CG_EHIP;
    }
    cus_ = prop.multiProcessorCount;
    arch_ = prop.gcnArchName;
    // graphs are captured and replayed on a private stream (the runs' stream
    // may be the legacy default stream, which cannot be captured), ordered
    // with the runs' stream by events; default priority
    if (hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_out_, hipEventDisableTiming) != hipSuccess) {
      *err = "stream/event creation failed";
      return CG_EHIP;
    }
    const size_t dbytes = dim_ == 3 ? sizeof(RunDesc<Real, 3>) : sizeof(RunDesc<Real, 2>);
    for (int q = 0; q < 2; ++q) {
      descs_[q] = al_->get(dbytes * runs_.size());
      if (!descs_[q]) {
        *err = "device allocation failed";
        return CG_ENOMEM;
      }
      owned_.push_back(descs_[q]);
    }
    int rc = upload_descs();
    if (rc != CG_OK) return rc;
    for (int st = 0; st < ST_COUNT; ++st) cfg_[st] = StageCfg{256, 0};
    total_nodes_ = 0;
    for (Eng* r : runs_) total_nodes_ += r->params().N;
    load_tuning();
    return CG_OK;
  }

  // A run stepped on its own, or given new parameters, since the tables were
  // written: rewrite them.
  int refresh() {
    for (size_t r = 0; r < runs_.size(); ++r)
      if (runs_[r]->t != t_expect_[r] || runs_[r]->params_version != v_expect_[r]) return upload_descs();
    return CG_OK;
  }

  int step(int64_t n) override {
    if (n <= 0) return CG_OK;
    {
      int rc = refresh();
      if (rc != CG_OK) return rc;
    }
    // runs holding a state set from the host take their first step on their own
    bool any_pre = false;
    for (Eng* r : runs_) any_pre = any_pre || r->pre();
    if (any_pre) {
      for (Eng* r : runs_) {
        int rc = r->step(1);
        if (rc != CG_OK) {
          err_ = r->err_;
          return rc;
        }
      }
      --n;
      int rc = upload_descs();
      if (rc != CG_OK) return rc;
    }
    if (use_graph_ && n >= 2) {
      if (!graph_exec_[par_]) {
        int rc = capture(par_);
        if (rc != CG_OK) return rc;
      }
      if (hipEventRecord(ev_in_, stream_) != hipSuccess || hipStreamWaitEvent(cap_stream_, ev_in_, 0) != hipSuccess)
        return hip_fail("stream ordering");
      // an even count of steps starts and ends on the same parity
      for (int64_t k = 0; k + 1 < n; k += 2) {
        if (hipGraphLaunch(graph_exec_[par_], cap_stream_) != hipSuccess) return hip_fail("hipGraphLaunch");
      }
      if (hipEventRecord(ev_out_, cap_stream_) != hipSuccess || hipStreamWaitEvent(stream_, ev_out_, 0) != hipSuccess)
        return hip_fail("stream ordering");
      for (Eng* r : runs_) r->advance(n & ~int64_t(1));
      if (n & 1) {
        enqueue_step(par_);
        for (Eng* r : runs_) r->advance(1);
        par_ ^= 1;
      }
    } else {
      for (int64_t k = 0; k < n; ++k) {
        enqueue_step(par_);
        par_ ^= 1;
      }
      for (Eng* r : runs_) r->advance(n);
    }
    for (size_t r = 0; r < runs_.size(); ++r) t_expect_[r] = runs_[r]->t;
    if (hipGetLastError() != hipSuccess) return hip_fail("batch launch");
    return CG_OK;
  }

  int sync() override {
    if (hipStreamSynchronize(stream_) != hipSuccess) return hip_fail("stream sync");
    return CG_OK;
  }

  void set_graph(bool on) override {
    use_graph_ = on;
    drop_graphs();
  }

  int64_t captures() const override { return captures_; }

  int64_t total_nodes() const override { return total_nodes_; }

  // Autotuner: for each stage, time every (block size, persistent grid)
  // candidate over `reps` launches on the batch's real data and keep the
  // fastest; the choice is cached per (arch, lattice, precision, batch size
  // class) in a text file.
  int tune(int reps, std::string* report) override {
    std::ostringstream os;
    const int bss[3] = {64, 128, 256};
    const int mults[5] = {0, 4, 8, 16, 32};
    // the tables must describe the runs' current state: a run whose state
    // was set from the host takes its first step (on its own) here
    {
      bool any_pre = false;
      for (Eng* r : runs_) any_pre = any_pre || r->pre();
      int rc = any_pre ? step(1) : refresh();
      if (rc != CG_OK) return rc;
    }
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return hip_fail("event");
    // all stages depend on the previous ones only through data; timing one
    // stage repeatedly on a valid state is safe (table par_ reads the
    // current buffer; the main stage writes the other ping-pong buffer and
    // does not change its own input)
    for (int st = 0; st < ST_COUNT; ++st) {
      double best = 1e30;
      StageCfg bc = cfg_[st];
      for (int bs : bss) {
        for (int m : mults) {
          StageCfg c{bs, m * cus_};
          launch_stage(st, par_, c);  // warm-up
          (void)hipEventRecord(a, stream_);
          for (int k = 0; k < reps; ++k) launch_stage(st, par_, c);
          (void)hipEventRecord(b, stream_);
          if (hipEventSynchronize(b) != hipSuccess) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return hip_fail("tune sync");
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, a, b);
          const double per = ms / reps;
          if (per < best) {
            best = per;
            bc = c;
          }
        }
      }
      cfg_[st] = bc;
      os << kStageNames[st] << ": block " << bc.bs << " grid " << (bc.grid ? std::to_string(bc.grid) : "tiles")
         << " " << best * 1e3 << " us; ";
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    drop_graphs();
    save_tuning();
    if (report) *report = os.str();
    return CG_OK;
  }

  void get_config(int* bs, int* grid) const override {
    for (int st = 0; st < ST_COUNT; ++st) {
      bs[st] = cfg_[st].bs;
      grid[st] = cfg_[st].grid;
    }
  }

 private:
  std::vector<Eng*> runs_;
  Alloc* al_ = nullptr;
  std::vector<void*> owned_;
  hipStream_t stream_ = nullptr;
  int dim_ = 3, cus_ = 256;
  std::string arch_;
  void* descs_[2] = {nullptr, nullptr};
  StageCfg cfg_[ST_COUNT];
  bool any_face_ = false;
  // tile tables per (node/sb, block size)
  std::map<std::pair<int, int>, std::pair<int2*, int>> tiles_;
  bool use_graph_ = true;
  hipStream_t cap_stream_ = nullptr;
  hipEvent_t ev_in_ = nullptr, ev_out_ = nullptr;
  // graph p replays two steps starting from descriptor table p
  hipGraph_t graph_[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec_[2] = {nullptr, nullptr};
  int par_ = 0;  // descriptor table of the next step
  int64_t captures_ = 0;
  int64_t total_nodes_ = 0;
  std::vector<int64_t> t_expect_;
  std::vector<uint64_t> v_expect_;

  int hip_fail(const char* what) {
    err_ = std::string(what) + ": " + hipGetErrorString(hipGetLastError());
    return CG_EHIP;
  }

  // Destroys both graphs once every replay queued on either stream is done.
  void drop_graphs() {
    if (!graph_exec_[0] && !graph_exec_[1]) return;
    if (cap_stream_) (void)hipStreamSynchronize(cap_stream_);
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (int p = 0; p < 2; ++p) {
      if (graph_exec_[p]) (void)hipGraphExecDestroy(graph_exec_[p]);
      if (graph_[p]) (void)hipGraphDestroy(graph_[p]);
      graph_exec_[p] = nullptr;
      graph_[p] = nullptr;
    }
  }

  // descriptor table q drives the step in which each run reads buffer cur ^ q
  // (cur as it is when the tables are written; par_ restarts at 0)
  template <int D>
  int upload_descs_d() {
    std::vector<RunDesc<Real, D>> h(runs_.size());
    for (int q = 0; q < 2; ++q) {
      for (size_t r = 0; r < runs_.size(); ++r) {
        Eng* e = runs_[r];
        const int c = e->cur() ^ q;
        h[r] = RunDesc<Real, D>{e->params(), e->geo(), e->grids(), e->template in_at<D>(c),
                                e->template out_at<D>(c)};
        // single-precision runs with Zou-He faces need the face stage
        if (sizeof(Real) == 4 && e->params().n_in + e->params().n_out > 0) any_face_ = true;
      }
      if (hipMemcpy(descs_[q], h.data(), sizeof(RunDesc<Real, D>) * h.size(), hipMemcpyHostToDevice) !=
          hipSuccess)
        return hip_fail("descriptor upload");
    }
    return CG_OK;
  }
  int upload_descs() {
    // queued launches (graph replays included) read the tables: let them
    // finish before the contents change
    if (cap_stream_ && hipStreamSynchronize(cap_stream_) != hipSuccess) return hip_fail("stream sync");
    if (stream_ && hipStreamSynchronize(stream_) != hipSuccess) return hip_fail("stream sync");
    t_expect_.resize(runs_.size());
    v_expect_.resize(runs_.size());
    for (size_t r = 0; r < runs_.size(); ++r) {
      t_expect_[r] = runs_[r]->t;
      v_expect_[r] = runs_[r]->params_version;
    }
    par_ = 0;
    return dim_ == 3 ? upload_descs_d<3>() : upload_descs_d<2>();
  }

  std::pair<int2*, int> tiles(bool sb, int bs) {
    auto key = std::make_pair(sb ? 1 : 0, bs);
    auto it = tiles_.find(key);
    if (it != tiles_.end()) return it->second;
    std::vector<int2> h;
    for (size_t r = 0; r < runs_.size(); ++r) {
      const int count = sb ? runs_[r]->params().nsb : runs_[r]->params().N;
      for (int s = 0; s < count; s += bs) h.push_back(make_int2((int)r, s));
    }
    int2* d = nullptr;
    if (!h.empty()) {
      d = (int2*)al_->get(sizeof(int2) * h.size());
      if (d) {
        owned_.push_back(d);
        if (hipMemcpy(d, h.data(), sizeof(int2) * h.size(), hipMemcpyHostToDevice) != hipSuccess) d = nullptr;
      }
    }
    auto v = std::make_pair(d, d ? (int)h.size() : 0);
    tiles_[key] = v;
    return v;
  }

  template <int D, int BS>
  void launch_bs(int st, int q, int grid, hipStream_t stream_) {
    auto tl = tiles(stage_on_sb(st), BS);
    if (tl.second == 0) return;
    const int ntiles = tl.second;
    const int g = grid > 0 ? std::min(grid, ntiles) : ntiles;
    const int per = (ntiles + g - 1) / g;
    const auto* d = (const RunDesc<Real, D>*)descs_[q];
    switch (st) {
      case ST_PHASE:
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_PHASE>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles, per);
        break;
      case ST_FACE:
        if (!any_face_) break;
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_FACE>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles, per);
        break;
      case ST_SB_PHI:
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_SB_PHI>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles,
                           per);
        break;
      case ST_NORMAL:
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_NORMAL>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles,
                           per);
        break;
      case ST_SB_N:
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_SB_N>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles, per);
        break;
        break;
      default:
        hipLaunchKernelGGL((kb_stage<Real, D, BS, ST_MAIN>), dim3(g), dim3(BS), 0, stream_, d, tl.first, ntiles, per);
    }
  }
  template <int D>
  void launch_stage_d(int st, int q, const StageCfg& c, hipStream_t s) {
    if (c.bs == 64)
      launch_bs<D, 64>(st, q, c.grid, s);
    else if (c.bs == 128)
      launch_bs<D, 128>(st, q, c.grid, s);
    else
      launch_bs<D, 256>(st, q, c.grid, s);
  }
  void launch_stage(int st, int q, const StageCfg& c, hipStream_t s = nullptr) {
    if (!s) s = stream_;
    if (dim_ == 3)
      launch_stage_d<3>(st, q, c, s);
    else
      launch_stage_d<2>(st, q, c, s);
  }
  void enqueue_step(int q, hipStream_t s = nullptr) {
    for (int st = 0; st < ST_COUNT; ++st) launch_stage(st, q, cfg_[st], s);
  }

  int capture(int p) {
    // build every tile table first: capture must not allocate or copy
    for (int st = 0; st < ST_COUNT; ++st) tiles(stage_on_sb(st), cfg_[st].bs);
    if (hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return hip_fail("begin capture");
    enqueue_step(p, cap_stream_);
    enqueue_step(p ^ 1, cap_stream_);
    if (hipStreamEndCapture(cap_stream_, &graph_[p]) != hipSuccess) return hip_fail("end capture");
    if (hipGraphInstantiate(&graph_exec_[p], graph_[p], nullptr, nullptr, 0) != hipSuccess) {
      graph_exec_[p] = nullptr;
      return hip_fail("graph instantiate");
    }
    ++captures_;
    return CG_OK;
  }

  // ---- tuning cache
  std::string cache_path() const {
    const char* p = std::getenv("CGLBM_TUNE_CACHE");
    if (p && *p) return p;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/cglbm_autotune.txt";
  }
  std::string key() const {
    // geometry class: lattice, precision, run count and total nodes (log2)
    int lg = 0;
    for (int64_t v = total_nodes_; v > 1; v >>= 1) ++lg;
    std::ostringstream os;
    os << arch_ << "|stages" << ST_COUNT << "|D" << (dim_ == 3 ? "3Q19" : "2Q9") << "|" << (sizeof(Real) == 4 ? "f32" : "f64") << "|runs"
       << runs_.size() << "|n2^" << lg;
    return os.str();
  }
  void load_tuning() {
    std::ifstream f(cache_path());
    std::string line;
    const std::string k = key();
    while (std::getline(f, line)) {
      std::istringstream is(line);
      std::string kk;
      int st, bs, grid;
      if (is >> kk >> st >> bs >> grid && kk == k && st >= 0 && st < ST_COUNT &&
          (bs == 64 || bs == 128 || bs == 256) && grid >= 0)
        cfg_[st] = StageCfg{bs, grid};
    }
  }
  void save_tuning() const {
    const std::string path = cache_path();
    std::vector<std::string> keep;
    {
      std::ifstream f(path);
      std::string line;
      while (std::getline(f, line))
        if (line.rfind(key() + " ", 0) != 0) keep.push_back(line);
    }
    const auto slash = path.rfind('/');
    if (slash != std::string::npos) (void)::mkdir(path.substr(0, slash).c_str(), 0755);
    std::ofstream o(path, std::ios::trunc);
    for (auto& l : keep) o << l << "\n";
    for (int st = 0; st < ST_COUNT; ++st) o << key() << " " << st << " " << cfg_[st].bs << " " << cfg_[st].grid << "\n";
  }
};

}  // namespace cg
