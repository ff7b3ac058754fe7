// Precision-independent interface of the batched engine (see batch.hpp).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "engine_base.hpp"

namespace cg {

struct BatchBase {
  virtual ~BatchBase() = default;
  virtual int init(const std::vector<EngineBase*>& runs, Alloc* al, std::string* err) = 0;
  virtual int step(int64_t n) = 0;
  virtual int sync() = 0;
  virtual void set_graph(bool on) = 0;
  virtual int64_t total_nodes() const = 0;
  virtual int tune(int reps, std::string* report) = 0;
  virtual void get_config(int* bs, int* grid) const = 0;
  // graphs captured so far (two at most while the configuration is unchanged)
  virtual int64_t captures() const = 0;
  std::string err_;
};

BatchBase* make_batch_f64();
BatchBase* make_batch_f32();

}  // namespace cg
