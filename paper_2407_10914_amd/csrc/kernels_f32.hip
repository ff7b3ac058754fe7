// Single-precision engine (compact state, contraction allowed).
#include "batch.hpp"

namespace cg {
EngineBase* make_engine_f32() { return new Engine<float>(); }
BatchBase* make_batch_f32() { return new Batch<float>(); }
}  // namespace cg
