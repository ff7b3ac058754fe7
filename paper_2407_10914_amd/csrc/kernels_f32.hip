// Single-precision engine (compact state, contraction allowed).
#include "engine.hpp"

namespace cg {
EngineBase* make_engine_f32() { return new Engine<float>(); }
}  // namespace cg
