// Double-precision engine.  Built with -ffp-contract=off: every product and
// sum is rounded on its own, in the order written.
#include "engine.hpp"

namespace cg {
EngineBase* make_engine_f64() { return new Engine<double>(); }
}  // namespace cg
