// Double-precision engine.  Built with -ffp-contract=off: every product and
// sum is rounded on its own, in the order written.
#include "batch.hpp"

namespace cg {
EngineBase* make_engine_f64() { return new Engine<double>(); }
BatchBase* make_batch_f64() { return new Batch<double>(); }
}  // namespace cg
