// MLP surrogate of the greedy indicator (placeholder until the kernels land).
#include "offline.h"

namespace rb {
struct Surrogate::Impl {};
Surrogate::Surrogate(GreedyState& g, const double*, int p) : gs(g), P(p) {
  throw Error{RB_EUNSUPPORTED, "surrogate greedy not built yet"};
}
Surrogate::~Surrogate() = default;
int Surrogate::step(int, double*) { return -1; }
}  // namespace rb
