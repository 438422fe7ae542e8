// ops3d_f64_strat.hip -- the 3D solver's kernels and launch sequences, double precision,
// Boussinesq (velocity and buoyancy).
#include "ops3d_impl.h"

namespace fs {
template Ops ops3_of<double, true>(int);
}  // namespace fs
