// ops3d_f32_strat.hip -- the 3D solver's kernels and launch sequences, single precision,
// Boussinesq (velocity and buoyancy).
#include "ops3d_impl.h"

namespace fs {
template Ops ops3_of<float, true>(int);
}  // namespace fs
