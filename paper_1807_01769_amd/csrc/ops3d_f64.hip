// ops3d_f64.hip -- the 3D solver's kernels and launch sequences, double precision,
// velocity only.
#include "ops3d_impl.h"

namespace fs {
template Ops ops3_of<double, false>(int);
}  // namespace fs
