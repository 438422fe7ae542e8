// ops3d_f32.hip -- the 3D solver's kernels and launch sequences, single precision,
// velocity only.
#include "ops3d_impl.h"

namespace fs {
template Ops ops3_of<float, false>(int);
}  // namespace fs
