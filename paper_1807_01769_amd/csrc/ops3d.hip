// ops3d.hip -- the 3D solver's ops table by precision and state size (the
// kernels and launch sequences are compiled in ops3d_f32*.hip, ops3d_f64*.hip).
#include "fs_internal.h"

namespace fs {

template <typename T, bool STRAT>
Ops ops3_of(int n);

template <typename T>
Ops make_ops3(int n, int nfield) {
  return nfield == 4 ? ops3_of<T, true>(n) : ops3_of<T, false>(n);
}

template Ops make_ops3<float>(int, int);
template Ops make_ops3<double>(int, int);

}  // namespace fs
