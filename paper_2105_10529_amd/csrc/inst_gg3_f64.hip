// Kernel instance: gg3_f64 (g g -> t t~ g g g, FP64 amplitudes and colour sum
// on the FP64 matrix cores), evaluated by the staged kernels of gg3.h.
#include "gg3.h"

namespace mf {
Launchers launchers_gg3_f64() { return g3::launchers<double>(); }
}  // namespace mf
