// Kernel instance: gg2s_f64 (g g -> t t~ g g, FP64 amplitudes, colour sum on
// the FP64 matrix cores), gg2s.h.
#include "gg2s.h"
namespace mf {
Launchers launchers_gg2s_f64() { return s2::launchers<double>(); }
}  // namespace mf
