// Kernel instance: gg2_f64 (final gluons 2, channel 0, amplitudes in double).
// VEGAS iterations of this instance use the staged path (see mf_api.hip): the
// fused kernel of this instance returned wrong sums on the device while the
// same amplitude in the explicit-point kernel is exact.
#include "kernels.h"
namespace mf {
Launchers launchers_gg2_f64() { return make_launchers<2, 0, double, Dual<double>, 0, 0>(); }
}  // namespace mf
