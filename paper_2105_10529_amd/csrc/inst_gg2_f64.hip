// Kernel instance: gg2_f64 (final gluons 2, channel 0, amplitudes in double).
#include "kernels.h"
namespace mf {
Launchers launchers_gg2_f64() { return make_launchers<2, 0, double, Dual<double>, 0>(); }
}  // namespace mf
