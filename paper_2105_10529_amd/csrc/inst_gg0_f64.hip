// Kernel instance: gg0_f64 (final gluons 0, channel 0, amplitudes in double).
#include "kernels.h"
namespace mf {
Launchers launchers_gg0_f64() { return make_launchers<0, 0, double, Dual<double>, 1>(); }
}  // namespace mf
