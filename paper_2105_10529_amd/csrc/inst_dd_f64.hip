// Kernel instance: dd_f64 (final gluons 0, channel 2, amplitudes in double).
#include "kernels.h"
namespace mf {
Launchers launchers_dd_f64() { return make_launchers<0, 2, double, Dual<double>, 1>(); }
}  // namespace mf
