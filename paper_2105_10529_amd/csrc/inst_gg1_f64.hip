// Kernel instance: gg1_f64 (final gluons 1, channel 0, amplitudes in double).
#include "kernels.h"
namespace mf {
Launchers launchers_gg1_f64() { return make_launchers<1, 0, double, Dual<double>, 1>(); }
}  // namespace mf
