// Kernel instance: uu_f64 (final gluons 0, channel 1, amplitudes in double).
#include "kernels.h"
namespace mf {
Launchers launchers_uu_f64() { return make_launchers<0, 1, double, Dual<double>, 1>(); }
}  // namespace mf
