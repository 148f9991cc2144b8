// Kernel instance: gg0_f32 (final gluons 0, channel 0, amplitudes in float).
#include "kernels.h"
namespace mf {
Launchers launchers_gg0_f32() { return make_launchers<0, 0, float, Dual<double>, 1>(); }
}  // namespace mf
