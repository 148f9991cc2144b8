// Kernel instance: gg1_f32 (final gluons 1, channel 0, amplitudes in float).
#include "kernels.h"
namespace mf {
Launchers launchers_gg1_f32() { return make_launchers<1, 0, float, Dual<float>, 1>(); }
}  // namespace mf
