// Kernel instance: gg2_f32 (final gluons 2, channel 0, amplitudes in float).
#include "kernels.h"
namespace mf {
Launchers launchers_gg2_f32() { return make_launchers<2, 0, float, Dual<float>, 0>(); }
}  // namespace mf
