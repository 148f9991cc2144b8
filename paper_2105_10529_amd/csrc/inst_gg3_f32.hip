// Kernel instance: gg3_f32 (g g -> t t~ g g g, FP32 amplitudes, FP64
// kinematics, PDFs and weights), evaluated by the staged kernels of gg3.h.
#include "gg3.h"

namespace mf {
Launchers launchers_gg3_f32() { return g3::launchers<float>(); }
}  // namespace mf
