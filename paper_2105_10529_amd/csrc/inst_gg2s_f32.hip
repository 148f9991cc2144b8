// Kernel instance: gg2s_f32 (g g -> t t~ g g, FP32 amplitudes, colour sum on
// the FP32 matrix cores; FP64 kinematics, PDFs and weights), gg2s.h.
#include "gg2s.h"
namespace mf {
Launchers launchers_gg2s_f32() { return s2::launchers<float>(); }
}  // namespace mf
