// Kernel instance: uug_f64 (u u~ -> t t~ g; one final light parton, channel 1,
// amplitudes in double; derivatives included).
#include "kernels.h"
namespace mf {
Launchers launchers_uug_f64() { return make_launchers<1, 1, double, Dual<double>, 1>(); }
}  // namespace mf
