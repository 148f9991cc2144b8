// Kernel instance: ddg_f64 (d d~ -> t t~ g; one final light parton, channel 2,
// amplitudes in double; derivatives included).
#include "kernels.h"
namespace mf {
Launchers launchers_ddg_f64() { return make_launchers<1, 2, double, Dual<double>, 1>(); }
}  // namespace mf
