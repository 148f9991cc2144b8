// Kernel instance: qg_f64 (q g -> t t~ q and q~ g -> t t~ q~; one final light parton, channel 3,
// amplitudes in double; derivatives included).
#include "kernels.h"
namespace mf {
Launchers launchers_qg_f64() { return make_launchers<1, 3, double, Dual<double>, 1>(); }
}  // namespace mf
