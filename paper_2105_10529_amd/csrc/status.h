// Error reporting shared by the translation units behind the C ABI: the
// message of the last failing call, per host thread (mf_last_error).
#pragma once
#include "../../include/mf.h"

namespace mf {
mf_status set_error(mf_status s, const char* fmt, ...);
void clear_error();
}  // namespace mf
