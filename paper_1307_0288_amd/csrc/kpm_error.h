// Error reporting shared by the host translation units of the C ABI: the
// message is returned by kpm_last_error() on the calling thread.
#pragma once

#include "kpm.h"

namespace kpm_detail {
kpm_status set_error(kpm_status st, const char *msg);
// set_error with a printf-style message
kpm_status fail(kpm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
}
