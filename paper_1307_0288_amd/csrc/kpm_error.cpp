// Thread-local error message of the C ABI and the version string (host only).
#include "kpm_error.h"

#include <cstdarg>
#include <cstdio>
#include <string>

namespace {
thread_local std::string g_err;
}

kpm_status kpm_detail::set_error(kpm_status st, const char *msg) {
    g_err = msg;
    return st;
}

kpm_status kpm_detail::fail(kpm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

extern "C" {
const char *kpm_last_error(void) { return g_err.c_str(); }
const char *kpm_version(void) { return "kpm-mi355x 0.2 (gfx950)"; }
}
