// Error reporting and version of the nvr C ABI.
#include "common.hpp"

#include <cstdarg>
#include <cstdio>

namespace nvr {

static thread_local char g_error[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

}  // namespace nvr

extern "C" const char *nvr_last_error(void) { return nvr::g_error; }

extern "C" const char *nvr_version(void) { return "nvr 0.1.0 (gfx950)"; }
