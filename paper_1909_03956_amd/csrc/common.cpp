#include "common.h"

#include <cstdarg>
#include <cstdio>

namespace swv {

static thread_local char g_msg[1024] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = '\0'; }

}  // namespace swv

extern "C" const char* swv_last_error(void) { return swv::g_msg; }

extern "C" int swv_version(int* major, int* minor) {
    if (!major || !minor) return swv::fail(SWV_EINVAL, "swv_version: null pointer");
    *major = SWV_VERSION_MAJOR;
    *minor = SWV_VERSION_MINOR;
    swv::clear_error();
    return SWV_OK;
}
