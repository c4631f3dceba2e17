// Thread-local error reporting for the C ABI.
#include <cstdarg>
#include <string>

#include "hrir_internal.h"

namespace hrir {
namespace {
thread_local std::string t_err;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }

const char* last_error() { return t_err.c_str(); }

}  // namespace hrir

extern "C" const char* hrir_last_error(void) { return hrir::last_error(); }
