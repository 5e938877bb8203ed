// Error reporting shared by the C ABI entry points.
#include <stdarg.h>
#include <string.h>

#include "common.h"

namespace ligate {

static thread_local char g_last_error[512] = "";

void set_last_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_error("%s: %s", what, hipGetErrorString(e));
        return DOCK_ERR_HIP;
    }
    return DOCK_OK;
}

}  // namespace ligate

extern "C" const char *dock_error_string(int code) {
    switch (code) {
        case DOCK_OK: return "ok";
        case DOCK_ERR_INVALID_ARG: return "invalid argument";
        case DOCK_ERR_LIMIT: return "limit exceeded";
        case DOCK_ERR_HIP: return "HIP runtime error";
        case DOCK_ERR_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

extern "C" const char *dock_last_error(void) { return ligate::g_last_error; }
