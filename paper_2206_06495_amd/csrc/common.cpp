// Thread-local error message and version query of the C ABI.
#include "common.h"

namespace rbf {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace rbf

extern "C" const char *rbf_last_error(void) { return rbf::g_last_error.c_str(); }

extern "C" int32_t rbf_abi_version(void) { return RBF_ABI_VERSION; }
