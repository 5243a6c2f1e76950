// Error reporting, version and shared host helpers of the C ABI.
#include <math.h>

#include "common.hpp"

namespace srk {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// T = floor(sqrt(c) * 2^32), at most 2^32 - 1: a walk continues iff its
// 32-bit draw is below T (Section 2.2: stop with probability 1 - sqrt(c)).
uint32_t continue_threshold(double c) {
    double t = floor(sqrt(c) * 4294967296.0);
    if (t > 4294967295.0) t = 4294967295.0;
    if (t < 0.0) t = 0.0;
    return (uint32_t)t;
}

}  // namespace srk

extern "C" const char *simrank_last_error(void) { return srk::g_last_error.c_str(); }

extern "C" const char *simrank_version(void) { return "simrank-mi355x 0.1 (gfx950)"; }
