// Error reporting of the C ABI: negative codes plus a message kept per
// context (and per thread for calls without a context).
#pragma once

#include <cstdarg>
#include <cstdio>

#include "ofm.h"

namespace ofm {

// Records the message for ctx (or the calling thread) and returns code.
int fail(ofm_ctx* ctx, int code, const char* fmt, ...);

}  // namespace ofm
