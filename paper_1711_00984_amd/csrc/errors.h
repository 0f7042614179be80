// errors.h -- thread-local error message behind dpg_last_error().
#pragma once

namespace dpg {

// Record a printf-style message for the calling thread and return code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
const char* last_error();

}  // namespace dpg
