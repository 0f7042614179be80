// errors.cpp -- thread-local error message behind dpg_last_error().
#include "errors.h"

#include <cstdarg>
#include <cstdio>

namespace dpg {

namespace {
thread_local char g_err[512];   // fixed storage: recording an error allocates nothing
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char* last_error() { return g_err; }

}  // namespace dpg
