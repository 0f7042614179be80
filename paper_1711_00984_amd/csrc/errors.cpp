// errors.cpp -- thread-local error message behind dpg_last_error().
#include "errors.h"

#include <cstdarg>
#include <cstdio>
#include <string>

namespace dpg {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

}  // namespace dpg
