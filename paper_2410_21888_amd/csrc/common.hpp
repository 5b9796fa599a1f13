// Error reporting shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

namespace rimp2 {

// Message of the calling thread's last non-OK return.
inline thread_local char g_err[512] = "";

inline int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int code, const char* fmt, ...) {
  char buf[sizeof g_err];   // the arguments may include g_err itself
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  memcpy(g_err, buf, sizeof buf);
  return code;
}

}  // namespace rimp2

#define HIP_TRY(call)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return ::rimp2::fail(-4, "%s: %s", #call, hipGetErrorString(e_));       \
  } while (0)
