// Error reporting, version and the per-device conversion workspace.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace argcsr {

namespace {
thread_local std::string g_last_error;
std::mutex g_ws_mutex;
std::vector<Workspace> g_ws;   // indexed by device ordinal
}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

int device_workspace(size_t bytes, void** out) {
  int dev = 0;
  ARGCSR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  Workspace& w = g_ws[dev];
  if (w.bytes < bytes) {
    if (w.ptr) {
      // the previous workspace may still be read by queued conversion work
      ARGCSR_HIP(hipDeviceSynchronize());
      ARGCSR_HIP(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipMalloc(&w.ptr, want) != hipSuccess) {
      w.ptr = nullptr;
      return fail(ARGCSR_ENOMEM, "workspace allocation of %zu bytes failed", want);
    }
    w.bytes = want;
  }
  *out = w.ptr;
  return ARGCSR_OK;
}

}  // namespace argcsr

extern "C" const char* argcsr_last_error(void) { return argcsr::last_error(); }

extern "C" int argcsr_version(void) { return 100; }
