// Status strings and thread-local error reporting for the C ABI.
#include <stdio.h>
#include <string.h>

#include "kfhost.h"

namespace {
thread_local char g_last_error[512] = "";
}

int kf_check(hipError_t e) {
  if (e == hipSuccess) return KF_OK;
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
  return KF_E_HIP;
}

int kf_check_launch() { return kf_check(hipGetLastError()); }

int kf_fail(int status, const char* msg) {
  snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
  return status;
}

extern "C" const char* kf_status_string(int status) {
  switch (status) {
    case KF_OK: return "ok";
    case KF_E_INVALID_ARG: return "invalid argument";
    case KF_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case KF_E_HIP: return "HIP error";
    case KF_E_UNSUPPORTED: return "unsupported parameter";
    default: return "unknown status";
  }
}

extern "C" int kf_last_error(char* buf, size_t n) {
  int len = (int)strlen(g_last_error);
  if (buf && n > 0) {
    size_t m = (size_t)len < n - 1 ? (size_t)len : n - 1;
    memcpy(buf, g_last_error, m);
    buf[m] = '\0';
  }
  return len;
}
