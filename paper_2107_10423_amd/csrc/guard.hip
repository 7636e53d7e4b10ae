// Host-side launch guards shared by every kernel wrapper (see gw_internal.h).
#include <cstdio>
#include <string>

#include "gw_internal.h"

namespace gw {

namespace {
bool g_audit = false;
long g_audit_count = 0;
thread_local std::string g_launch_err;
}  // namespace

bool audit_mode() { return g_audit; }
void set_audit_mode(bool on) { g_audit = on; }
const char* launch_error() { return g_launch_err.c_str(); }
long audit_count() { return g_audit_count; }
void audit_note() { ++g_audit_count; }

bool guard(const char* kernel, const char* buffer, long max_index, long extent) {
  if (max_index >= -1 && max_index < extent) return true;
  char buf[256];
  snprintf(buf, sizeof buf, "%s: launch would reach element %ld of %s (extent %ld)", kernel,
           max_index, buffer, extent);
  g_launch_err = buf;
  return false;
}

hipError_t refuse(const char* kernel, const char* why) {
  g_launch_err = std::string(kernel) + ": " + why;
  return hipErrorInvalidValue;
}

}  // namespace gw
