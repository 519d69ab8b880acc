// Optional roctx ranges around the library's calls, so that a timeline taken
// with rocprofv3 --marker-trace shows which call launched which kernels. Off
// unless the environment variable NTT_ROCTX is set (to anything but "0") when
// the library first checks it; then each entry point pushes a range named for
// the call and pops it when the call returns (ranges cover the host side of a
// call: its launches, not the kernels' execution).
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdlib>
#include <cstring>

namespace ntti {

inline bool roctx_on() {
  static const bool on = [] {
    const char* e = std::getenv("NTT_ROCTX");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}

struct Range {
  bool on;
  explicit Range(const char* name) : on(roctx_on()) {
    if (on) roctxRangePushA(name);
  }
  ~Range() {
    if (on) roctxRangePop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

}  // namespace ntti
