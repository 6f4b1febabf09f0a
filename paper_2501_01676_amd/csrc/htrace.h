// Optional host-side timeline (environment variable ABDDC_HOST_TRACE=1):
// each mark prints the host time spent since the previous mark to stderr.
// It shows host work and synchronisations that leave the GPU idle.
#pragma once

#include <chrono>
#include <cstdio>
#include <cstdlib>

namespace abddc {

struct HostTrace {
  bool on;
  std::chrono::steady_clock::time_point last;
  HostTrace() : on(enabled()), last(on ? std::chrono::steady_clock::now() : std::chrono::steady_clock::time_point()) {}
  static bool enabled() {
    static const bool e = std::getenv("ABDDC_HOST_TRACE") != nullptr;   // read once per process
    return e;
  }
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[host] %-40s %9.1f us\n", what,
                 std::chrono::duration<double, std::micro>(now - last).count());
    last = now;
  }
};

}  // namespace abddc
