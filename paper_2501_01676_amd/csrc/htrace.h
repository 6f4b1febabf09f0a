// Optional host-side timeline (environment variable ABDDC_HOST_TRACE=1):
// each mark prints the host time spent since the previous mark, and the
// minor page faults taken meanwhile, to stderr.
// It shows host work and synchronisations that leave the GPU idle.
#pragma once

#include <sys/resource.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>

namespace abddc {

struct HostTrace {
  bool on;
  std::chrono::steady_clock::time_point last;
  long faults = 0;   // minor page faults of the process at the last mark
  HostTrace() : on(enabled()), last(on ? std::chrono::steady_clock::now() : std::chrono::steady_clock::time_point()) {
    if (on) faults = minor_faults();
  }
  static long minor_faults() {
    rusage u{};
    getrusage(RUSAGE_SELF, &u);
    return u.ru_minflt;
  }
  static bool enabled() {
    static const bool e = std::getenv("ABDDC_HOST_TRACE") != nullptr;   // read once per process
    return e;
  }
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    const long f = minor_faults();
    std::fprintf(stderr, "[host] %-40s %9.1f us %7ld faults\n", what,
                 std::chrono::duration<double, std::micro>(now - last).count(), f - faults);
    last = now;
    faults = f;
  }
};

}  // namespace abddc
