// Optional host-side timeline (environment variable ABDDC_HOST_TRACE=1):
// each mark prints the host time spent since the previous mark of any trace
// on the calling thread (one continuous timeline), the minor page faults
// taken meanwhile and the mark's steady-clock time, to stderr.
// It shows host work and synchronisations that leave the GPU idle.
#pragma once

#include <sys/resource.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>

namespace abddc {

struct HostTrace {
  bool on;
  HostTrace() : on(enabled()) {
    if (on && last().time_since_epoch().count() == 0) {
      last() = std::chrono::steady_clock::now();
      faults() = minor_faults();
    }
  }
  // the thread's previous mark and the process's minor page faults then
  static std::chrono::steady_clock::time_point& last() {
    static thread_local std::chrono::steady_clock::time_point t;
    return t;
  }
  static long& faults() {
    static thread_local long f = 0;
    return f;
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
    std::fprintf(stderr, "[host] %-40s %9.1f us %7ld faults @ %.1f us\n", what,
                 std::chrono::duration<double, std::micro>(now - last()).count(), f - faults(),
                 std::chrono::duration<double, std::micro>(now.time_since_epoch()).count());
    last() = now;
    faults() = f;
  }
};

}  // namespace abddc
