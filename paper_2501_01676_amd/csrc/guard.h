// Exception-to-error-code guard shared by the C ABI entry points.
#pragma once

#include <new>
#include <string>

#include "internal.h"

namespace abddc {

extern thread_local std::string g_last_error;
int fail(int code, const std::string& msg);

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ABDDC_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ABDDC_EDEVICE, e.what());
  }
}

}  // namespace abddc
