// Shared host-side helpers: status handling, small complex type, HIP checks.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tn.h"

namespace tn {

using cd = std::complex<double>;

// Error carried from the C++ core to the C ABI, where it becomes a status.
struct Error : std::runtime_error {
  tn_status code;
  Error(tn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define TN_REQUIRE(cond, code, msg)                      \
  do {                                                   \
    if (!(cond)) throw ::tn::Error((code), (msg));       \
  } while (0)

#define TN_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::tn::Error(TN_ERR_DEVICE, std::string(#call) + ": " +            \
                                           hipGetErrorString(e_));            \
  } while (0)

// Run a body and map exceptions to status codes (used by every extern "C").
template <class F>
tn_status guarded(F&& f) {
  try {
    f();
    set_last_error("");
    return TN_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return TN_ERR_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return TN_ERR_ARG;
  }
}

}  // namespace tn
