// Shared helpers for the PNK-CCSD library: error handling, device types.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace pnk {

// A failed HIP call or an invalid internal state. Caught at the C boundary
// and turned into a status code; never crosses it.
struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};
struct ArgError : std::runtime_error {
  explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};
struct OomError : std::runtime_error {
  explicit OomError(const std::string& s) : std::runtime_error(s) {}
};

#define PNK_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::pnk::HipError(std::string(#call) + " failed: " +                 \
                            hipGetErrorString(e_) + " (" + __FILE__ + ":" +    \
                            std::to_string(__LINE__) + ")");                   \
  } while (0)

#define PNK_CHECK_LAUNCH() PNK_HIP(hipGetLastError())

#define PNK_REQUIRE(cond, msg)                                                 \
  do {                                                                         \
    if (!(cond)) throw ::pnk::ArgError(msg);                                   \
  } while (0)

// Storage / compute precisions of a contraction.
enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2 };

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pnk
