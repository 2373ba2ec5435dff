// Error plumbing shared by the host sources: HIP failures become DeviceError, which the
// C-ABI layer turns into MG_EDEVICE with the HIP error string.
#pragma once
#include <hip/hip_runtime_api.h>

#include <stdexcept>
#include <string>

namespace decmg {

struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

inline void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw DeviceError(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace decmg
