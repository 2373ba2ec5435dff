// The binary16 weight type of the row kernels (device code).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace decmg {
namespace {

// An IEEE binary16 weight, widened exactly to FP32 or FP64.  A named type rather than _Float16,
// so that the kernels instantiated on it keep demangled names in profiler output.
struct Half16 {
  uint16_t bits;
  __device__ __forceinline__ explicit operator float() const {
    return static_cast<float>(__builtin_bit_cast(_Float16, bits));
  }
  __device__ __forceinline__ explicit operator double() const {
    return static_cast<double>(__builtin_bit_cast(_Float16, bits));
  }
};

}  // namespace
}  // namespace decmg
