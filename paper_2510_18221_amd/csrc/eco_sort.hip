// eco_sort.hip -- init-time placement sort (library radix sort of 64-bit keys).
//
// Placement takes, per world, the cells with the smallest (Philox key, cell)
// pairs; sorting the packed 64-bit keys gives that order.  Init only: never on
// the step path.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

namespace eco {

hipError_t sort_keys_temp_bytes(uint32_t n, size_t* bytes) {
  *bytes = 0;
  return hipcub::DeviceRadixSort::SortKeys(nullptr, *bytes, (const unsigned long long*)nullptr,
                                           (unsigned long long*)nullptr, (int)n, 0, 64, (hipStream_t)0);
}

hipError_t sort_keys(void* tmp, size_t bytes, const unsigned long long* in, unsigned long long* out, uint32_t n,
                     hipStream_t s) {
  size_t b = bytes;
  return hipcub::DeviceRadixSort::SortKeys(tmp, b, in, out, (int)n, 0, 64, s);
}

}  // namespace eco
