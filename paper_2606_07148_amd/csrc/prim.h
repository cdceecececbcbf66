// Device-wide primitives of the build and the export, called on rocPRIM
// directly: radix sort of 64-bit keys, selection of unique keys, exclusive
// prefix sum of 64-bit counts.  Each follows rocPRIM's two-call protocol
// (temp == nullptr: *bytes receives the temporary storage needed); counts
// are size_t, so no input size is narrowed to int.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

namespace abc {
namespace prim {

// Stable LSD radix sort of n keys on bits [begin, end).
inline hipError_t sort_keys(void *temp, size_t &bytes, const uint64_t *in, uint64_t *out,
                            size_t n, int begin, int end, hipStream_t s) {
  return rocprim::radix_sort_keys(temp, bytes, in, out, n, (unsigned)begin, (unsigned)end, s);
}

// The first key of every run of equal keys, in order; *count their number.
inline hipError_t unique(void *temp, size_t &bytes, const uint64_t *in, uint64_t *out,
                         int *count, size_t n, hipStream_t s) {
  return rocprim::unique(temp, bytes, in, out, count, n, rocprim::equal_to<uint64_t>(), s);
}

// out[i] = in[0] + ... + in[i - 1] (out[0] = 0).
inline hipError_t exclusive_sum(void *temp, size_t &bytes, const int64_t *in, int64_t *out,
                                size_t n, hipStream_t s) {
  return rocprim::exclusive_scan(temp, bytes, in, out, (int64_t)0, n, rocprim::plus<int64_t>(),
                                 s);
}

}  // namespace prim
}  // namespace abc
