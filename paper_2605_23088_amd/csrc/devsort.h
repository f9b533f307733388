// Device sort / scan helpers of the index builders (rocPRIM), and the
// temporary-memory arena they draw from.  No paper arithmetic here.
#pragma once

#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include <algorithm>
#include <vector>

namespace yasps {
namespace devsort {

constexpr int DI_BLOCK = 256;
constexpr int PIN_INTS = 64;  // size of the pinned read-back scratch the builders are given

inline int bits_for(long long v) {  // bits needed for values 0 .. v
  int b = 1;
  while ((1ll << b) <= v) ++b;
  return b;
}

inline int grid_of(long long m) { return (int)std::max<long long>(1, (m + DI_BLOCK - 1) / DI_BLOCK); }

// Temporaries of one build, carved from the caller's arena while it lasts
// (256-byte aligned), else allocated and freed when done; `used` is the arena
// size the whole build needs.
struct Temp {
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  int* pin = nullptr;  // pinned host scratch (PIN_INTS ints) for the builds' read-backs
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <class T>
  T* get(size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    void* p = nullptr;
    if (used + bytes <= cap) {
      p = arena + used;
    } else if (err == hipSuccess) {
      err = hipMalloc(&p, bytes);
      if (p) ptrs.push_back(p);
    }
    used += bytes;
    return static_cast<T*>(p);
  }
  ~Temp() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// Stable radix sort of (key, value) pairs over key bits [0, end_bit).  rocPRIM
// sorts up to 2^20 items by merging sorted blocks (about two launches per
// doubling of the sorted run past 1024 items) unless told otherwise; its
// one-sweep LSD sort takes about three launches per 8-bit digit.  The cheaper
// of the two by that count is taken (one-sweep for keys of few bits).
template <class Config, class K, class V>
hipError_t sort_pairs_with(Temp& tmp, const K* ki, K* ko, const V* vi, V* vo, long long m, int end_bit,
                           hipStream_t s) {
  size_t bytes = 0;
  hipError_t e =
      rocprim::radix_sort_pairs<Config>(nullptr, bytes, ki, ko, vi, vo, (size_t)m, 0u, (unsigned)end_bit, s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::radix_sort_pairs<Config>(store, bytes, ki, ko, vi, vo, (size_t)m, 0u, (unsigned)end_bit, s);
}

template <class K, class V>
hipError_t sort_pairs(Temp& tmp, const K* ki, K* ko, const V* vi, V* vo, long long m, int end_bit, hipStream_t s) {
  if (m == 0) return hipSuccess;
  int merges = 0;
  for (long long run = 1024; run < m; run *= 2) ++merges;
  const int digits = (end_bit + 7) / 8;
  if (m <= (1ll << 20) && 3 * digits + 2 < 2 * merges + 1) {
    using onesweep = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                rocprim::default_config, 0>;
    return sort_pairs_with<onesweep>(tmp, ki, ko, vi, vo, m, end_bit, s);
  }
  return sort_pairs_with<rocprim::default_config>(tmp, ki, ko, vi, vo, m, end_bit, s);
}

// in[k] for k < m, 0 at k = m: the input of an exclusive scan of m + 1 values
struct PaddedInput {
  const int32_t* in;
  size_t m;
  __host__ __device__ int32_t operator()(size_t k) const { return k < m ? in[k] : 0; }
};

// out[0] = 0, out[k + 1] = in[0] + ... + in[k]  (k < m): one exclusive scan
// of m + 1 values (no separate launch for out[0])
inline hipError_t prefix(Temp& tmp, const int32_t* in, int32_t* out, long long m, hipStream_t s) {
  const auto src =
      rocprim::make_transform_iterator(rocprim::make_counting_iterator<size_t>(0), PaddedInput{in, (size_t)m});
  size_t bytes = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, bytes, src, out, int32_t(0), (size_t)m + 1,
                                         rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::exclusive_scan(store, bytes, src, out, int32_t(0), (size_t)m + 1, rocprim::plus<int32_t>(), s);
}

inline hipError_t inclusive(Temp& tmp, const int32_t* in, int32_t* out, long long m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  size_t bytes = 0;
  hipError_t e = rocprim::inclusive_scan(nullptr, bytes, in, out, (size_t)m, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::inclusive_scan(store, bytes, in, out, (size_t)m, rocprim::plus<int32_t>(), s);
}

}  // namespace devsort
}  // namespace yasps
