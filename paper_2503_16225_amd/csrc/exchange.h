// Exchange slots between the work-groups of a cooperative kernel: every value
// that one wave hands to others has a slot of its own (per step), filled
// beforehand with a signalling-NaN pattern that no arithmetic produces.
// Producers store with device-scope atomic stores, and consumers poll the
// slot with device-scope atomic loads until the pattern is gone, so no
// barrier is needed.  Waits are bounded (kXchSpin polls); a timeout is
// reported through ok.
#pragma once

#include "devcommon.h"

namespace eahp {
namespace xch {

constexpr unsigned long long kEmpty = 0x7FF4A5A5A5A5A5A5ull;
constexpr int kXchSpin = 1 << 20;

__device__ __forceinline__ void put_z(z64* p, z64 v) {
  unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
  unsigned long long x = (unsigned long long)__double_as_longlong(v.x);
  unsigned long long y = (unsigned long long)__double_as_longlong(v.y);
  if (x == kEmpty) x = 0x7FF8000000000000ull;
  if (y == kEmpty) y = 0x7FF8000000000000ull;
  __hip_atomic_store(u, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(u + 1, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ z64 poll_z(const z64* p, bool& ok) {
  const unsigned long long* u = reinterpret_cast<const unsigned long long*>(p);
  unsigned long long x = kEmpty, y = kEmpty;
  for (int spins = 0;; ++spins) {
    x = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    y = __hip_atomic_load(u + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (x != kEmpty && y != kEmpty) break;
    if (spins > kXchSpin) {
      ok = false;
      break;
    }
  }
  return mk<double>(__longlong_as_double((long long)x), __longlong_as_double((long long)y));
}

// Polls the n <= N slots p, p + stride, ... together: the loads of every
// slot not yet filled are in flight at once, so a wave waits about one
// round trip for all of them instead of one per slot.  v[j] is slot j's value.
template <int N>
__device__ __forceinline__ void poll_zn(const z64* p, int64_t stride, int n, z64 (&v)[N], bool& ok) {
  unsigned long long x[N], y[N];
  bool done[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    x[j] = y[j] = 0;
    done[j] = j >= n;
  }
  for (int spins = 0;; ++spins) {
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (!done[j]) {
        const unsigned long long* u = reinterpret_cast<const unsigned long long*>(p + j * stride);
        x[j] = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        y[j] = __hip_atomic_load(u + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    bool all = true;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (!done[j]) {
        if (x[j] != kEmpty && y[j] != kEmpty) done[j] = true;
        else all = false;
      }
    if (all) break;
    if (spins > kXchSpin) {
      ok = false;
      break;
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = mk<double>(__longlong_as_double((long long)x[j]), __longlong_as_double((long long)y[j]));
}

}  // namespace xch
}  // namespace eahp
