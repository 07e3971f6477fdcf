// Single-pass scan shared by decode's records and text modes: blocks of
// 1024 values, claimed in order, chained by a decoupled look-back.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_internal.h"

namespace spv {

constexpr int kRecThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanBlock = kRecThreads * kScanPerThread;  // values per scan block
constexpr int kRStateStride = 16;                          // one 128-byte line per block state
constexpr unsigned long long kRAgg = 1ull << 62, kRIncl = 2ull << 62, kRMask = 3ull << 62;
constexpr unsigned long long kRSum = (1ull << 62) - 1;

__device__ __forceinline__ unsigned long long ld_state_r(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_state_r(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single-pass exclusive scan of n 64-bit values (in may alias out): out[i] =
// sum of in[0 .. i), out[n] = the total.  Blocks claim their chunk from
// ctrl[claim]; states[] (kRStateStride words per block) must be zero.
__device__ inline void scan_block(const unsigned long long* in, int64_t n, unsigned long long* out,
                           unsigned long long* states, uint32_t* claim, uint32_t* spin_err) {
  __shared__ uint32_t s_bid;
  __shared__ unsigned long long s_w[kRecThreads / 64];
  __shared__ unsigned long long s_pre;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(claim, 1u);
  __syncthreads();
  const long long b = s_bid;
  const int64_t i0 = int64_t(b) * kScanBlock + int64_t(tid) * kScanPerThread;
  unsigned long long v[kScanPerThread], t = 0;
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) {
    v[k] = (i0 + k < n) ? in[i0 + k] : 0ull;
    t += v[k];
  }
  unsigned long long inc = t;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  unsigned long long wpre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kRecThreads / 64; ++w) {
    if (w < wave) wpre += s_w[w];
    tot += s_w[w];
  }
  if (tid == 64) st_state_r(&states[b * kRStateStride], kRAgg | tot);
  if (wave == 0) {
    unsigned long long prefix = 0;
    long long hi = b - 1;
    uint32_t spins = 0;
    while (hi >= 0) {
      const long long u = hi - lane;
      const unsigned long long st = (u >= 0) ? ld_state_r(&states[u * kRStateStride]) : kRIncl;
      const unsigned long long f = st & kRMask;
      const uint64_t stopm = __ballot(f == kRIncl);
      const uint64_t unpub = __ballot(f == 0);
      const int sl = stopm ? int(__builtin_ctzll(stopm)) : 64;
      const uint64_t need = (sl >= 63) ? ~0ull : ((2ull << sl) - 1ull);
      if (unpub & need) {
        if (++spins > kSpinLimit) {
          if (lane == 0) atomicOr(spin_err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      unsigned long long c = (lane <= sl) ? (st & kRSum) : 0ull;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
      prefix += c;
      if (sl < 64) break;
      hi -= 64;
    }
    if (lane == 0) {
      st_state_r(&states[b * kRStateStride], kRIncl | (prefix + tot));
      s_pre = prefix;
    }
  }
  __syncthreads();
  unsigned long long run = s_pre + wpre + (inc - t);
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) {
    if (i0 + k < n) out[i0 + k] = run;
    run += v[k];
  }
  // the total, after the last value
  if (i0 <= n && n < i0 + kScanPerThread) out[n] = run;
}

}  // namespace spv
