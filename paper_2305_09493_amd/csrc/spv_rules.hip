// Module-level rules (section "Validation Rules"): a module that passed every
// structural and ID check must declare a capability (OpCapability, 17),
// define its memory model (OpMemoryModel, 14), declare a function
// (OpFunction, 54) and declare an entry point (OpEntryPoint, 15).
//
// The rules read the instruction index that the validate call wrote: module
// m's opcodes are idx_op[mod_off[m] .. mod_off[m] + n_inst).  Two kernels on
// the call's stream after its own:
//   k_rules_scan : each wave takes 4096 consecutive index entries.  A chunk
//                  inside one passing module's index prefix is read with
//                  coalesced 16-byte loads; the block's such chunks are
//                  combined in LDS and flushed once per module.  Any other
//                  chunk is walked by its lanes, 64 entries each, across
//                  module boundaries (modules found by binary search over
//                  mod_off).  The rule opcodes seen are ORed into presence
//                  bits (sem_mask bits 8..11 of passing modules, whose
//                  sem_mask is otherwise 0) with device atomics; a flush
//                  that a plain read shows adds no new bit is skipped.
//   k_rules_fin  : per module, presence bits -> SPV_E_MODULE_RULES with the
//                  missing rules as 8 (capability) | 16 (memory model) |
//                  32 (function) | 64 (entry point).
// Bytes per index entry: 2 (opcode), plus 16 per module for the results.
#include <hip/hip_runtime.h>

#include "spv_internal.h"

namespace spv {

constexpr int kRulesBlock = 256;
constexpr int kRulesPer = 64;                    // index entries per thread
constexpr int64_t kRulesWave = 64 * kRulesPer;   // entries per wave chunk
constexpr uint32_t kPresentShift = 8;

__device__ __forceinline__ uint32_t rule_bit(uint32_t op) {
  return op == 17u ? 1u : (op == 14u ? 2u : (op == 54u ? 4u : (op == 15u ? 8u : 0u)));
}

// ORs presence bits into module m's sem_mask, unless a plain (cached) read
// already shows them: a stale read only costs a redundant atomic.
__device__ __forceinline__ void rules_flush(spv_result* results, int64_t m, uint32_t bits) {
  if (bits == 0) return;
  uint32_t* dst = &results[m].sem_mask;
  const uint32_t want = bits << kPresentShift;
  if ((*dst & want) != want) atomicOr(dst, want);
}

// The last module starting at or before i (module 0 if none does).
__device__ __forceinline__ int64_t module_at(const int64_t* mod_off, int64_t M, int64_t i) {
  int64_t lo = 0, hi = M - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (mod_off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t bits) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) bits |= uint32_t(__shfl_xor(int(bits), d));
  return bits;
}

__global__ __launch_bounds__(kRulesBlock) void k_rules_scan(const uint16_t* idx_op, const int64_t* mod_off,
                                                            spv_result* results, int64_t M, int64_t W) {
  constexpr int kWaves = kRulesBlock / 64;
  __shared__ long long s_m[kWaves];
  __shared__ uint32_t s_bits[kWaves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = (int64_t(blockIdx.x) * kWaves + wave) * kRulesWave;
  // bits of a wave whose whole chunk lies in one module's index prefix;
  // combined over the block and flushed once per module below
  long long fm = -1;
  uint32_t fbits = 0;
  if (c0 < W) {
    const int64_t c1 = (c0 + kRulesWave < W) ? c0 + kRulesWave : W;
    // the chunk's module (the same in every lane)
    const int64_t mc = module_at(mod_off, M, c0);
    const int64_t bc = mod_off[mc], ec = mod_off[mc + 1];
    const bool live_c = results[mc].code == SPV_OK;
    const int64_t lim_c = bc + int64_t(results[mc].n_inst);
    const bool aligned = (reinterpret_cast<uintptr_t>(idx_op) & 15u) == 0;
    if (c0 >= bc && c1 <= ec && (!live_c || c0 >= lim_c)) {
      // inside one module and outside its valid prefix: nothing to read
    } else if (aligned && live_c && c1 - c0 == kRulesWave && c0 >= bc && c1 <= lim_c) {
      // a full chunk inside one module's index prefix: coalesced 16-byte loads
      const uint4* src = reinterpret_cast<const uint4*>(idx_op + c0);
      uint32_t bits = 0;
#pragma unroll
      for (int j = 0; j < kRulesPer / 8; ++j) {
        const uint4 v = src[j * 64 + lane];
        const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) bits |= rule_bit(x[k] & 0xFFFFu) | rule_bit(x[k] >> 16);
      }
      fbits = wave_or(bits);
      fm = mc;
    } else {
      // general chunk: each lane walks its own consecutive entries across
      // module boundaries
      const int64_t i0 = c0 + int64_t(lane) * kRulesPer;
      int64_t m = -1;
      uint32_t bits = 0;
      if (i0 < c1) {
        m = module_at(mod_off, M, i0);
        int64_t b = mod_off[m], e = mod_off[m + 1];
        bool live = results[m].code == SPV_OK;
        int64_t lim = b + int64_t(results[m].n_inst);
        const int64_t i1 = (i0 + kRulesPer < c1) ? i0 + kRulesPer : c1;
        for (int64_t i = i0; i < i1; ++i) {
          while (i >= e && m + 1 < M) {
            rules_flush(results, m, bits);
            bits = 0;
            ++m;
            b = mod_off[m];
            e = mod_off[m + 1];
            live = results[m].code == SPV_OK;
            lim = b + int64_t(results[m].n_inst);
          }
          if (i >= e) break;  // past the last module
          if (i < b) {        // before the first module
            i = b - 1;
            continue;
          }
          if (!live || i >= lim) {  // the rest of this module holds no entries
            i = e - 1;
            continue;
          }
          bits |= rule_bit(idx_op[i]);
        }
      }
      // a wave whose lanes all end in one module flushes once
      const long long m0 = __shfl(static_cast<long long>(m), 0);
      if (__ballot(m != m0) == 0) {
        bits = wave_or(bits);
        if (lane == 0 && m >= 0) rules_flush(results, m, bits);
      } else if (m >= 0) {
        rules_flush(results, m, bits);
      }
    }
  }
  if (lane == 0) {
    s_m[wave] = fm;
    s_bits[wave] = fbits;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long cur = -1;
    uint32_t acc = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (s_m[w] != cur) {
        if (cur >= 0) rules_flush(results, cur, acc);
        cur = s_m[w];
        acc = 0;
      }
      acc |= s_bits[w];
    }
    if (cur >= 0) rules_flush(results, cur, acc);
  }
}

__global__ __launch_bounds__(kRulesBlock) void k_rules_fin(spv_result* results, int64_t M) {
  for (int64_t m = int64_t(blockIdx.x) * kRulesBlock + threadIdx.x; m < M; m += int64_t(gridDim.x) * kRulesBlock) {
    if (results[m].code != SPV_OK) continue;
    const uint32_t present = (results[m].sem_mask >> kPresentShift) & 15u;
    const uint32_t missing = ((present & 1u) ? 0u : 8u) | ((present & 2u) ? 0u : 16u) | ((present & 4u) ? 0u : 32u) |
                             ((present & 8u) ? 0u : 64u);
    results[m].sem_mask = missing;
    if (missing) results[m].code = SPV_E_MODULE_RULES;
  }
}

void launch_rules(const uint16_t* idx_op, const int64_t* mod_off, spv_result* results, int64_t M, int64_t W,
                  hipStream_t s) {
  if (M <= 0) return;
  if (W > 0) {
    const int64_t per_block = (kRulesBlock / 64) * kRulesWave;
    const int64_t g = (W + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_rules_scan, dim3(unsigned(g)), dim3(kRulesBlock), 0, s, idx_op, mod_off, results, M, W);
  }
  int64_t g = (M + kRulesBlock - 1) / kRulesBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_rules_fin, dim3(unsigned(g)), dim3(kRulesBlock), 0, s, results, M);
}

}  // namespace spv
