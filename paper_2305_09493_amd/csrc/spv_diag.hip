// Semantic positions and the defined-before-use mode of spv_validate
// (options SPV_OPT_SEM_OFFSETS and SPV_OPT_DEF_BEFORE_USE), for gfx950.
//
// What is computed (Beehive SPIR-V Toolkit paper, arXiv 2305.09493): the ID
// rules of the semantic stage (each result ID defined once and every used ID
// defined, the SSA rule of section "Enabling Function Composition"; IDs
// below the header's bound, section "SPIR-V Library"), now with the word
// offset of the first instruction, in module order, that breaks the primary
// rule, and optionally the stricter reading that a use needs a definition
// earlier in the module (OpName targets and OpEntryPoint functions may still
// name later definitions).
//
// How: these kernels run after a validate call has written its results and
// index, over the modules that reached the semantic stage.  Each such module's
// part of the ID-set workspace (8 bytes per word) becomes an open-addressing
// table of its result IDs: slot = ID << 32 | word offset, claimed by a CAS
// and lowered by a 64-bit atomicMin, which keeps the ID's first definition
// (an instruction defining a result has at least two words, so the table is
// at most half full).  A second pass over the instructions lowers the
// module's first out-of-bound, duplicate and undefined offsets with atomicMin,
// and a last pass rewrites the results.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_internal.h"

namespace spv {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// Operand roles of the grammar's opcodes: operand words before the string
// (all of them for an instruction without one) and 2 bits per slot (0 literal,
// 1 ID use, 2 result ID).
struct DiagOp {
  uint32_t nfix, roles;
};

__device__ __forceinline__ DiagOp diag_op(uint32_t op) {
  switch (op) {
    case 5: return {1, 1u};                                      // OpName: target
    case 15: return {2, 1u << 2};                                // OpEntryPoint: model, function
    case 21: return {3, 2u};                                     // OpTypeInt
    case 43: return {3, 1u | (2u << 2)};                         // OpConstant
    case 54: return {4, 1u | (2u << 2) | (1u << 6)};             // OpFunction
    case 61: return {3, 1u | (2u << 2) | (1u << 4)};             // OpLoad
    case 62: return {2, 1u | (1u << 2)};                         // OpStore
    case 128: return {4, 1u | (2u << 2) | (1u << 4) | (1u << 6)};  // OpIAdd
    case 248: return {1, 2u};                                    // OpLabel
    default: return {0, 0u};  // OpCapability, OpMemoryModel, OpFunctionEnd, OpReturn: no IDs
  }
}

// A use that may name a later definition.
__device__ __forceinline__ bool forward_use(uint32_t op, uint32_t slot) {
  return (op == 5u && slot == 0u) || (op == 15u && slot == 1u);
}

// Modules whose results come from the semantic stage (codes 0 and 8..11).
__device__ __forceinline__ bool semantic_reached(uint32_t code) {
  return code == SPV_OK || (code >= SPV_E_ID_OUT_OF_BOUND && code <= SPV_E_MODULE_RULES);
}

__device__ __forceinline__ uint32_t diag_hash(uint32_t v) {
  uint32_t h = v * 0x9E3779B1u;  // Fibonacci hashing (Knuth's multiplicative method)
  return h ^ (h >> 15);
}

// Module of word g (the last m with mod_off[m] <= g among the modules that
// have words).
__device__ __forceinline__ int64_t diag_module(const int64_t* mod_off, int64_t M, int64_t g) {
  int64_t lo = 0, hi = M - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (mod_off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Instruction j = g - mod_off[m] of the module that owns word g, when g's
// module reached the semantic stage and has a j-th instruction.
struct DiagInst {
  bool ok;
  int64_t m, base, n;
  uint32_t pos, bound;
};

__device__ __forceinline__ DiagInst diag_inst(const VParams& P, int64_t g) {
  DiagInst d;
  d.ok = false;
  d.m = diag_module(P.mod_off, P.M, g);
  d.base = P.mod_off[d.m];
  d.n = P.mod_off[d.m + 1] - d.base;
  const spv_result r = P.results[d.m];
  if (!semantic_reached(r.code) || uint64_t(g - d.base) >= uint64_t(r.n_inst)) return d;
  d.pos = P.idx_off[g];
  d.bound = P.mods[d.m].bound;
  d.ok = true;
  return d;
}

}  // namespace

// Per-module first offsets to none; the ID tables of the modules that reached
// the semantic stage to empty.
__global__ __launch_bounds__(256) void k_diag_init(VParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t m = gtid; m < P.M; m += nth) P.diag[m] = make_uint4(kNone, kNone, kNone, 0u);
  for (int64_t g = gtid; g < P.W; g += nth) P.idmap[g] = 0ull;
}

// Every in-bound result ID with the offset of its first definition.
__global__ __launch_bounds__(256) void k_diag_defs(VParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t g = gtid; g < P.W; g += nth) {
    const DiagInst d = diag_inst(P, g);
    if (!d.ok) continue;
    const uint32_t* w = P.words + d.base + d.pos;
    const DiagOp o = diag_op(w[0] & 0xFFFFu);
    for (uint32_t s = 0; s < o.nfix; ++s) {
      if (((o.roles >> (2 * s)) & 3u) != 2u) continue;
      const uint32_t v = w[1 + s];
      if (v == 0u || v >= d.bound) continue;
      unsigned long long* tab = P.idmap + d.base;
      const unsigned long long val = ((unsigned long long)v << 32) | d.pos;
      uint64_t h = diag_hash(v) % uint64_t(d.n);
      while (true) {
        const unsigned long long prev = atomicCAS(&tab[h], 0ull, val);
        if (prev == 0ull) break;
        if (uint32_t(prev >> 32) == v) {
          atomicMin(&tab[h], val);  // same ID: the smaller offset stays
          break;
        }
        h = (h + 1 == uint64_t(d.n)) ? 0 : h + 1;
      }
    }
  }
}

// The first out-of-bound, duplicate and undefined offsets of every module.
__global__ __launch_bounds__(256) void k_diag_scan(VParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  const bool before_use = P.before_use != 0;
  for (int64_t g = gtid; g < P.W; g += nth) {
    const DiagInst d = diag_inst(P, g);
    if (!d.ok) continue;
    const uint32_t* w = P.words + d.base + d.pos;
    const uint32_t op = w[0] & 0xFFFFu;
    const DiagOp o = diag_op(op);
    const unsigned long long* tab = P.idmap + d.base;
    bool oob = false, dup = false, undef = false;
    for (uint32_t s = 0; s < o.nfix; ++s) {
      const uint32_t role = (o.roles >> (2 * s)) & 3u;
      if (role == 0u) continue;
      const uint32_t v = w[1 + s];
      if (v == 0u || v >= d.bound) {
        oob = true;
        continue;
      }
      // offset of v's first definition, or none
      uint32_t first = kNone;
      uint64_t h = diag_hash(v) % uint64_t(d.n);
      while (true) {
        const unsigned long long e = tab[h];
        if (e == 0ull) break;
        if (uint32_t(e >> 32) == v) {
          first = uint32_t(e);
          break;
        }
        h = (h + 1 == uint64_t(d.n)) ? 0 : h + 1;
      }
      if (role == 2u) dup |= first < d.pos;
      else undef |= first == kNone || (before_use && !forward_use(op, s) && first >= d.pos);
    }
    uint4* st = &P.diag[d.m];
    if (oob) atomicMin(&st->x, d.pos);
    if (dup) atomicMin(&st->y, d.pos);
    if (undef) atomicMin(&st->z, d.pos);
  }
}

// Results of the modules that reached the semantic stage: the classes from
// the offsets (with defined-before-use, a forward use is undefined), the code
// by the priority out of bound > duplicate > undefined, and with
// SPV_OPT_SEM_OFFSETS the first offset of the primary class in err_word.  A
// module with no semantic failure keeps its result (0, or the module rules'
// code 11).
__global__ __launch_bounds__(256) void k_diag_final(VParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t m = gtid; m < P.M; m += nth) {
    spv_result r = P.results[m];
    if (!semantic_reached(r.code)) continue;
    const uint4 st = P.diag[m];
    const uint32_t mask = (st.x != kNone ? 1u : 0u) | (st.y != kNone ? 2u : 0u) | (st.z != kNone ? 4u : 0u);
    if (!mask) continue;
    r.sem_mask = mask;
    r.code = (mask & 1u) ? SPV_E_ID_OUT_OF_BOUND : (mask & 2u) ? SPV_E_DUPLICATE_ID : SPV_E_UNDEFINED_ID;
    r.err_word = P.sem_offsets ? ((mask & 1u) ? st.x : (mask & 2u) ? st.y : st.z) : kNone;
    P.results[m] = r;
  }
}

void launch_diag(const VParams& p, hipStream_t s) {
  auto grid = [](int64_t n) {
    const int64_t g = n / 256 + 1;
    return int(g > 8192 ? 8192 : g);
  };
  const int64_t n = p.W > p.M ? p.W : p.M;
  hipLaunchKernelGGL(k_diag_init, dim3(grid(n)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_diag_defs, dim3(grid(p.W)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_diag_scan, dim3(grid(p.W)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_diag_final, dim3(grid(p.M)), dim3(256), 0, s, p);
}

}  // namespace spv
