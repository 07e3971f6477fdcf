// Batched SPIR-V encode for gfx950: the library's binary write step.
//
// What is computed (Beehive SPIR-V Toolkit paper, arXiv 2305.09493): every
// instruction writes its first word (word count << 16 | opcode) and its
// operands, operands report their word counts so the module size is known
// before writing (section "Parsing Operand Kinds"), and the header's bound
// is recomputed right before the module is written (section "SPIR-V
// Library", header listing and initial-bound paragraph).
//
// How: record r's output position is 5 * (m + 1) + S(r), where m is its
// module and S(r) the sum of the word counts of all records before r - a
// plain exclusive scan, computed in one pass with a decoupled look-back over
// blocks of records, followed by the scatter in the same pass.  Module
// failures (rare) are found in the same pass; a module that fails writes no
// words, so when any module fails a compaction kernel closes the gaps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_internal.h"

namespace spv {

namespace {

constexpr int kEncThreads = 256;
constexpr uint32_t kMagicE = 0x07230203u;

struct EGEnt {
  uint16_t op;
  uint8_t n_ops;   // non-string operand words
  uint8_t idmask;  // operand s (0-based) is an ID (use or result) when bit s is set
  uint8_t is_name;
};
__device__ __constant__ EGEnt kEncGrammar[12] = {
    {5, 1, 0x1, 1},    // OpName          id, string
    {14, 2, 0x0, 0},   // OpMemoryModel
    {17, 1, 0x0, 0},   // OpCapability
    {21, 3, 0x1, 0},   // OpTypeInt       result, width, signedness
    {43, 3, 0x3, 0},   // OpConstant      type, result, value
    {54, 4, 0xB, 0},   // OpFunction      type, result, control, fn type
    {56, 0, 0x0, 0},   // OpFunctionEnd
    {61, 3, 0x7, 0},   // OpLoad          type, result, pointer
    {62, 2, 0x3, 0},   // OpStore         pointer, object
    {128, 4, 0xF, 0},  // OpIAdd          type, result, a, b
    {248, 1, 0x1, 0},  // OpLabel         result
    {253, 0, 0x0, 0},  // OpReturn
};

// packed LDS table entry for opcode < 256: bit 15 known, bits 0..3 n_ops,
// bits 4..7 ID mask, bit 8 OpName
__device__ __forceinline__ void enc_table(uint16_t* tbl) {
  for (int i = threadIdx.x; i < 257; i += blockDim.x) tbl[i] = 0;
  __syncthreads();
  if (threadIdx.x < 12) {
    EGEnt g = kEncGrammar[threadIdx.x];
    tbl[g.op] = uint16_t(0x8000u | g.n_ops | (uint32_t(g.idmask) << 4) | (uint32_t(g.is_name) << 8));
  }
  __syncthreads();
}

// block states carry their whole message: relaxed device-scope atomics
__device__ __forceinline__ unsigned long long ld_state_e(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_state_e(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr unsigned long long kEAgg = 1ull << 62, kEIncl = 2ull << 62, kEMask = 3ull << 62;
constexpr unsigned long long kESum = (1ull << 62) - 1;

// module of record r, searching forward from a module known to start at or before r
__device__ __forceinline__ int64_t module_of(const int64_t* rec_mod_off, int64_t M, int64_t m, int64_t r) {
  while (m + 1 < M && rec_mod_off[m + 1] <= r) ++m;
  return m;
}

}  // namespace

__global__ __launch_bounds__(256) void k_enc_init(EParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (gtid == 0) {
    P.ctrl[0] = 0;
    P.ctrl[1] = 0;
    P.ctrl[2] = 0;
  }
  for (int64_t i = gtid; i < P.n_blocks; i += nth) P.blk[i] = 0;
  for (int64_t m = gtid; m < P.M; m += nth) {
    P.mod_bad[m] = ~0ull;
    P.mod_maxid[m] = 0;
    P.mod_words[m] = -1;
  }
}

// One pass: per-record word counts and checks, exclusive scan with look-back,
// scatter of every record's words.
__global__ __launch_bounds__(kEncThreads) void k_enc_main(EParams P) {
  __shared__ uint16_t tbl[257];
  __shared__ long long s_b;
  __shared__ unsigned long long s_wsum[kEncThreads / 64];
  __shared__ unsigned long long s_prefix;
  __shared__ long long s_m0;
  enc_table(tbl);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int rpt = P.block_records / kEncThreads;

  for (;;) {
    if (tid == 0) s_b = atomicAdd(&P.ctrl[0], 1u);
    __syncthreads();
    const long long b = s_b;
    if (b >= P.n_blocks) break;
    const int64_t r0 = b * P.block_records;
    const int64_t r1 = (r0 + P.block_records < P.N) ? r0 + P.block_records : P.N;
    if (tid == 0) {
      // module of r0: last m with rec_mod_off[m] <= r0
      int64_t lo = 0, hi = P.M - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (P.rec_mod_off[mid] <= r0) lo = mid;
        else hi = mid - 1;
      }
      s_m0 = lo;
    }
    __syncthreads();
    const int64_t rb = r0 + int64_t(tid) * rpt;
    // pass 1 over this thread's records: word counts
    unsigned long long mysum = 0;
    for (int k = 0; k < rpt; ++k) {
      int64_t r = rb + k;
      if (r >= r1) break;
      uint32_t op = P.op[r];
      int64_t n_ops = int64_t(P.opnd_off[r + 1]) - P.opnd_off[r];
      int64_t L = int64_t(P.str_off[r + 1]) - P.str_off[r];
      uint32_t e = tbl[op < 256u ? op : 256u];
      bool name = (e >> 8) & 1u;
      mysum += uint64_t(1 + n_ops + ((name || L > 0) ? L / 4 + 1 : 0));
    }
    // block exclusive scan of the thread sums
    unsigned long long inc = mysum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      unsigned long long u = __shfl_up(inc, d);
      if (lane >= d) inc += u;
    }
    if (lane == 63) s_wsum[wave] = inc;
    __syncthreads();
    unsigned long long wpre = 0, tot = 0;
    for (int w = 0; w < kEncThreads / 64; ++w) {
      if (w < wave) wpre += s_wsum[w];
      tot += s_wsum[w];
    }
    if (wave == 0) {
      // look-back over 64 predecessor blocks per round trip
      if (lane == 0) st_state_e(&P.blk[b], kEAgg | tot);
      unsigned long long prefix = 0;
      long long hi = b - 1;
      uint32_t spins = 0;
      while (hi >= 0) {
        long long u = hi - lane;
        unsigned long long st = (u >= 0) ? ld_state_e(&P.blk[u]) : kEIncl;
        unsigned long long f = st & kEMask;
        uint64_t stopm = __ballot(f == kEIncl);
        uint64_t unpub = __ballot(f == 0);
        int sl = stopm ? int(__builtin_ctzll(stopm)) : 64;
        uint64_t need = (sl >= 63) ? ~0ull : ((2ull << sl) - 1ull);
        if (unpub & need) {
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicOr(&P.ctrl[2], 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        unsigned long long c = (lane <= sl) ? (st & kESum) : 0ull;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
        prefix += c;
        if (sl < 64) break;
        hi -= 64;
      }
      if (lane == 0) {
        st_state_e(&P.blk[b], kEIncl | (prefix + tot));
        s_prefix = prefix;
      }
    }
    __syncthreads();
    unsigned long long S = s_prefix + wpre + (inc - mysum);  // words of all records before rb
    // pass 2: checks and scatter
    int64_t m = module_of(P.rec_mod_off, P.M, s_m0, rb < r1 ? rb : r0);
    uint32_t maxid = 0;
    int64_t maxid_m = m;
    for (int k = 0; k < rpt; ++k) {
      int64_t r = rb + k;
      if (r >= r1) break;
      m = module_of(P.rec_mod_off, P.M, m, r);
      if (m != maxid_m) {
        if (maxid) atomicMax(&P.mod_maxid[maxid_m], maxid);
        maxid = 0;
        maxid_m = m;
      }
      if (r == P.rec_mod_off[m]) {
        // first record of module m (and of the empty modules just before it)
        for (int64_t mm = m; mm >= 0 && P.rec_mod_off[mm] == r; --mm) P.mod_words[mm] = int64_t(S);
      }
      uint32_t op = P.op[r];
      int64_t o0 = P.opnd_off[r];
      int64_t n_ops = int64_t(P.opnd_off[r + 1]) - o0;
      int64_t s0 = P.str_off[r];
      int64_t L = int64_t(P.str_off[r + 1]) - s0;
      uint32_t e = tbl[op < 256u ? op : 256u];
      bool known = (e & 0x8000u) != 0;
      bool name = (e >> 8) & 1u;
      uint32_t idm = (e >> 4) & 0xFu;
      int64_t sw = (name || L > 0) ? L / 4 + 1 : 0;
      int64_t wc = 1 + n_ops + sw;
      uint32_t code = 0;
      if (!known) code = SPV_ENC_UNKNOWN_OPCODE;
      else if (n_ops != int64_t(e & 0xFu)) code = SPV_ENC_OPERAND_COUNT;
      else if (!name && L > 0) code = SPV_ENC_BAD_STRING;
      else {
        for (int64_t i = 0; i < L && code == 0; ++i)
          if (P.chars[s0 + i] == 0) code = SPV_ENC_BAD_STRING;
        if (code == 0 && wc > 65535) code = SPV_ENC_TOO_LONG;
      }
      int64_t base = 5 * (m + 1) + int64_t(S);
      bool fits = base + wc <= P.words_cap;
      if (fits) P.words_out[base] = uint32_t((wc & 0xFFFF) << 16) | (op & 0xFFFFu);
      for (int64_t i = 0; i < n_ops; ++i) {
        uint32_t v = P.opnd[o0 + i];
        if (code == 0 && i < 4 && ((idm >> i) & 1u)) {
          if (v == 0xFFFFFFFFu) code = SPV_ENC_BAD_ID;
          else if (v + 1u > maxid) maxid = v + 1u;
        }
        if (fits) P.words_out[base + 1 + i] = v;
      }
      for (int64_t s = 0; s < sw; ++s) {
        uint32_t word = 0;
        for (int bb = 0; bb < 4; ++bb) {
          int64_t ci = 4 * s + bb;
          uint32_t byte = ci < L ? P.chars[s0 + ci] : 0u;
          word |= byte << (8 * bb);
        }
        if (fits) P.words_out[base + 1 + n_ops + s] = word;
      }
      if (code) atomicMin(&P.mod_bad[m], ((unsigned long long)(r - P.rec_mod_off[m]) << 8) | code);
      S += uint64_t(wc);
    }
    if (maxid) atomicMax(&P.mod_maxid[maxid_m], maxid);
    __syncthreads();
  }
}

// Per module: status, header, optimistic offsets; counts failing modules.
__global__ __launch_bounds__(256) void k_enc_fin(EParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  unsigned long long total = 0;
  if (P.n_blocks > 0) total = P.blk[P.n_blocks - 1] & kESum;
  for (int64_t m = gtid; m < P.M; m += nth) {
    int64_t s_m = P.mod_words[m];
    if (s_m < 0) s_m = int64_t(total);  // trailing modules without records
    int64_t s_n;
    if (m + 1 < P.M) {
      s_n = P.mod_words[m + 1];
      if (s_n < 0) s_n = int64_t(total);
    } else {
      s_n = int64_t(total);
    }
    int64_t base = 5 * m + s_m;
    int64_t end = 5 * (m + 1) + s_n;
    unsigned long long bad = P.mod_bad[m];
    uint32_t code = 0;
    int64_t badrec = -1;
    if (bad != ~0ull) {
      code = uint32_t(bad & 0xFFu);
      badrec = int64_t(bad >> 8);
    } else if (end > P.words_cap) {
      code = 6;  // output capacity: the module does not fit in words_cap
    }
    if (P.ctrl[2]) code = kSpinFailCode;
    P.enc_code[m] = code;
    P.enc_bad[m] = badrec;
    P.word_mod_off[m] = base;  // optimistic; rewritten by the compaction if any module failed
    if (m == P.M - 1) P.word_mod_off[P.M] = end;
    if (code == 0) {
      uint32_t* w = P.words_out + base;
      w[0] = kMagicE;
      w[1] = P.version_word;
      w[2] = P.generator_word;
      w[3] = P.mod_maxid[m] ? P.mod_maxid[m] : 1u;
      w[4] = 0;
    } else {
      atomicAdd(&P.ctrl[1], 1u);
    }
  }
}

// Remove the words of failing modules (one block; runs only if one failed).
__global__ __launch_bounds__(256) void k_enc_compact(EParams P) {
  if (P.ctrl[1] == 0) return;
  __shared__ long long s_run;
  __shared__ long long s_scan[256];
  const int tid = threadIdx.x;
  if (tid == 0) s_run = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < P.M; c0 += 256) {
    int64_t m = c0 + tid;
    int64_t old_b = 0, size = 0;
    if (m < P.M) {
      old_b = P.word_mod_off[m];
      int64_t old_e = (m + 1 < P.M) ? P.word_mod_off[m + 1] : P.word_mod_off[P.M];
      size = (P.enc_code[m] == 0) ? old_e - old_b : 0;
    }
    s_scan[tid] = size;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      long long v = (tid >= d) ? s_scan[tid - d] : 0;
      __syncthreads();
      s_scan[tid] += v;
      __syncthreads();
    }
    long long new_b = s_run + s_scan[tid] - size;
    long long chunk_total = s_scan[255];
    __syncthreads();
    // move the modules of this chunk, in order, left (new_b <= old_b)
    for (int k = 0; k < 256; ++k) {
      int64_t mk = c0 + k;
      if (mk >= P.M) break;
      __shared__ long long s_ob, s_nb, s_sz;
      if (tid == k) {
        s_ob = old_b;
        s_nb = new_b;
        s_sz = size;
      }
      __syncthreads();
      long long ob = s_ob, nb = s_nb, sz = s_sz;
      for (long long i = 0; i < sz; i += 256) {
        uint32_t v = (i + tid < sz) ? P.words_out[ob + i + tid] : 0u;
        __syncthreads();
        if (i + tid < sz) P.words_out[nb + i + tid] = v;
        __syncthreads();
      }
      if (tid == k) P.word_mod_off[mk] = new_b;
      __syncthreads();
    }
    if (tid == 0) s_run += chunk_total;
    __syncthreads();
  }
  if (tid == 0) P.word_mod_off[P.M] = s_run;
}

void launch_encode(const EParams& p, int grid, hipStream_t s) {
  int64_t gi = (p.M > p.n_blocks ? p.M : p.n_blocks) / 256 + 1;
  int ginit = int(gi > 4096 ? 4096 : gi);
  hipLaunchKernelGGL(k_enc_init, dim3(ginit), dim3(256), 0, s, p);
  if (p.n_blocks > 0) hipLaunchKernelGGL(k_enc_main, dim3(grid), dim3(kEncThreads), 0, s, p);
  int64_t gf = p.M / 256 + 1;
  hipLaunchKernelGGL(k_enc_fin, dim3(int(gf > 4096 ? 4096 : gf)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_enc_compact, dim3(1), dim3(256), 0, s, p);
}

}  // namespace spv
