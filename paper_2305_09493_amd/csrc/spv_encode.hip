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
// plain exclusive scan.  Three passes with no waiting between blocks: word
// totals per block of records, a scan of those totals (blocks of 256
// totals chained by a decoupled look-back), and the scatter, in which every
// block re-derives its records' word counts and positions.  Records are
// handed to threads in slices of 256 consecutive records, so every load of a
// record field is coalesced.  Module failures (rare) are found in the
// scatter; a module that fails writes no words, so when any module fails a
// compaction kernel closes the gaps.
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
constexpr int kEncOps = 13;
__device__ __constant__ EGEnt kEncGrammar[kEncOps] = {
    {5, 1, 0x1, 1},    // OpName          id, string
    {14, 2, 0x0, 0},   // OpMemoryModel
    {15, 2, 0x2, 1},   // OpEntryPoint    execution model, function, string
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
// bits 4..7 ID mask, bit 8 string operand (OpName, OpEntryPoint)
__device__ __forceinline__ void enc_table(uint16_t* tbl) {
  for (int i = threadIdx.x; i < 257; i += blockDim.x) tbl[i] = 0;
  __syncthreads();
  if (threadIdx.x < kEncOps) {
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
constexpr int kEStateStride = 16;  // one 128-byte line per scan-block state
constexpr unsigned long long kESum = (1ull << 62) - 1;

}  // namespace

__global__ __launch_bounds__(256) void k_enc_init(EParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (gtid == 0) {
    P.ctrl[0] = 0;
    P.ctrl[1] = 0;
    P.ctrl[2] = 0;
    P.ctrl[3] = 0;
  }
  for (int64_t i = gtid; i < P.n_blocks / kEncThreads + 2; i += nth) P.sstate[i * kEStateStride] = 0;
  for (int64_t m = gtid; m < P.M; m += nth) {
    P.mod_bad[m] = ~0ull;
    P.mod_maxid[m] = 0;
    P.mod_words[m] = -1;
  }
  // module of each block's first record: the last m with rec_mod_off[m] <= r0
  // (the non-empty module holding r0); all blocks search at once
  for (int64_t b = gtid; b < P.n_blocks; b += nth) {
    const int64_t r0 = b * P.block_records;
    int64_t lo = 0, hi = P.M - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (P.rec_mod_off[mid] <= r0) lo = mid;
      else hi = mid - 1;
    }
    P.bmod[b] = lo;
  }
}

constexpr int kEncMaxSlices = 16;  // records per thread of a block (block_records / 256)

// Word count of record r (first word + operand words + string words).
__device__ __forceinline__ uint32_t enc_wc(const EParams& P, const uint16_t* tbl, int64_t r) {
  const uint32_t op = P.op[r];
  const int64_t n_ops = int64_t(P.opnd_off[r + 1]) - P.opnd_off[r];
  const int64_t L = int64_t(P.str_off[r + 1]) - P.str_off[r];
  const uint32_t e = tbl[op < 256u ? op : 256u];
  const bool name = (e >> 8) & 1u;
  return uint32_t(1 + n_ops + ((name || L > 0) ? L / 4 + 1 : 0));
}

__device__ __forceinline__ uint32_t enc_wave_incl(uint32_t x) {
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(x, d);
    if (lane >= d) x += u;
  }
  return x;
}

// Pass 1: word total of each block of records.
__global__ __launch_bounds__(kEncThreads) void k_enc_count(EParams P) {
  __shared__ uint16_t tbl[257];
  __shared__ unsigned long long s_w[kEncThreads / 64];
  enc_table(tbl);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rpt = P.block_records / kEncThreads;
  for (long long b = blockIdx.x; b < P.n_blocks; b += gridDim.x) {
    const int64_t r0 = b * P.block_records;
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < kEncMaxSlices; ++k) {
      const int64_t r = r0 + int64_t(k) * kEncThreads + tid;
      if (k < rpt && r < P.N) sum += enc_wc(P, tbl, r);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d);
    if (lane == 0) s_w[wave] = sum;
    __syncthreads();
    if (tid == 0) {
      unsigned long long tot = 0;
      for (int w = 0; w < kEncThreads / 64; ++w) tot += s_w[w];
      P.blk[b] = tot;
    }
    __syncthreads();
  }
}

// Pass 2: exclusive scan of the block totals into blkx (blocks of 256 totals,
// claimed in order, chained by a decoupled look-back); blkx[n_blocks] is the
// grand total.
__global__ __launch_bounds__(kEncThreads) void k_enc_scan(EParams P) {
  __shared__ uint32_t s_bid;
  __shared__ unsigned long long s_w[kEncThreads / 64];
  __shared__ unsigned long long s_pre;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(&P.ctrl[3], 1u);
  __syncthreads();
  const long long sb = s_bid;
  const long long i = sb * kEncThreads + tid;
  const unsigned long long v = (i < P.n_blocks) ? P.blk[i] : 0ull;
  unsigned long long inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  unsigned long long wpre = 0, tot = 0;
  for (int w = 0; w < kEncThreads / 64; ++w) {
    if (w < wave) wpre += s_w[w];
    tot += s_w[w];
  }
  if (tid == 64) st_state_e(&P.sstate[sb * kEStateStride], kEAgg | tot);
  if (wave == 0) {
    unsigned long long prefix = 0;
    long long hi = sb - 1;
    uint32_t spins = 0;
    while (hi >= 0) {
      const long long u = hi - lane;
      const unsigned long long st = (u >= 0) ? ld_state_e(&P.sstate[u * kEStateStride]) : kEIncl;
      const unsigned long long f = st & kEMask;
      const uint64_t stopm = __ballot(f == kEIncl);
      const uint64_t unpub = __ballot(f == 0);
      const int sl = stopm ? int(__builtin_ctzll(stopm)) : 64;
      const uint64_t need = (sl >= 63) ? ~0ull : ((2ull << sl) - 1ull);
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
      st_state_e(&P.sstate[sb * kEStateStride], kEIncl | (prefix + tot));
      s_pre = prefix;
    }
  }
  __syncthreads();
  const unsigned long long ex = s_pre + wpre + (inc - v);
  if (i <= P.n_blocks) P.blkx[i] = ex;  // (blkx[n_blocks]: the grand total)
}

// Pass 3: checks and scatter.  A block takes its records in steps of
// kEncChunk slices of 256 consecutive records: the record fields and the
// operands of all of a thread's records of the step are loaded before any is
// used, one block scan gives their positions, and every thread then writes
// its records' words.  One slice per step measured fastest: more slices cost
// more registers than the extra loads in flight gain.  Staging a step's
// operand, character and output runs in LDS (coalesced copies in and out)
// measured slower still: the scatter is bound by dependent memory round
// trips, and staging adds barriers without removing any.
constexpr int kEncChunk = 1;

// (six waves per SIMD: 80 registers; more resident waves hide more of the
// scatter's memory round trips, eight spill)
__global__ __launch_bounds__(kEncThreads, 6) void k_enc_scatter(EParams P) {
  __shared__ uint16_t tbl[257];
  __shared__ uint32_t s_w[kEncChunk][kEncThreads / 64];
  __shared__ int64_t s_off[kEncThreads + 1];  // rec_mod_off[m0 .. m0 + 256], past M: no start
  enc_table(tbl);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rpt = P.block_records / kEncThreads;
  const uint16_t* __restrict__ opc = P.op;
  const int32_t* __restrict__ ooff = P.opnd_off;
  const uint32_t* __restrict__ opnd = P.opnd;
  const int32_t* __restrict__ soff = P.str_off;
  uint32_t* __restrict__ out = P.words_out;
  for (long long b = blockIdx.x; b < P.n_blocks; b += gridDim.x) {
    const int64_t r0 = b * P.block_records;
    unsigned long long base_s = P.blkx[b];  // words of all records before this block
    const int64_t m0 = P.bmod[b];
    // starts of the modules from m0 on, so that finding a record's module
    // costs LDS reads when all the block's module starts are among them, else
    // the searches read HBM (a block-uniform choice: no access mixes the two)
    __syncthreads();  // the previous block's reads of s_off are done
    s_off[tid] = (m0 + tid <= P.M) ? P.rec_mod_off[m0 + tid] : INT64_MAX;
    if (tid == 0) s_off[kEncThreads] = (m0 + kEncThreads <= P.M) ? P.rec_mod_off[m0 + kEncThreads] : INT64_MAX;
    __syncthreads();
    const int64_t rblast = (r0 + P.block_records < P.N ? r0 + P.block_records : P.N) - 1;
    const bool lds_mods = s_off[kEncThreads] > rblast;
    int64_t ml = 0;  // this thread's current module, relative to m0
    for (int k0 = 0; k0 < rpt; k0 += kEncChunk) {
      int64_t r[kEncChunk], o0[kEncChunk], n_ops[kEncChunk], s0[kEncChunk], L[kEncChunk];
      uint32_t op[kEncChunk], wc[kEncChunk], e[kEncChunk];
      bool real[kEncChunk];
#pragma unroll
      for (int j = 0; j < kEncChunk; ++j) {
        r[j] = r0 + int64_t(k0 + j) * kEncThreads + tid;
        real[j] = (k0 + j < rpt) && r[j] < P.N;
        op[j] = real[j] ? opc[r[j]] : 0u;
        o0[j] = real[j] ? ooff[r[j]] : 0;
        n_ops[j] = real[j] ? int64_t(ooff[r[j] + 1]) - o0[j] : 0;
        s0[j] = real[j] ? soff[r[j]] : 0;
        L[j] = real[j] ? int64_t(soff[r[j] + 1]) - s0[j] : 0;
      }
      // operands of the common counts, loaded before anything is written
      uint32_t v[kEncChunk][4];
#pragma unroll
      for (int j = 0; j < kEncChunk; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[j][i] = (i < n_ops[j] && n_ops[j] <= 4) ? opnd[o0[j] + i] : 0u;
      uint32_t winc[kEncChunk];
#pragma unroll
      for (int j = 0; j < kEncChunk; ++j) {
        e[j] = tbl[op[j] < 256u ? op[j] : 256u];
        const bool name = (e[j] >> 8) & 1u;
        const int64_t sw = (name || L[j] > 0) ? L[j] / 4 + 1 : 0;
        wc[j] = real[j] ? uint32_t(1 + n_ops[j] + sw) : 0u;
        winc[j] = enc_wave_incl(wc[j]);
        if (lane == 63) s_w[j][wave] = winc[j];
      }
      __syncthreads();
      unsigned long long S[kEncChunk];
      {
        unsigned long long run = base_s;
#pragma unroll
        for (int j = 0; j < kEncChunk; ++j) {
          uint32_t wpre = 0, stot = 0;
#pragma unroll
          for (int w = 0; w < kEncThreads / 64; ++w) {
            if (w < wave) wpre += s_w[j][w];
            stot += s_w[j][w];
          }
          S[j] = run + wpre + (winc[j] - wc[j]);
          run += stot;
        }
        base_s = run;
      }
      __syncthreads();
      uint32_t maxid = 0;
      int64_t max_m = -1;
#pragma unroll
      for (int j = 0; j < kEncChunk; ++j) {
        if (!real[j]) continue;
        // module of r (forward from the block's first module)
        bool first;
        if (lds_mods) {
          while (m0 + ml + 1 < P.M && s_off[ml + 1] <= r[j]) ++ml;
          first = r[j] == s_off[ml];
        } else {
          while (m0 + ml + 1 < P.M && P.rec_mod_off[m0 + ml + 1] <= r[j]) ++ml;
          first = r[j] == P.rec_mod_off[m0 + ml];
        }
        const int64_t mr = m0 + ml;
        if (first) {
          for (int64_t mm = mr; mm >= 0 && P.rec_mod_off[mm] == r[j]; --mm) P.mod_words[mm] = int64_t(S[j]);
        }
        if (mr != max_m) {
          if (maxid) atomicMax(&P.mod_maxid[max_m], maxid);
          maxid = 0;
          max_m = mr;
        }
        const bool known = (e[j] & 0x8000u) != 0;
        const bool name = (e[j] >> 8) & 1u;
        const uint32_t idm = (e[j] >> 4) & 0xFu;
        const int64_t sw = (name || L[j] > 0) ? L[j] / 4 + 1 : 0;
        uint32_t code = 0;
        if (!known) code = SPV_ENC_UNKNOWN_OPCODE;
        else if (n_ops[j] != int64_t(e[j] & 0xFu)) code = SPV_ENC_OPERAND_COUNT;
        else if (!name && L[j] > 0) code = SPV_ENC_BAD_STRING;
        bool bad_id = false, nul = false;
        const int64_t base = 5 * (mr + 1) + int64_t(S[j]);
        const bool fits = base + 1 + n_ops[j] + sw <= P.words_cap;
        if (fits) out[base] = uint32_t(((1 + n_ops[j] + sw) & 0xFFFF) << 16) | (op[j] & 0xFFFFu);
        if (n_ops[j] <= 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (i < n_ops[j]) {
              if ((idm >> i) & 1u) {
                if (v[j][i] == 0xFFFFFFFFu) bad_id = true;
                else if (v[j][i] + 1u > maxid) maxid = v[j][i] + 1u;
              }
              if (fits) out[base + 1 + i] = v[j][i];
            }
          }
        } else {
          for (int64_t i = 0; i < n_ops[j]; ++i) {
            const uint32_t x = opnd[o0[j] + i];
            if (i < 4 && ((idm >> i) & 1u)) {
              if (x == 0xFFFFFFFFu) bad_id = true;
              else if (x + 1u > maxid) maxid = x + 1u;
            }
            if (fits) out[base + 1 + i] = x;
          }
        }
        // string words: little-endian packing of the characters, NUL padded;
        // a NUL among the characters is a bad string.  The characters are read
        // as aligned 32-bit words (an aligned word never crosses a page, so
        // the bytes around the string that share its first and last words are
        // safe to read), eight output words at a time, all loads issued before
        // use, and realigned with a byte funnel shift.
        if (sw > 0) {
          const uint32_t sh = uint32_t(reinterpret_cast<uintptr_t>(P.chars + s0[j]) & 3u);
          const uint32_t* cw = reinterpret_cast<const uint32_t*>(P.chars + s0[j] - sh);
          for (int64_t s8 = 0; s8 < sw; s8 += 8) {
            const int64_t need = (L[j] - 4 * s8 + int64_t(sh) + 3) / 4;  // aligned words holding characters
            uint32_t a[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) a[q] = (q < need) ? cw[s8 + q] : 0u;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              if (s8 + q < sw) {
                uint32_t word = __builtin_amdgcn_alignbyte(a[q + 1], a[q], sh);
                const int64_t rem = L[j] - 4 * (s8 + q);  // characters left in this word
                const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : ((1u << (8 * rem)) - 1u));
                word &= keep;
                const uint32_t probe = word | ~keep;  // positions past the string never read as NUL
                nul |= ((probe - 0x01010101u) & ~probe & 0x80808080u) != 0;
                if (fits) out[base + 1 + n_ops[j] + s8 + q] = word;
              }
            }
          }
        }
        // checks in the order of the record contract: grammar, string, length, IDs
        if (code == 0 && nul) code = SPV_ENC_BAD_STRING;
        if (code == 0 && 1 + n_ops[j] + sw > 65535) code = SPV_ENC_TOO_LONG;
        if (code == 0 && bad_id) code = SPV_ENC_BAD_ID;
        if (code) atomicMin(&P.mod_bad[mr], ((unsigned long long)(r[j] - P.rec_mod_off[mr]) << 8) | code);
      }
      // bound: max ID + 1 per module (one atomic per wave when the wave's
      // records of this step are in one module)
      const int64_t mlead = __shfl(max_m, 0);
      if (__ballot(max_m != mlead) == 0 && mlead >= 0) {
        uint32_t mx = maxid;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
          const uint32_t o = __shfl_xor(mx, d);
          mx = o > mx ? o : mx;
        }
        if (lane == 0 && mx) atomicMax(&P.mod_maxid[mlead], mx);
      } else if (maxid) {
        atomicMax(&P.mod_maxid[max_m], maxid);
      }
    }
  }
}

// Per module: status, header, optimistic offsets; counts failing modules.
__global__ __launch_bounds__(256) void k_enc_fin(EParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  unsigned long long total = 0;
  if (P.n_blocks > 0) total = P.blkx[P.n_blocks];
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
      code = SPV_ENC_CAPACITY;  // the module does not fit in words_cap
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

int encode_occupancy(int pass) {
  int n = 0;
  const void* k = pass == 0 ? reinterpret_cast<const void*>(k_enc_count) : reinterpret_cast<const void*>(k_enc_scatter);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kEncThreads, 0) != hipSuccess) return 0;
  return n;
}

void launch_encode(const EParams& p, int grid_count, int grid_scatter, hipStream_t s) {
  int64_t gi = (p.M > p.n_blocks ? p.M : p.n_blocks) / 256 + 1;
  int ginit = int(gi > 4096 ? 4096 : gi);
  hipLaunchKernelGGL(k_enc_init, dim3(ginit), dim3(256), 0, s, p);
  if (p.n_blocks > 0) {
    hipLaunchKernelGGL(k_enc_count, dim3(grid_count), dim3(kEncThreads), 0, s, p);
    hipLaunchKernelGGL(k_enc_scan, dim3(int(p.n_blocks / kEncThreads + 1)), dim3(kEncThreads), 0, s, p);
    hipLaunchKernelGGL(k_enc_scatter, dim3(grid_scatter), dim3(kEncThreads), 0, s, p);
  }
  int64_t gf = p.M / 256 + 1;
  hipLaunchKernelGGL(k_enc_fin, dim3(int(gf > 4096 ? 4096 : gf)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_enc_compact, dim3(1), dim3(256), 0, s, p);
}

}  // namespace spv
