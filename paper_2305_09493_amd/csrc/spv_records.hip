// Decode's records mode for gfx950: the instructions that decode found,
// turned back into the encoder's record layout (opcode, non-string operand
// words, string bytes), so that encoding the records of a valid module gives
// its words again.
//
// What is computed (Beehive SPIR-V Toolkit paper, arXiv 2305.09493): the
// disassembler's instruction view of a binary (section "Dis/Assembler") in the
// form the library's writer takes (section "SPIR-V Library"; operand words
// and strings as in section "Parsing Operand Kinds").  Module m contributes
// the records of its valid instruction prefix: results[m].n_inst records,
// or none when its header check failed.
//
// How: one scan over the modules gives each module's first record; a count
// pass gives every record's operand and character counts (a string
// was validated by decode, so its length follows from its last word alone)
// and the totals of blocks of 1024 records; a scan of those totals and an
// in-block scan in the scatter give both offset arrays while it writes the
// records.  The scans over many values are single-pass: blocks of 1024
// values, claimed in order, chained by a decoupled look-back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_internal.h"
#include "spv_scan.h"

namespace spv {

namespace {

// Module of global record r: the last m with rec_mod_off[m] <= r among the
// modules with records (binary search; rec_mod_off is non-decreasing).
__device__ __forceinline__ int64_t rec_module(const int64_t* rec_mod_off, int64_t M, int64_t r) {
  int64_t lo = 0, hi = M - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rec_mod_off[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A record's instruction: its first word's position and the word.
struct RecInst {
  int64_t pos;
  uint32_t w0;
};

__device__ __forceinline__ RecInst rec_inst(const RParams& P, int64_t r) {
  const int64_t m = rec_module(P.rec_mod_off, P.M, r);
  const int64_t j = r - P.rec_mod_off[m];
  const int64_t base = P.mod_off[m];
  RecInst ri;
  ri.pos = base + int64_t(P.idx_off[base + j]);
  ri.w0 = P.words[ri.pos];
  return ri;
}

// Operand words before the string of a string-bearing instruction (OpName:
// its target; OpEntryPoint: execution model and entry function), 0 for the
// others.
__device__ __forceinline__ uint32_t rec_str_operands(uint32_t op) {
  return op == uint32_t(kOpName) ? 1u : (op == uint32_t(kOpEntryPoint) ? 2u : 0u);
}

// Operand words and string bytes of a record.  A string-bearing instruction
// has its fixed operands and then the string, whose first NUL lies in its
// last word (decode checked that), so its length is 4 * (string words - 1)
// plus the bytes of the last word before the NUL.
__device__ __forceinline__ void rec_counts(const RParams& P, const RecInst& ri, uint32_t& n_opnd, uint32_t& n_chars) {
  const uint32_t wc = ri.w0 >> 16, op = ri.w0 & 0xFFFFu;
  const uint32_t k0 = rec_str_operands(op);
  if (k0) {
    const uint32_t last = P.words[ri.pos + wc - 1];
    uint32_t k = 0;
    while (k < 4 && ((last >> (8 * k)) & 0xFFu) != 0) ++k;
    n_opnd = k0;
    n_chars = 4 * (wc - 2 - k0) + k;
  } else {
    n_opnd = wc - 1;
    n_chars = 0;
  }
}

}  // namespace

// Clears the scan states and claim counters; per module, its record count.
__global__ __launch_bounds__(kRecThreads) void k_rec_init(RParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (gtid < 4) P.ctrl[gtid] = 0;
  const int64_t ns = (P.M + 1) / kScanBlock + 2, nr = (P.cap_records / kScanBlock + 1) / kScanBlock + 2;
  for (int64_t i = gtid; i < ns; i += nth) P.mstate[i * kRStateStride] = 0;
  for (int64_t i = gtid; i < nr; i += nth) P.rstate[i * kRStateStride] = 0;
  for (int64_t m = gtid; m < P.M; m += nth) {
    const spv_result r = P.results[m];
    const bool hdr_ok = r.code == SPV_OK || (r.code >= SPV_E_BAD_WORD_COUNT && r.code <= SPV_E_MODULE_RULES);
    P.mscan[m] = hdr_ok ? (unsigned long long)r.n_inst : 0ull;
  }
}

// rec_mod_off = exclusive scan of the module record counts.
__global__ __launch_bounds__(kRecThreads) void k_rec_modscan(RParams P) {
  scan_block(P.mscan, P.M, P.mscan, P.mstate, &P.ctrl[0], &P.ctrl[2]);
}

// Packed counts of every record (operand words << 32 | string bytes) and
// the total of every block of kScanBlock records.
__global__ __launch_bounds__(kRecThreads) void k_rec_count(RParams P) {
  __shared__ unsigned long long s_w[kRecThreads / 64];
  if (P.ctrl[2]) return;  // the module scan gave up: rec_mod_off is not valid
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t N = min(P.rec_mod_off[P.M], P.cap_records);
  const int64_t nb = N / kScanBlock + 1;  // (the last block may be empty)
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      if (r < N) {
        const RecInst ri = rec_inst(P, r);
        uint32_t no, nc;
        rec_counts(P, ri, no, nc);
        const unsigned long long x = ((unsigned long long)no << 32) | nc;
        P.rscan[r] = x;
        sum += x;
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d);
    if (lane == 0) s_w[wave] = sum;
    __syncthreads();
    if (tid == 0) {
      unsigned long long t = 0;
#pragma unroll
      for (int w = 0; w < kRecThreads / 64; ++w) t += s_w[w];
      P.btot[b] = t;
    }
    __syncthreads();
  }
}

// rec_mod_off (int64) from the module scan.
__global__ __launch_bounds__(kRecThreads) void k_rec_offsets(RParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t m = gtid; m <= P.M; m += nth) P.rec_mod_off[m] = int64_t(P.mscan[m]);
}

// Exclusive scan of the record blocks' packed totals (both halves at once:
// neither half's total reaches 2^32).
__global__ __launch_bounds__(kRecThreads) void k_rec_scan(RParams P) {
  if (P.ctrl[2]) return;
  const int64_t N = min(P.rec_mod_off[P.M], P.cap_records);
  const int64_t nb = N / kScanBlock + 1;
  if (int64_t(blockIdx.x) * kScanBlock > nb) return;  // (the grid is sized for the largest N)
  scan_block(P.btot, nb, P.btot, P.rstate, &P.ctrl[1], &P.ctrl[2]);
}

// Records: opcode, offsets, operand words, string bytes.  A block takes a
// block of kScanBlock records in slices of 256: the slice's packed counts,
// scanned in the block, plus the block's prefix give each record's offsets.
// (Recomputing the counts here instead of storing them measured slower: it
// puts the dependent loads of every record before the block scan.)
__global__ __launch_bounds__(kRecThreads) void k_rec_scatter(RParams P) {
  __shared__ unsigned long long s_w[kRecThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (P.ctrl[2]) {  // a scan gave up waiting: no valid output
    const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + tid;
    const int64_t nth = int64_t(gridDim.x) * blockDim.x;
    for (int64_t m = gtid; m <= P.M; m += nth) P.rec_mod_off[m] = -1;
    return;
  }
  const int64_t N = min(P.rec_mod_off[P.M], P.cap_records);
  const int64_t nb = N / kScanBlock + 1;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    unsigned long long base = P.btot[b];
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      const unsigned long long x = (r < N) ? P.rscan[r] : 0ull;
      unsigned long long inc = x;
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
      __syncthreads();  // s_w is free for the next slice
      const unsigned long long ex = base + wpre + (inc - x);
      base += tot;
      if (r > N) continue;
      const int32_t oo = int32_t(ex >> 32), so = int32_t(ex & 0xFFFFFFFFull);
      P.opnd_off[r] = oo;  // (r == N: the totals)
      P.str_off[r] = so;
      if (r == N) continue;
      const RecInst ri = rec_inst(P, r);
      const uint32_t wc = ri.w0 >> 16, op = ri.w0 & 0xFFFFu;
      P.op[r] = uint16_t(op);
      const uint32_t k0 = rec_str_operands(op);
      if (k0) {
        for (uint32_t i = 0; i < k0; ++i) P.opnd[oo + i] = P.words[ri.pos + 1 + i];
        const uint32_t nc = uint32_t(x & 0xFFFFFFFFull);
        for (uint32_t c = 0; c < nc; c += 4) {
          const uint32_t w = P.words[ri.pos + 1 + k0 + c / 4];
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q)
            if (c + q < nc) P.chars[so + c + q] = uint8_t(w >> (8 * q));
        }
      } else {
        for (uint32_t i = 1; i < wc; ++i) P.opnd[oo + i - 1] = P.words[ri.pos + i];
      }
    }
  }
}

int records_grid(int64_t n) {
  const int64_t g = n / kRecThreads + 1;
  return int(g > 4096 ? 4096 : g);
}

void launch_records(const RParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_init, dim3(records_grid(p.M > p.cap_records / kScanBlock ? p.M : p.cap_records / kScanBlock)),
                     dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_rec_modscan, dim3(int(p.M / kScanBlock + 1)), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_rec_offsets, dim3(records_grid(p.M + 1)), dim3(kRecThreads), 0, s, p);
  const int64_t nb = p.cap_records / kScanBlock + 1;  // record blocks, at most
  const int gb = int(nb > 4096 ? 4096 : nb);
  hipLaunchKernelGGL(k_rec_count, dim3(gb), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_rec_scan, dim3(int(nb / kScanBlock + 1)), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_rec_scatter, dim3(gb), dim3(kRecThreads), 0, s, p);
}

}  // namespace spv
