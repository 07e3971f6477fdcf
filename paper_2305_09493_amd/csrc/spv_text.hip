// Decode's text mode for gfx950: the instructions that decode found, printed
// as SPIR-V assembly text.
//
// What is computed (Beehive SPIR-V Toolkit paper, arXiv 2305.09493, section
// "Dis/Assembler"): the disassembler maps every opcode and operand of a binary
// back to text, under five switches (syntax highlight, inline names,
// indentation off, grouping, header off; option bits 1, 2, 4, 8, 16 in that
// order).  The text format:
//   - a module whose header check failed gives no text; otherwise its text
//     covers its valid instruction prefix (results[m].n_inst instructions);
//   - unless bit 16, five comment lines: "; SPIR-V", "; Version: M.m",
//     "; Generator: g", "; Bound: b", "; Schema: s" (decimal);
//   - per instruction one line: [padding][%r = ]OpName[ operand]...\n; the
//     result ID moves left of " = ", the other operands keep their order;
//     unless bit 4 the line is padded with spaces so that the opcode name
//     starts at column 15 (no padding when "%r = " is 15 wide or wider);
//   - an ID prints as %<decimal>, or with bit 2 as %<name> when the module's
//     first OpName of that ID carries a usable name (non-empty, only
//     [A-Za-z0-9_], not starting with a digit); names are not made unique;
//   - literals print in decimal or as the enumerant of the SPIR-V
//     specification (capability, addressing model, memory model, execution
//     model; function control as None or its bits joined by '|');
//   - strings print between double quotes, '"' and '\' escaped by '\';
//   - bit 8 adds an empty line before each OpFunction and OpLabel;
//   - bit 1 wraps every opcode name, ID, literal and string in an ANSI colour
//     (ESC[36m, 33m, 34m, 32m) and a reset ESC[0m; padding ignores the codes.
//
// How: a scan over the modules gives each module's first instruction and
// header bytes; with inline names, the OpName instructions are gathered into
// a list and inserted into an open-addressing hash keyed by (module, ID),
// where atomicMin keeps each ID's first OpName; a length pass sizes every
// line (the same line writer run into a counting sink) and totals blocks of
// 1024 lines; a scan of those totals and an in-block scan in the scatter place
// every line.  The scatter writes a slice of 256 lines into LDS at the byte
// alignment they have in the text and stores the slice with aligned 32-bit
// stores (byte stores only at its two ends); a slice too wide for LDS writes
// its lines straight to memory.  Module headers and text_mod_off come last,
// so the header bytes overwrite whatever a slice's store left between lines.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spv_internal.h"
#include "spv_scan.h"

namespace spv {

namespace {

constexpr uint64_t kInstMask = (1ull << 29) - 1;  // low bits of the module scan: instructions
constexpr int kHdrShift = 29;                      // high bits: header bytes
constexpr int kStageBytes = 40960;                 // LDS staging per slice of 256 lines

// One opcode of the grammar: its name, the operand words before its string
// (all operand words for an instruction without one), whether a string
// follows, operand roles (2 bits per slot: 0 literal, 1 ID use, 2 result ID)
// and literal kinds (3 bits per slot: 0 decimal, 1 capability, 2 addressing
// model, 3 memory model, 4 execution model, 5 function control).
struct TxtOp {
  const char* name;
  uint32_t nfix, str, roles, lits;
};

__device__ __forceinline__ TxtOp txt_op(uint32_t op) {
  switch (op) {
    case 5: return {"OpName", 1, 1, 1u, 0u};
    case 14: return {"OpMemoryModel", 2, 0, 0u, 2u | (3u << 3)};
    case 15: return {"OpEntryPoint", 2, 1, 1u << 2, 4u};
    case 17: return {"OpCapability", 1, 0, 0u, 1u};
    case 21: return {"OpTypeInt", 3, 0, 2u, 0u};
    case 43: return {"OpConstant", 3, 0, 1u | (2u << 2), 0u};
    case 54: return {"OpFunction", 4, 0, 1u | (2u << 2) | (1u << 6), 5u << 6};
    case 56: return {"OpFunctionEnd", 0, 0, 0u, 0u};
    case 61: return {"OpLoad", 3, 0, 1u | (2u << 2) | (1u << 4), 0u};
    case 62: return {"OpStore", 2, 0, 1u | (1u << 2), 0u};
    case 128: return {"OpIAdd", 4, 0, 1u | (2u << 2) | (1u << 4) | (1u << 6), 0u};
    case 248: return {"OpLabel", 1, 0, 2u, 0u};
    default: return {"OpReturn", 0, 0, 0u, 0u};  // 253: decode admits no other opcode
  }
}

// Enumerant names of the SPIR-V specification; nullptr where the table has
// no entry (the value prints in decimal).
__device__ __forceinline__ const char* txt_enum(uint32_t kind, uint32_t v) {
  if (kind == 1) {
    switch (v) {
      case 0: return "Matrix";
      case 1: return "Shader";
      case 2: return "Geometry";
      case 3: return "Tessellation";
      case 4: return "Addresses";
      case 5: return "Linkage";
      case 6: return "Kernel";
      case 7: return "Vector16";
      case 8: return "Float16Buffer";
      case 9: return "Float16";
      case 10: return "Float64";
      case 11: return "Int64";
      case 12: return "Int64Atomics";
      case 22: return "Int16";
      case 39: return "Int8";
      default: return nullptr;
    }
  }
  if (kind == 2) {
    switch (v) {
      case 0: return "Logical";
      case 1: return "Physical32";
      case 2: return "Physical64";
      default: return nullptr;
    }
  }
  if (kind == 3) {
    switch (v) {
      case 0: return "Simple";
      case 1: return "GLSL450";
      case 2: return "OpenCL";
      case 3: return "Vulkan";
      default: return nullptr;
    }
  }
  if (kind == 4) {
    switch (v) {
      case 0: return "Vertex";
      case 1: return "TessellationControl";
      case 2: return "TessellationEvaluation";
      case 3: return "Geometry";
      case 4: return "Fragment";
      case 5: return "GLCompute";
      case 6: return "Kernel";
      default: return nullptr;
    }
  }
  return nullptr;
}

// Output sinks of the line writer: a counter (lengths only), LDS staging, and
// global memory clipped at the caller's capacity.  o is the position of the
// next byte; put_at writes at a position already counted.
struct CountSink {
  static constexpr bool kWrite = false;
  uint32_t o;
  __device__ __forceinline__ void put(uint32_t) { ++o; }
  __device__ __forceinline__ void put_at(uint32_t, uint32_t) {}
};
struct LdsSink {
  static constexpr bool kWrite = true;
  uint8_t* p;
  uint32_t o;
  __device__ __forceinline__ void put(uint32_t c) { p[o++] = uint8_t(c); }
  __device__ __forceinline__ void put_at(uint32_t k, uint32_t c) { p[k] = uint8_t(c); }
};
struct GlobalSink {
  static constexpr bool kWrite = true;
  uint8_t* p;
  int64_t g, cap;
  uint32_t o;
  __device__ __forceinline__ void put(uint32_t c) {
    if (g + o < cap) p[g + o] = uint8_t(c);
    ++o;
  }
  __device__ __forceinline__ void put_at(uint32_t k, uint32_t c) {
    if (g + k < cap) p[g + k] = uint8_t(c);
  }
};

__device__ __forceinline__ uint32_t ndigits(uint32_t v) {
  uint32_t d = 1;
  while (v >= 10u) {
    v /= 10u;
    ++d;
  }
  return d;
}

template <class S>
__device__ __forceinline__ void put_dec(S& s, uint32_t v) {
  const uint32_t d = ndigits(v);
  if constexpr (S::kWrite) {
    uint32_t k = s.o + d;
    do {
      s.put_at(--k, '0' + v % 10u);
      v /= 10u;
    } while (v);
  }
  s.o += d;
}

template <class S>
__device__ __forceinline__ void put_cstr(S& s, const char* c) {
  for (; *c; ++c) s.put(uint8_t(*c));
}

template <class S>
__device__ __forceinline__ void color_on(S& s, uint32_t digit) {
  s.put(0x1b);
  s.put('[');
  s.put('3');
  s.put(digit);
  s.put('m');
}

template <class S>
__device__ __forceinline__ void color_off(S& s) {
  s.put(0x1b);
  s.put('[');
  s.put('0');
  s.put('m');
}

// The name an ID prints with: its first OpName's word position and the
// name's length (0: print the number).
struct IdName {
  uint32_t pos, len;
};

// MurmurHash3's 64-bit finaliser (fmix64), a published bit mixer.
__device__ __forceinline__ unsigned long long txt_mix(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Slots in use: the smallest power of two >= 2 * the OpName count (>= 64).
__device__ __forceinline__ unsigned long long txt_slots(const TParams& P) {
  const unsigned long long c = P.ctrl[3];
  unsigned long long s = 64;
  while (s < 2 * c) s <<= 1;
  return s < (unsigned long long)P.slot_cap ? s : (unsigned long long)P.slot_cap;
}

__device__ __forceinline__ IdName txt_name(const TParams& P, unsigned long long nslots, uint32_t m, uint32_t v) {
  const unsigned long long key = ((unsigned long long)m << 32) | v;
  unsigned long long h = txt_mix(key) & (nslots - 1);
  while (true) {  // the table is at most half full, so an empty slot ends every probe
    const unsigned long long k = P.slots[h].key;
    if (k == key) return IdName{P.slots[h].pos, P.slots[h].len};
    if (k == kTxtEmpty) return IdName{0u, 0u};
    h = (h + 1) & (nslots - 1);
  }
}

template <class S>
__device__ __forceinline__ void put_id(S& s, const TParams& P, bool hl, IdName nm, uint32_t v) {
  if (hl) color_on(s, '3');
  s.put('%');
  if (nm.len) {
    if constexpr (S::kWrite) {
      const uint32_t* w = P.words + nm.pos + 2;  // OpName: first word, target, then the name
      for (uint32_t i = 0; i < nm.len; ++i) s.put((w[i >> 2] >> (8 * (i & 3))) & 0xFFu);
    } else {
      s.o += nm.len;
    }
  } else {
    put_dec(s, v);
  }
  if (hl) color_off(s);
}

template <class S>
__device__ __forceinline__ void put_lit(S& s, bool hl, uint32_t kind, uint32_t v) {
  if (hl) color_on(s, '4');
  if (kind == 5) {  // function control: a bit mask
    if (v == 0) {
      put_cstr(s, "None");
    } else if (v & ~0xFu) {
      put_dec(s, v);
    } else {
      bool first = true;
      for (uint32_t b = 0; b < 4; ++b) {
        if (!(v & (1u << b))) continue;
        if (!first) s.put('|');
        put_cstr(s, b == 0 ? "Inline" : b == 1 ? "DontInline" : b == 2 ? "Pure" : "Const");
        first = false;
      }
    }
  } else {
    const char* e = txt_enum(kind, v);
    if (e) put_cstr(s, e);
    else put_dec(s, v);
  }
  if (hl) color_off(s);
}

// A string literal (decode checked that it ends in a NUL within its last
// word), quoted, with '"' and '\' escaped.
template <class S>
__device__ __forceinline__ void put_string(S& s, const uint32_t* w) {
  for (uint32_t i = 0;; ++i) {
    const uint32_t x = w[i];
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t c = (x >> (8 * q)) & 0xFFu;
      if (c == 0) return;
      if (c == '"' || c == '\\') s.put('\\');
      s.put(c);
    }
  }
}

// The text line of the instruction at word position pos of module m.
template <class S>
__device__ void txt_line(const TParams& P, unsigned long long nslots, uint32_t m, int64_t pos, S& s) {
  const uint32_t w0 = P.words[pos], op = w0 & 0xFFFFu;
  const TxtOp d = txt_op(op);
  const uint32_t opt = P.options;
  const bool hl = (opt & kTxtHighlight) != 0, names = (opt & kTxtInlineNames) != 0;
  uint32_t v[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) v[k] = k < d.nfix ? P.words[pos + 1 + k] : 0u;
  bool has_res = false;
  uint32_t rv = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k)
    if (((d.roles >> (2 * k)) & 3u) == 2u) {
      has_res = true;
      rv = v[k];
    }
  if ((opt & kTxtGroup) && (op == 54u || op == 248u)) s.put('\n');
  IdName rn{0u, 0u};
  if (has_res && names) rn = txt_name(P, nslots, m, rv);
  if (!(opt & kTxtNoIndent)) {
    const uint32_t width = has_res ? 4u + (rn.len ? rn.len : ndigits(rv)) : 0u;  // "%" token " = "
    for (uint32_t c = width; c < 15u; ++c) s.put(' ');
  }
  if (has_res) {
    put_id(s, P, hl, rn, rv);
    s.put(' ');
    s.put('=');
    s.put(' ');
  }
  if (hl) color_on(s, '6');
  put_cstr(s, d.name);
  if (hl) color_off(s);
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    if (k >= d.nfix) break;
    const uint32_t role = (d.roles >> (2 * k)) & 3u;
    if (role == 2u) continue;
    s.put(' ');
    if (role == 1u) {
      const IdName nm = names ? txt_name(P, nslots, m, v[k]) : IdName{0u, 0u};
      put_id(s, P, hl, nm, v[k]);
    } else {
      put_lit(s, hl, (d.lits >> (3 * k)) & 7u, v[k]);
    }
  }
  if (d.str) {
    s.put(' ');
    if (hl) color_on(s, '2');
    s.put('"');
    put_string(s, P.words + pos + 1 + d.nfix);
    s.put('"');
    if (hl) color_off(s);
  }
  s.put('\n');
}

// The five header comment lines of module m.
template <class S>
__device__ void txt_header(const TParams& P, int64_t m, S& s) {
  const uint32_t* w = P.words + P.mod_off[m];
  put_cstr(s, "; SPIR-V\n; Version: ");
  put_dec(s, (w[1] >> 16) & 0xFFu);
  s.put('.');
  put_dec(s, (w[1] >> 8) & 0xFFu);
  put_cstr(s, "\n; Generator: ");
  put_dec(s, w[2]);
  put_cstr(s, "\n; Bound: ");
  put_dec(s, w[3]);
  put_cstr(s, "\n; Schema: ");
  put_dec(s, w[4]);
  s.put('\n');
}

// Module of instruction r: the last m in [lo, hi] whose first instruction is
// at or before r (requires that of lo to be).
__device__ __forceinline__ int64_t txt_module(const unsigned long long* mscan, int64_t lo, int64_t hi, int64_t r) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (int64_t(mscan[mid] & kInstMask) <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t txt_count(const TParams& P) {
  const int64_t n = int64_t(P.mscan[P.M] & kInstMask);
  return n < P.cap_inst ? n : P.cap_inst;
}

// Modules owning the first and last instruction of block b (in LDS).
__device__ __forceinline__ void txt_bracket(const TParams& P, int64_t b, int64_t N, int64_t* s_mb) {
  if (threadIdx.x == 0) {
    const int64_t r0 = b * kScanBlock;
    const int64_t r1 = (r0 + kScanBlock < N ? r0 + kScanBlock : N) - 1;
    s_mb[0] = txt_module(P.mscan, 0, P.M - 1, r0);
    s_mb[1] = txt_module(P.mscan, s_mb[0], P.M - 1, r1);
  }
  __syncthreads();
}

// Word position of instruction r of module m (decode's gapped index).
__device__ __forceinline__ int64_t txt_pos(const TParams& P, int64_t m, int64_t r) {
  const int64_t base = P.mod_off[m];
  const int64_t j = r - int64_t(P.mscan[m] & kInstMask);
  return base + int64_t(P.idx_off[base + j]);
}

}  // namespace

// Clears the scan states and counters; per module, its header bytes and
// instruction count (none when its header check failed).
__global__ __launch_bounds__(kRecThreads) void k_txt_init(TParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (gtid < 4) P.ctrl[gtid] = 0;
  const int64_t ns = (P.M + 1) / kScanBlock + 2, nbs = (P.cap_inst / kScanBlock + 1) / kScanBlock + 2;
  for (int64_t i = gtid; i < ns; i += nth) P.mstate[i * kRStateStride] = 0;
  for (int64_t i = gtid; i < nbs; i += nth) P.bstate[i * kRStateStride] = 0;
  for (int64_t m = gtid; m < P.M; m += nth) {
    const spv_result r = P.results[m];
    const bool hdr_ok = r.code == SPV_OK || (r.code >= SPV_E_BAD_WORD_COUNT && r.code <= SPV_E_MODULE_RULES);
    unsigned long long hb = 0;
    if (hdr_ok && !(P.options & kTxtNoHeader)) {
      CountSink c{0};
      txt_header(P, m, c);
      hb = c.o;
    }
    P.mscan[m] = hdr_ok ? (hb << kHdrShift) | (unsigned long long)r.n_inst : 0ull;
  }
}

__global__ __launch_bounds__(kRecThreads) void k_txt_modscan(TParams P) {
  scan_block(P.mscan, P.M, P.mscan, P.mstate, &P.ctrl[0], &P.ctrl[2]);
}

// Inline names, step 1: the list of OpName instructions.
__global__ __launch_bounds__(kRecThreads) void k_txt_collect(TParams P) {
  __shared__ int64_t s_mb[2];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    txt_bracket(P, b, N, s_mb);
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      int64_t m = 0, pos = 0;
      bool is_name = false;
      if (r < N) {
        m = txt_module(P.mscan, s_mb[0], s_mb[1], r);
        pos = txt_pos(P, m, r);
        is_name = (P.words[pos] & 0xFFFFu) == uint32_t(kOpName);
      }
      const uint64_t bal = __ballot(is_name);
      if (bal) {
        const int leader = __builtin_ctzll(bal);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&P.ctrl[3], uint32_t(__builtin_popcountll(bal)));
        base = __shfl(base, leader);
        if (is_name) {
          const uint32_t rank = uint32_t(__builtin_popcountll(bal & ((1ull << lane) - 1ull)));
          P.nlist[base + rank] = make_uint2(uint32_t(m), uint32_t(pos));
        }
      }
    }
    __syncthreads();  // s_mb is rewritten for the next block
  }
}

// Inline names, step 2: empty the slots in use.
__global__ __launch_bounds__(kRecThreads) void k_txt_hclear(TParams P) {
  if (P.ctrl[2]) return;
  const unsigned long long ns = txt_slots(P);
  const unsigned long long gtid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long nth = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = gtid; i < ns; i += nth) {
    P.slots[i].key = kTxtEmpty;
    P.slots[i].pos = 0xFFFFFFFFu;
    P.slots[i].len = 0u;
  }
}

// Inline names, step 3: insert every OpName by (module, target); the slot
// keeps the smallest word position, i.e. the module's first OpName.
__global__ __launch_bounds__(kRecThreads) void k_txt_insert(TParams P) {
  if (P.ctrl[2]) return;
  const unsigned long long ns = txt_slots(P);
  const uint32_t n = P.ctrl[3];
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (uint32_t i = gtid; i < n; i += nth) {
    const uint2 e = P.nlist[i];
    const unsigned long long key = ((unsigned long long)e.x << 32) | P.words[e.y + 1];
    unsigned long long h = txt_mix(key) & (ns - 1);
    while (true) {
      const unsigned long long prev = atomicCAS(&P.slots[h].key, kTxtEmpty, key);
      if (prev == kTxtEmpty || prev == key) {
        atomicMin(&P.slots[h].pos, e.y);
        break;
      }
      h = (h + 1) & (ns - 1);
    }
  }
}

// Inline names, step 4: the length of each kept name, 0 when it is not usable.
__global__ __launch_bounds__(kRecThreads) void k_txt_nlen(TParams P) {
  if (P.ctrl[2]) return;
  const unsigned long long ns = txt_slots(P);
  const unsigned long long gtid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long nth = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = gtid; i < ns; i += nth) {
    if (P.slots[i].key == kTxtEmpty) continue;
    const uint32_t* w = P.words + P.slots[i].pos + 2;
    uint32_t len = 0;
    bool ok = true;
    for (uint32_t k = 0;; ++k) {
      const uint32_t x = w[k >> 2];
      const uint32_t c = (x >> (8 * (k & 3))) & 0xFFu;
      if (c == 0) break;
      const bool alpha = (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || c == '_';
      const bool digit = c >= '0' && c <= '9';
      if (!(alpha || (digit && k > 0))) ok = false;
      ++len;
    }
    P.slots[i].len = (ok && len > 0) ? len : 0u;
  }
}

// Line lengths, and the total of every block of 1024 lines.
__global__ __launch_bounds__(kRecThreads) void k_txt_lens(TParams P) {
  __shared__ int64_t s_mb[2];
  __shared__ unsigned long long s_w[kRecThreads / 64];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  const unsigned long long ns = (P.options & kTxtInlineNames) ? txt_slots(P) : 1;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    txt_bracket(P, b, N, s_mb);
    unsigned long long sum = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      if (r < N) {
        const int64_t m = txt_module(P.mscan, s_mb[0], s_mb[1], r);
        CountSink c{0};
        txt_line(P, ns, uint32_t(m), txt_pos(P, m, r), c);
        P.lens[r] = c.o;
        sum += c.o;
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

// Exclusive scan of the block totals (btot[nb] receives the grand total).
__global__ __launch_bounds__(kRecThreads) void k_txt_bscan(TParams P) {
  if (P.ctrl[2]) return;
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  if (int64_t(blockIdx.x) * kScanBlock > nb) return;  // (the grid is sized for the largest count)
  scan_block(P.btot, nb, P.btot, P.bstate, &P.ctrl[1], &P.ctrl[2]);
}

// The lines.  lens[r] becomes line r's offset within its block of 1024.
__global__ __launch_bounds__(kRecThreads) void k_txt_scatter(TParams P) {
  __shared__ uint32_t s_stage[kStageBytes / 4];
  __shared__ int64_t s_mb[2];
  __shared__ unsigned long long s_w[kRecThreads / 64];
  __shared__ long long s_g[2];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  const unsigned long long ns = (P.options & kTxtInlineNames) ? txt_slots(P) : 1;
  uint8_t* stage = reinterpret_cast<uint8_t*>(s_stage);
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    txt_bracket(P, b, N, s_mb);
    const unsigned long long bbase = P.btot[b];
    unsigned long long inblk = 0;  // bytes of the block's earlier slices
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r0 = b * kScanBlock + int64_t(k) * kRecThreads;
      if (r0 >= N) break;  // (uniform over the block)
      const int64_t r = r0 + tid;
      const bool valid = r < N;
      const uint32_t L = valid ? P.lens[r] : 0u;
      int64_t m = 0;
      if (valid) m = txt_module(P.mscan, s_mb[0], s_mb[1], r);
      unsigned long long inc = L;
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
      const unsigned long long off = inblk + wpre + (inc - L);  // offset within the block
      int64_t g = 0;
      if (valid) {
        g = int64_t(bbase + off + (P.mscan[m + 1] >> kHdrShift));
        P.lens[r] = uint32_t(off);
        if (tid == 0) s_g[0] = g;
        if (r == N - 1 || tid == kRecThreads - 1) s_g[1] = g + L;
      }
      __syncthreads();
      const int64_t G0 = s_g[0], G1 = s_g[1], G0a = G0 & ~int64_t(3);
      const bool staged = G1 - G0a <= kStageBytes;
      if (valid) {
        if (staged) {
          LdsSink sk{stage, uint32_t(g - G0a)};
          txt_line(P, ns, uint32_t(m), txt_pos(P, m, r), sk);
        } else {
          GlobalSink sk{P.text, g, P.text_cap, 0u};
          txt_line(P, ns, uint32_t(m), txt_pos(P, m, r), sk);
        }
      }
      __syncthreads();
      if (staged) {
        const int64_t nw = (G1 - G0a + 3) >> 2;
        for (int64_t i = tid; i < nw; i += kRecThreads) {
          const int64_t A = G0a + 4 * i;
          const uint32_t x = s_stage[i];
          if (A >= G0 && A + 4 <= G1 && A + 4 <= P.text_cap) {
            *reinterpret_cast<uint32_t*>(P.text + A) = x;
          } else {
            for (int q = 0; q < 4; ++q)
              if (A + q >= G0 && A + q < G1 && A + q < P.text_cap) P.text[A + q] = uint8_t(x >> (8 * q));
          }
        }
      }
      __syncthreads();  // the stage, s_w and s_g are rewritten by the next slice
      inblk += tot;
    }
  }
}

// text_mod_off and the module headers (after the lines: a header overwrites
// whatever a staged slice stored in the gap it fills).
__global__ __launch_bounds__(kRecThreads) void k_txt_modules(TParams P) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (P.ctrl[2]) {  // a scan gave up waiting: no valid output
    for (int64_t m = gtid; m <= P.M; m += nth) P.text_mod_off[m] = -1;
    return;
  }
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  for (int64_t m = gtid; m <= P.M; m += nth) {
    const unsigned long long sm = P.mscan[m];
    const int64_t r0 = int64_t(sm & kInstMask);
    const unsigned long long lx = r0 < N ? P.btot[r0 / kScanBlock] + P.lens[r0] : P.btot[nb];
    const int64_t off = int64_t(lx + (sm >> kHdrShift));
    P.text_mod_off[m] = off;
    if (m < P.M && (P.mscan[m + 1] >> kHdrShift) > (sm >> kHdrShift)) {
      GlobalSink sk{P.text, off, P.text_cap, 0u};
      txt_header(P, m, sk);
    }
  }
}

void launch_text(const TParams& p, hipStream_t s) {
  auto grid = [](int64_t n) {
    const int64_t g = n / kRecThreads + 1;
    return int(g > 4096 ? 4096 : g);
  };
  const int64_t nb = p.cap_inst / kScanBlock + 1;  // blocks of instructions, at most
  const int gb = int(nb > 4096 ? 4096 : nb);
  hipLaunchKernelGGL(k_txt_init, dim3(grid(p.M > nb ? p.M : nb)), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_modscan, dim3(int(p.M / kScanBlock + 1)), dim3(kRecThreads), 0, s, p);
  if (p.options & kTxtInlineNames) {
    hipLaunchKernelGGL(k_txt_collect, dim3(gb), dim3(kRecThreads), 0, s, p);
    hipLaunchKernelGGL(k_txt_hclear, dim3(grid(p.slot_cap)), dim3(kRecThreads), 0, s, p);
    hipLaunchKernelGGL(k_txt_insert, dim3(grid(p.cap_inst / 3 + 1)), dim3(kRecThreads), 0, s, p);
    hipLaunchKernelGGL(k_txt_nlen, dim3(grid(p.slot_cap)), dim3(kRecThreads), 0, s, p);
  }
  hipLaunchKernelGGL(k_txt_lens, dim3(gb), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_bscan, dim3(int(nb / kScanBlock + 1)), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_scatter, dim3(gb), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_modules, dim3(grid(p.M + 1)), dim3(kRecThreads), 0, s, p);
}

}  // namespace spv
