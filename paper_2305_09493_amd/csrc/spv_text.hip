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
// per-block regions of a list and inserted into an open-addressing hash keyed
// by (module, ID), where a 64-bit atomicMin on (position, name length) keeps
// each ID's first OpName, and into a 2 MB bit filter that answers most IDs
// (those without a name) without a probe of the table; a length pass sizes every
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
constexpr int kStageBytes = 30720;                 // LDS staging per slice of 256 lines
constexpr uint32_t kLenBits = 28;  // a line's length (< 2^20: at most 4 names and a string of 65533 words); above it, its name bits

// Every fixed token the lines print, concatenated: opcode names (ids 0..12),
// capabilities 0..12, 22, 39 (13..27), addressing models 0..2 (28..30), memory
// models 0..3 (31..34), execution models 0..6 (35..41), function control None,
// Inline, DontInline, Pure, Const (42..46).  Enumerant names are those of the
// SPIR-V specification.
constexpr const char* kTokStr[] = {
    "OpName", "OpMemoryModel", "OpEntryPoint", "OpCapability", "OpTypeInt", "OpConstant", "OpFunction",
    "OpFunctionEnd", "OpLoad", "OpStore", "OpIAdd", "OpLabel", "OpReturn",
    "Matrix", "Shader", "Geometry", "Tessellation", "Addresses", "Linkage", "Kernel", "Vector16",
    "Float16Buffer", "Float16", "Float64", "Int64", "Int64Atomics", "Int16", "Int8",
    "Logical", "Physical32", "Physical64",
    "Simple", "GLSL450", "OpenCL", "Vulkan",
    "Vertex", "TessellationControl", "TessellationEvaluation", "Geometry", "Fragment", "GLCompute", "Kernel",
    "None", "Inline", "DontInline", "Pure", "Const"};
constexpr int kNumTok = int(sizeof(kTokStr) / sizeof(kTokStr[0]));
constexpr int kTokCap = 512;

struct TokTable {
  uint16_t off[kNumTok];
  uint8_t len[kNumTok];
  char chars[kTokCap];
};

constexpr TokTable make_tok_table() {
  TokTable t{};
  int o = 0;
  for (int i = 0; i < kNumTok; ++i) {
    int n = 0;
    while (kTokStr[i][n]) ++n;
    t.off[i] = uint16_t(o);
    t.len[i] = uint8_t(n);
    for (int k = 0; k < n; ++k) t.chars[o + k] = kTokStr[i][k];
    o += n;
  }
  return t;
}

__constant__ TokTable kTok = make_tok_table();

// One opcode of the grammar: its name's token, the operand words before its
// string (all operand words for an instruction without one), whether a
// string follows, operand roles (2 bits per slot: 0 literal, 1 ID use, 2
// result ID) and literal kinds (3 bits per slot: 0 decimal, 1 capability, 2
// addressing model, 3 memory model, 4 execution model, 5 function control).
struct TxtOp {
  uint32_t tok, nfix, str, roles, lits;
};

__device__ __forceinline__ TxtOp txt_op(uint32_t op) {
  switch (op) {
    case 5: return {0, 1, 1, 1u, 0u};
    case 14: return {1, 2, 0, 0u, 2u | (3u << 3)};
    case 15: return {2, 2, 1, 1u << 2, 4u};
    case 17: return {3, 1, 0, 0u, 1u};
    case 21: return {4, 3, 0, 2u, 0u};
    case 43: return {5, 3, 0, 1u | (2u << 2), 0u};
    case 54: return {6, 4, 0, 1u | (2u << 2) | (1u << 6), 5u << 6};
    case 56: return {7, 0, 0, 0u, 0u};
    case 61: return {8, 3, 0, 1u | (2u << 2) | (1u << 4), 0u};
    case 62: return {9, 2, 0, 1u | (1u << 2), 0u};
    case 128: return {10, 4, 0, 1u | (2u << 2) | (1u << 4) | (1u << 6), 0u};
    case 248: return {11, 1, 0, 2u, 0u};
    default: return {12, 0, 0, 0u, 0u};  // 253: decode admits no other opcode
  }
}

// Token of enumerant v of literal kind 1..4, or -1 (the value prints in
// decimal).
__device__ __forceinline__ int txt_enum(uint32_t kind, uint32_t v) {
  if (kind == 1) return v <= 12u ? 13 + int(v) : v == 22u ? 26 : v == 39u ? 27 : -1;
  if (kind == 2) return v <= 2u ? 28 + int(v) : -1;
  if (kind == 3) return v <= 3u ? 31 + int(v) : -1;
  if (kind == 4) return v <= 6u ? 35 + int(v) : -1;
  return -1;
}

// Output sinks of the line writer: a counter (lengths only), LDS staging, and
// global memory clipped at the caller's capacity.  o is the position of the
// next byte; put_at writes at a position already counted.
struct CountSink {
  static constexpr bool kWrite = false;
  uint32_t o;
  const char* tok;
  __device__ __forceinline__ void put(uint32_t) { ++o; }
  __device__ __forceinline__ void put_at(uint32_t, uint32_t) {}
};
struct LdsSink {
  static constexpr bool kWrite = true;
  uint8_t* p;
  uint32_t o;
  const char* tok;  // the token characters, staged in LDS
  __device__ __forceinline__ void put(uint32_t c) { p[o++] = uint8_t(c); }
  __device__ __forceinline__ void put_at(uint32_t k, uint32_t c) { p[k] = uint8_t(c); }
};
struct GlobalSink {
  static constexpr bool kWrite = true;
  uint8_t* p;
  int64_t g, cap;
  uint32_t o;
  const char* tok;
  __device__ __forceinline__ void put(uint32_t c) {
    if (g + o < cap) p[g + o] = uint8_t(c);
    ++o;
  }
  __device__ __forceinline__ void put_at(uint32_t k, uint32_t c) {
    if (g + k < cap) p[g + k] = uint8_t(c);
  }
};

__device__ __forceinline__ uint32_t ndigits(uint32_t v) {
  return v < 10u ? 1u : v < 100u ? 2u : v < 1000u ? 3u : v < 10000u ? 4u : v < 100000u ? 5u
       : v < 1000000u ? 6u : v < 10000000u ? 7u : v < 100000000u ? 8u : v < 1000000000u ? 9u : 10u;
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
__device__ __forceinline__ void put_tok(S& s, int id) {
  const uint32_t n = kTok.len[id];
  if constexpr (S::kWrite) {
    const char* c = s.tok + kTok.off[id];
    for (uint32_t k = 0; k < n; ++k) s.put(uint8_t(c[k]));
  } else {
    s.o += n;
  }
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

// Bit of (module, ID) in the name filter: the mixed key's high bits (the
// table slot takes its low bits).
__device__ __forceinline__ uint32_t txt_fbit(unsigned long long mixed) { return uint32_t(mixed >> 40); }

__device__ __forceinline__ IdName txt_name(const TParams& P, unsigned long long nslots, uint32_t m, uint32_t v) {
  const unsigned long long key = ((unsigned long long)m << 32) | v;
  const unsigned long long mixed = txt_mix(key);
  // most IDs have no name: the filter (in L2) answers them without a probe
  const uint32_t fb = txt_fbit(mixed);
  if (!((P.nfilter[fb >> 5] >> (fb & 31u)) & 1u)) return IdName{0u, 0u};
  unsigned long long h = mixed & (nslots - 1);
  while (true) {  // the table is at most half full, so an empty slot ends every probe
    const unsigned long long k = P.slots[h].key;
    if (k == key) {
      const unsigned long long pl = P.slots[h].pl;
      return IdName{uint32_t(pl >> 32), uint32_t(pl)};
    }
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
      // (one load per word of the name)
      for (uint32_t j = 0; 4 * j < nm.len; ++j) {
        const uint32_t x = w[j];
        if (4 * j + 4 <= nm.len) {
          s.put(x & 0xFFu);
          s.put((x >> 8) & 0xFFu);
          s.put((x >> 16) & 0xFFu);
          s.put(x >> 24);
        } else {
          for (uint32_t q = 0; 4 * j + q < nm.len; ++q) s.put((x >> (8 * q)) & 0xFFu);
        }
      }
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
      put_tok(s, 42);
    } else if (v & ~0xFu) {
      put_dec(s, v);
    } else {
      bool first = true;
      for (int b = 0; b < 4; ++b) {
        if (!(v & (1u << b))) continue;
        if (!first) s.put('|');
        put_tok(s, 43 + b);
        first = false;
      }
    }
  } else {
    const int e = txt_enum(kind, v);
    if (e >= 0) put_tok(s, e);
    else put_dec(s, v);
  }
  if (hl) color_off(s);
}

// 0x80 in every byte of t that is zero, 0 elsewhere (exact per byte).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t t) {
  return ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t | 0x7F7F7F7Fu);
}

// Bytes of the last word of a string before its NUL (decode checked that the
// first NUL lies in the last word).
__device__ __forceinline__ uint32_t last_word_bytes(uint32_t x) {
  return uint32_t(__builtin_ctz(zero_bytes(x) | 0x80000000u)) >> 3;
}

// A string literal of nw words, quoted, with '"' and '\' escaped.  The
// counter works on whole words: the length from the last word, the escapes by
// byte compares.
template <class S>
__device__ __forceinline__ void put_string(S& s, const uint32_t* w, uint32_t nw) {
  if constexpr (S::kWrite) {
#pragma unroll 4
    for (uint32_t i = 0; i < nw; ++i) {
      const uint32_t x = w[i];
      const uint32_t nb = i + 1 < nw ? 4u : last_word_bytes(x);
      const uint32_t esc = zero_bytes(x ^ 0x22222222u) | zero_bytes(x ^ 0x5C5C5C5Cu);
      if (nb == 4u && esc == 0u) {
        // (a whole word with nothing to escape: four bytes, no per-byte branch)
        s.put(x & 0xFFu);
        s.put((x >> 8) & 0xFFu);
        s.put((x >> 16) & 0xFFu);
        s.put(x >> 24);
        continue;
      }
      for (uint32_t q = 0; q < nb; ++q) {
        const uint32_t c = (x >> (8 * q)) & 0xFFu;
        if (c == '"' || c == '\\') s.put('\\');
        s.put(c);
      }
    }
  } else {
    uint32_t n = 0;
#pragma unroll 4
    for (uint32_t i = 0; i < nw; ++i) {
      const uint32_t x = w[i];
      const uint32_t nb = i + 1 < nw ? 4u : last_word_bytes(x);
      const uint32_t live = nb == 4u ? 0x80808080u : (0x80808080u & ((1u << (8 * nb)) - 1u));
      const uint32_t esc = zero_bytes(x ^ 0x22222222u) | zero_bytes(x ^ 0x5C5C5C5Cu);
      n += nb + uint32_t(__builtin_popcount(esc & live));
    }
    s.o += n;
  }
}

// An instruction's first word and the four words after it (loaded together,
// before the line is built; words past the batch read as 0, words of the
// next instruction are not used).
struct InstWords {
  uint32_t w[5];
};

__device__ __forceinline__ InstWords load_inst(const TParams& P, int64_t pos) {
  InstWords iw;
#pragma unroll
  for (int q = 0; q < 5; ++q) iw.w[q] = pos + q < P.cap_inst ? P.words[pos + q] : 0u;
  return iw;
}

// The text line of the instruction at word position pos of module m.
// nmask: bit k set when operand k's ID has a name.  The length pass (kFind)
// looks every ID up and sets the bits; the scatter looks up only the IDs
// whose bit is set (the others print as numbers).
template <bool kFind, class S>
__device__ __forceinline__ void txt_line(const TParams& P, unsigned long long nslots, uint32_t m, int64_t pos,
                                         const InstWords& iw, S& s, uint32_t& nmask) {
  const uint32_t w0 = iw.w[0], op = w0 & 0xFFFFu;
  const TxtOp d = txt_op(op);
  const uint32_t opt = P.options;
  const bool hl = (opt & kTxtHighlight) != 0, names = (opt & kTxtInlineNames) != 0;
  uint32_t v[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) v[k] = k < d.nfix ? iw.w[1 + k] : 0u;
  bool has_res = false;
  uint32_t rv = 0, rk = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k)
    if (((d.roles >> (2 * k)) & 3u) == 2u) {
      has_res = true;
      rv = v[k];
      rk = k;
    }
  auto name_of = [&](uint32_t k, uint32_t id) -> IdName {
    if (!kFind && !((nmask >> k) & 1u)) return IdName{0u, 0u};
    const IdName nm = txt_name(P, nslots, m, id);
    if (kFind && nm.len) nmask |= 1u << k;
    return nm;
  };
  if ((opt & kTxtGroup) && (op == 54u || op == 248u)) s.put('\n');
  IdName rn{0u, 0u};
  if (has_res && names) rn = name_of(rk, rv);
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
  put_tok(s, int(d.tok));
  if (hl) color_off(s);
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    if (k >= d.nfix) break;
    const uint32_t role = (d.roles >> (2 * k)) & 3u;
    if (role == 2u) continue;
    s.put(' ');
    if (role == 1u) {
      const IdName nm = names ? name_of(k, v[k]) : IdName{0u, 0u};
      put_id(s, P, hl, nm, v[k]);
    } else {
      put_lit(s, hl, (d.lits >> (3 * k)) & 7u, v[k]);
    }
  }
  if (d.str) {
    s.put(' ');
    if (hl) color_on(s, '2');
    s.put('"');
    put_string(s, P.words + pos + 1 + d.nfix, (w0 >> 16) - 1 - d.nfix);
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
      CountSink c{0, nullptr};
      txt_header(P, m, c);
      hb = c.o;
    }
    P.mscan[m] = hdr_ok ? (hb << kHdrShift) | (unsigned long long)r.n_inst : 0ull;
  }
}

__global__ __launch_bounds__(kRecThreads) void k_txt_modscan(TParams P) {
  scan_block(P.mscan, P.M, P.mscan, P.mstate, &P.ctrl[0], &P.ctrl[2]);
}

// Inline names, step 1: the OpName instructions of every block of 1024
// instructions, compacted into that block's own region of the list (no
// shared counter), and their number.
__global__ __launch_bounds__(kRecThreads) void k_txt_collect(TParams P) {
  __shared__ int64_t s_mb[2];
  __shared__ uint32_t s_wc[kRecThreads / 64];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    txt_bracket(P, b, N, s_mb);
    uint32_t run = 0;  // names in the block's earlier slices
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
      if (lane == 0) s_wc[wave] = uint32_t(__builtin_popcountll(bal));
      __syncthreads();
      uint32_t before = run, tot = 0;
#pragma unroll
      for (int w = 0; w < kRecThreads / 64; ++w) {
        if (w < wave) before += s_wc[w];
        tot += s_wc[w];
      }
      if (is_name) {
        const uint32_t rank = before + uint32_t(__builtin_popcountll(bal & ((1ull << lane) - 1ull)));
        P.nlist[b * kScanBlock + rank] = make_uint2(uint32_t(m), uint32_t(pos));
      }
      run += tot;
      __syncthreads();  // s_wc is rewritten by the next slice
    }
    if (tid == 0) P.bcount[b] = run;
  }
}

// Inline names, step 2: the number of OpName instructions (one block).
__global__ __launch_bounds__(1024) void k_txt_ncount(TParams P) {
  __shared__ uint32_t s_w[16];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x;
  const int64_t nb = (txt_count(P) + kScanBlock - 1) / kScanBlock;
  uint32_t sum = 0;
  for (int64_t b = tid; b < nb; b += 1024) sum += P.bcount[b];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d);
  if ((tid & 63) == 0) s_w[tid >> 6] = sum;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int w = 0; w < 16; ++w) t += s_w[w];
    P.ctrl[3] = t;
  }
}

// Inline names, step 3: empty the slots in use.
__global__ __launch_bounds__(kRecThreads) void k_txt_hclear(TParams P) {
  if (P.ctrl[2]) return;
  const unsigned long long ns = txt_slots(P);
  const unsigned long long gtid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long nth = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = gtid; i < ns; i += nth) {
    P.slots[i].key = kTxtEmpty;
    P.slots[i].pl = ~0ull;
  }
  for (unsigned long long i = gtid; i < kTxtFilterBits / 32; i += nth) P.nfilter[i] = 0u;
}

// Inline names, step 4: insert every OpName by (module, target) with its
// name's length (0 when the name is not usable: empty, a character outside
// [A-Za-z0-9_], or a leading digit); a 64-bit atomicMin on (word position <<
// 32 | length) keeps the module's first OpName of each target.
__global__ __launch_bounds__(kRecThreads) void k_txt_insert(TParams P) {
  if (P.ctrl[2]) return;
  const unsigned long long ns = txt_slots(P);
  const int64_t n = ((txt_count(P) + kScanBlock - 1) / kScanBlock) * kScanBlock;
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = gtid; i < n; i += nth) {
    if (uint32_t(i % kScanBlock) >= P.bcount[i / kScanBlock]) continue;
    const uint2 e = P.nlist[i];
    const uint32_t nw = (P.words[e.y] >> 16) - 2;  // the name's words
    const uint32_t* w = P.words + e.y + 2;
    uint32_t len = 0;
    // (all four bytes of a word tested, the ones past the string masked; the
    // flag an integer: no per-byte branches or lane-mask merging)
    uint32_t bad = 0;
#pragma unroll 4
    for (uint32_t k = 0; k < nw; ++k) {
      const uint32_t x = w[k];
      const uint32_t nb = k + 1 < nw ? 4u : last_word_bytes(x);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t c = (x >> (8 * q)) & 0xFFu;
        const uint32_t alpha = (c - 'a' < 26u || c - 'A' < 26u || c == '_') ? 1u : 0u;
        const uint32_t digit = (c - '0' < 10u && (k | q) != 0u) ? 1u : 0u;
        bad |= (q < nb && (alpha | digit) == 0u) ? 1u : 0u;
      }
      len += nb;
    }
    const unsigned long long val = ((unsigned long long)e.y << 32) | (bad ? 0u : len);
    const unsigned long long key = ((unsigned long long)e.x << 32) | P.words[e.y + 1];
    const unsigned long long mixed = txt_mix(key);
    const uint32_t fb = txt_fbit(mixed);
    atomicOr(&P.nfilter[fb >> 5], 1u << (fb & 31u));
    unsigned long long h = mixed & (ns - 1);
    while (true) {
      const unsigned long long prev = atomicCAS(&P.slots[h].key, kTxtEmpty, key);
      if (prev == kTxtEmpty || prev == key) {
        atomicMin(&P.slots[h].pl, val);
        break;
      }
      h = (h + 1) & (ns - 1);
    }
  }
}

// Line lengths, and the total of every block of 1024 lines.
// (eight waves per SIMD, 64 registers: the pass waits on dependent loads, and
// more resident waves hide more of them)
__global__ __launch_bounds__(kRecThreads, 8) void k_txt_lens(TParams P) {
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
    // the thread's four lines: positions, then all their words, then the
    // lengths (the loads of the four are in flight together)
    int64_t mk[kScanPerThread], pk[kScanPerThread];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      mk[k] = 0;
      pk[k] = -1;
      if (r < N) {
        mk[k] = txt_module(P.mscan, s_mb[0], s_mb[1], r);
        pk[k] = txt_pos(P, mk[k], r);
      }
    }
    InstWords iw[kScanPerThread];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)
      if (pk[k] >= 0) iw[k] = load_inst(P, pk[k]);
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      if (pk[k] >= 0) {
        CountSink c{0, nullptr};
        uint32_t nmask = 0;
        txt_line<true>(P, ns, uint32_t(mk[k]), pk[k], iw[k], c, nmask);
        P.lens[r] = c.o | (nmask << kLenBits);  // (the scatter reads the name bits back)
        P.lpos[r] = uint32_t(pk[k]);
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
__global__ __launch_bounds__(kRecThreads, 5) void k_txt_scatter(TParams P) {
  __shared__ uint32_t s_stage[kStageBytes / 4];
  __shared__ int64_t s_mb[2];
  __shared__ unsigned long long s_w[kRecThreads / 64];
  __shared__ long long s_g[2];
  __shared__ char s_tok[kTokCap];
  if (P.ctrl[2]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < kTokCap; i += kRecThreads) s_tok[i] = kTok.chars[i];
  __syncthreads();
  const int64_t N = txt_count(P);
  const int64_t nb = (N + kScanBlock - 1) / kScanBlock;
  const unsigned long long ns = (P.options & kTxtInlineNames) ? txt_slots(P) : 1;
  uint8_t* stage = reinterpret_cast<uint8_t*>(s_stage);
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    txt_bracket(P, b, N, s_mb);
    const unsigned long long bbase = P.btot[b];
    unsigned long long inblk = 0;  // bytes of the block's earlier slices
    // the thread's four lines' lengths and positions first (loads in flight
    // together); each slice's instruction words are loaded before its scan
    uint32_t Lk[kScanPerThread], pk[kScanPerThread];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r = b * kScanBlock + int64_t(k) * kRecThreads + tid;
      Lk[k] = r < N ? P.lens[r] : 0u;  // length | name bits << kLenBits
      pk[k] = r < N ? P.lpos[r] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
      const int64_t r0 = b * kScanBlock + int64_t(k) * kRecThreads;
      if (r0 >= N) break;  // (uniform over the block)
      const int64_t r = r0 + tid;
      const bool valid = r < N;
      const uint32_t L = Lk[k] & ((1u << kLenBits) - 1u);
      uint32_t nmask = Lk[k] >> kLenBits;
      InstWords iwk;
      if (valid) iwk = load_inst(P, int64_t(pk[k]));
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
          LdsSink sk{stage, uint32_t(g - G0a), s_tok};
          txt_line<false>(P, ns, uint32_t(m), int64_t(pk[k]), iwk, sk, nmask);
        } else {
          GlobalSink sk{P.text, g, P.text_cap, 0u, s_tok};
          txt_line<false>(P, ns, uint32_t(m), int64_t(pk[k]), iwk, sk, nmask);
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
      GlobalSink sk{P.text, off, P.text_cap, 0u, nullptr};
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
    hipLaunchKernelGGL(k_txt_ncount, dim3(1), dim3(1024), 0, s, p);
    hipLaunchKernelGGL(k_txt_hclear, dim3(grid(p.slot_cap > int64_t(kTxtFilterBits / 32) ? p.slot_cap : int64_t(kTxtFilterBits / 32))),
                       dim3(kRecThreads), 0, s, p);
    hipLaunchKernelGGL(k_txt_insert, dim3(grid(p.cap_inst)), dim3(kRecThreads), 0, s, p);
  }
  hipLaunchKernelGGL(k_txt_lens, dim3(gb), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_bscan, dim3(int(nb / kScanBlock + 1)), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_scatter, dim3(gb), dim3(kRecThreads), 0, s, p);
  hipLaunchKernelGGL(k_txt_modules, dim3(grid(p.M + 1)), dim3(kRecThreads), 0, s, p);
}

}  // namespace spv
