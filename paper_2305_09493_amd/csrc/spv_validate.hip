// Batched SPIR-V decode / validate kernels for gfx950 (CDNA4, wave64).
//
// What is computed (Beehive SPIR-V Toolkit paper, arXiv 2305.09493): the
// disassembler's walk over a module's instructions (section "Dis/Assembler"),
// where each instruction's first word carries its word count and opcode
// (section "Parsing Operand Kinds"), after the 5-word header (section "SPIR-V
// Library", header listing), and the validation the library performs before
// storing a module (section "Validation Rules") together with the SSA rule
// that every ID is defined once (section "Enabling Function Composition").
//
// How (MI355X design):
//   * The batch's words are cut into tiles of 4096 words, 16 per lane, 256
//     lanes per block; tiles ignore module boundaries.
//   * Instruction-boundary recovery is pointer jumping over
//     next(i) = i + (w[i] >> 16).  Each lane derives its transfer function
//     "entry offset -> exit offset" over its 16 words: by following the
//     chain from its first plausible start when every plausible start lies on
//     that chain (chains that start on operand words die at once, so this is
//     the common case and the exit does not depend on the entry), else by a
//     backward recurrence that packs the exits of the 15 following positions
//     as 4-bit nibbles in a 64-bit register.
//   * Three passes when every tile settles this way (the common case): the
//     chain pass computes every tile's exit, its lanes' starts and its
//     per-module start counts, each tile on its own; the resolve pass scans
//     the tile summaries (a segmented scan chained by a decoupled look-back)
//     into every tile's exact entry and instruction-count prefix; the walk
//     then checks, indexes and marks result IDs with no waiting between
//     tiles.  Otherwise (a tile with an instruction of 15+ words on a
//     candidate chain, crowded module starts, a lane that stays ambiguous)
//     the whole batch takes the single-pass walk, in which tiles chain
//     through a decoupled look-back on aggregate / full states; tiles that
//     even this cannot settle are walked serially by one thread.
//   * Result-ID define-once checks use 64-bit bitmaps (or a hash table when
//     the bound is much larger than the module) with atomics, accumulated in
//     LDS windows first; the undefined-ID check is skipped for modules whose
//     result IDs cover [1, bound) (no use can then be undefined) and
//     otherwise runs as a second pass against the completed bitmap.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "spv_internal.h"

namespace spv {

namespace {

constexpr uint32_t kMagic = 0x07230203u;

// grammar: opcode, smallest word count, count of accepted word counts,
// result-ID slot mask, ID-use slot mask (slot s <-> bit s-1), and the
// module-level rule the opcode satisfies (section "Validation Rules": 1
// capability, 2 memory model, 4 function, 8 entry point)
struct GEnt {
  uint16_t op;
  uint8_t lo;
  uint16_t nok;
  uint8_t def;
  uint8_t use;
  uint8_t rule;
};
constexpr int kNumOps = 13;
__device__ __constant__ GEnt kGrammar[kNumOps] = {
    {5, 3, 65533, 0x0, 0x1, 0},   // OpName          U S...
    {14, 3, 1, 0x0, 0x0, 2},      // OpMemoryModel   L L
    {15, 4, 65532, 0x0, 0x2, 8},  // OpEntryPoint    L U S...
    {17, 2, 1, 0x0, 0x0, 1},      // OpCapability    L
    {21, 4, 1, 0x1, 0x0, 0},      // OpTypeInt       D L L
    {43, 4, 1, 0x2, 0x1, 0},      // OpConstant      U D L
    {54, 5, 1, 0x2, 0x9, 4},      // OpFunction      U D L U
    {56, 1, 1, 0x0, 0x0, 0},      // OpFunctionEnd
    {61, 4, 1, 0x2, 0x5, 0},      // OpLoad          U D U
    {62, 3, 1, 0x0, 0x3, 0},      // OpStore         U U
    {128, 5, 1, 0x2, 0xD, 0},     // OpIAdd          U D U U
    {248, 2, 1, 0x1, 0x0, 0},     // OpLabel         D
    {253, 1, 1, 0x0, 0x0, 0},     // OpReturn
};

// LDS grammar entry of an opcode (0 = unknown): bits 0..2 smallest word
// count, bit 3 string operand, bits 4..7 module-level rule bits, bits 8..23
// count of accepted word counts, bits 24..27 result-ID slots, bits 28..31
// ID-use slots.  The instructions with a string (OpName, OpEntryPoint) have
// a variable word count whose smallest value is their fixed operands, one
// string word and the first word, so their string starts at operand slot
// lo - 1.
constexpr uint32_t kEntStr = 0x8u;
__device__ __forceinline__ uint32_t str_slot(uint32_t e) { return (e & 0x7u) - 1u; }
__device__ __forceinline__ uint32_t ent_str(uint32_t e) { return (e >> 3) & 1u; }
__device__ __forceinline__ uint32_t ent_rules(uint32_t e) { return (e >> 4) & 0xFu; }

__device__ __forceinline__ void init_table(uint32_t* tbl) {
  for (int i = threadIdx.x; i < 257; i += blockDim.x) tbl[i] = 0;
  __syncthreads();
  if (threadIdx.x < kNumOps) {
    GEnt g = kGrammar[threadIdx.x];
    tbl[g.op] = uint32_t(g.lo) | (g.nok > 1 ? kEntStr : 0u) | (uint32_t(g.rule) << 4) | (uint32_t(g.nok) << 8) |
                (uint32_t(g.def) << 24) | (uint32_t(g.use) << 28);
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t tbl_lookup(const uint32_t* tbl, uint32_t op) { return tbl[op < 256u ? op : 256u]; }
__device__ __forceinline__ bool tbl_plausible(uint32_t e, uint32_t wc) {
  return (wc - (e & 0x7u)) < ((e >> 8) & 0xFFFFu);
}

// Tile states carry their whole message in one 64-bit word, so relaxed
// device-scope atomics suffice: no reader depends on other data written
// before the state.  (Acquire / release here would cost an L2 invalidate or
// a full L2 write-back on every poll and publish.)
__device__ __forceinline__ unsigned long long ld_state(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_state(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Module of word x: the last m < M with mod_off[m] <= x (mod_off[0] = 0 <= x).
// An 8-way search: each round loads seven probes together and keeps the
// eighth of the range that holds the answer, so a batch of 4096 modules takes
// five rounds of loads instead of a binary search's twelve.
__device__ __forceinline__ int64_t find_module(const int64_t* mod_off, int64_t M, int64_t x) {
  int64_t lo = 0, hi = M - 1;  // mod_off[lo] <= x, answer in [lo, hi]
  while (hi - lo >= 8) {
    const int64_t step = (hi - lo + 1) >> 3;
    int64_t v[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = mod_off[lo + (k + 1) * step];
    int n = 0;  // probes at or below x (a prefix: the offsets do not decrease)
#pragma unroll
    for (int k = 0; k < 7; ++k) n += v[k] <= x ? 1 : 0;
    const int64_t nlo = lo + n * step;
    if (n < 7) hi = nlo + step - 1;
    lo = nlo;
  }
  int64_t v[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = (lo + 1 + k <= hi) ? mod_off[lo + 1 + k] : INT64_MAX;
  int n = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) n += v[k] <= x ? 1 : 0;
  return lo + n;
}

// A string operand: bytes little-endian within each word, terminated by the
// first NUL, which must be in the last word, followed only by NUL padding.
__device__ __forceinline__ bool string_ok_global(const uint32_t* w, int64_t n_words) {
  for (int64_t i = 0; i + 1 < n_words; ++i) {
    uint32_t x = w[i];
    if (((x - 0x01010101u) & ~x & 0x80808080u) != 0) return false;  // a NUL before the last word
  }
  uint32_t x = w[n_words - 1];
  uint32_t z = (x - 0x01010101u) & ~x & 0x80808080u;  // lowest set flag marks the first NUL byte exactly
  if (z == 0) return false;
  int k = __builtin_ctz(z) >> 3;
  return (x >> (8 * k)) == 0;
}

// Exact parse-stage code of a candidate start (0 if it is a valid
// instruction).  end = end of its module (absolute word index).
__device__ __forceinline__ uint32_t start_code(const uint32_t* words, const uint32_t* tbl, int64_t pos, int64_t end) {
  uint32_t w0 = words[pos];
  uint32_t wc = w0 >> 16, op = w0 & 0xFFFFu;
  if (wc == 0 || pos + wc > end) return SPV_E_BAD_WORD_COUNT;
  uint32_t e = tbl_lookup(tbl, op);
  if (((e >> 8) & 0xFFFFu) == 0) return SPV_E_UNKNOWN_OPCODE;
  if (!tbl_plausible(e, wc)) return SPV_E_BAD_WORD_COUNT;
  if ((e & kEntStr) && !string_ok_global(words + pos + str_slot(e), wc - str_slot(e))) return SPV_E_BAD_STRING;
  return 0;
}

// ---- ID sets ---------------------------------------------------------------
// Bitmap mode: module m's bitmap is idmap[off_m .. off_m + ceil(bound/64)).
// Hash mode: module m owns n_m 64-bit slots idmap[off_m .. off_m + n_m),
// slot = id | (flags << 32), flags bit 0 defined, bit 1 used, 0 = empty.
__device__ __forceinline__ uint32_t hash_slot(uint32_t v, int64_t n) {
  return uint32_t((uint64_t(v * 2654435761u) * uint64_t(n)) >> 32);
}

// Insert id v into a hash-mode module; returns the old flag bits of v.
__device__ __forceinline__ uint32_t hash_insert(unsigned long long* slots, int64_t n, uint32_t v, uint32_t flag) {
  int64_t h = hash_slot(v, n);
  for (int64_t probe = 0; probe < n; ++probe) {
    unsigned long long cur = __hip_atomic_load(&slots[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (uint32_t(cur) == 0u) {
      unsigned long long prev = atomicCAS(&slots[h], 0ull, (unsigned long long)v);
      if (prev == 0ull || uint32_t(prev) == v) cur = v;
    }
    if (uint32_t(cur) == v) {
      unsigned long long old = atomicOr(&slots[h], (unsigned long long)flag << 32);
      return uint32_t(old >> 32);
    }
    h = (h + 1 == n) ? 0 : h + 1;
  }
  return 0;  // unreachable: a module has more slots than distinct IDs
}

// ---- per-tile module list -------------------------------------------------
struct LEnt {
  int32_t rel;     // start - t0 (clamped to -1 below the tile)
  int32_t mod;     // module index, -1 for the batch end
  int64_t off;     // module start
  int64_t end;     // module end
  uint32_t bound;
  uint32_t info;   // bits 0..2 header length min(5, n); bit 3 batch end; bit 4 header ok; bit 5 hash mode
};
constexpr uint32_t kInfoEnd = 8u, kInfoHdrOk = 16u, kInfoSparse = 32u;
constexpr int kWinWords = 128;  // LDS window of 8192 result IDs per tile
constexpr uint32_t kNoBound = 0xFFFFFFFFu;  // no load-time bound test (bound - 1 is never this)
constexpr int kTwTail = 32;     // words past the tile end kept in LDS
// LDS index of tile position q: one pad word after every 16, so that the 64
// lanes of a wave, 16 words apart, read a position each from distinct banks
__device__ __forceinline__ int twx(int q) { return q + (q >> 4); }
constexpr int kTwSize = (kTileWords + kTwTail) + (kTileWords + kTwTail) / 16 + 1;

struct Shared {
  uint32_t tw[kTwSize] __attribute__((aligned(16)));  // the tile's words (+ the next 32), padded (twx)
  uint32_t stage[kTileWords];  // staged index entries: tile position | opcode << 16
  uint32_t tbl[257];
  LEnt list[kListMax];
  int K;
  int crowded;
  long long t;
  long long tnext;             // next tile, claimed ahead
  uint32_t wagg[kWaves];       // wave exit when independent of the wave entry, else 0xFF
  uint32_t wflags[kWaves];     // bit 0: far candidate in the wave
  uint32_t wcnt[kWaves];       // wave count aggregate (bit 31 = module start inside)
  uint32_t wst[kWaves];        // per-wave totals of instruction starts (plain scan)
  uint32_t wref[kWaves];       // per-wave first result ID of the window module
  uint32_t E;                  // tile entry offset (exact) or kExitDead
  uint32_t prefix;             // count of the module open at t0 before t0
  int serial;
  int jw;                      // list index of the module whose result IDs use the LDS window
  uint32_t spill[kBlock];      // role bits of words 16..19 of each lane: def | use << 4
  uint32_t modflags[kListMax];
  uint32_t moddef[kListMax];
  uint32_t slot0[kListMax];    // first staging slot of each module's starts in this tile
  static constexpr int kWins = 1;     // one window: module jw
  static constexpr int kWinW = kWinWords;
  unsigned long long win[kWinWords];  // result-ID window bitmap of module jw
  uint32_t wmin[1];
  uint32_t nname;              // string-bearing starts compacted into stage[] for the string checks
  uint32_t badb[kTileWords / 32];  // tile positions whose string is malformed
  LEnt cache;                  // module containing the previous tile's start
  int cache_ok;
  int32_t rl_mod;               // rule presence bits this block has flushed, and their module
  uint32_t rl_bits;
};

// Shared state of the resolved walk: no staging of index entries (they are
// written directly), OpName starts in a short list (a tile with more checks
// its strings lane by lane), so that six blocks fit on a CU.
constexpr int kNameCap = 1024;
struct WalkShared {
  uint32_t tw[kTwSize] __attribute__((aligned(16)));
  uint16_t names[kNameCap];
  uint32_t tbl[257];
  LEnt list[kListMax];
  int K;
  int crowded;
  long long t;
  long long tnext;
  uint32_t wagg[kWaves];
  uint32_t wflags[kWaves];
  uint32_t wcnt[kWaves];
  uint32_t wst[kWaves];
  uint32_t wref[kWaves];
  uint32_t E;
  uint32_t prefix;
  int serial;
  int jw;
  uint32_t spill[kBlock];
  uint32_t modflags[kListMax];
  uint32_t moddef[kListMax];
  static constexpr int kWins = 2;     // windows of list entries 0 and 1, 4096 result IDs each
  static constexpr int kWinW = 64;
  unsigned long long win[kWins * kWinW];
  uint32_t wmin[kWins];               // smallest anchoring result ID of each window's module
  uint32_t nname;
  uint32_t badb[kTileWords / 32];
  int32_t rl_mod;               // rule presence bits this block has flushed, and their module
  uint32_t rl_bits;
  LEnt cache;
  int cache_ok;
  // bound - 1 of the module that covers this block's next tile and the 16
  // words after it, when that is the module of its current list entry 0 and
  // it keeps its result IDs in a bitmap; kNoBound otherwise
  uint32_t nbm1;
};

// Build the list of non-empty modules overlapping [t0, t1 + 16] (wave 0).
template <class SH>
__device__ __forceinline__ void build_list(SH& S, const VParams& P, long long t, int64_t t0, int64_t t1) {
  const int lane = lane_id();
  // a block's previous tile may have lain in a module that also covers this
  // whole tile window: then that module is the only list entry
  if (S.cache_ok && S.cache.off <= t0 && S.cache.end > t1 + 16) {
    if (lane == 0) {
      LEnt e = S.cache;
      e.rel = int32_t(e.off - t0 < -1 ? -1 : e.off - t0);
      S.list[0] = e;
      S.K = 1;
      S.crowded = 0;
    }
    return;
  }
  int64_t m0 = P.tfm[t];
  if (lane == 0) {
    const ModState& ms = P.mods[m0];
    int64_t off = P.mod_off[m0], end = P.mod_off[m0 + 1];
    LEnt e;
    e.rel = int32_t(off - t0 < -1 ? -1 : off - t0);
    e.mod = int32_t(m0);
    e.off = off;
    e.end = end;
    e.bound = ms.bound;
    int64_t n = end - off;
    e.info = uint32_t(n < 5 ? n : 5) | ((ms.flags & kModHdrOk) ? kInfoHdrOk : 0u) |
             ((ms.flags & kModSparse) ? kInfoSparse : 0u);
    S.list[0] = e;
  }
  int K = 1;
  int crowded = 0;
  const int64_t lim = t1 + 16;
  for (int64_t base = m0 + 1; base < P.M; base += 64) {
    int64_t m = base + lane;
    bool valid = m < P.M;
    int64_t off = valid ? P.mod_off[m] : INT64_MAX;
    int64_t end = valid ? P.mod_off[m + 1] : INT64_MAX;
    bool in = valid && off <= lim;
    bool take = in && end > off;
    uint64_t tm = __ballot(take);
    uint64_t im = __ballot(in);
    int pos = K + __popcll(tm & ((1ull << lane) - 1ull));
    if (take && pos < kListMax) {
      const ModState& ms = P.mods[m];
      LEnt e;
      e.rel = int32_t(off - t0);
      e.mod = int32_t(m);
      e.off = off;
      e.end = end;
      e.bound = ms.bound;
      int64_t n = end - off;
      e.info = uint32_t(n < 5 ? n : 5) | ((ms.flags & kModHdrOk) ? kInfoHdrOk : 0u) |
               ((ms.flags & kModSparse) ? kInfoSparse : 0u);
      S.list[pos] = e;
    }
    K += __popcll(tm);
    if (K > kListMax - 1) {
      crowded = 1;
      break;
    }
    if (im != ~0ull) break;
  }
  if (!crowded && P.W <= lim) {
    if (lane == 0) {
      LEnt e;
      e.rel = int32_t(P.W - t0);
      e.mod = -1;
      e.off = P.W;
      e.end = P.W;
      e.bound = 0;
      e.info = kInfoEnd;
      S.list[K] = e;
    }
    K += 1;
  }
  if (lane == 0) {
    S.K = K;
    S.crowded = crowded;
    S.cache = S.list[0];
    S.cache_ok = 1;
  }
}

template <class SH>
__device__ __forceinline__ int list_find(const SH& S, int32_t rel) {
  // largest j with list[j].rel <= rel (list[0].rel <= 0 <= rel)
  int lo = 0, hi = S.K - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (S.list[mid].rel <= rel) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v |= uint32_t(__shfl_xor(int(v), d));
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Count look-back (called by a whole wave): instruction starts of the module
// open at tile t's start that lie before it.  The wave reads 256 predecessor
// states per round trip (4 per lane, nearest first) and stops at the nearest
// inclusive state or the nearest aggregate of a tile in which a module
// starts.
__device__ __forceinline__ uint32_t count_lookback(const VParams& P, const unsigned long long* states, long long t) {
  const int lane = lane_id();
  uint32_t prefix = 0;
  long long hi = t - 1;
  uint32_t spins = 0;
  while (hi >= 0) {
    unsigned long long st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const long long u = hi - lane - 64 * k;
      st[k] = (u >= 0) ? ld_state(&states[u * kStateStride]) : kFlagFull;
    }
    int k = 0;
    for (; k < 4; ++k) {
      const uint64_t f = st[k] & kFlagMask;
      const bool stop = f == kFlagFull || (f == kFlagAgg && (st[k] & kResetBit));
      const uint64_t stopm = __ballot(stop);
      const uint64_t unpub = __ballot(f == 0);
      const int sl = stopm ? int(__builtin_ctzll(stopm)) : 64;
      const uint64_t need = (sl >= 63) ? ~0ull : ((2ull << sl) - 1ull);
      if (unpub & need) break;
      prefix += wave_sum_u32(lane <= sl ? uint32_t(st[k]) : 0u);
      if (sl < 64) return prefix;
      hi -= 64;
    }
    if (k == 4) continue;
    if (++spins > kSpinLimit) {
      if (lane == 0) atomicOr(&P.ctrl[kCtlSpinErr], 1u);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return prefix;
}

// Entry look-back (wave 0): exact entry offset of tile t, or kExitDead.
// Returns 0xFFFFFFFE when the entry cannot be had from aggregates and the
// full state of t-1 was awaited and found; all lanes get the same value.
__device__ __forceinline__ uint32_t entry_lookback(const VParams& P, long long t) {
  const int lane = lane_id();
  for (uint32_t spins = 0;; ++spins) {
    if (spins > kSpinLimit) {
      if (lane == 0) atomicOr(&P.ctrl[kCtlSpinErr], 1u);
      return kExitDead;
    }
    long long u = t - 1 - lane;
    bool real = lane < kMaxSpanTiles && u >= 0;
    unsigned long long st = real ? ld_state(&P.tileA[(u) * kStateStride]) : kFlagAgg;
    unsigned long long st0 = __shfl(st, 0);
    if ((st0 & kFlagMask) == kFlagFull) return uint32_t(st0);
    bool pub = (st & kFlagMask) != 0;
    if (__ballot(!pub) == 0) {
      uint32_t X = uint32_t(st0) & 15u;
      bool far_before = __ballot(lane >= 1 && real && (st & kFarBit)) != 0;
      if (X != kFar && !far_before) return X == kDead ? kExitDead : X;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

__device__ __forceinline__ uint32_t nib(uint64_t r, uint32_t k) { return uint32_t(r >> (4u * k)) & 15u; }

// Apply a lane transfer function (nibble e = exit for entry e) to an entry.
__device__ __forceinline__ uint32_t apply_fn(uint64_t F, uint32_t e) {
  if (e == kDead) return kDead;
  if (e >= kFar) return kFar;
  return nib(F, e);
}

struct Lane {
  uint32_t w[kLaneWords];
  int64_t a;         // absolute start of the lane segment
  int j0;            // list index of the module open at a
  uint32_t bm;       // window [0, 32): module starts and the batch end
  uint32_t hdr;      // bm & 0xFFFF : positions that are not instruction starts
  uint32_t rst;      // module starts (not the batch end) in [0, 16)
  uint32_t rstbits;  // first-instruction positions of modules starting in [0, 16)
  uint32_t plmask;   // plausible instruction starts
  uint32_t farmask;  // plausible starts with word count >= 15
  uint32_t namemask; // candidate starts of string-bearing instructions (OpName, OpEntryPoint)
  uint32_t rolep[kLaneWords / 4];  // role bits per position (8 bits: result slots | use slots << 4)
  uint64_t F;        // transfer function
  uint32_t reach0;   // fast lanes: chain from the first candidate
  bool slow;         // transfer function from the nibble recurrence
  bool conv;
  uint32_t X;
  bool far_cand;
};

// Module-window masks of a lane.
template <class SH>
__device__ __forceinline__ void lane_window(const SH& S, Lane& L, int32_t lrel) {
  L.j0 = (S.K == 1) ? 0 : list_find(S, lrel);
  L.bm = 0;
  L.rst = 0;
  L.rstbits = 0;
  if (S.K > 1 || S.list[0].rel >= lrel) {
    for (int j = L.j0; j < S.K; ++j) {
      int32_t r = S.list[j].rel - lrel;
      if (r < 0) continue;
      if (r >= 32) break;
      L.bm |= 1u << r;
      if (r < 16 && !(S.list[j].info & kInfoEnd)) {
        L.rst |= 1u << r;
        L.rstbits |= 1u << (r + (S.list[j].info & 7u));
      }
    }
  }
  L.hdr = L.bm & 0xFFFFu;
}

// list index of the module that owns position p (0..15) of the lane
__device__ __forceinline__ int lane_mod_at(const Lane& L, int p) {
  // modules starting at positions in (0, p] of the lane advance the index
  uint32_t below = L.rst & ((2u << p) - 1u);
  int n = __popc(below);
  // a module starting exactly at position 0 is already list entry j0
  if (L.rst & 1u) n -= 1;
  return L.j0 + n;
}

// Backward pass: plausibility of every position and the lane's transfer
// function.  ex[p] = exit offset reached from position p (see kFar/kDead).
template <bool kBounds>
__device__ __forceinline__ void lane_dp(const Shared& S, const VParams& P, Lane& L) {
  // pass 1: every position as a candidate instruction start; all grammar
  // lookups are issued before any is used
  uint32_t e[kLaneWords];
#pragma unroll
  for (int p = 0; p < kLaneWords; ++p) e[p] = tbl_lookup(S.tbl, L.w[p] & 0xFFFFu);
  uint32_t pl_m = 0, far_m = 0, name_m = 0;
#pragma unroll
  for (int p = 0; p < kLaneWords; ++p) {
    const uint32_t wc = L.w[p] >> 16;
    bool pl = tbl_plausible(e[p], wc);
    if (kBounds) {
      // an instruction may not run past its module's end, and module starts
      // (headers) and the batch end are not instruction starts
      uint64_t span = (wc >= 2) ? ((wc - 1 >= 40) ? ~0ull : ((1ull << (wc - 1)) - 1ull)) : 0ull;
      pl = pl && ((((uint64_t)L.bm >> (p + 1)) & span) == 0);
      pl = pl && !((L.hdr >> p) & 1u);
    }
    pl_m |= uint32_t(pl) << p;
    far_m |= uint32_t(pl && wc >= 15u) << p;
    name_m |= ent_str(e[p]) << p;
    if ((p & 3) == 0) L.rolep[p >> 2] = 0;
    L.rolep[p >> 2] |= (e[p] >> 24) << (8 * (p & 3));
  }
  // long instructions (only string-bearing ones can be; rare): kept only when they
  // stay inside their module and the string words before the last hold no
  // NUL byte
  L.far_cand = false;
  if (far_m) {
    uint32_t fm = far_m;
    while (fm) {
      const int p = __builtin_ctz(fm);
      fm &= fm - 1;
      const int64_t pos = L.a + p;
      const uint32_t w0 = P.words[pos];
      const uint32_t wc = w0 >> 16;
      const int jm = kBounds ? lane_mod_at(L, p) : L.j0;
      bool ok = pos + int64_t(wc) <= S.list[jm].end;
      const uint32_t lim = wc - 1 < 18u ? wc - 1 : 18u;
      for (uint32_t k = str_slot(tbl_lookup(S.tbl, w0 & 0xFFFFu)); ok && k < lim; ++k) {
        uint32_t x = P.words[pos + k];
        ok = ((x - 0x01010101u) & ~x & 0x80808080u) == 0;
      }
      if (!ok) {
        pl_m &= ~(1u << p);
        far_m &= ~(1u << p);
      }
    }
    L.far_cand = far_m != 0;
  }
  L.plmask = pl_m;
  L.farmask = far_m;
  L.namemask = name_m;
  // pass 2: exits, backwards; nibble k of R is the exit of position p + k
  uint64_t R = 0xEDCBA98765432100ull;  // positions 16..30: exit offsets 0..13, 14 = far
  bool forced = false;
  uint32_t fval = 0;
#pragma unroll
  for (int p = kLaneWords - 1; p >= 0; --p) {
    const uint32_t wc = L.w[p] >> 16;
    const bool pl = (pl_m >> p) & 1u;
    const bool far = (far_m >> p) & 1u;
    uint32_t val = pl ? (far ? kFar : nib(R, wc & 15u)) : kDead;
    if (kBounds) {
      if ((L.hdr >> p) & 1u) {
        // at a module start the chain restarts after the header; whatever the
        // previous module's chain does, the lane's exit is decided from here
        uint32_t v;
        if (!((L.rst >> p) & 1u)) {
          v = kDead;  // batch end: nothing follows
        } else {
          uint32_t hl = S.list[lane_mod_at(L, p)].info & 7u;
          v = (p + hl < 16u) ? nib(R, hl) : (p + hl - 16u);
        }
        forced = true;
        fval = v;
        val = v;
      } else if (forced) {
        val = fval;
      }
    }
    R = (R | val) << 4;
  }
  L.F = R >> 4;
  // convergence: all entries 0..13 that survive reach the same exit
  const uint64_t kNib14 = 0x00FFFFFFFFFFFFFFull, kOnes14 = 0x0011111111111111ull;
  uint64_t f = L.F & kNib14;
  if (kBounds && L.hdr) {
    L.conv = (fval != kFar);
    L.X = fval;
    return;
  }
  uint64_t nd = ~f & kNib14;
  uint64_t alive = (nd | (nd >> 1) | (nd >> 2) | (nd >> 3)) & kOnes14;
  uint64_t xf = (f ^ (kOnes14 * kFar)) & kNib14;
  uint64_t notfar = (xf | (xf >> 1) | (xf >> 2) | (xf >> 3)) & kOnes14;
  bool anyfar = notfar != kOnes14;
  if (alive == 0) {
    L.conv = true;
    L.X = kDead;
  } else {
    uint32_t X = uint32_t(f >> __builtin_ctzll(alive)) & 15u;
    uint64_t xd = (f ^ (kOnes14 * X)) & kNib14;
    uint64_t differ = (xd | (xd >> 1) | (xd >> 2) | (xd >> 3)) & kOnes14;
    L.conv = !anyfar && (differ & alive) == 0;
    L.X = X;
  }
}

// Forward pass from a known entry: chain nodes of the lane (bit p = position
// p of the window; bit 31 is the sink of dead or long chains).
__device__ __forceinline__ uint32_t lane_forward(const Lane& L, uint32_t ent) {
  uint32_t reach = (ent < 14u ? (1u << ent) : 0u) | L.rstbits;
  const uint32_t okm = L.plmask & ~L.farmask;
#pragma unroll
  for (int p = 0; p < kLaneWords; ++p) {
    uint32_t go = ((reach & okm) >> p) & 1u;
    reach |= go << (p + (L.w[p] >> 16));
  }
  return reach;
}

// ---- lean lane pipeline of the main pass --------------------------------
// Lane i of a wave receives the value of lane i-1 (lane 0 gets `first`).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x, uint32_t first) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(first), int(x), 0x138, 0xF, 0xF, false));
}

// Inclusive wave sum over lanes 0..i (row shifts within 16-lane rows, then
// row broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xF, 0xF, false));
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xF, 0xF, false));
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xF, 0xF, false));
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xF, 0xF, false));
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xA, 0xF, false));
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xC, 0xF, false));
  return x;
}

// Inclusive segmented wave sum (bit 31 of a value: a segment starts there;
// the count restarts at it), by the same row shifts and row broadcasts as
// wave_incl_sum: the combining step is associative, so the same pattern
// applies, and a lane that receives nothing gets 0, which changes nothing.
__device__ __forceinline__ uint32_t seg_step(uint32_t x, uint32_t u) {
  return (x & 0x80000000u) ? x : (x + (u & 0x7FFFFFFFu)) | (u & 0x80000000u);
}
__device__ __forceinline__ uint32_t wave_incl_segsum(uint32_t x) {
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xF, 0xF, false)));
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xF, 0xF, false)));
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xF, 0xF, false)));
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xF, 0xF, false)));
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xA, 0xF, false)));
  x = seg_step(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xC, 0xF, false)));
  return x;
}

// Candidate starts of a lane: grammar lookups of all 16 positions (kept in
// e[] for the result-ID roles), plausibility, long (word count >= 15) and
// string-operand candidates.
template <bool kBounds, bool kNames = true, class SH>
__device__ __forceinline__ void lane_scan(const SH& S, const VParams& P, Lane& L, uint32_t (&e)[kLaneWords]) {
#pragma unroll
  for (int p = 0; p < kLaneWords; ++p) e[p] = tbl_lookup(S.tbl, L.w[p] & 0xFFFFu);
  uint32_t pl_m = 0, far_m = 0, name_m = 0;
#pragma unroll
  for (int p = 0; p < kLaneWords; ++p) {
    const uint32_t wc = L.w[p] >> 16;
    bool pl = tbl_plausible(e[p], wc);
    if (kBounds) {
      uint64_t span = (wc >= 2) ? ((wc - 1 >= 40) ? ~0ull : ((1ull << (wc - 1)) - 1ull)) : 0ull;
      pl = pl && ((((uint64_t)L.bm >> (p + 1)) & span) == 0);
      pl = pl && !((L.hdr >> p) & 1u);
    }
    pl_m |= uint32_t(pl) << p;
    far_m |= uint32_t(pl && wc >= 15u) << p;
    if (kNames) name_m |= ent_str(e[p]) << p;
  }
  L.far_cand = false;
  if (far_m) {
    uint32_t fm = far_m;
    while (fm) {
      const int p = __builtin_ctz(fm);
      fm &= fm - 1;
      const int64_t pos = L.a + p;
      const uint32_t w0 = P.words[pos];
      const uint32_t wc = w0 >> 16;
      const int jm = kBounds ? lane_mod_at(L, p) : L.j0;
      bool ok = pos + int64_t(wc) <= S.list[jm].end;
      const uint32_t lim = wc - 1 < 18u ? wc - 1 : 18u;
      for (uint32_t k = str_slot(tbl_lookup(S.tbl, w0 & 0xFFFFu)); ok && k < lim; ++k) {
        uint32_t x = P.words[pos + k];
        ok = ((x - 0x01010101u) & ~x & 0x80808080u) == 0;
      }
      if (!ok) {
        pl_m &= ~(1u << p);
        far_m &= ~(1u << p);
      }
    }
    L.far_cand = far_m != 0;
  }
  L.plmask = pl_m;
  L.farmask = far_m;
  L.namemask = name_m;
}

// Lane transfer function by the backward nibble recurrence (lanes with a
// module start or a long candidate, or whose candidates form more than one
// chain).
template <class SH>
__device__ __forceinline__ void lane_dp_full(const SH& S, Lane& L) {
  const uint32_t pl_m = L.plmask, far_m = L.farmask;
  uint64_t R = 0xEDCBA98765432100ull;  // positions 16..30: exit offsets 0..13, 14 = far
  bool forced = false;
  uint32_t fval = 0;
#pragma unroll
  for (int p = kLaneWords - 1; p >= 0; --p) {
    const uint32_t wc = L.w[p] >> 16;
    const bool pl = (pl_m >> p) & 1u;
    const bool far = (far_m >> p) & 1u;
    uint32_t val = pl ? (far ? kFar : nib(R, wc & 15u)) : kDead;
    if ((L.hdr >> p) & 1u) {
      uint32_t v;
      if (!((L.rst >> p) & 1u)) {
        v = kDead;
      } else {
        uint32_t hl = S.list[lane_mod_at(L, p)].info & 7u;
        v = (p + hl < 16u) ? nib(R, hl) : (p + hl - 16u);
      }
      forced = true;
      fval = v;
      val = v;
    } else if (forced) {
      val = fval;
    }
    R = (R | val) << 4;
  }
  L.F = R >> 4;
  const uint64_t kNib14 = 0x00FFFFFFFFFFFFFFull, kOnes14 = 0x0011111111111111ull;
  uint64_t f = L.F & kNib14;
  if (L.hdr) {
    L.conv = (fval != kFar);
    L.X = fval;
    return;
  }
  uint64_t nd = ~f & kNib14;
  uint64_t alive = (nd | (nd >> 1) | (nd >> 2) | (nd >> 3)) & kOnes14;
  uint64_t xf = (f ^ (kOnes14 * kFar)) & kNib14;
  uint64_t notfar = (xf | (xf >> 1) | (xf >> 2) | (xf >> 3)) & kOnes14;
  bool anyfar = notfar != kOnes14;
  if (alive == 0) {
    L.conv = true;
    L.X = kDead;
  } else {
    uint32_t X = uint32_t(f >> __builtin_ctzll(alive)) & 15u;
    uint64_t xd = (f ^ (kOnes14 * X)) & kNib14;
    uint64_t differ = (xd | (xd >> 1) | (xd >> 2) | (xd >> 3)) & kOnes14;
    L.conv = !anyfar && (differ & alive) == 0;
    L.X = X;
  }
}

// Transfer function of a lane.  Fast case (no module start in the lane, no
// long candidate): follow the chain from the first candidate among entry
// offsets 0..13; when every candidate there lies on that chain, each entry
// either joins it (same exit) or is not a plausible start (dead), so the
// lane's exit does not depend on its entry.  Otherwise the nibble
// recurrence decides.
template <class SH>
__device__ __forceinline__ void lane_chain(const SH& S, Lane& L) {
  L.slow = L.hdr != 0 || L.farmask != 0;
  if (!L.slow) {
    const uint32_t pl_m = L.plmask;
    const uint32_t cand = pl_m & 0x3FFFu;
    uint32_t reach = cand ? (1u << __builtin_ctz(cand)) : 0u;
#pragma unroll
    for (int p = 0; p < kLaneWords; ++p) {
      const uint32_t go = ((reach & pl_m) >> p) & 1u;
      reach |= go << ((p + (L.w[p] >> 16)) & 31u);  // word counts <= 14 here: p + wc <= 29
    }
    L.reach0 = reach;
    if ((cand & ~reach) == 0) {
      const uint32_t beyond = reach >> 16;
      L.conv = true;
      L.X = beyond ? uint32_t(__builtin_ctz(beyond)) : kDead;
    } else {
      L.slow = true;
    }
  }
  if (L.slow) lane_dp_full(S, L);
}

// Chain nodes of a fast lane from its exact entry (see lane_forward).
__device__ __forceinline__ uint32_t fast_reach(const Lane& L, uint32_t ent) {
  if (ent >= 14u) return 0u;
  if ((L.reach0 >> ent) & 1u) return L.reach0 & (~0u << ent);
  return 1u << ent;  // not a plausible start: the chain ends here with an error
}

__device__ __forceinline__ void report_error(ModState& ms, uint32_t rel, uint32_t code, uint32_t rank) {
  atomicMin(&ms.err_key, ((unsigned long long)rel << 8) | code);
  atomicMin(&ms.err_rank, ((unsigned long long)rel << 32) | rank);
}

// ID check of one ID word in module ms (bitmap or hash mode).
__device__ __forceinline__ void id_check(const VParams& P, const LEnt& le, uint32_t v, bool is_def, uint32_t* flags,
                                         uint32_t* defcnt) {
  if (v == 0u || v >= le.bound) {
    atomicOr(flags, kModOOB);
    return;
  }
  unsigned long long* base = P.idmap + le.off;
  if (le.info & kInfoSparse) {
    uint32_t old = hash_insert(base, le.end - le.off, v, is_def ? 1u : 2u);
    if (is_def && (old & 1u)) atomicOr(flags, kModDup);
    return;
  }
  if (!is_def) return;
  unsigned long long bit = 1ull << (v & 63u);
  unsigned long long old = atomicOr(&base[v >> 6], bit);
  if (old & bit) atomicOr(flags, kModDup);
  else atomicAdd(defcnt, 1u);
}

// Serial path for one tile (thread 0): exact walk from entry E.
template <bool kSem, bool kIdx>
__device__ __forceinline__ void serial_tile(Shared& S, const VParams& P, long long t, int64_t t0, int64_t t1, uint32_t E) {
  // called by the whole block; wave 0 fetches the count prefix, thread 0 walks
  if (threadIdx.x < 64) {
    uint32_t pre = (P.mod_off[P.tfm[t]] == t0) ? 0u : count_lookback(P, P.tileB, t);
    if (threadIdx.x == 0) S.prefix = pre;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t m = P.tfm[t];
  int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
  int64_t pos;
  uint32_t cnt;
  if (off == t0) {
    int64_t n = end - off;
    pos = off + (n < 5 ? n : 5);
    cnt = 0;
  } else {
    pos = (E == kExitDead) ? -1 : t0 + int64_t(E);
    cnt = S.prefix;
  }
  bool far = false;
  for (;;) {
    ModState& ms = P.mods[m];
    bool hdr_ok = (ms.flags & kModHdrOk) != 0;
    LEnt le;
    le.off = off;
    le.end = end;
    le.bound = ms.bound;
    le.info = (ms.flags & kModSparse) ? kInfoSparse : 0u;
    while (pos >= 0 && pos < end && pos < t1) {
      uint32_t code = start_code(P.words, S.tbl, pos, end);
      uint32_t rel = uint32_t(pos - off);
      if (code) {
        report_error(ms, rel, code, cnt);
        pos = -1;
        break;
      }
      uint32_t w0 = P.words[pos];
      uint32_t wc = w0 >> 16, op = w0 & 0xFFFFu;
      if (wc >= 15u) far = true;
      if (kIdx && hdr_ok) {
        P.idx_off[off + cnt] = rel;
        P.idx_op[off + cnt] = uint16_t(op);
      }
      if (kSem && hdr_ok) {
        uint32_t e = tbl_lookup(S.tbl, op);
        if (ent_rules(e)) atomicOr(&ms.flags, ent_rules(e) << kModRuleShift);
        uint32_t dm = (e >> 24) & 0xFu, um = (e >> 28) & 0xFu;
        for (uint32_t s = 1; s <= 4; ++s) {
          bool d = (dm >> (s - 1)) & 1u, u = (um >> (s - 1)) & 1u;
          if (d || u) id_check(P, le, P.words[pos + s], d, &ms.flags, &ms.def_count);
        }
      }
      ++cnt;
      pos += wc;
    }
    if (end <= t1) {
      ms.n_total = cnt;  // the module's last word is in this tile
      int64_t m2 = m + 1;
      while (m2 < P.M && P.mod_off[m2 + 1] == P.mod_off[m2]) ++m2;
      if (m2 >= P.M) {
        pos = -1;
        m = -1;
        break;
      }
      m = m2;
      off = P.mod_off[m];
      end = P.mod_off[m + 1];
      cnt = 0;
      if (off >= t1) {
        pos = -1;
        break;
      }
      int64_t n = end - off;
      pos = off + (n < 5 ? n : 5);
      continue;
    }
    break;
  }
  uint32_t exitv = (pos >= 0) ? uint32_t(pos - t1) : kExitDead;
  st_state(&P.tileA[(t) * kStateStride], kFlagFull | (far ? kFarBit : 0ull) | exitv);
  st_state(&P.tileB[(t) * kStateStride], kFlagFull | cnt);
}

}  // namespace

// ---------------------------------------------------------------------------
// plan: header stage, per-module state, tile -> module map, tile states and
// ID-set regions cleared.
__global__ __launch_bounds__(256) void k_plan(VParams P, int64_t chunk) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  if (gtid == 0) {
    P.ctrl[kCtlClaim] = 0;
    P.ctrl[kCtlClaim2] = 0;
    P.ctrl[kCtlPass2] = 0;
    P.ctrl[kCtlSpinErr] = 0;
    P.ctrl[kCtlMode] = 0;
    P.ctrl[kCtlClaimR] = 0;
    P.ctrl[kCtlDoneR] = 0;
    P.ctrl[kCtlP2Tiles] = 0;
    P.ctrl[kCtlP2Done] = 0;
  }
  for (int64_t m = gtid; m < P.M; m += nth) {
    int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
    int64_t n = end - off;
    const uint32_t* w = P.words + off;
    uint32_t code = 0, err = 0xFFFFFFFFu, bound = 0;
    if (n < 5) {
      code = SPV_E_TRUNCATED_HEADER;
      err = uint32_t(n);
    } else if (w[0] != kMagic) {
      code = SPV_E_BAD_MAGIC;
      err = 0;
    } else if ((w[1] & 0xFF0000FFu) != 0 || ((w[1] >> 16) & 0xFFu) != 1u || ((w[1] >> 8) & 0xFFu) > 6u) {
      code = SPV_E_BAD_VERSION;
      err = 1;
    } else if (w[4] != 0) {
      code = SPV_E_BAD_SCHEMA;
      err = 4;
    }
    if (n >= 4) bound = w[3];
    ModState s;
    s.err_key = ~0ull;
    s.err_rank = ~0ull;
    s.flags = (code == 0 ? kModHdrOk : 0u) | ((uint64_t(bound) > 64ull * uint64_t(n)) ? kModSparse : 0u);
    s.def_count = 0;
    s.n_total = 0;
    s.bound = bound;
    s.hdr_code = code;
    s.hdr_err = err;
    s.pad[0] = s.pad[1] = 0;
    P.mods[m] = s;
  }
  for (int64_t b = gtid; b < P.n_tiles / kResolveTiles + 2; b += nth) P.rstate[b * kStateStride] = 0;
  for (int64_t t = gtid; t < P.n_tiles; t += nth) {
    P.tileA[(t) * kStateStride] = 0;
    P.tileB[(t) * kStateStride] = 0;
    // module containing word t * T: last m with mod_off[m] <= tT
    P.tfm[t] = int32_t(find_module(P.mod_off, P.M, t * kTileWords));
  }
  if (!P.semantic) return;
  // clear the ID sets of header-valid modules, chunk by chunk of idmap
  __shared__ int64_t s_m0;
  int64_t n_chunks = (P.W + chunk - 1) / chunk;
  for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    int64_t cs = c * chunk, ce = cs + chunk < P.W ? cs + chunk : P.W;
    if (threadIdx.x == 0) s_m0 = find_module(P.mod_off, P.M, cs);
    __syncthreads();
    for (int64_t m = s_m0; m < P.M; ++m) {
      int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
      if (off >= ce) break;
      int64_t n = end - off;
      if (n < 5) continue;
      const uint32_t* w = P.words + off;
      bool ok = w[0] == kMagic && (w[1] & 0xFF0000FFu) == 0 && ((w[1] >> 16) & 0xFFu) == 1u &&
                ((w[1] >> 8) & 0xFFu) <= 6u && w[4] == 0;
      if (!ok) continue;
      uint64_t bound = w[3];
      int64_t need = (bound > 64ull * uint64_t(n)) ? n : int64_t((bound + 63) / 64);
      int64_t zs = off > cs ? off : cs, ze = off + need < ce ? off + need : ce;
      for (int64_t i = zs + threadIdx.x; i < ze; i += blockDim.x) P.idmap[i] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Chain pass: for every tile, independently of all other tiles, the lane
// transfer functions, each lane's exact instruction starts and parse-error
// nodes (every lane but the tile's first, whose entry comes from the previous
// tile), and a summary: the tile's exit (it does not depend on the tile's
// entry), the first lane's candidate chain, and the per-module start counts.
// Tiles this cannot settle (crowded, a long instruction candidate, a chain
// that stays ambiguous over a whole lane) are flagged, and the batch then
// takes the single-pass walk.
struct ChainShared {
  uint32_t tbl[257];
  LEnt list[kListMax];
  int K;
  int crowded;
  uint32_t wagg[kWaves];
  uint32_t wflags[kWaves];
  uint32_t wcnt[kWaves];
  uint32_t whead[kWaves];
  uint32_t bad;
  LEnt cache;
  int cache_ok;
};

// (6 waves per SIMD: the pass has little shared state, so more resident
// blocks hide the load latency of each tile)
__global__ __launch_bounds__(kBlock, 24 / kWaves) void k_chain(VParams P) {
  __shared__ ChainShared S;
  if (threadIdx.x == 0) S.cache_ok = 0;
  init_table(S.tbl);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  for (long long t = blockIdx.x; t < P.n_tiles; t += gridDim.x) {
    const int64_t t0 = t * kTileWords;
    const int64_t t1 = (t0 + kTileWords < P.W) ? t0 + kTileWords : P.W;
    Lane L;
    L.a = t0 + int64_t(tid) * kLaneWords;
    if (L.a + kLaneWords <= P.W) {
      const uint4* src = reinterpret_cast<const uint4*>(P.words + L.a);
#pragma unroll
      for (int i = 0; i < kLaneWords / 4; ++i) {
        uint4 v = src[i];
        L.w[4 * i] = v.x;
        L.w[4 * i + 1] = v.y;
        L.w[4 * i + 2] = v.z;
        L.w[4 * i + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kLaneWords; ++i) L.w[i] = (L.a + i < P.W) ? P.words[L.a + i] : 0u;
    }
    __syncthreads();  // the previous tile is done with the shared state
    if (wave == 0) build_list(S, P, t, t0, t1);
    if (tid == 0) S.bad = 0;
    __syncthreads();
    uint32_t* sum = P.tsum + 4 * t;
    if (S.crowded) {
      if (tid == 0) sum[0] = kSumFallback;
      continue;
    }
    const int32_t lrel = tid * kLaneWords;
    lane_window(S, L, lrel);
    uint32_t e[kLaneWords];
    const bool any_bounds = __ballot(L.bm != 0) != 0;
    if (any_bounds) lane_scan<true, false>(S, P, L, e);
    else lane_scan<false, false>(S, P, L, e);
    lane_chain(S, L);

    // exits inside each wave, independent of the wave entry where possible
    bool known = L.conv;
    uint32_t ex = L.conv ? L.X : 0u;
    for (;;) {
      uint32_t pex = wave_shr1(ex, 0u);
      bool pk = wave_shr1(known ? 1u : 0u, 0u) != 0;
      bool nw = !known && pk;
      if (nw) {
        ex = apply_fn(L.F, pex);
        known = true;
      }
      if (__ballot(nw) == 0) break;
    }
    // the tile's first lane must not pass its entry on to the next lane
    if (wave == 0 && __ballot(!known) != 0 && lane == 0) S.bad = 1;
    const bool wave_far = __ballot(L.far_cand) != 0;
    if (lane == 63) S.wagg[wave] = known ? ex : 0xFFu;
    if (lane == 0) S.wflags[wave] = wave_far ? 1u : 0u;
    __syncthreads();
    bool bad = S.bad != 0;
    for (int w = 0; w < kWaves; ++w) {
      bad |= S.wflags[w] != 0;
      if (w >= 1 && S.wagg[w - 1] == 0xFFu) bad = true;
    }
    const uint32_t X = S.wagg[kWaves - 1];
    if (X == 0xFFu || X == kFar) bad = true;
    if (bad) {
      if (tid == 0) sum[0] = kSumFallback;
      continue;
    }
    // entries of every lane but the tile's first
    const uint32_t Ew = (wave == 0) ? kDead : S.wagg[wave - 1];
    if (lane == 0 && wave > 0 && !known) {
      ex = apply_fn(L.F, Ew);
      known = true;
    }
    for (;;) {
      uint32_t pex = wave_shr1(ex, 0u);
      bool pk = wave_shr1(known ? 1u : 0u, 0u) != 0;
      bool nw = !known && pk;
      if (nw) {
        ex = apply_fn(L.F, pex);
        known = true;
      }
      if (__ballot(nw) == 0) break;
    }
    const uint32_t ent = wave_shr1(ex, Ew);
    uint32_t starts, errs, mask0 = 0;
    bool ok0 = true;
    if (tid != 0) {
      const uint32_t reach = L.slow ? lane_forward(L, ent == kDead ? 99u : ent) : fast_reach(L, ent);
      starts = reach & L.plmask & ~L.farmask & ~L.hdr & 0xFFFFu;
      errs = reach & ~L.plmask & ~L.hdr & 0xFFFFu;
    } else {
      // first lane: the chain from its entry, up to its first module start,
      // is kept as a candidate mask (every candidate there on one chain, so an
      // entry either joins it or is not a plausible start); starts after a
      // module start do not depend on the entry
      if (!L.slow) {
        // plausible chain nodes (bits 0..15) and the node where the chain
        // meets an invalid start (bits 16..31; the chain stops there)
        mask0 = (L.reach0 & L.plmask & 0xFFFFu) | ((L.reach0 & ~L.plmask & 0xFFFFu) << 16);
        starts = 0;
        errs = 0;
      } else if (L.hdr && L.farmask == 0) {
        const uint32_t h0 = uint32_t(__builtin_ctz(L.hdr));
        const uint32_t hm = (1u << h0) - 1u;
        const uint32_t cand = L.plmask & 0x3FFFu & hm;
        uint32_t reach = cand ? (1u << __builtin_ctz(cand)) : 0u;
#pragma unroll
        for (int p = 0; p < kLaneWords; ++p) {
          const uint32_t go = ((reach & L.plmask & hm) >> p) & 1u;
          reach |= go << ((p + (L.w[p] >> 16)) & 31u);
        }
        ok0 = (cand & ~reach) == 0;
        mask0 = (reach & L.plmask & hm) | ((reach & ~L.plmask & hm) << 16);
        const uint32_t fr = lane_forward(L, 99u);
        starts = fr & L.plmask & ~L.farmask & ~L.hdr & 0xFFFFu;
        errs = fr & ~L.plmask & ~L.hdr & 0xFFFFu;
      } else {
        ok0 = false;
        starts = 0;
        errs = 0;
      }
    }
    // per-module counts: segmented by module starts (as in the main pass);
    // a plain sum when no module starts in the tile
    const uint32_t rst = L.rst;
    const uint32_t nst = __popc(starts);
    uint32_t inc;
    if (S.K > 1 || S.list[0].rel >= 0) {
      uint32_t cval;
      if (rst) {
        int last = 31 - __builtin_clz(rst);
        cval = 0x80000000u | uint32_t(__popc(starts & ~((2u << last) - 1u)));
      } else {
        cval = nst;
      }
      inc = cval;
      // (rounds of lane shifts: the row-broadcast form of this scan costs the
      // pass more registers than it has)
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(inc, d);
        if (lane >= d) inc = seg_step(inc, u);
      }
    } else {
      inc = wave_incl_sum(nst);
    }
    const uint32_t excl = wave_shr1(inc, 0u);
    if (lane == 63) S.wcnt[wave] = inc;
    if (tid == 0 && !ok0) S.bad = 1;
    __syncthreads();
    if (S.bad) {
      if (tid == 0) sum[0] = kSumFallback;
      continue;
    }
    if (!(S.K > 1 || S.list[0].rel >= 0)) {
      // no module starts in the tile: every start belongs to the module open
      // at its start, so the count of those starts is the tile total, and
      // no further barrier is needed (the next tile begins with one)
      P.lst[t * kBlock + tid] = starts | (errs << 16);
      if (tid == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += S.wcnt[w];
        sum[0] = X;
        sum[1] = mask0;
        sum[2] = tot;
        sum[3] = tot;
      }
      continue;
    }
    uint32_t wpre = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      uint32_t v = S.wcnt[w];
      if (w < wave) wpre = (v & 0x80000000u) ? v : (wpre + v) | (wpre & 0x80000000u);
      tot = (v & 0x80000000u) ? v : (tot + v) | (tot & 0x80000000u);
    }
    const uint32_t lex = (excl & 0x80000000u) ? excl : (wpre + excl) | (wpre & 0x80000000u);
    // starts of the module open at the tile start
    uint32_t head = 0;
    if (!(lex & 0x80000000u)) head = rst ? uint32_t(__popc(starts & ((1u << __builtin_ctz(rst)) - 1u))) : nst;
    head = wave_sum_u32(head);
    if (lane == 0) S.whead[wave] = head;
    P.lst[t * kBlock + tid] = starts | (errs << 16);
    __syncthreads();
    if (tid == 0) {
      uint32_t c_head = 0;
      for (int w = 0; w < kWaves; ++w) c_head += S.whead[w];
      sum[0] = X | ((S.list[0].rel == 0) ? kSumModStart : 0u) | ((tot & 0x80000000u) ? kSumReset : 0u);
      sum[1] = mask0;
      sum[2] = c_head;
      sum[3] = tot & 0x7FFFFFFFu;
    }
  }
}

// Resolve pass: each tile's exact entry (the previous tile's exit) and the
// count of starts of the module open at its start that lie before it: a
// segmented scan over the tiles (blocks of kResolveTiles tiles, claimed in
// order, chained by a decoupled look-back).  The last block to finish sets
// kCtlMode when no tile was flagged and every exit is a plain offset.
constexpr int kResolveBlock = kResolveTiles;

__global__ __launch_bounds__(kResolveBlock) void k_resolve(VParams P) {
  __shared__ uint32_t s_bid;
  __shared__ uint32_t s_wagg[kResolveBlock / 64];
  __shared__ uint32_t s_pre;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(&P.ctrl[kCtlClaimR], 1u);
  __syncthreads();
  const long long bid = s_bid;
  const long long t = bid * kResolveBlock + tid;
  const bool real = t < P.n_tiles;
  const uint4* T = reinterpret_cast<const uint4*>(P.tsum);
  const uint4 v = real ? T[t] : make_uint4(0u, 0u, 0u, 0u);
  const uint32_t px = (real && t > 0) ? T[t - 1].x : 0u;
  bool bad = false;
  uint32_t E = kExitDead;
  if (real && !(v.x & kSumModStart) && t > 0) {
    E = px & 0xFFu;
    if (px & kSumFallback) bad = true;
    if (E == kDead) E = kExitDead;
    else if (E >= kFar) bad = true;
  }
  if (real && (v.x & kSumFallback)) bad = true;
  const uint32_t c0 = (E < 14u && ((v.y >> E) & 1u)) ? uint32_t(__popc((v.y & 0xFFFFu) >> E)) : 0u;
  const bool rs = real && (v.x & kSumReset);
  const uint32_t val = real ? (rs ? v.w : v.z + c0) : 0u;
  // inclusive segmented scan (bit 31: a module starts in the range)
  const uint32_t inc = wave_incl_segsum((rs ? 0x80000000u : 0u) | val);
  if (lane == 63) s_wagg[wave] = inc;
  __syncthreads();
  uint32_t wpre = 0, btot = 0;
  for (int w = 0; w < kResolveBlock / 64; ++w) {
    uint32_t a = s_wagg[w];
    if (w < wave) wpre = (a & 0x80000000u) ? a : (wpre + a) | (wpre & 0x80000000u);
    btot = (a & 0x80000000u) ? a : (btot + a) | (btot & 0x80000000u);
  }
  if (tid == 64)
    st_state(&P.rstate[bid * kStateStride], kFlagAgg | ((btot & 0x80000000u) ? kResetBit : 0ull) | (btot & 0x7FFFFFFFu));
  if (wave == 0) {
    const uint32_t pre = count_lookback(P, P.rstate, bid);
    if (lane == 0) {
      s_pre = pre;
      const uint32_t incl = (btot & 0x80000000u) ? (btot & 0x7FFFFFFFu) : pre + btot;
      st_state(&P.rstate[bid * kStateStride], kFlagFull | incl);
    }
  }
  const bool any_bad = __syncthreads_or(bad);
  // exclusive value of this tile within the block, then with the block prefix
  uint32_t ex = wave_shr1(inc, 0u);
  ex = (ex & 0x80000000u) ? ex : (wpre + ex) | (wpre & 0x80000000u);
  const uint32_t prefix = (ex & 0x80000000u) ? (ex & 0x7FFFFFFFu) : s_pre + ex;
  if (real) reinterpret_cast<uint2*>(P.tres)[t] = make_uint2(E, (v.x & kSumModStart) ? 0u : prefix);
  if (tid == 0) {
    const uint32_t old = atomicAdd(&P.ctrl[kCtlDoneR], 1u + (any_bad ? (1u << 20) : 0u));
    if ((old & 0xFFFFFu) == gridDim.x - 1 && (old >> 20) == 0 && !any_bad) P.ctrl[kCtlMode] = kModeResolved;
  }
}

// ---------------------------------------------------------------------------
// main pass: boundary recovery, parse checks, instruction index, result-ID
// checks.
// kRes: entries and count prefixes come from the resolve pass (tiles in
// block order, no look-back, no waiting on other tiles); otherwise the
// single-pass walk with decoupled look-back.
template <bool kSem, bool kIdx, bool kRes, class SH, bool kRules = false>
__device__ __forceinline__ void main_body(SH& S, const VParams& P) {
  // (the resolved walk accounts the module-level rules only in its rules
  // instantiation: the code costs registers even when not run; the
  // single-pass walk checks the option at run time)
  const bool rules_on = kRes ? kRules : (P.rules != 0);
  if (threadIdx.x == 0) S.cache_ok = 0;
  init_table(S.tbl);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  // LDS copy of the tile's words, then the next tile's first words, with a
  // pad word after every 16 (twx).  (A column-major copy measured slower in
  // the resolved walk, 199 against 183 us: its 16-byte stores conflict.)
  auto tw_store4 = [&](int l, int i, const uint4& v) {
    const int q = twx(l * kLaneWords + 4 * i);
    S.tw[q] = v.x;
    S.tw[q + 1] = v.y;
    S.tw[q + 2] = v.z;
    S.tw[q + 3] = v.w;
  };
  // the first tile is claimed here, each later one near the end of the tile
  // before it
  if (tid == 0)
    S.tnext = (kRes || P.sched_static) ? (long long)blockIdx.x : (long long)atomicAdd(&P.ctrl[kCtlClaim], 1u);
  // result-ID window flush of the previous tile: issued at its end, its
  // returned words are examined at the start of the next tile
  // (windows: SH::kWins of SH::kWinW words; thread tid flushes word
  // k * kBlock + tid - kFlOff of slot k, whose window is aligned to its wave)
  constexpr int kWW = SH::kWinW;
  constexpr int kNW = SH::kWins * kWW;
  constexpr int kSlots = (kNW + kBlock - 1) / kBlock;
  constexpr int kFlOff = kNW < kBlock ? kBlock - kNW : 0;
  unsigned long long fl_old[kSlots], fl_bits[kSlots];
  int32_t fl_mk[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    fl_old[k] = 0;
    fl_bits[k] = 0;
    fl_mk[k] = -1;
  }
  // new result IDs of the window are counted per block and added to the
  // module's count when the module changes or the block ends (one device
  // atomic per module run instead of one per tile)
  int64_t dc_mod = -1;
  uint32_t dc_cnt = 0;
  if (tid == 0) {
    S.rl_mod = -1;
    S.rl_bits = 0;
  }
  if constexpr (kRes) {
    if (tid == 0) S.nbm1 = kNoBound;
  }
  // words of the next tile, loaded during the tail of the current one
  uint4 pf[kLaneWords / 4];
  uint32_t pf_tail = 0;  // (threads below kTwTail) a word past the next tile's end
  long long pf_tile = -1;

  for (;;) {
    __syncthreads();
    const long long t = S.tnext;
    // fold the previous tile's flush into its module's state
    if (kSem) {
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        if (fl_mk[k] >= 0) {  // the same in the whole wave
          const bool dup = (fl_old[k] & fl_bits[k]) != 0;
          uint32_t cnt = wave_sum_u32(uint32_t(__popcll(fl_bits[k] & ~fl_old[k])));
          const bool d = __ballot(dup) != 0;
          if (lane == 0) {
            if (cnt) {
              if (fl_mk[k] != dc_mod) {
                if (dc_cnt) atomicAdd(&P.mods[dc_mod].def_count, dc_cnt);
                dc_mod = fl_mk[k];
                dc_cnt = 0;
              }
              dc_cnt += cnt;
            }
            if (d) atomicOr(&P.mods[fl_mk[k]].flags, kModDup);
          }
        }
        fl_mk[k] = -1;
      }
    }
    if (t >= P.n_tiles) break;
    const int64_t t0 = t * kTileWords;
    const int64_t t1 = (t0 + kTileWords < P.W) ? t0 + kTileWords : P.W;

    Lane L;
    L.a = t0 + int64_t(tid) * kLaneWords;
    // coalesced 16-byte loads of the lane's 16 words, kept in registers and
    // in LDS (strings and rare paths read the LDS copy)
    // (pf_tile is the same in every thread, so the prefetched branch is
    // taken by the whole block)
    if (pf_tile == t) {
#pragma unroll
      for (int i = 0; i < kLaneWords / 4; ++i) {
        const uint4 v = pf[i];
        L.w[4 * i] = v.x;
        L.w[4 * i + 1] = v.y;
        L.w[4 * i + 2] = v.z;
        L.w[4 * i + 3] = v.w;
        tw_store4(tid, i, v);
      }
    } else if (L.a + kLaneWords <= P.W) {
      const uint4* src = reinterpret_cast<const uint4*>(P.words + L.a);
      // resolved walk, a tile inside the module of the block's previous
      // tile: the bound test of all 16 words as they arrive (bit p: word p
      // is 0 or at least the bound), kept in the pad word after the lane's
      // words for the ID checks
      uint32_t nb = kNoBound;
      if constexpr (kRes && kSem) nb = S.nbm1;
      uint32_t badw = 0;
#pragma unroll
      for (int i = 0; i < kLaneWords / 4; ++i) {
        const uint4 v = src[i];
        L.w[4 * i] = v.x;
        L.w[4 * i + 1] = v.y;
        L.w[4 * i + 2] = v.z;
        L.w[4 * i + 3] = v.w;
        tw_store4(tid, i, v);
        badw |= (uint32_t(v.x - 1u >= nb) | (uint32_t(v.y - 1u >= nb) << 1) | (uint32_t(v.z - 1u >= nb) << 2) |
                 (uint32_t(v.w - 1u >= nb) << 3)) << (4 * i);
      }
      if constexpr (kRes && kSem) {
        if (nb != kNoBound) S.tw[tid * (kLaneWords + 1) + kLaneWords] = badw;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kLaneWords; ++i) {
        L.w[i] = (L.a + i < P.W) ? P.words[L.a + i] : 0u;
        S.tw[twx(tid * kLaneWords + i)] = L.w[i];
      }
    }
    if (tid < kTwTail) S.tw[twx(kTileWords + tid)] = (pf_tile == t) ? pf_tail : ((t1 + tid < P.W) ? P.words[t1 + tid] : 0u);
    // resolved walk: the chain pass's lane record and the tile's resolved
    // entry, count prefix and first-lane chain, loaded with the words (the
    // per-tile values through scalar loads)
    uint32_t h_rec = 0, h_pre = 0, h_E = 0, h_m0 = 0;
    if constexpr (kRes) {
      h_rec = P.lst[t * kBlock + tid];
      const uint32_t tl = __builtin_amdgcn_readfirstlane(uint32_t(t));
      const uint32_t th = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(t) >> 32));
      const long long tu = (long long)(((uint64_t)th << 32) | tl);
      h_pre = P.tres[2 * tu + 1];
      h_E = P.tres[2 * tu];
      h_m0 = P.tsum[4 * tu + 1];
    }
    if (wave == 0) build_list(S, P, t, t0, t1);
    if (tid < kListMax) {
      S.modflags[tid] = 0;
      S.moddef[tid] = 0;
      if constexpr (!kRes) S.slot0[tid] = 0xFFFFFFFFu;
    }
    if (kSem) {
      for (int i = tid; i < kNW; i += kBlock) S.win[i] = 0;
      if (tid < SH::kWins) S.wmin[tid] = 0xFFFFFFFFu;
    }
    if (tid < kTileWords / 32) S.badb[tid] = 0;
    if (tid == 0) {
      S.serial = 0;
      S.nname = 0;
    }
    __syncthreads();

    // The next tile: block order (static) or claimed now by the last wave,
    // whose answer is read before the scans barrier; the next tile's words
    // are then loaded during the second half of this tile.
    long long claim_tn = 0;
    if (tid == kBlock - 1)
      claim_tn = (kRes || P.sched_static) ? t + gridDim.x : (long long)atomicAdd(&P.ctrl[kCtlClaim], 1u);

    // Every way into the serial path leaves the block below with go_serial
    // set (one call site keeps a single inlined copy of it).
    uint32_t serialE = kExitDead;
    bool go_serial = false;
    do {
    if (!kRes && S.crowded) {
      if (tid == 0) st_state(&P.tileA[(t) * kStateStride], kFlagAgg | kFarBit | kFar);
      if (wave == 0) serialE = (S.list[0].rel == 0) ? kExitDead : entry_lookback(P, t);
      go_serial = true;
      break;
    }

    if (tid == 0) {
      // module whose result IDs go through the LDS window: the one at the
      // middle of the tile, when its IDs are kept in a bitmap
      int j = list_find(S, kTileWords / 2);
      const LEnt& le = S.list[j];
      S.jw = (le.mod >= 0 && (le.info & kInfoHdrOk) && !(le.info & kInfoSparse)) ? j : -1;
    }
    const int32_t lrel = tid * kLaneWords;
    lane_window(S, L, lrel);
    uint32_t e[kLaneWords];
    uint32_t starts, errs;
    uint32_t reach = 0, ent = 0, E = kExitDead;
    uint32_t res_pre = 0;
    if constexpr (kRes) {
      // starts and parse-error nodes from the chain pass; the first lane adds
      // the part of its candidate chain that its resolved entry reaches
      const uint32_t rec = h_rec;
      res_pre = h_pre;
      starts = rec & 0xFFFFu;
      errs = rec >> 16;
      if (tid == 0) {
        const uint32_t Et = h_E;
        const uint32_t m0 = h_m0;
        const uint32_t h0 = L.hdr ? uint32_t(__builtin_ctz(L.hdr)) : 16u;
        if (Et < 14u && Et < h0) {
          if ((m0 >> Et) & 1u) {
            // the entry is on the first lane's candidate chain: its starts
            // and its error node from the entry on
            starts |= m0 & 0xFFFFu & (~0u << Et);
            errs |= (m0 >> 16) & (~0u << Et);
          }
          else errs |= 1u << Et;
        }
      }
    } else {
      const bool any_bounds = __ballot(L.bm != 0) != 0;
      if (any_bounds) lane_scan<true>(S, P, L, e);
      else lane_scan<false>(S, P, L, e);
      lane_chain(S, L);

      // ---- wave-level resolution independent of the wave entry
      bool known = L.conv;
      uint32_t ex = L.conv ? L.X : 0u;
      for (;;) {
        uint32_t pex = wave_shr1(ex, 0u);
        bool pk = wave_shr1(known ? 1u : 0u, 0u) != 0;
        bool nw = !known && pk;
        if (nw) {
          ex = apply_fn(L.F, pex);
          known = true;
        }
        if (__ballot(nw) == 0) break;
      }
      const bool wave_far = __ballot(L.far_cand) != 0;
      if (lane == 63) S.wagg[wave] = known ? ex : 0xFFu;
      if (lane == 0) S.wflags[wave] = wave_far ? 1u : 0u;
      __syncthreads();

      // ---- tile aggregate (published from wave 1: wave 0's polls below then
      // do not wait for this store to complete)
      if (tid == 64) {
        bool any_far = false, serial = false;
        for (int w = 0; w < kWaves; ++w) {
          any_far |= (S.wflags[w] & 1u) != 0;
          if (w >= 1 && S.wagg[w - 1] == 0xFFu) serial = true;  // a wave entry that needs the previous wave's entry
        }
        uint32_t X = S.wagg[kWaves - 1];
        uint32_t agg = (serial || any_far || X == 0xFFu || X == kFar) ? kFar : X;
        st_state(&P.tileA[(t) * kStateStride], kFlagAgg | (any_far ? kFarBit : 0ull) | agg);
        S.serial = serial ? 1 : 0;
      }
      // ---- exact tile entry
      if (wave == 0) {
        uint32_t E = (S.list[0].rel == 0) ? kExitDead : entry_lookback(P, t);
        if (lane == 0) S.E = E;
      }
      __syncthreads();
      E = S.E;
      if (S.serial || (E != kExitDead && E >= kFar)) {
        serialE = E;
        go_serial = true;
        break;
      }

      // ---- entries of every lane
      uint32_t Ew = (wave == 0) ? (E == kExitDead ? kDead : E) : S.wagg[wave - 1];
      if (lane == 0 && !known) {
        ex = apply_fn(L.F, Ew);
        known = true;
      }
      for (;;) {
        uint32_t pex = wave_shr1(ex, 0u);
        bool pk = wave_shr1(known ? 1u : 0u, 0u) != 0;
        bool nw = !known && pk;
        if (nw) {
          ex = apply_fn(L.F, pex);
          known = true;
        }
        if (__ballot(nw) == 0) break;
      }
      ent = wave_shr1(ex, Ew);
      reach = L.slow ? lane_forward(L, ent == kDead ? 99u : ent) : fast_reach(L, ent);
      const uint32_t hdr = L.hdr;
      starts = uint32_t(reach) & L.plmask & ~L.farmask & ~hdr & 0xFFFFu;
      errs = uint32_t(reach) & ~L.plmask & ~hdr & 0xFFFFu;
    }
    // ID slots of this lane's instructions (bit q <-> word q of the lane
    // window; words 16..19 belong to the next lane)
    uint32_t defm = 0, usem = 0;
    if (kSem && !kRes) {
      uint32_t rules = 0;
#pragma unroll
      for (int p = 0; p < kLaneWords; ++p) {
        if ((starts >> p) & 1u) {
          defm |= ((e[p] >> 24) & 0xFu) << (p + 1);
          usem |= (e[p] >> 28) << (p + 1);
          if (rules_on) {
            if (L.rst == 0) rules |= ent_rules(e[p]);
            else if (ent_rules(e[p])) atomicOr(&S.modflags[lane_mod_at(L, p)], ent_rules(e[p]) << kModRuleShift);
          }
        }
      }
      S.spill[tid] = ((defm >> 16) & 0xFu) | (((usem >> 16) & 0xFu) << 4);
      // module-level rule presence (section "Validation Rules")
      if (rules) atomicOr(&S.modflags[L.j0], rules << kModRuleShift);
    }
    // a long instruction on the chain sends the tile to the serial path; only
    // tiles with a long candidate can have one
    uint32_t tile_far = 0;
    if (!kRes) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) tile_far |= S.wflags[w];
    }
    if (tile_far != 0) {
      const bool far_hit = (uint32_t(reach) & L.farmask & 0xFFFFu) != 0 || ent == kFar;
      if (__syncthreads_or(far_hit)) {
        serialE = E;
        go_serial = true;
        break;
      }
    }
    // starts of string-bearing instructions are compacted for the string checks
    if constexpr (!kRes) {
      uint32_t ns = starts & L.namemask;
      if (ns) {
        uint32_t b = atomicAdd(&S.nname, uint32_t(__popc(ns)));
        while (ns) {
          const int p = __builtin_ctz(ns);
          ns &= ns - 1;
          S.stage[b++] = uint32_t(lrel + p);
        }
      }
    }
    if (!kRes && tid == kBlock - 1) {
      // the tile's exit: chain node of the last lane beyond position 15
      uint32_t beyond = reach >> 16;
      uint32_t xv = beyond ? uint32_t(__builtin_ctz(beyond)) : kExitDead;
      if (xv != kExitDead && xv >= 14u) xv = kExitDead;  // the sink
      st_state(&P.tileA[(t) * kStateStride],
               kFlagFull | (tile_far ? kFarBit : 0ull) | xv);
    }

    // ---- scans over lanes: per-module instruction counts (segmented by
    // module starts) and tile-local staging slots (plain)
    const uint32_t rst = L.rst;
    const uint32_t nst = __popc(starts);
    const uint32_t sinc = wave_incl_sum(nst);
    uint32_t inc, excl;
    if (S.K > 1 || S.list[0].rel >= 0) {
      // a module starts in the tile: counts restart at module starts
      uint32_t cval;
      if (rst) {
        int last = 31 - __builtin_clz(rst);
        cval = 0x80000000u | uint32_t(__popc(starts & ~((2u << last) - 1u)));
      } else {
        cval = nst;
      }
      inc = wave_incl_segsum(cval);
      excl = wave_shr1(inc, 0u);
    } else {
      inc = sinc;
      excl = sinc - nst;
    }
    if (lane == 63) {
      S.wcnt[wave] = inc;
      S.wst[wave] = sinc;
    }
    if (tid == kBlock - 1) S.tnext = claim_tn;
    __syncthreads();
    // the next tile's words, loaded during the rest of this one (the
    // single-pass walk only: the resolved walk runs more blocks per CU and
    // hides the load latency with them instead of with registers)
    auto issue_prefetch = [&]() {
      const long long tn = S.tnext;
      const int64_t an = tn * kTileWords + int64_t(tid) * kLaneWords;
      if (tn < P.n_tiles) {
        if (an + kLaneWords <= P.W) {
          const uint4* src = reinterpret_cast<const uint4*>(P.words + an);
#pragma unroll
          for (int i = 0; i < kLaneWords / 4; ++i) pf[i] = src[i];
        } else {
          // the batch's last, partial tile: words past the end read as 0
#pragma unroll
          for (int i = 0; i < kLaneWords / 4; ++i) {
            uint32_t x[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = (an + 4 * i + j < P.W) ? P.words[an + 4 * i + j] : 0u;
            pf[i] = make_uint4(x[0], x[1], x[2], x[3]);
          }
        }
        if (tid < kTwTail) {
          const int64_t e1 = (tn + 1) * kTileWords;
          pf_tail = (e1 + tid < P.W) ? P.words[e1 + tid] : 0u;
        }
        pf_tile = tn;
      }
    };
    if constexpr (!kRes) issue_prefetch();
    uint32_t wpre = 0, tot = 0, sbase = sinc - nst, n_slots = 0;
    for (int w = 0; w < kWaves; ++w) {
      uint32_t v = S.wcnt[w];
      if (w < wave) {
        wpre = (v & 0x80000000u) ? v : (wpre + v) | (wpre & 0x80000000u);
        sbase += S.wst[w];
      }
      tot = (v & 0x80000000u) ? v : (tot + v) | (tot & 0x80000000u);
      n_slots += S.wst[w];
    }
    if (!kRes && tid == 64)
      st_state(&P.tileB[(t) * kStateStride], kFlagAgg | ((tot & 0x80000000u) ? kResetBit : 0ull) | (tot & 0x7FFFFFFFu));
    // starts of the module open at this lane's start, before it, inside this
    // tile; for list entry 0 the tile prefix is added once it is known
    const uint32_t lex = (excl & 0x80000000u) ? excl : (wpre + excl) | (wpre & 0x80000000u);
    const uint32_t pre_local = lex & 0x7FFFFFFFu;
    const bool lane_in_first = !(lex & 0x80000000u);  // module open at the lane start is list entry 0
    auto rank_local = [&](int p) -> uint32_t {
      uint32_t below = starts & ((1u << p) - 1u);
      uint32_t rb = rst & ((2u << p) - 1u);
      if (rb == 0) return pre_local + __popc(below);
      int r = 31 - __builtin_clz(rb);
      return __popc(below & ~((1u << r) - 1u));
    };
    // is the start at p in list entry 0 (ranks continue the tile prefix)?
    auto in_first = [&](int p) -> bool { return lane_in_first && (rst & ((2u << p) - 1u)) == 0; };

    // ---- strings (OpName, OpEntryPoint): one lane per compacted start, on the LDS copy of
    // the words; malformed ones are marked in badb and reported with the
    // parse errors
    // one string-bearing start at tile position q: its string, on the LDS copy of the
    // words; malformed ones are marked in badb and reported with the parse
    // errors
    auto check_name = [&](const int q) {
      const uint32_t ss = str_slot(tbl_lookup(S.tbl, S.tw[twx(q)] & 0xFFFFu));
      const uint32_t nw = (S.tw[twx(q)] >> 16) - ss;  // string words: 1..12 on this path
      uint32_t x[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) x[k] = (uint32_t(k) < nw) ? S.tw[twx(q + int(ss) + k)] : 0u;
      bool ok = true;
      uint32_t last = 0;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        uint32_t z = (x[k] - 0x01010101u) & ~x[k] & 0x80808080u;
        if (uint32_t(k) + 1 < nw) ok = ok && z == 0;
        if (uint32_t(k) + 1 == nw) last = x[k];
      }
      uint32_t z = (last - 0x01010101u) & ~last & 0x80808080u;
      ok = ok && z != 0 && (last >> (8 * (__builtin_ctz(z | 0x80000000u) >> 3))) == 0;
      if (!ok) atomicOr(&S.badb[q >> 5], 1u << (q & 31));
    };
    auto check_names = [&](uint32_t own) {
      const uint32_t nn = S.nname;
      if constexpr (kRes) {
        if (nn <= uint32_t(kNameCap)) {
          for (uint32_t i = tid; i < nn; i += kBlock) check_name(int(S.names[i]));
        } else {
          while (own) {
            const int p = __builtin_ctz(own);
            own &= own - 1;
            check_name(lrel + p);
          }
        }
      } else {
        for (uint32_t i = tid; i < nn; i += kBlock) check_name(int(S.stage[i]));
      }
    };
    if constexpr (!kRes) check_names(0u);

    uint32_t own_names = 0;
    // resolved walk: one pass over the lane's starts for the grammar entry,
    // the ID slots, the string marks and the instruction index (the tile
    // prefix is already known)
    if constexpr (kRes) {
      uint32_t name_m = 0, rules = 0;
      uint32_t sm = starts;
      uint32_t k = 0;
      // lanes inside one module: index entries at dst0 + k, values val0 + p
      int64_t dst0 = 0;
      uint32_t val0 = 0;
      bool ok0 = false;
      if (kIdx && rst == 0) {
        const LEnt& le = S.list[L.j0];
        ok0 = (le.info & kInfoHdrOk) != 0;
        dst0 = le.off + pre_local + (lane_in_first ? res_pre : 0u);
        val0 = uint32_t(t0 + lrel - le.off);
      }
      // (a wave with no module start in its lanes runs a copy of the loop
      // without the module-start branches)
      auto starts_loop = [&](auto plain_t) {
        constexpr bool kPlain = decltype(plain_t)::value;
        while (sm) {
          const int p = __builtin_ctz(sm);
          sm &= sm - 1;
          const uint32_t w0 = S.tw[twx(lrel + p)];
          const uint32_t ee = tbl_lookup(S.tbl, w0 & 0xFFFFu);
          name_m |= ent_str(ee) << p;
          if (kSem) {
            defm |= ((ee >> 24) & 0xFu) << (p + 1);
            usem |= (ee >> 28) << (p + 1);
            // module-level rule presence (section "Validation Rules")
            if (rules_on) {
              if (kPlain || rst == 0) rules |= ent_rules(ee);
              else if (ent_rules(ee)) atomicOr(&S.modflags[lane_mod_at(L, p)], ent_rules(ee) << kModRuleShift);
            }
          }
          if (kIdx) {
            if (kPlain || rst == 0) {
              if (ok0) {
                P.idx_off[dst0 + k] = val0 + uint32_t(p);
                P.idx_op[dst0 + k] = uint16_t(w0 & 0xFFFFu);
              }
            } else {
              const int jm = lane_mod_at(L, p);
              const LEnt& le = S.list[jm];
              if (le.info & kInfoHdrOk) {
                const int64_t dst = le.off + rank_local(p) + (in_first(p) ? res_pre : 0u);
                P.idx_off[dst] = uint32_t(t0 + lrel + p - le.off);
                P.idx_op[dst] = uint16_t(w0 & 0xFFFFu);
              }
            }
          }
          ++k;
        }
      };
      if (__ballot(rst != 0) == 0) starts_loop(std::true_type{});
      else starts_loop(std::false_type{});
      if (kSem) {
        S.spill[tid] = ((defm >> 16) & 0xFu) | (((usem >> 16) & 0xFu) << 4);
        if (rules_on) {
          // one LDS atomic per wave when the wave's lanes are in one module
          if (S.K == 1) {
            rules = wave_or_u32(rules);
            if (lane == 0 && rules) atomicOr(&S.modflags[0], rules << kModRuleShift);
          } else if (rules) {
            atomicOr(&S.modflags[L.j0], rules << kModRuleShift);
          }
        }
      }
      uint32_t ns = name_m;
      if (ns) {
        uint32_t b = atomicAdd(&S.nname, uint32_t(__popc(ns)));
        while (ns) {
          const int p = __builtin_ctz(ns);
          ns &= ns - 1;
          if (b < uint32_t(kNameCap)) S.names[b] = uint16_t(lrel + p);
          ++b;
        }
      }
      own_names = name_m;
      if (!kSem) {
        __syncthreads();
        check_names(own_names);
      }
    }

    // ---- result-ID checks
    if (kSem) {
      // LDS windows for the result IDs of this tile.  One window: module jw,
      // anchored at the first result ID found by the lowest wave that has
      // one.  Several: list entries 0.., each anchored at the smallest first
      // result ID of its lanes.
      const int jw = S.jw;
      // a tile inside one module has one window over the whole window space
      const bool one = SH::kWins == 1 || S.K == 1;
      if (one) {
        const uint32_t dw = (L.rst == 0 && L.j0 == jw) ? (defm & 0xFFFFu) : 0u;
        const uint32_t first = dw ? S.tw[twx(lrel + __builtin_ctz(dw))] : 0u;
        uint64_t bal = __ballot(dw != 0);
        uint32_t ref = 0xFFFFFFFFu;
        if (bal) ref = __shfl(first, int(__builtin_ctzll(bal)));
        if (lane == 0) S.wref[wave] = ref;
      } else {
        const uint32_t dw = defm & 0xFFFFu;
        if (L.rst == 0 && L.j0 < SH::kWins && dw) {
          const LEnt& le = S.list[L.j0];
          const uint32_t v = S.tw[twx(lrel + __builtin_ctz(dw))];
          if (le.mod >= 0 && (le.info & kInfoHdrOk) && !(le.info & kInfoSparse) && v != 0u && v < le.bound)
            atomicMin(&S.wmin[L.j0], v);
        }
      }
      __syncthreads();
      if constexpr (kRes) check_names(own_names);
      if (tid > 0) {
        uint32_t sp = S.spill[tid - 1];
        defm |= sp & 0xFu;
        usem |= (sp >> 4) & 0xFu;
      }
      defm &= 0xFFFFu;
      usem &= 0xFFFFu;
      uint32_t ref1 = 0xFFFFFFFFu;
      if (one) {
        for (int w = kWaves - 1; w >= 0; --w)
          if (S.wref[w] != 0xFFFFFFFFu) ref1 = S.wref[w];
      }
      // words of a window, window of list entry j (-1: none), its base
      const uint32_t wsz = one ? uint32_t(kNW) : uint32_t(kWW);
      auto win_of = [&](int j) -> int {
        if (one) return (jw >= 0 && ref1 != 0xFFFFFFFFu && j == jw) ? 0 : -1;
        return (j < SH::kWins && S.wmin[j] != 0xFFFFFFFFu) ? j : -1;
      };
      auto win_base = [&](int w) -> uint32_t {
        const uint32_t r = one ? ref1 : S.wmin[w];
        return (r > 16u * wsz ? r - 16u * wsz : 0u) & ~63u;  // a quarter of the window below the anchor
      };
      // set result ID v in window w (v inside it); true if it was set before
      auto win_set = [&](int w, uint32_t base, uint32_t v) -> bool {
        const unsigned long long bit = 1ull << (v & 63u);
        return (atomicOr(&S.win[w * wsz + ((v - base) >> 6)], bit) & bit) != 0;
      };
      // Lanes inside one bitmap-mode module: bound check of every ID word,
      // LDS-window insertion of the result IDs.  Every other ID word (result
      // outside the window, hash-mode module, lanes with a module start) is
      // collected in `rare` and handled below.
      uint32_t rare = 0;
      if (L.rst == 0) {
        const int j0 = L.j0;
        const uint32_t info = S.list[j0].info, bound = S.list[j0].bound;
        if ((info & kInfoHdrOk) && !(info & kInfoSparse)) {
          const uint32_t bm1 = bound ? bound - 1u : 0u;  // v - 1 >= bm1  <=>  v == 0 or v >= bound
          const uint32_t idm = defm | usem;
          bool oob = false;
          if constexpr (kRes) {
            // (the resolved walk keeps the words in LDS only; flags gathered
            // under per-lane branches are integers, not booleans: they stay in
            // vector registers, with no lane-mask merging at every branch)
            if (S.nbm1 != kNoBound) {
              // (the bound test of the words, taken at their load)
              oob = (idm & S.tw[tid * (kLaneWords + 1) + kLaneWords]) != 0;
            } else {
              uint32_t oobm = 0;
#pragma unroll
              for (int p = 0; p < kLaneWords; ++p)
                if ((idm >> p) & 1u) oobm |= (S.tw[twx(lrel + p)] - 1u >= bm1) ? 1u : 0u;
              oob = oobm != 0;
            }
          } else {
#pragma unroll
            for (int p = 0; p < kLaneWords; ++p) oob |= ((idm >> p) & 1u) && (L.w[p] - 1u >= bm1);
          }
          const int wj = win_of(j0);
          const uint32_t base = wj >= 0 ? win_base(wj) : 0u;
          uint32_t dupm = 0;
          uint32_t dm = defm;
          const uint32_t wlim = wj >= 0 ? 64u * wsz : 0u;
          while (dm) {
            const int p = __builtin_ctz(dm);
            dm &= dm - 1;
            const uint32_t v = S.tw[twx(lrel + p)];
            const uint32_t inb = (v - 1u < bm1) ? 1u : 0u;  // in bound (the others were flagged above)
            const uint32_t inw = inb & ((v - base < wlim) ? 1u : 0u);
            rare |= (inb & (inw ^ 1u)) << p;
            if (inw) {
              const unsigned long long bit = 1ull << (v & 63u);
              dupm |= uint32_t((atomicOr(&S.win[wj * wsz + ((v - base) >> 6)], bit) >> (v & 63u)) & 1ull);
            }
          }
          bool dup = dupm != 0;
          if (oob || dup) atomicOr(&S.modflags[j0], (oob ? kModOOB : 0u) | (dup ? kModDup : 0u));
        } else if (info & kInfoHdrOk) {
          rare = defm | usem;
        }
      } else {
        rare = defm | usem;
      }
      while (rare) {
        int p = __builtin_ctz(rare);
        rare &= rare - 1;
        int jm = lane_mod_at(L, p);
        const LEnt& le = S.list[jm];
        if (!(le.info & kInfoHdrOk)) continue;
        uint32_t v = S.tw[twx(lrel + p)];
        bool is_def = (defm >> p) & 1u;
        const int wj = win_of(jm);
        const uint32_t base = wj >= 0 ? win_base(wj) : 0u;
        if (wj >= 0 && is_def && v != 0u && v < le.bound && v >= base && v - base < 64u * wsz) {
          if (win_set(wj, base, v)) atomicOr(&S.modflags[jm], kModDup);
        } else {
          id_check(P, le, v, is_def, &S.modflags[jm], &S.moddef[jm]);
        }
      }
      // the tile's last lane also checks the words of its last instruction
      // that lie in the next tile
      if (tid == kBlock - 1) {
        uint32_t sp = S.spill[tid];
        for (int k = 0; k < 4; ++k) {
          bool d = (sp >> k) & 1u, u = (sp >> (4 + k)) & 1u;
          if (!(d || u)) continue;
          int jm = lane_mod_at(L, 15);
          const LEnt& le = S.list[jm];
          if (!(le.info & kInfoHdrOk)) continue;
          const uint32_t v = S.tw[twx(kTileWords + k)];
          const int wj = win_of(jm);
          const uint32_t base = wj >= 0 ? win_base(wj) : 0u;
          if (d && wj >= 0 && v != 0u && v < le.bound && v >= base && v - base < 64u * wsz) {
            if (win_set(wj, base, v)) atomicOr(&S.modflags[jm], kModDup);
          } else {
            id_check(P, le, v, d, &S.modflags[jm], &S.moddef[jm]);
          }
        }
      }
      __syncthreads();
      // window flush: one device atomic per 64 result IDs, issued by the last
      // waves (wave 0 polls other tiles' states next); the returned words are
      // examined at the start of the next tile
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int i = k * kBlock + tid - kFlOff;
        fl_mk[k] = -1;
        fl_bits[k] = 0;
        fl_old[k] = 0;
        if (i >= 0 && i < kNW) {
          const int w = one ? 0 : i / kWW;
          const int jl = one ? jw : w;
          if (win_of(jl) >= 0) {
            const LEnt& le = S.list[jl];
            fl_mk[k] = le.mod;
            fl_bits[k] = S.win[i];
            if (fl_bits[k])
              fl_old[k] = atomicOr(&P.idmap[le.off + (win_base(w) >> 6) + (i - w * int(wsz))], fl_bits[k]);
          }
        }
      }
      if (tid < S.K && S.list[tid].mod >= 0) {
        ModState& ms = P.mods[S.list[tid].mod];
        uint32_t f = S.modflags[tid];
        // rule presence bits: every tile of a large module has the same ones,
        // and device atomics on one address serialize, so a block flushes
        // each module's bits once (the module of its list entry 0 is
        // remembered from tile to tile)
        if (rules_on && tid == 0) {
          const uint32_t rb = f & (15u << kModRuleShift);
          if (S.list[0].mod == S.rl_mod && (rb & ~S.rl_bits) == 0) f &= ~(15u << kModRuleShift);
          if (S.list[0].mod != S.rl_mod) {
            S.rl_mod = S.list[0].mod;
            S.rl_bits = 0;
          }
          S.rl_bits |= rb;
        }
        if (f) atomicOr(&ms.flags, f);
        if (S.moddef[tid]) atomicAdd(&ms.def_count, S.moddef[tid]);
      }
    }

    // ---- index entries staged in LDS in tile order (slot = plain scan)
    if constexpr (kIdx && !kRes) {
      if (!kSem) __syncthreads();  // the string checks above read stage[]
#pragma unroll
      for (int p = 0; p < kLaneWords; ++p) {
        if ((starts >> p) & 1u) S.stage[sbase + __popc(starts & ((1u << p) - 1u))] = uint32_t(lrel + p) | (L.w[p] << 16);
      }
      // first slot of each module in this tile: the first start of the module
      // open at this lane's start when no earlier lane had one, and the first
      // start after each module start inside the lane
      if (starts) {
        const uint32_t first_rst = rst ? uint32_t(__builtin_ctz(rst)) : 32u;
        if (pre_local == 0 && (starts & ((first_rst >= 32u) ? ~0u : ((1u << first_rst) - 1u))))
          S.slot0[L.j0] = sbase;
        uint32_t rr = rst;
        while (rr) {
          const int r = __builtin_ctz(rr);
          rr &= rr - 1;
          const uint32_t upto = rr ? ((1u << __builtin_ctz(rr)) - 1u) : 0xFFFFu;
          if (starts & upto & ~((2u << r) - 1u)) S.slot0[lane_mod_at(L, r)] = sbase + __popc(starts & ((1u << r) - 1u));
        }
      }
    }

    // ---- tile prefix of list entry 0 (count look-back), inclusive state
    if (kRes) {
      // (all threads hold the prefix)
    } else if (wave == 0) {
      uint32_t prefix = (S.list[0].rel == 0) ? 0u : count_lookback(P, P.tileB, t);
      if (lane == 0) {
        S.prefix = prefix;
        uint32_t incl = (tot & 0x80000000u) ? (tot & 0x7FFFFFFFu) : prefix + tot;
        st_state(&P.tileB[(t) * kStateStride], kFlagFull | incl);
      }
    }
    // the resolved walk with result-ID checks has passed a barrier since the
    // string checks; the others wait here for the prefix or the string marks
    if (!kRes || !kSem) __syncthreads();
    const uint32_t prefix = kRes ? res_pre : S.prefix;

    // ---- instruction index: coalesced stores of the staged entries
    if constexpr (kIdx && !kRes) {
      const int K = S.K;
      for (uint32_t sl = tid; sl < n_slots; sl += kBlock) {
        // modules with starts in this tile own consecutive slot ranges in
        // list order; modules without starts keep slot0 = 0xFFFFFFFF
        int jm = 0;
        for (int j = 1; j < K; ++j)
          if (S.slot0[j] <= sl) jm = j;
        const LEnt& le = S.list[jm];
        if (le.info & kInfoHdrOk) {
          uint32_t v = S.stage[sl];
          int64_t dst = le.off + (jm == 0 ? prefix : 0u) + (sl - S.slot0[jm]);
          P.idx_off[dst] = uint32_t(t0 + (v & 0xFFFFu) - le.off);
          P.idx_op[dst] = uint16_t(v >> 16);
        }
      }
    }

    // (the resolved walk does not prefetch: the registers cost more occupancy
    // than the early loads gain)

    // ---- module ends owned by this lane: positions 1..16 of the window
    {
      uint32_t ends = (L.bm >> 1) & 0xFFFFu;  // bit k <-> end at position k+1
      while (ends) {
        int k = __builtin_ctz(ends);
        ends &= ends - 1;
        int e = k + 1;
        // module open just before position e
        uint32_t rb = rst & ((1u << e) - 1u);  // module starts in [0, e)
        uint32_t below = starts & ((1u << e) - 1u);
        uint32_t c;
        int jm;
        if (rb == 0) {
          c = pre_local + __popc(below) + (lane_in_first ? prefix : 0u);
          jm = L.j0;
        } else {
          int r = 31 - __builtin_clz(rb);
          c = __popc(below & ~((1u << r) - 1u));
          jm = lane_mod_at(L, r);
        }
        const LEnt& le = S.list[jm];
        if (le.mod >= 0) P.mods[le.mod].n_total = c;
      }
    }

    // ---- parse errors: chain nodes that are not valid instructions, and
    // string-bearing starts whose string is malformed
    {
      const uint32_t bad_names = (S.badb[lrel >> 5] >> (lrel & 31)) & 0xFFFFu;
      uint32_t ee = errs | bad_names;
      while (ee) {
        int p = __builtin_ctz(ee);
        ee &= ee - 1;
        int jm = lane_mod_at(L, p);
        const LEnt& le = S.list[jm];
        int64_t pos = L.a + p;
        if (pos >= P.W || le.mod < 0) continue;
        uint32_t code = ((bad_names >> p) & 1u) ? uint32_t(SPV_E_BAD_STRING) : start_code(P.words, S.tbl, pos, le.end);
        if (code == 0) code = SPV_E_BAD_WORD_COUNT;  // not reachable: implausible implies a failing check
        uint32_t rank = rank_local(p) + (in_first(p) ? prefix : 0u);
        report_error(P.mods[le.mod], uint32_t(pos - le.off), code, rank);
      }
    }
    } while (false);
    // the bound for the next tile's load-time test (list entry 0 is read
    // before the next tile rebuilds the list, behind the loop's barrier)
    if constexpr (kRes && kSem) {
      if (tid == 0) {
        const long long tn = t + gridDim.x;
        uint32_t nb = kNoBound;
        if (tn < P.n_tiles) {
          const int64_t t0n = tn * kTileWords;
          const int64_t t1n = (t0n + kTileWords < P.W) ? t0n + kTileWords : P.W;
          const LEnt& c = S.list[0];
          if (c.mod >= 0 && c.off <= t0n && c.end > t1n + 16 && (c.info & kInfoHdrOk) && !(c.info & kInfoSparse))
            nb = c.bound ? c.bound - 1u : 0u;
        }
        S.nbm1 = nb;
      }
    }
    if constexpr (!kRes) {
      if (go_serial) {
        if (tid == kBlock - 1) S.tnext = claim_tn;
        serial_tile<kSem, kIdx>(S, P, t, t0, t1, serialE);
      }
    }
  }
  if (kSem && dc_cnt) atomicAdd(&P.mods[dc_mod].def_count, dc_cnt);
}

template <bool kSem, bool kIdx>
__global__ __launch_bounds__(kBlock, 16 / kWaves) void k_main(VParams P) {
  __shared__ Shared S;
  if (P.ctrl[kCtlMode] == kModeResolved) return;  // the resolved walk ran
  main_body<kSem, kIdx, false>(S, P);
}

template <bool kSem, bool kIdx, bool kRules>
__global__ __launch_bounds__(kBlock, 24 / kWaves) void k_walk(VParams P) {
  __shared__ WalkShared S;
  if (P.ctrl[kCtlMode] != kModeResolved) return;  // the single-pass walk runs next
  main_body<kSem, kIdx, true, WalkShared, kRules>(S, P);
}

// ---------------------------------------------------------------------------
// Result of module m from its state (the second finalize phase).
__device__ __forceinline__ void finalize_module(const VParams& P, int64_t m) {
  const ModState& ms = P.mods[m];
  spv_result r;
  if (ms.hdr_code != 0) {
    r.code = ms.hdr_code;
    r.sem_mask = 0;
    r.err_word = ms.hdr_err;
    r.n_inst = 0;
  } else if (ms.err_key != ~0ull) {
    r.code = uint32_t(ms.err_key & 0xFFu);
    r.sem_mask = 0;
    r.err_word = uint32_t(ms.err_key >> 8);
    r.n_inst = uint32_t(ms.err_rank & 0xFFFFFFFFu);
  } else {
    uint32_t sem = P.semantic ? (ms.flags & 7u) : 0u;
    r.code = (sem & 1u) ? SPV_E_ID_OUT_OF_BOUND : (sem & 2u) ? SPV_E_DUPLICATE_ID : (sem & 4u) ? SPV_E_UNDEFINED_ID : 0u;
    r.sem_mask = sem;
    r.err_word = 0xFFFFFFFFu;
    r.n_inst = ms.n_total;
    if (P.rules && r.code == 0) {
      // module-level rules (section "Validation Rules"): a capability, the
      // memory model, a function and an entry point
      const uint32_t present = (ms.flags >> kModRuleShift) & 15u;
      const uint32_t missing = ((present & 1u) ? 0u : 8u) | ((present & 2u) ? 0u : 16u) |
                               ((present & 4u) ? 0u : 32u) | ((present & 8u) ? 0u : 64u);
      if (missing) {
        r.code = SPV_E_MODULE_RULES;
        r.sem_mask = missing;
      }
    }
  }
  if (P.ctrl[kCtlSpinErr]) r.code = kSpinFailCode;
  P.results[m] = r;
}

// finalize: phase 1 marks modules whose undefined-ID check needs the second
// pass; phase 2 writes spv_result.
__global__ __launch_bounds__(256) void k_finalize(VParams P, int phase) {
  const int64_t gtid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = int64_t(gridDim.x) * blockDim.x;
  for (int64_t m = gtid; m < P.M; m += nth) {
    if (phase == 2) {
      finalize_module(P, m);
      continue;
    }
    ModState& ms = P.mods[m];
    if (ms.hdr_code == 0 && ms.err_key == ~0ull) {
      bool need;
      if (ms.flags & kModSparse) need = true;
      else need = ms.bound > 1u && ms.def_count < ms.bound - 1u;
      if (need) {
        ms.flags |= kModPass2;
        atomicAdd(&P.ctrl[kCtlPass2], 1u);
        // the module's tiles join the second pass's list
        const int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
        if (end > off) {
          const int64_t a = off / kTileWords, b = (end - 1) / kTileWords;
          const uint32_t base = atomicAdd(&P.ctrl[kCtlP2Tiles], uint32_t(b - a + 1));
          for (int64_t i = 0; i <= b - a; ++i) P.p2list[base + i] = uint32_t(a + i);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// second pass: undefined-ID check for modules marked in phase 1.
__global__ __launch_bounds__(kBlock) void k_pass2(VParams P) {
  __shared__ Shared S;
  // small batches (p1_inline, at most kBlock modules): every block decides
  // for itself which modules the pass needs and lists their tiles in LDS
  // (the first finalize phase's work, no launch of it); the need flags are
  // read from LDS, never from module state that other blocks write.  The
  // second finalize phase runs at the end, in one block.
  __shared__ uint32_t s_need[kBlock / 32];
  __shared__ uint32_t s_tpre[kBlock + 1];  // listed tiles before module m
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  long long n_list;
  if (P.p1_inline) {
    uint32_t nt = 0;
    bool need = false;
    if (tid < P.M) {
      const ModState& ms = P.mods[tid];
      if (ms.hdr_code == 0 && ms.err_key == ~0ull)
        need = (ms.flags & kModSparse) || (ms.bound > 1u && ms.def_count < ms.bound - 1u);
      const int64_t off = P.mod_off[tid], end = P.mod_off[tid + 1];
      if (need && end > off) nt = uint32_t((end - 1) / kTileWords - off / kTileWords + 1);
    }
    const uint64_t nb = __ballot(need);
    if (lane == 0) {
      s_need[2 * wave] = uint32_t(nb);
      s_need[2 * wave + 1] = uint32_t(nb >> 32);
    }
    const uint32_t inc = wave_incl_sum(nt);
    if (lane == 63) S.wcnt[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (w < wave) pre += S.wcnt[w];
      tot += S.wcnt[w];
    }
    s_tpre[tid] = pre + inc - nt;
    if (tid == 0) s_tpre[kBlock] = tot;
    __syncthreads();
    n_list = tot;
    if (n_list == 0) {  // the same in every block: no second pass, block 0 writes the results
      if (blockIdx.x == 0 && tid < P.M) finalize_module(P, tid);
      return;
    }
  } else {
    if (P.ctrl[kCtlPass2] == 0) return;
    n_list = P.ctrl[kCtlP2Tiles];
  }
  auto marked = [&](int64_t m) -> bool {
    return P.p1_inline ? ((s_need[m >> 5] >> (m & 31)) & 1u) != 0 : (P.mods[m].flags & kModPass2) != 0;
  };
  if (threadIdx.x == 0) S.cache_ok = 0;
  init_table(S.tbl);
  // the resolved walk ran (the chain pass's lane records are exact)
  const bool resolved = P.ctrl[kCtlMode] == kModeResolved;
  // tiles of the marked modules, listed by the first finalize phase, in
  // block order (a tile of two marked modules may come twice: the checks
  // only set flags)
  for (long long li = blockIdx.x; li < n_list; li += gridDim.x) {
    long long t;
    if (P.p1_inline) {
      int lo = 0, hi = int(P.M) - 1;  // last module with s_tpre[m] <= li
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_tpre[mid] <= uint32_t(li)) lo = mid;
        else hi = mid - 1;
      }
      t = P.mod_off[lo] / kTileWords + (li - s_tpre[lo]);
    } else {
      t = P.p2list[li];
    }
    const int64_t t0 = t * kTileWords;
    const int64_t t1 = (t0 + kTileWords < P.W) ? t0 + kTileWords : P.W;
    if (wave == 0) build_list(S, P, t, t0, t1);
    __syncthreads();
    // any module of this tile marked?
    bool mark = false;
    for (int j = 0; j < (S.crowded ? 0 : S.K); ++j)
      if (S.list[j].mod >= 0 && marked(S.list[j].mod)) mark = true;
    if (S.crowded) mark = true;
    if (!mark) {
      __syncthreads();
      continue;
    }
    // hash-mode modules: scan their slots within this tile's word range
    if (S.crowded) {
      // serial fallback over the modules of the tile
      if (tid == 0) {
        int64_t m = P.tfm[t];
        for (; m < P.M && P.mod_off[m] < t1; ++m) {
          ModState& ms = P.mods[m];
          if (!marked(m)) continue;
          int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
          if (ms.flags & kModSparse) {
            int64_t s0 = off > t0 ? off : t0, s1 = end < t1 ? end : t1;
            for (int64_t i = s0; i < s1; ++i) {
              uint32_t f = uint32_t(P.idmap[i] >> 32);
              if ((f & 2u) && !(f & 1u)) atomicOr(&ms.flags, kModUndef);
            }
          }
        }
      }
      __syncthreads();
      // bitmap-mode modules of crowded tiles are walked serially below
    } else {
      for (int j = 0; j < S.K; ++j) {
        const LEnt& le = S.list[j];
        if (le.mod < 0 || !(le.info & kInfoSparse)) continue;
        ModState& ms = P.mods[le.mod];
        if (!marked(le.mod)) continue;
        int64_t s0 = le.off > t0 ? le.off : t0, s1 = le.end < t1 ? le.end : t1;
        bool bad = false;
        for (int64_t i = s0 + tid; i < s1; i += kBlock) {
          uint32_t f = uint32_t(P.idmap[i] >> 32);
          bad |= (f & 2u) && !(f & 1u);
        }
        if (bad) atomicOr(&ms.flags, kModUndef);
      }
    }
    // bitmap-mode modules: walk the chain from the exact entry and test uses
    uint32_t E;
    if (S.list[0].rel == 0 || t == 0) E = kExitDead;
    else if (resolved) E = P.tres[2 * t];
    else {
      unsigned long long st = ld_state(&P.tileA[(t - 1) * kStateStride]);
      E = uint32_t(st);
    }
    bool serial = S.crowded || (E != kExitDead && E >= kFar);
    // uses of the lane's starts (use slots as bits 1..19 of the lane window;
    // those past the lane go to the next one): each use of a marked
    // bitmap-mode module must be a set bit of its bitmap (block-wide: every
    // thread calls it)
    auto test_uses = [&](const Lane& L, uint32_t usem) {
      S.spill[tid] = (usem >> 16) & 0xFu;
      __syncthreads();
      if (tid > 0) usem |= S.spill[tid - 1];
      auto test = [&](int jm, uint32_t v) {
        const LEnt& le = S.list[jm];
        if (le.mod < 0 || (le.info & kInfoSparse) || !(le.info & kInfoHdrOk)) return;
        ModState& ms = P.mods[le.mod];
        if (!marked(le.mod)) return;
        if (v == 0u || v >= le.bound) return;
        unsigned long long word = P.idmap[le.off + (v >> 6)];
        if (!((word >> (v & 63u)) & 1ull)) atomicOr(&ms.flags, kModUndef);
      };
#pragma unroll
      for (int p = 0; p < kLaneWords; ++p)
        if ((usem >> p) & 1u) test(lane_mod_at(L, p), L.w[p]);
      if (tid == kBlock - 1) {
        uint32_t sp = S.spill[tid];
        for (int k = 0; k < 4; ++k)
          if ((sp >> k) & 1u) test(lane_mod_at(L, 15), P.words[L.a + 16 + k]);
      }
    };
    if (!serial && resolved) {
      // resolved batches: the chain pass's lane starts give the instruction
      // starts (the first lane adds the part of its candidate chain that the
      // resolved entry reaches, as the resolved walk does), so the lanes need
      // no transfer functions
      Lane L;
      L.a = t0 + int64_t(tid) * kLaneWords;
#pragma unroll
      for (int i = 0; i < kLaneWords; ++i) L.w[i] = (L.a + i < P.W) ? P.words[L.a + i] : 0u;
      lane_window(S, L, tid * kLaneWords);
      uint32_t starts = P.lst[t * kBlock + tid] & 0xFFFFu;
      if (tid == 0) {
        const uint32_t m0 = P.tsum[4 * t + 1];
        const uint32_t h0 = L.hdr ? uint32_t(__builtin_ctz(L.hdr)) : 16u;
        if (E < 14u && E < h0 && ((m0 >> E) & 1u)) starts |= m0 & 0xFFFFu & (~0u << E);
      }
      uint32_t usem = 0;
#pragma unroll
      for (int p = 0; p < kLaneWords; ++p)
        if ((starts >> p) & 1u) usem |= (tbl_lookup(S.tbl, L.w[p] & 0xFFFFu) >> 28) << (p + 1);
      test_uses(L, usem);
    } else if (!serial) {
      Lane L;
      L.a = t0 + int64_t(tid) * kLaneWords;
#pragma unroll
      for (int i = 0; i < kLaneWords; ++i) L.w[i] = (L.a + i < P.W) ? P.words[L.a + i] : 0u;
      lane_window(S, L, tid * kLaneWords);
      const bool any_bounds = __ballot(L.bm != 0) != 0;
      if (any_bounds) lane_dp<true>(S, P, L);
      else lane_dp<false>(S, P, L);
      bool known = L.conv;
      uint32_t ex = L.conv ? L.X : 0u;
      for (;;) {
        uint32_t pex = __shfl_up(ex, 1);
        bool pk = __shfl_up(known ? 1 : 0, 1) != 0 && lane > 0;
        bool nw = !known && pk;
        if (nw) {
          ex = apply_fn(L.F, pex);
          known = true;
        }
        if (__ballot(nw) == 0) break;
      }
      if (lane == 63) S.wagg[wave] = known ? ex : 0xFFu;
      __syncthreads();
      bool amb = false;
      for (int w = 1; w < kWaves; ++w) amb |= S.wagg[w - 1] == 0xFFu;
      if (!amb) {
        uint32_t Ew = (wave == 0) ? (E == kExitDead ? kDead : E) : S.wagg[wave - 1];
        if (lane == 0 && !known) {
          ex = apply_fn(L.F, Ew);
          known = true;
        }
        for (;;) {
          uint32_t pex = __shfl_up(ex, 1);
          bool pk = __shfl_up(known ? 1 : 0, 1) != 0 && lane > 0;
          bool nw = !known && pk;
          if (nw) {
            ex = apply_fn(L.F, pex);
            known = true;
          }
          if (__ballot(nw) == 0) break;
        }
        uint32_t ent = __shfl_up(ex, 1);
        if (lane == 0) ent = Ew;
        const uint32_t reach = lane_forward(L, ent == kDead ? 99u : ent);
        const uint32_t starts = uint32_t(reach) & L.plmask & ~L.farmask & ~L.hdr & 0xFFFFu;
        const bool far_hit = (uint32_t(reach) & L.farmask & 0xFFFFu) != 0 || ent == kFar;
        amb = __syncthreads_or(far_hit);
        if (!amb) {
          uint32_t usem = 0;
#pragma unroll
          for (int p = 0; p < kLaneWords; ++p)
            if ((starts >> p) & 1u) usem |= ((L.rolep[p >> 2] >> (8 * (p & 3) + 4)) & 0xFu) << (p + 1);
          test_uses(L, usem);
        }
      }
      serial = amb;
    }
    __syncthreads();
    if (serial && tid == 0) {
      // exact serial walk over the tile, testing uses of marked modules
      int64_t m = P.tfm[t];
      int64_t off = P.mod_off[m], end = P.mod_off[m + 1];
      int64_t pos;
      if (off == t0) {
        int64_t n = end - off;
        pos = off + (n < 5 ? n : 5);
      } else {
        pos = (E == kExitDead) ? -1 : t0 + int64_t(E);
      }
      for (;;) {
        ModState& ms = P.mods[m];
        bool act = marked(m) && !(ms.flags & kModSparse);
        while (pos >= 0 && pos < end && pos < t1) {
          if (start_code(P.words, S.tbl, pos, end)) {
            pos = -1;
            break;
          }
          uint32_t w0 = P.words[pos];
          uint32_t wc = w0 >> 16;
          if (act) {
            uint32_t um = (tbl_lookup(S.tbl, w0 & 0xFFFFu) >> 28) & 0xFu;
            for (uint32_t s = 1; s <= 4; ++s) {
              if (!((um >> (s - 1)) & 1u)) continue;
              uint32_t v = P.words[pos + s];
              if (v == 0u || v >= ms.bound) continue;
              unsigned long long word = P.idmap[off + (v >> 6)];
              if (!((word >> (v & 63u)) & 1ull)) atomicOr(&ms.flags, kModUndef);
            }
          }
          pos += wc;
        }
        if (end <= t1) {
          int64_t m2 = m + 1;
          while (m2 < P.M && P.mod_off[m2 + 1] == P.mod_off[m2]) ++m2;
          if (m2 >= P.M) break;
          m = m2;
          off = P.mod_off[m];
          end = P.mod_off[m + 1];
          if (off >= t1) break;
          int64_t n = end - off;
          pos = off + (n < 5 ? n : 5);
          continue;
        }
        break;
      }
    }
    __syncthreads();
  }
  if (P.p1_inline) {
    // the last block to finish writes the results: every block's module-state
    // updates are complete and visible (fence, barrier) before it counts
    // itself, and the last one reads them after its own fence
    __shared__ uint32_t s_last;
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = (atomicAdd(&P.ctrl[kCtlP2Done], 1u) == gridDim.x - 1) ? 1u : 0u;
    __syncthreads();
    if (s_last) {
      __threadfence();
      if (tid < P.M) finalize_module(P, tid);
    }
  }
}

// ---------------------------------------------------------------------------
void launch_plan(const VParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_plan, dim3(grid), dim3(256), 0, s, p, int64_t(16384));
}

hipError_t launch_main(const VParams& p, int grid, hipStream_t s) {
  const void* f = p.semantic ? (p.index ? reinterpret_cast<const void*>(k_main<true, true>)
                                        : reinterpret_cast<const void*>(k_main<true, false>))
                             : (p.index ? reinterpret_cast<const void*>(k_main<false, true>)
                                        : reinterpret_cast<const void*>(k_main<false, false>));
  VParams q = p;
  void* args[] = {&q};
  return hipLaunchKernel(f, dim3(grid), dim3(kBlock), args, 0, s);
}

void launch_walk(const VParams& p, int grid, hipStream_t s) {
  if (p.semantic) {
    if (p.rules) {
      if (p.index) hipLaunchKernelGGL((k_walk<true, true, true>), dim3(grid), dim3(kBlock), 0, s, p);
      else hipLaunchKernelGGL((k_walk<true, false, true>), dim3(grid), dim3(kBlock), 0, s, p);
    } else {
      if (p.index) hipLaunchKernelGGL((k_walk<true, true, false>), dim3(grid), dim3(kBlock), 0, s, p);
      else hipLaunchKernelGGL((k_walk<true, false, false>), dim3(grid), dim3(kBlock), 0, s, p);
    }
  } else {
    if (p.index) hipLaunchKernelGGL((k_walk<false, true, false>), dim3(grid), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL((k_walk<false, false, false>), dim3(grid), dim3(kBlock), 0, s, p);
  }
}

void launch_chain(const VParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_chain, dim3(grid), dim3(kBlock), 0, s, p);
}

void launch_resolve(const VParams& p, hipStream_t s) {
  int64_t g = p.n_tiles / kResolveTiles + 1;
  hipLaunchKernelGGL(k_resolve, dim3(int(g)), dim3(kResolveBlock), 0, s, p);
}

void launch_finalize(const VParams& p, int phase, hipStream_t s) {
  int64_t g = (p.M + 255) / 256;
  int grid = int(g < 1 ? 1 : (g > 4096 ? 4096 : g));
  hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, s, p, phase);
}

void launch_pass2(const VParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pass2, dim3(grid), dim3(kBlock), 0, s, p);
}

}  // namespace spv

namespace spv {
int walk_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(k_walk<true, true, false>), kBlock, 0) !=
      hipSuccess)
    return 0;
  return n;
}
int chain_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(k_chain), kBlock, 0) != hipSuccess)
    return 0;
  return n;
}
int main_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(k_main<true, true>), kBlock, 0) !=
      hipSuccess)
    return 0;
  return n;
}
}  // namespace spv
