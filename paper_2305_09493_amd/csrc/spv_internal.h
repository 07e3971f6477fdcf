// Internal definitions shared by the spvgpu kernels and the C ABI.
//
// Batch model: module m is words[mod_off[m] .. mod_off[m+1]).  A SPIR-V
// module is a 5-word header followed by instructions whose first word is
// (word count << 16) | opcode (Beehive SPIR-V Toolkit paper, section "SPIR-V
// Library" header listing and section "Parsing Operand Kinds").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spvgpu.h"

namespace spv {

// ---- tiling --------------------------------------------------------------
constexpr int kLaneWords = 16;                    // words owned by one lane
#ifndef SPV_TILE_WAVES
#define SPV_TILE_WAVES 4
#endif
constexpr int kWaves = SPV_TILE_WAVES;            // waves per tile block
constexpr int kBlock = 64 * kWaves;               // threads per tile block
constexpr int kTileWords = kLaneWords * kBlock;   // words per tile
constexpr int kListMax = 64;                      // module starts per tile window (fast path)
constexpr int kMaxSpanTiles = (65535 + kTileWords - 1) / kTileWords + 1;  // tiles a 65535-word instruction spans
static_assert(kMaxSpanTiles <= 64, "the entry look-back reads one tile per lane of a wave");

// 4-bit exit codes of a lane transfer function: 0..13 exit offset into the
// next lane, kFar = exit not representable (long instruction), kDead = the
// chain ends (invalid start) before leaving the lane.
constexpr uint32_t kFar = 14, kDead = 15;

// ---- tile state words (uint64, one pair per tile) --------------------------
// A[t] (entry/exit):  bits 62..63 flag: 1 = aggregate, 2 = full.
//   aggregate: bits 0..3 exit offset if the exit does not depend on the
//   tile's entry (0..13), kDead (no chain leaves), or kFar meaning "depends
//   on the entry / unknown: wait for full".
//   full: bits 0..31 exact exit offset relative to the next tile start, or
//   0xFFFFFFFF when no chain leaves the tile.
//   bit 33 (both forms): the tile holds a plausible instruction start whose
//   word count is >= 15 (a long instruction could reach past the next tile's
//   first 14 words).
// B[t] (instruction counts of the module open at the tile end):
//   flag 1 = aggregate: bit 32 = a module starts inside the tile, bits 0..31
//   = starts after the last module start (or all starts if none); flag 2 =
//   inclusive: bits 0..31 = starts of that module up to the tile end.
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagFull = 2ull << 62, kFlagMask = 3ull << 62;
constexpr uint64_t kFarBit = 1ull << 33;
constexpr uint64_t kResetBit = 1ull << 32;
constexpr uint32_t kExitDead = 0xFFFFFFFFu;

// ---- per-module state in the workspace ------------------------------------
enum : uint32_t {
  kModOOB = 1u,
  kModDup = 2u,
  kModUndef = 4u,
  kModSparse = 8u,     // IDs kept in a hash table (bound > 64 * words)
  kModPass2 = 16u,     // undefined-ID check needs the second pass
  kModHdrOk = 32u,
};

// Module-level rule presence bits (section "Validation Rules") in
// ModState::flags: 1 capability, 2 memory model, 4 function, 8 entry point,
// shifted by kModRuleShift.
constexpr uint32_t kModRuleShift = 8;

struct ModState {
  unsigned long long err_key;   // (offset << 8) | code of the first failing instruction (atomicMin)
  unsigned long long err_rank;  // (offset << 32) | instructions before it (atomicMin)
  uint32_t flags;               // kMod* bits and rule presence bits (atomicOr)
  uint32_t def_count;           // distinct in-bound result IDs (atomicAdd)
  uint32_t n_total;             // instructions of a module whose parse did not fail
  uint32_t bound;               // header word 3
  uint32_t hdr_code;            // header-stage code
  uint32_t hdr_err;             // header-stage err_word
  uint32_t pad[2];
};
static_assert(sizeof(ModState) == 48, "ModState layout");

// ---- workspace layout ----------------------------------------------------
struct Layout {
  size_t ctrl, tileA, tileB, tfm, mods, idmap, tsum, lst, tres, rstate, p2list, diag, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// tiles per block of the resolve pass
constexpr int kResolveTiles = 256;

// Tile states are polled and written by many blocks with device-scope
// operations, which the memory system serializes per 128-byte line: each
// tile's state gets a line of its own (stride in 64-bit words).
constexpr int kStateStride = 16;

inline Layout make_layout(int64_t n_modules, int64_t n_words) {
  Layout L;
  int64_t n_tiles = (n_words + kTileWords - 1) / kTileWords;
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + 256);
  L.tileA = off;
  off = align256(off + 8 * kStateStride * size_t(n_tiles + 1));
  L.tileB = off;
  off = align256(off + 8 * kStateStride * size_t(n_tiles + 1));
  L.tfm = off;
  off = align256(off + 4 * size_t(n_tiles + 1));
  L.mods = off;
  off = align256(off + sizeof(ModState) * size_t(n_modules + 1));
  L.idmap = off;
  off = align256(off + 8 * size_t(n_words + 1));
  L.tsum = off;
  off = align256(off + 16 * size_t(n_tiles + 1));
  L.lst = off;
  off = align256(off + 4 * size_t(kBlock) * size_t(n_tiles + 1));
  L.tres = off;
  off = align256(off + 8 * size_t(n_tiles + 1));
  L.rstate = off;
  off = align256(off + 8 * kStateStride * size_t(n_tiles / kResolveTiles + 2));
  L.p2list = off;
  off = align256(off + 4 * size_t(n_tiles + n_modules + 2));
  L.diag = off;
  off = align256(off + 16 * size_t(n_modules + 1));
  L.total = off;
  return L;
}

// control words (uint32) at the start of the workspace
enum {
  kCtlClaim = 0,
  kCtlClaim2 = 1,
  kCtlPass2 = 2,
  kCtlSpinErr = 3,
  kCtlMode = 4,
  kCtlClaimR = 5,
  kCtlDoneR = 6,
  kCtlP2Tiles = 7,  // entries of the second pass's tile list
  kCtlP2Done = 8,   // blocks of the second pass that have finished (small batches)
  kCtlDebug = 15    // status word of the SPV_OPT_DEBUG_CHECKS offset check
};
// kCtlMode: kModeResolved when the chain and resolve passes settled every
// tile's entry and count prefix (the main pass then walks without look-back);
// anything else selects the single-pass walk with look-back.
constexpr uint32_t kModeResolved = 1u;
// per-tile summary of the chain pass (4 words): word 0 = exit offset (bits
// 0..7) | flags, word 1 = candidate chain of lane 0 before its first module
// start (bits 0..15: its plausible nodes; bits 16..31: the invalid node that
// ends it, if any), word 2 = starts of the module open at the tile start (lane 0's
// entry-dependent ones excluded), word 3 = starts after the tile's last
// module start
constexpr uint32_t kSumFallback = 1u << 31, kSumModStart = 1u << 30, kSumReset = 1u << 29;

// Every wait on another tile's published state gives up after this many
// polls (seconds of waiting) and flags kCtlSpinErr instead of hanging; the
// finalize kernel then marks every result with kSpinFailCode.
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr uint32_t kSpinFailCode = SPV_E_SPIN_LIMIT;

struct VParams {
  const uint32_t* words;
  const int64_t* mod_off;
  int64_t M, W, n_tiles;
  uint32_t* idx_off;
  uint16_t* idx_op;
  spv_result* results;
  uint32_t* ctrl;
  unsigned long long* tileA;
  unsigned long long* tileB;
  int32_t* tfm;
  ModState* mods;
  unsigned long long* idmap;
  uint32_t* tsum;   // chain-pass tile summaries (4 words per tile)
  uint32_t* lst;    // chain-pass lane records: starts | parse-error nodes << 16
  uint32_t* tres;   // resolved tile entry and count prefix (2 words per tile)
  unsigned long long* rstate;  // resolve-pass block states (look-back)
  uint32_t* p2list;  // tiles of the modules that need the undefined-ID pass
  int semantic;
  int index;
  // single-pass walk: 1, tile t is processed by block t mod gridDim.x; 0,
  // tiles are claimed in order from a counter (the resolved walk always takes
  // tiles t, t + gridDim.x, ...: its tiles do not wait on each other)
  int sched_static;
  // at most 256 modules: k_pass2 computes finalize phase 1 itself and its
  // last block writes the results (no k_finalize launch at all)
  int p1_inline;
  int rules;      // finalize applies the module-level rules
  // semantic positions / defined-before-use (kernels of spv_diag.hip, after
  // the finalize): per module, the first out-of-bound, duplicate and
  // undefined offsets
  uint4* diag;
  int sem_offsets;
  int before_use;
};

// Grammar entry for opcode < 256 (index 256 = any other opcode):
//   bits 0..7  lo      smallest word count
//   bits 8..23 n_ok    number of accepted word counts starting at lo
//                      (1 for fixed-size instructions, 0 = opcode unknown)
//   bits 24..27 result-ID slots (bit s-1 = operand word s is a result ID)
//   bits 28..31 ID-use slots
// A word w at a candidate start is a plausible instruction iff
// (wc - lo) < n_ok (unsigned) with wc = w >> 16.
constexpr int kOpName = 5;
constexpr int kOpEntryPoint = 15;

struct Params;  // forward

void launch_plan(const VParams& p, int grid, hipStream_t s);
hipError_t launch_main(const VParams& p, int grid, hipStream_t s);
void launch_chain(const VParams& p, int grid, hipStream_t s);
void launch_walk(const VParams& p, int grid, hipStream_t s);
void launch_resolve(const VParams& p, hipStream_t s);
void launch_finalize(const VParams& p, int phase, hipStream_t s);
void launch_pass2(const VParams& p, int grid, hipStream_t s);
void launch_diag(const VParams& p, hipStream_t s);

struct EParams {
  const uint16_t* op;
  const int32_t* opnd_off;
  const uint32_t* opnd;
  const int32_t* str_off;
  const uint8_t* chars;
  const int64_t* rec_mod_off;
  int64_t M, N;  // modules, records
  uint32_t version_word, generator_word;
  uint32_t* words_out;
  int64_t* word_mod_off;
  int64_t words_cap;
  uint32_t* enc_code;
  int64_t* enc_bad;
  // workspace
  uint32_t* ctrl;
  unsigned long long* blk;    // per block of records: word total
  unsigned long long* blkx;   // per block of records: words of all records before it (+ grand total)
  unsigned long long* sstate; // look-back states of the scan of the totals
  int64_t* bmod;              // per block of records: module of its first record
  unsigned long long* mod_bad;   // per module: (record << 8) | code, atomicMin
  uint32_t* mod_maxid;        // per module: max ID operand + 1 (atomicMax)
  int64_t* mod_words;         // per module: optimistic start offset of its first record
  uint32_t* stage;            // words staging for compaction
  int64_t n_blocks;
  int block_records;
};

struct ELayout {
  size_t ctrl, blk, blkx, sstate, bmod, mod_bad, mod_maxid, mod_words, total;
};

inline ELayout make_elayout(int64_t n_modules, int64_t n_records, int block_records) {
  ELayout L;
  int64_t nb = (n_records + block_records - 1) / block_records;
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + 256);
  L.blk = off;
  off = align256(off + 8 * size_t(nb + 1));
  L.blkx = off;
  off = align256(off + 8 * size_t(nb + 2));
  L.sstate = off;
  off = align256(off + 128 * size_t(nb / 256 + 2));
  L.bmod = off;
  off = align256(off + 8 * size_t(nb + 1));
  L.mod_bad = off;
  off = align256(off + 8 * size_t(n_modules + 1));
  L.mod_maxid = off;
  off = align256(off + 4 * size_t(n_modules + 1));
  L.mod_words = off;
  off = align256(off + 8 * size_t(n_modules + 1));
  L.total = off;
  return L;
}

void launch_encode(const EParams& p, int grid_count, int grid_scatter, hipStream_t s);

// decode's records mode
struct RParams {
  const uint32_t* words;
  const int64_t* mod_off;
  int64_t M;
  int64_t cap_records;  // n_words: no batch has more records
  const uint32_t* idx_off;
  const spv_result* results;
  uint16_t* op;
  int32_t* opnd_off;
  uint32_t* opnd;
  int32_t* str_off;
  uint8_t* chars;
  int64_t* rec_mod_off;
  // workspace
  uint32_t* ctrl;               // 0, 1: scan claims; 2: a scan gave up waiting
  unsigned long long* mscan;    // per module: record count, then its exclusive scan
  unsigned long long* mstate;   // look-back states of the module scan
  unsigned long long* rscan;    // per record: packed counts (operand words << 32 | string bytes)
  unsigned long long* btot;     // per block of 1024 records: packed total, then its exclusive scan
  unsigned long long* rstate;   // look-back states of the block-total scan
};

struct RLayout {
  size_t ctrl, mscan, mstate, rscan, btot, rstate, total;
};

inline RLayout make_rlayout(int64_t n_modules, int64_t n_words) {
  RLayout L;
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + 256);
  L.mscan = off;
  off = align256(off + 8 * size_t(n_modules + 1));
  L.mstate = off;
  off = align256(off + 128 * size_t((n_modules + 1) / 1024 + 2));
  L.rscan = off;
  off = align256(off + 8 * size_t(n_words + 1));
  const int64_t nb = n_words / 1024 + 1;  // blocks of 1024 records, at most
  L.btot = off;
  off = align256(off + 8 * size_t(nb + 1));
  L.rstate = off;
  off = align256(off + 128 * size_t(nb / 1024 + 2));
  L.total = off;
  return L;
}

void launch_records(const RParams& p, hipStream_t s);

// decode's text mode (disassembly to text)
enum : uint32_t {
  kTxtHighlight = 1u,
  kTxtInlineNames = 2u,
  kTxtNoIndent = 4u,
  kTxtGroup = 8u,
  kTxtNoHeader = 16u,
};
// Inline-name hash slot: key (module << 32 | target ID) and, for the
// module's first OpName of that target (atomicMin), its word position << 32 |
// the length of its name when usable (0 = print the number).
struct TxtSlot {
  unsigned long long key;
  unsigned long long pl;
};
constexpr unsigned long long kTxtEmpty = ~0ull;
struct TParams {
  const uint32_t* words;
  const int64_t* mod_off;
  int64_t M;
  int64_t cap_inst;  // n_words: no batch has more instructions
  const uint32_t* idx_off;
  const spv_result* results;
  uint32_t options;
  uint8_t* text;
  int64_t text_cap;
  int64_t* text_mod_off;
  // workspace
  uint32_t* ctrl;               // 0, 1: scan claims; 2: a scan gave up waiting; 3: OpName count
  unsigned long long* mscan;    // per module: header bytes << 29 | instructions, then the exclusive scan
  unsigned long long* mstate;   // look-back states of the module scan
  uint32_t* lens;               // per instruction: line bytes; after the scatter, offset in its block
  uint32_t* lpos;               // per instruction: word position of its first word
  unsigned long long* btot;     // per block of 1024 instructions: bytes, then the exclusive scan
  unsigned long long* bstate;   // look-back states of the block scan
  TxtSlot* slots;               // inline-name hash (slot_cap slots, a power of two)
  int64_t slot_cap;
  uint2* nlist;                 // OpName instructions (module, word position), 1024 entries per block
  uint32_t* bcount;             // OpName instructions per block of 1024 instructions
  uint32_t* nfilter;            // kTxtFilterBits bits: a (module, ID) that some OpName targets has its bit set
};
constexpr uint32_t kTxtFilterBits = 1u << 24;  // 2 MB: stays in L2
struct TLayout {
  size_t ctrl, mscan, mstate, lens, lpos, btot, bstate, slots, nlist, bcount, nfilter, total;
  int64_t slot_cap;
};
inline TLayout make_tlayout(int64_t n_modules, int64_t n_words, uint32_t options) {
  TLayout L;
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + 256);
  L.mscan = off;
  off = align256(off + 8 * size_t(n_modules + 1));
  L.mstate = off;
  off = align256(off + 128 * size_t((n_modules + 1) / 1024 + 2));
  L.lens = off;
  off = align256(off + 4 * size_t(n_words + 1));
  L.lpos = off;
  off = align256(off + 4 * size_t(n_words + 1));
  const int64_t nb = n_words / 1024 + 1;  // blocks of 1024 instructions, at most
  L.btot = off;
  off = align256(off + 8 * size_t(nb + 1));
  L.bstate = off;
  off = align256(off + 128 * size_t(nb / 1024 + 2));
  // an OpName has at least 3 words
  const int64_t max_names = (options & kTxtInlineNames) ? n_words / 3 + 1 : 0;
  int64_t cap = 64;
  while (cap < 2 * max_names) cap <<= 1;
  L.slot_cap = (options & kTxtInlineNames) ? cap : 0;
  L.slots = off;
  off = align256(off + sizeof(TxtSlot) * size_t(L.slot_cap));
  const bool names = (options & kTxtInlineNames) != 0;
  L.nlist = off;
  off = align256(off + (names ? 8 * size_t(nb) * 1024 : 0));
  L.bcount = off;
  off = align256(off + (names ? 4 * size_t(nb) : 0));
  L.nfilter = off;
  off = align256(off + (names ? size_t(kTxtFilterBits) / 8 : 0));
  L.total = off;
  return L;
}
void launch_text(const TParams& p, hipStream_t s);

}  // namespace spv
