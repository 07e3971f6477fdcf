/*
 * spvgpu -- batched SPIR-V decode, validate and encode on AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * What the library computes comes from the Beehive SPIR-V Toolkit paper
 * (arXiv 2305.09493): SPIR-V modules are streams of 32-bit words that begin
 * with a 5-word header (magic, version, generator, bound, schema; section
 * "SPIR-V Library", header listing) followed by instructions whose first word
 * holds the word count (high 16 bits) and opcode (low 16 bits); every
 * instruction and operand writes its own words and reports its word count
 * (section "Parsing Operand Kinds"); IDs are allocated once per module and
 * each is assigned once (section "Enabling Function Composition"); the bound
 * is recomputed when the module is written; the disassembler turns binaries
 * back into instructions (section "Dis/Assembler") and the library validates
 * modules before storing them (section "Validation Rules").
 *
 * Batches are CSR-packed: module m is words[mod_off[m] .. mod_off[m+1]).
 * All pointers to batch data, outputs and the workspace are DEVICE pointers
 * (hipMalloc'd or torch CUDA tensors) owned by the caller; the library owns
 * only the context.  Every call is asynchronous on the given stream
 * (hipStream_t passed as void*; NULL = the default stream), performs no host
 * synchronisation and no allocation, and may be captured into a HIP graph.
 * Calls that share a workspace must be ordered (same stream or events).
 *
 * Return values are synchronous and report argument / environment problems
 * only (SPV_ERR_*).  Problems in the data never fail a call: they are
 * reported per module in spv_result / the encode status arrays.
 */
#ifndef SPVGPU_H
#define SPVGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- call status ------------------------------------------------------- */
#define SPV_SUCCESS 0
#define SPV_ERR_INVALID_ARG (-1) /* null pointer, negative size, misaligned words, bad flags */
#define SPV_ERR_CAPACITY (-2)    /* idx_cap < n_words, or words_cap < 5*n_modules + n_records */
#define SPV_ERR_WORKSPACE (-3)   /* ws too small (see spv_workspace_size) or null */
#define SPV_ERR_HIP (-4)         /* a HIP runtime call failed; see spv_last_hip_error */
#define SPV_ERR_LIMIT (-5)       /* a module has >= 2^32 words, or too many modules */
#define SPV_ERR_CANCELED (-6)    /* (server completion status) the request was cancelled before a batch took it */

/* ---- per-module result codes (decode / validate) ------------------------
 * Checks run in stages; the first failing stage decides the code.
 *   header : n < 5 -> TRUNCATED_HEADER (err_word = n); magic != 0x07230203
 *            -> BAD_MAGIC (0); version word with non-zero reserved bytes,
 *            major != 1 or minor > 6 -> BAD_VERSION (1); schema != 0 ->
 *            BAD_SCHEMA (4).
 *   parse  : walk from word 5; at each instruction start p, in this order:
 *            word count 0 or past the module end -> BAD_WORD_COUNT; opcode
 *            not in the grammar table -> UNKNOWN_OPCODE; word count not the
 *            table's -> BAD_WORD_COUNT; string (OpName, OpEntryPoint) not
 *            NUL-terminated in its last word with zero padding -> BAD_STRING.  err_word = p
 *            (word offset in the module), n_inst = instructions before p.
 *   semantic (validate only): over ID-role words, id == 0 or id >= bound ->
 *            OOB (mask 1); a result ID defined twice -> DUP (mask 2); an ID
 *            used but defined nowhere in the module -> UNDEF (mask 4).
 *            code = first of OOB > DUP > UNDEF; err_word = 0xFFFFFFFF.
 * For SPV_OK and semantic codes err_word is 0xFFFFFFFF.                    */
#define SPV_OK 0
#define SPV_E_TRUNCATED_HEADER 1
#define SPV_E_BAD_MAGIC 2
#define SPV_E_BAD_VERSION 3
#define SPV_E_BAD_SCHEMA 4
#define SPV_E_BAD_WORD_COUNT 5
#define SPV_E_UNKNOWN_OPCODE 6
#define SPV_E_BAD_STRING 7
#define SPV_E_ID_OUT_OF_BOUND 8
#define SPV_E_DUPLICATE_ID 9
#define SPV_E_UNDEFINED_ID 10
/* (spv_validate with SPV_OPT_MODULE_RULES) a module that passed every check
 * above lacks what section "Validation Rules" requires of every module:
 * sem_mask = 8 no OpCapability | 16 no OpMemoryModel | 32 no OpFunction |
 * 64 no OpEntryPoint. */
#define SPV_E_MODULE_RULES 11

/* spv_validate options (option_flags, a bit set):
 *   SPV_OPT_NO_SEMANTIC  stop after the parse stage: the call is spv_decode
 *                        (section "Parsing Operand Kinds"); cannot be combined
 *                        with the options of the semantic stage below
 *                        (SPV_ERR_INVALID_ARG);
 *   SPV_OPT_MODULE_RULES hold modules that pass every check to the
 *                        module-level rules of section "Validation Rules"
 *                        (SPV_E_MODULE_RULES);
 *   SPV_OPT_DEBUG_CHECKS before anything else, a device check of mod_off:
 *                        mod_off[0] == 0, non-decreasing, every module below
 *                        2^32 words, mod_off[n_modules] == n_words.  On a
 *                        violation nothing else runs and the call returns
 *                        SPV_ERR_INVALID_ARG.  The check reads its status word
 *                        back, so the call synchronises its stream, and under
 *                        stream capture it returns SPV_ERR_INVALID_ARG;
 *   SPV_OPT_SEM_OFFSETS  a module that fails the semantic stage gets in
 *                        err_word the word offset (within the module) of the
 *                        first instruction, in module order, that breaks
 *                        the rule of its primary code: an ID operand out of
 *                        bound, a result ID that an earlier instruction
 *                        already defines, a used ID that is not defined;
 *   SPV_OPT_DEF_BEFORE_USE the stricter reading of the SSA rule of section
 *                        "Enabling Function Composition": a used ID must be
 *                        defined by an earlier instruction (OpName targets
 *                        and OpEntryPoint functions may still name later
 *                        definitions); other uses are SPV_E_UNDEFINED_ID.
 * The last two run extra kernels after the call's results are written; they
 * need the instruction index (idx_off / idx_op, else SPV_ERR_INVALID_ARG)
 * and reuse the workspace's ID sets. */
#define SPV_OPT_NO_SEMANTIC 1u
#define SPV_OPT_MODULE_RULES 2u
#define SPV_OPT_DEBUG_CHECKS 4u
#define SPV_OPT_SEM_OFFSETS 8u
#define SPV_OPT_DEF_BEFORE_USE 16u

/* ---- encode status codes (per module) ---------------------------------- */
#define SPV_ENC_OK 0
#define SPV_ENC_UNKNOWN_OPCODE 1 /* opcode not in the grammar table */
#define SPV_ENC_OPERAND_COUNT 2  /* non-string operand count differs from the table (OpName 1, OpEntryPoint 2) */
#define SPV_ENC_BAD_STRING 3     /* string on a record without a string operand, or a NUL inside a string */
#define SPV_ENC_TOO_LONG 4       /* word count would exceed 65535 */
#define SPV_ENC_BAD_ID 5         /* an ID operand equals 0xFFFFFFFF (bound not representable) */
#define SPV_ENC_CAPACITY 6       /* the module would end past words_cap (its words are not kept) */

/* Result code (decode / validate code or encode status) of every module of a
 * call in which a kernel's wait on another block exceeded its spin limit
 * (a scheduling failure, not a property of the input); the call's outputs
 * are then not valid and the call may be repeated. */
#define SPV_E_SPIN_LIMIT 0xDEAD

/* Grammar table (the twelve opcodes of the synthetic workloads and
 * OpEntryPoint): opcode, word count, operand roles (U = ID use, D = result
 * ID, L = literal, S = string words):
 *   OpName 5 (>=3, U S...), OpMemoryModel 14 (3, L L), OpEntryPoint 15
 *   (>=4, L U S...; its string must end in its last word: the interface IDs
 *   SPIR-V allows after the name are not part of this table), OpCapability 17
 *   (2, L), OpTypeInt 21 (4, D L L), OpConstant 43 (4, U D L), OpFunction
 *   54 (5, U D L U), OpFunctionEnd 56 (1), OpLoad 61 (4, U D U), OpStore 62
 *   (3, U U), OpIAdd 128 (5, U D U U), OpLabel 248 (2, D), OpReturn 253 (1). */

typedef struct spv_ctx spv_ctx;

/* 16 bytes per module. */
typedef struct {
  uint32_t code;     /* SPV_OK or SPV_E_* */
  uint32_t sem_mask; /* 1 OOB | 2 DUP | 4 UNDEF (validate); missing rules (SPV_E_MODULE_RULES); else 0 */
  uint32_t err_word; /* offending word offset within the module, or 0xFFFFFFFF */
  uint32_t n_inst;   /* instructions decoded (before the failing one, if any) */
} spv_result;

/* Create a context on HIP device `hip_device` (holds device properties and
 * launch tuning).  *out receives the handle.  SPV_ERR_HIP if the device
 * cannot be used. */
int spv_create(spv_ctx **out, int hip_device);
int spv_destroy(spv_ctx *ctx);

/* Device-side error text of the last failing HIP call on this context. */
const char *spv_last_hip_error(spv_ctx *ctx);

/* Launch tuning (0 = keep the built-in default).  blocks_per_cu sets the
 * persistent grid of the single-pass decode/validate walk (the fallback when
 * some tile's entry cannot be settled in advance); encode_block sets the
 * records per encode block (a multiple of 256, at most 4096, default 4096;
 * SPV_ERR_INVALID_ARG otherwise). */
int spv_set_tuning(spv_ctx *ctx, int blocks_per_cu, int encode_block);
/* Current launch tuning of the context. */
int spv_get_tuning(spv_ctx *ctx, int *blocks_per_cu, int *encode_block);

/* Grids of the two kernels that run on every decode/validate call whose
 * tiles settle (0 = keep): blocks per CU of the chain pass and of the
 * resolved walk, each 1..64 (SPV_ERR_INVALID_ARG otherwise).  Both take
 * their tiles in a static order, so any grid is correct; the default is the
 * kernels' resident blocks per CU. */
int spv_set_grids(spv_ctx *ctx, int chain_blocks_per_cu, int walk_blocks_per_cu);
/* Current grids (blocks per CU) of the chain pass and the resolved walk. */
int spv_get_grids(spv_ctx *ctx, int *chain_blocks_per_cu, int *walk_blocks_per_cu);

/* Bytes of workspace that spv_decode / spv_validate need for a batch of
 * n_modules modules and n_words words (about 8 bytes per word plus small
 * per-module and per-tile state).  The workspace needs no initialisation
 * and may be reused by later calls on the same stream. */
int spv_workspace_size(spv_ctx *ctx, int64_t n_modules, int64_t n_words, size_t *bytes);

/* Decode: the header and parse stages of the validator (section "Validation
 * Rules": the library checks a module before it stores it), reading the
 * binary as the disassembler does (section "Dis/Assembler") with the header
 * fields of section "SPIR-V Library" and the operand word counts of section
 * "Parsing Operand Kinds".  results[m] for every module, and, when
 * idx_off / idx_op are non-NULL, the instruction index in gapped CSR form:
 * module m's instruction j is idx_off[mod_off[m] + j] (word offset of its
 * first word within the module) and idx_op[mod_off[m] + j] (opcode), for
 * j < results[m].n_inst.  Entries past n_inst are unspecified.  idx_cap must
 * be >= n_words when the index is requested.
 *   words   : uint32[n_words], 16-byte aligned
 *   mod_off : int64[n_modules+1], mod_off[0] = 0, non-decreasing,
 *             mod_off[n_modules] = n_words; each module < 2^32 words
 *   results : spv_result[n_modules]
 *   ws      : workspace of ws_bytes >= spv_workspace_size(...)          */
int spv_decode(spv_ctx *ctx, const uint32_t *words, const int64_t *mod_off, int64_t n_modules, int64_t n_words,
               uint32_t *idx_off, uint16_t *idx_op, int64_t idx_cap, spv_result *results, void *ws,
               size_t ws_bytes, void *stream);

/* Validate: decode plus the semantic stage: every ID below the header's
 * bound (section "SPIR-V Library", bound paragraph), each result ID defined
 * once and every used ID defined somewhere in the module (the SSA rule of
 * section "Enabling Function Composition").  Same arguments as spv_decode,
 * plus option_flags, a set of SPV_OPT_* bits (SPV_ERR_INVALID_ARG for others). */
int spv_validate(spv_ctx *ctx, const uint32_t *words, const int64_t *mod_off, int64_t n_modules, int64_t n_words,
                 uint32_t *idx_off, uint16_t *idx_op, int64_t idx_cap, spv_result *results, uint32_t option_flags,
                 void *ws, size_t ws_bytes, void *stream);

/* spv_validate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same call without a workspace argument.  Its workspace is the
 * library's own scratch array, SPV_NOALLOC_SCRATCH_BYTES per GPU, which each
 * GPU the library runs on holds until the process ends; its address on a
 * device is resolved by spv_create.  The call allocates nothing, creates no
 * event (timing is not recorded on this path) and needs no initialised
 * scratch.  Every call on one GPU shares that GPU's scratch, so calls that
 * overlap on one GPU (different streams without ordering) race: order them.
 * Arguments and results as for spv_validate; SPV_ERR_WORKSPACE when the
 * batch needs more than the scratch holds (spv_workspace_size(...) >
 * SPV_NOALLOC_SCRATCH_BYTES: about 7.5M words for one module), SPV_ERR_HIP
 * when the scratch address could not be resolved on the context's device. */
#define SPV_NOALLOC_SCRATCH_BYTES (64u << 20)
int spv_validate_noalloc(spv_ctx *ctx, const uint32_t *words, const int64_t *mod_off, int64_t n_modules,
                         int64_t n_words, uint32_t *idx_off, uint16_t *idx_op, int64_t idx_cap, spv_result *results,
                         uint32_t option_flags, void *stream);

/* Bytes of workspace spv_decode_records needs. */
int spv_records_workspace_size(spv_ctx *ctx, int64_t n_modules, int64_t n_words, size_t *bytes);

/* Decode's records mode: the instructions a spv_decode / spv_validate call
 * found, in the record layout spv_encode takes (the disassembler's
 * instruction view, section "Dis/Assembler", in the form of the library's
 * writer, section "SPIR-V Library").  Module m contributes the records of
 * its valid instruction prefix, results[m].n_inst of them, or none when its
 * header check failed (codes 1..4).  Record r: op[r] = its opcode; its
 * non-string operand words opnd[opnd_off[r] .. opnd_off[r+1]) (OpName: its
 * target ID; OpEntryPoint: execution model and function ID); its string bytes
 * chars[str_off[r] .. str_off[r+1]) (OpName, OpEntryPoint: the name up to,
 * not including, its NUL; none otherwise).  rec_mod_off
 * receives the records' CSR by module; the record count is
 * rec_mod_off[n_modules] (all -1 if a kernel's wait exceeded its spin limit).
 * For a valid module, spv_encode of its records gives its words back.
 *   words, mod_off : the batch the index was computed on (as for spv_decode)
 *   idx_off, results : the index and results of that call (idx_op unused)
 *   op uint16[n_words], opnd_off int32[n_words+1], opnd uint32[n_words],
 *   str_off int32[n_words+1], chars uint8[4*n_words], rec_mod_off
 *   int64[n_modules+1]: device buffers owned by the caller.
 * n_words must be below 2^29 (SPV_ERR_LIMIT). */
int spv_decode_records(spv_ctx *ctx, const uint32_t *words, const int64_t *mod_off, int64_t n_modules,
                       int64_t n_words, const uint32_t *idx_off, const spv_result *results, uint16_t *op,
                       int32_t *opnd_off, uint32_t *opnd, int32_t *str_off, uint8_t *chars, int64_t *rec_mod_off,
                       void *ws, size_t ws_bytes, void *stream);

/* Options of spv_decode_text: the five switches of the disassembler's
 * options listing (section "Dis/Assembler"), in the listing's order. */
#define SPV_TEXT_HIGHLIGHT 1u    /* ANSI colours: opcode 36, IDs 33, literals 34, strings 32, reset 0 */
#define SPV_TEXT_INLINE_NAMES 2u /* %<name> for IDs that an OpName names */
#define SPV_TEXT_NO_INDENT 4u    /* no padding to column 15 */
#define SPV_TEXT_GROUP 8u        /* an empty line before each OpFunction and OpLabel */
#define SPV_TEXT_NO_HEADER 16u   /* no "; SPIR-V" header comment lines */

/* Bytes of workspace spv_decode_text needs (it depends on
 * SPV_TEXT_INLINE_NAMES: about 4 bytes per word without it, up to 32 with it). */
int spv_text_workspace_size(spv_ctx *ctx, int64_t n_modules, int64_t n_words, uint32_t options, size_t *bytes);

/* Decode's text mode: disassembly of the instructions a spv_decode /
 * spv_validate call found into SPIR-V assembly text (section "Dis/Assembler":
 * opcodes and operands mapped back to text, under the five switches of its
 * options listing).  Module m's text covers its valid instruction prefix
 * (results[m].n_inst instructions), or is empty when its header check failed
 * (codes 1..4).  The format:
 *   - unless SPV_TEXT_NO_HEADER: "; SPIR-V", "; Version: M.m",
 *     "; Generator: g", "; Bound: b", "; Schema: s" lines (decimal);
 *   - one line per instruction: [padding][%r = ]OpName[ operand]..."\n";
 *     the result ID moves left of " = " and the other operands keep their
 *     order; unless SPV_TEXT_NO_INDENT, spaces pad the line so that the
 *     opcode name starts at column 15 (none if "%r = " is 15 or wider);
 *   - IDs print as %<decimal>; with SPV_TEXT_INLINE_NAMES as %<name> when
 *     the module's first OpName of the ID has a usable name (non-empty, only
 *     [A-Za-z0-9_], not starting with a digit; not made unique);
 *   - literals print in decimal, or as their SPIR-V enumerant for the
 *     capability, addressing model, memory model and execution model operands
 *     of the table, and the function control mask as None or its bits
 *     (Inline|DontInline|Pure|Const) joined by '|';
 *   - strings print in double quotes with '"' and '\' escaped by '\';
 *   - SPV_TEXT_GROUP: an empty line before each OpFunction and OpLabel;
 *   - SPV_TEXT_HIGHLIGHT: ESC[3Xm ... ESC[0m around each opcode name, ID,
 *     literal and string (padding counts visible characters only).
 *   words, mod_off, idx_off, results : the batch and the index and results of
 *     the decode call made on it (the module rules code 11 counts as decoded)
 *   text : device buffer of text_cap bytes, 4-byte aligned; it receives the
 *     first min(total, text_cap) bytes of the whole text (a text_cap of 0 only
 *     sizes it)
 *   text_mod_off : int64[n_modules+1] device buffer; module m's text is
 *     text[text_mod_off[m] .. text_mod_off[m+1]), text_mod_off[n_modules] is
 *     the total; a module is complete in text iff text_mod_off[m+1] <=
 *     text_cap (all -1 if a kernel's wait exceeded its spin limit)
 * Asynchronous on stream; SPV_ERR_INVALID_ARG for unknown option bits or a
 * misaligned text, SPV_ERR_LIMIT for n_words >= 2^29 or n_modules >= 2^26,
 * SPV_ERR_WORKSPACE when ws is smaller than spv_text_workspace_size. */
int spv_decode_text(spv_ctx *ctx, const uint32_t *words, const int64_t *mod_off, int64_t n_modules, int64_t n_words,
                    const uint32_t *idx_off, const spv_result *results, uint32_t options, uint8_t *text,
                    int64_t text_cap, int64_t *text_mod_off, void *ws, size_t ws_bytes, void *stream);

/* Host-side upper bound on the words spv_encode may write:
 * 5*n_modules + n_records + n_opnd_words + n_string_records + n_chars/4. */
int spv_encode_bound(int64_t n_modules, int64_t n_records, int64_t n_opnd_words, int64_t n_string_records,
                     int64_t n_chars, int64_t *max_words);

/* Bytes of workspace spv_encode needs. */
int spv_encode_workspace_size(spv_ctx *ctx, int64_t n_modules, int64_t n_records, size_t *bytes);

/* Encode records to SPIR-V words (the library's write step, section "SPIR-V
 * Library": each record writes (wc << 16) | opcode, its operands and its
 * string packed little-endian and zero padded; the header gets magic,
 * version_word, generator_word, bound = 1 + the largest ID operand (1 if
 * none), schema 0).  Records are CSR by module: module m owns records
 * rec_mod_off[m] .. rec_mod_off[m+1]; record r has opcode op[r], operands
 * opnd[opnd_off[r] .. opnd_off[r+1]) and string bytes
 * chars[str_off[r] .. str_off[r+1]) (no NUL; only OpName and OpEntryPoint
 * may have one).
 * A module with a failing record writes no words; enc_code[m] /
 * enc_bad_record[m] (module-relative index of its first failing record, -1
 * if none) say why.  word_mod_off (n_modules+1) receives the dense output
 * CSR.  words_cap >= spv_encode_bound(...) always suffices; a smaller one
 * (at least 5*n_modules + n_records, else SPV_ERR_CAPACITY) is accepted, and
 * every module that would end past it gets SPV_ENC_CAPACITY (with a record
 * index of -1) and no words, the modules before it keeping theirs.
 * Device pointers: op uint16[n_records], opnd_off int32[n_records+1],
 * opnd uint32[opnd_off[n]], str_off int32[n_records+1], chars uint8,
 * rec_mod_off int64[n_modules+1], words_out uint32[words_cap],
 * word_mod_off int64[n_modules+1], enc_code uint32[n_modules],
 * enc_bad_record int64[n_modules]. */
int spv_encode(spv_ctx *ctx, const uint16_t *op, const int32_t *opnd_off, const uint32_t *opnd, const int32_t *str_off,
               const uint8_t *chars, const int64_t *rec_mod_off, int64_t n_modules, int64_t n_records,
               uint32_t version_word, uint32_t generator_word, uint32_t *words_out, int64_t *word_mod_off,
               int64_t words_cap, uint32_t *enc_code, int64_t *enc_bad_record, void *ws, size_t ws_bytes,
               void *stream);

/* Measurement hook.  When enabled, every spv_decode / spv_validate call on
 * this context records a pair of HIP events on the call's stream around its
 * boundary-recovery and walk kernels (chain pass, resolve pass, resolved
 * walk, single-pass walk: the bulk of the call); spv_read_timing waits
 * for those events, returns their summed duration in milliseconds and the
 * number of launches since the last read, and clears them.  Not for use
 * inside graph capture. */
int spv_set_timing(spv_ctx *ctx, int enable);
int spv_read_timing(spv_ctx *ctx, double *total_ms, int64_t *n_launches);

/* ---- serving: continuous batching over a stream of requests ------------
 * A server validates one SPIR-V module per request.  Requests (host word
 * buffers that the caller keeps alive until their completion is polled) carry
 * an arrival time; a worker thread admits arrived requests into `n_slots`
 * slots, each with its own stream, pinned staging and device buffers sized
 * from device_budget_bytes (the index stays on the device).  Whenever a slot
 * is free, every arrived request that fits joins that slot's next batch (at
 * most max_batch_modules; 1 gives one module per launch), which is copied in,
 * validated with spv_validate (or, with use_graphs, a HIP graph captured per
 * padded size bucket and replayed) and whose results are copied back while
 * other slots' batches run.  Latency = completion time - arrival time, on
 * the server's steady clock (ns since spv_server_start).  A request larger
 * than a slot completes with status SPV_ERR_CAPACITY.  The server keeps the
 * context; destroy the server before the context. */
typedef struct spv_server spv_server;

typedef struct {
  int64_t id;            /* caller's request id */
  spv_result result;     /* the module's validation result */
  int32_t status;        /* SPV_SUCCESS, SPV_ERR_CAPACITY, SPV_ERR_CANCELED or SPV_ERR_HIP */
  int32_t pad;
  int64_t t_arrival_ns;  /* arrival time */
  int64_t t_done_ns;     /* time the worker saw the batch complete */
  int64_t batch_modules; /* modules in the batch that carried this request */
} spv_completion;

int spv_server_create(spv_server **out, spv_ctx *ctx, int hip_device, size_t device_budget_bytes, int n_slots,
                      int64_t max_batch_modules, int64_t slot_max_modules, int use_graphs);
/* Start the worker; arrival times are relative to this call. */
int spv_server_start(spv_server *srv);
/* Queue n requests in arrival order: ids[i], host words[i] (n_words[i] words)
 * arriving at t_arrival_ns[i] (NULL or negative = now). */
int spv_server_submit(spv_server *srv, int64_t n, const int64_t *ids, const uint32_t *const *words,
                      const int64_t *n_words, const int64_t *t_arrival_ns);
/* Move up to max_out completions to out; *pending = submitted, not completed. */
/* Cancel queued requests by id: every listed request that no batch has taken
 * yet completes with status SPV_ERR_CANCELED (and a zero result) at the
 * worker's next step; ids of requests already in a batch, done or unknown
 * are ignored.  Cancels apply to requests submitted before the call. */
int spv_server_cancel(spv_server *srv, int64_t n, const int64_t *ids);
int spv_server_poll(spv_server *srv, spv_completion *out, int64_t max_out, int64_t *n_out, int64_t *pending);
int spv_server_stats(spv_server *srv, int64_t *n_batches, int64_t *n_modules, int64_t *n_words, int64_t *max_batch,
                     int64_t *slot_capacity_words);
/* Finish all queued work, then free the server. */
int spv_server_destroy(spv_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* SPVGPU_H */
