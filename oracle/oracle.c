/*
 * Sequential CPU oracle for batched SPIR-V decode, validate and encode.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant generator with the GPU path and includes
 * nothing from it.
 *
 * What it follows (Beehive SPIR-V Toolkit paper, arXiv 2305.09493):
 *   - header fields in the standard's order, bound recomputed when the module
 *     is written (section "SPIR-V Library", header-construction listing and
 *     the paragraph on the initial bound);
 *   - every instruction and operand writes its own 32-bit words and reports a
 *     word count that sizes the module (section "Parsing Operand Kinds");
 *   - IDs are requested once per module and each construct is assigned once,
 *     the SSA rule (section "Enabling Function Composition", SSA paragraph);
 *   - the disassembler turns the binary back into instructions (section
 *     "Dis/Assembler"); the library validates modules before storing them
 *     (section "Validation Rules").
 * SPIR-V binary facts used: magic 0x07230203, schema word 0, first word of an
 * instruction = (word count << 16) | opcode.  The grammar table below is this
 * file's own copy of the twelve opcodes of the synthetic workload plus
 * OpEntryPoint, which the module-level rules need.
 *
 * Where the paper is silent the readings are: word counts are in words and
 * include the first word; the undefined-ID rule means "defined anywhere in the
 * module"; checks run header -> parse (first failing instruction) -> semantic
 * (set of classes, primary code by OOB > DUP > UNDEF); at one instruction the
 * order is count/overrun -> opcode -> fixed count -> string; the version word
 * must have zero reserved bytes, major 1 and minor <= 6; ID 0 is invalid.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAGIC 0x07230203u

enum {
  ORC_OK = 0,
  ORC_TRUNCATED_HEADER = 1,
  ORC_BAD_MAGIC = 2,
  ORC_BAD_VERSION = 3,
  ORC_BAD_SCHEMA = 4,
  ORC_BAD_WORD_COUNT = 5,
  ORC_UNKNOWN_OPCODE = 6,
  ORC_BAD_STRING = 7,
  ORC_ID_OUT_OF_BOUND = 8,
  ORC_DUPLICATE_ID = 9,
  ORC_UNDEFINED_ID = 10,
  ORC_MODULE_RULES = 11,
};
enum {
  ORC_ENC_OK = 0,
  ORC_ENC_UNKNOWN_OPCODE = 1,
  ORC_ENC_OPERAND_COUNT = 2,
  ORC_ENC_BAD_STRING = 3,
  ORC_ENC_TOO_LONG = 4,
  ORC_ENC_BAD_ID = 5,
};

typedef struct {
  uint32_t code, sem_mask, err_word, n_inst;
} orc_result;

/* One grammar entry: opcode, word count (0 = variable: the operands before
 * the 'S' role, then a string that runs to the last word), and the role of
 * each operand word after the first word: 'U' ID use, 'D' result ID,
 * 'L' literal, 'S' string words to the end.  OpEntryPoint's interface IDs,
 * which in SPIR-V may follow its name, are not part of this grammar: its
 * string must end in its last word. */
typedef struct {
  uint16_t opcode;
  uint16_t word_count;
  const char *roles;
} orc_inst;

static const orc_inst GRAMMAR[] = {
    {5, 0, "US"},     /* OpName         */
    {14, 3, "LL"},    /* OpMemoryModel  */
    {15, 0, "LUS"},   /* OpEntryPoint   */
    {17, 2, "L"},     /* OpCapability   */
    {21, 4, "DLL"},   /* OpTypeInt      */
    {43, 4, "UDL"},   /* OpConstant     */
    {54, 5, "UDLU"},  /* OpFunction     */
    {56, 1, ""},      /* OpFunctionEnd  */
    {61, 4, "UDU"},   /* OpLoad         */
    {62, 3, "UU"},    /* OpStore        */
    {128, 5, "UDUU"}, /* OpIAdd         */
    {248, 2, "D"},    /* OpLabel        */
    {253, 1, ""},     /* OpReturn       */
};

static const orc_inst *lookup(uint32_t opcode) {
  for (size_t i = 0; i < sizeof(GRAMMAR) / sizeof(GRAMMAR[0]); ++i)
    if (GRAMMAR[i].opcode == opcode) return &GRAMMAR[i];
  return NULL;
}

/* Operand words before the string of a variable instruction (OpName 1,
 * OpEntryPoint 2); for a fixed one, all of its operand words. */
static uint32_t fixed_operands(const orc_inst *g) {
  uint32_t k = 0;
  while (g->roles[k] != '\0' && g->roles[k] != 'S') ++k;
  return k;
}

/* A literal string is stored as bytes little-endian within each word, ends
 * with a NUL byte, and is zero padded to a whole word.  So the first NUL must
 * lie in the last word and every byte after it must be zero. */
static int string_ok(const uint32_t *w, uint64_t n_words) {
  uint64_t n_bytes = 4 * n_words;
  uint64_t first_nul = n_bytes;
  for (uint64_t b = 0; b < n_bytes; ++b) {
    uint32_t byte = (w[b / 4] >> (8 * (b % 4))) & 0xFFu;
    if (byte == 0) {
      first_nul = b;
      break;
    }
  }
  if (first_nul == n_bytes) return 0;          /* no terminator */
  if (first_nul / 4 != n_words - 1) return 0;  /* terminator not in the last word */
  for (uint64_t b = first_nul; b < n_bytes; ++b)
    if (((w[b / 4] >> (8 * (b % 4))) & 0xFFu) != 0) return 0;
  return 1;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

static int contains(const uint32_t *sorted, uint64_t n, uint32_t v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (sorted[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && sorted[lo] == v;
}

/* Module-level rules (section "Validation Rules"), a stage after the
 * semantic one for a module that passed it: the module must declare a
 * capability (OpCapability, 17), define its memory model (OpMemoryModel, 14),
 * declare a function (OpFunction, 54) and declare an entry point
 * (OpEntryPoint, 15).  Returns the missing rules as 8 (capability) | 16
 * (memory model) | 32 (function) | 64 (entry point). */
static uint32_t missing_rules(const uint32_t *w, uint64_t n) {
  int capability = 0, memory_model = 0, function = 0, entry_point = 0;
  for (uint64_t p = 5; p < n; p += w[p] >> 16) {
    uint32_t op = w[p] & 0xFFFFu;
    if (op == 17) capability = 1;
    if (op == 14) memory_model = 1;
    if (op == 54) function = 1;
    if (op == 15) entry_point = 1;
  }
  return (capability ? 0u : 8u) | (memory_model ? 0u : 16u) | (function ? 0u : 32u) | (entry_point ? 0u : 64u);
}

/* Options of the semantic stage (bits of `opts`). */
enum { ORC_OPT_RULES = 1, ORC_OPT_OFFSETS = 2, ORC_OPT_BEFORE_USE = 4 };

/* An ID use that may name an ID defined later in the module: the target of
 * OpName and the function of OpEntryPoint (debug and mode-setting operands,
 * which SPIR-V places before the definitions they name). */
static int forward_use_ok(uint32_t op, uint32_t slot) { return (op == 5 && slot == 0) || (op == 15 && slot == 1); }

typedef struct {
  uint32_t v, pos;
} orc_def;

static int cmp_def(const void *a, const void *b) {
  const orc_def *x = (const orc_def *)a, *y = (const orc_def *)b;
  if (x->v != y->v) return (x->v > y->v) - (x->v < y->v);
  return (x->pos > y->pos) - (x->pos < y->pos);
}

/* Word offset of the first definition of v, or 0xFFFFFFFF if none (defs
 * sorted by ID, then position). */
static uint32_t first_def(const orc_def *d, uint64_t n, uint32_t v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (d[mid].v < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && d[lo].v == v) ? d[lo].pos : 0xFFFFFFFFu;
}

/* Semantic-stage positions of a module that passed the parse stage: the word
 * offset of the first instruction (module order) with an ID operand out of
 * bound, of the first whose in-bound result ID an earlier instruction already
 * defines, and of the first with an in-bound ID use that no instruction
 * defines, or, with before_use, that no earlier instruction defines (OpName
 * targets and OpEntryPoint functions may name later definitions).
 * 0xFFFFFFFF where there is none.  Returns 0, or -1 without memory. */
static int semantic_positions(const uint32_t *w, uint64_t n, uint32_t bound, int before_use, uint32_t *f_oob,
                              uint32_t *f_dup, uint32_t *f_undef) {
  orc_def *defs = (orc_def *)malloc((n + 1) * sizeof(orc_def));
  if (!defs) return -1;
  uint64_t nd = 0;
  *f_oob = *f_dup = *f_undef = 0xFFFFFFFFu;
  for (uint64_t p = 5; p < n; p += w[p] >> 16) {
    const orc_inst *g = lookup(w[p] & 0xFFFFu);
    for (uint32_t s = 0; g->roles[s] != '\0' && g->roles[s] != 'S'; ++s) {
      char role = g->roles[s];
      if (role != 'U' && role != 'D') continue;
      uint32_t v = w[p + 1 + s];
      if (v == 0 || v >= bound) {
        if (*f_oob == 0xFFFFFFFFu) *f_oob = (uint32_t)p;
      } else if (role == 'D') {
        defs[nd].v = v;
        defs[nd].pos = (uint32_t)p;
        ++nd;
      }
    }
  }
  qsort(defs, nd, sizeof(orc_def), cmp_def);
  for (uint64_t i = 1; i < nd; ++i) /* the second definition of an ID */
    if (defs[i].v == defs[i - 1].v && defs[i].pos < *f_dup) *f_dup = defs[i].pos;
  for (uint64_t p = 5; p < n && *f_undef == 0xFFFFFFFFu; p += w[p] >> 16) {
    uint32_t op = w[p] & 0xFFFFu;
    const orc_inst *g = lookup(op);
    for (uint32_t s = 0; g->roles[s] != '\0' && g->roles[s] != 'S'; ++s) {
      uint32_t v = w[p + 1 + s];
      if (g->roles[s] != 'U' || v == 0 || v >= bound) continue;
      uint32_t d = first_def(defs, nd, v);
      if (d == 0xFFFFFFFFu || (before_use && !forward_use_ok(op, s) && d >= p)) *f_undef = (uint32_t)p;
    }
  }
  free(defs);
  return 0;
}

/* Decode (and, if semantic != 0, validate) one module w[0..n).  Instruction
 * j of the valid prefix goes to idx_off[j] / idx_op[j] when they are given.
 * Options of the semantic stage (opts): ORC_OPT_BEFORE_USE counts a use
 * whose ID only a later instruction defines as undefined (the forward
 * operands of forward_use_ok aside); ORC_OPT_OFFSETS puts in err_word the
 * word offset of the first instruction of the primary semantic class;
 * ORC_OPT_RULES holds a module that passes every check to the module-level
 * rules.  Returns 0, or -1 if memory for the semantic stage could not be had. */
static int check_module(const uint32_t *w, uint64_t n, int semantic, int opts, uint32_t *idx_off, uint16_t *idx_op,
                        orc_result *r) {
  const int rules = (opts & ORC_OPT_RULES) != 0;
  r->code = ORC_OK;
  r->sem_mask = 0;
  r->err_word = 0xFFFFFFFFu;
  r->n_inst = 0;

  /* 1. header, first failure wins */
  if (n < 5) {
    r->code = ORC_TRUNCATED_HEADER;
    r->err_word = (uint32_t)n;
    return 0;
  }
  if (w[0] != ORC_MAGIC) {
    r->code = ORC_BAD_MAGIC;
    r->err_word = 0;
    return 0;
  }
  uint32_t major = (w[1] >> 16) & 0xFFu, minor = (w[1] >> 8) & 0xFFu;
  if ((w[1] & 0xFF0000FFu) != 0 || major != 1 || minor > 6) {
    r->code = ORC_BAD_VERSION;
    r->err_word = 1;
    return 0;
  }
  if (w[4] != 0) {
    r->code = ORC_BAD_SCHEMA;
    r->err_word = 4;
    return 0;
  }
  uint32_t bound = w[3];

  /* 2. walk the instruction chain from the first word after the header */
  uint64_t p = 5, k = 0;
  while (p < n) {
    uint32_t wc = w[p] >> 16, op = w[p] & 0xFFFFu;
    const orc_inst *g = lookup(op);
    uint32_t code = ORC_OK;
    if (wc == 0 || p + wc > n) code = ORC_BAD_WORD_COUNT;
    else if (g == NULL) code = ORC_UNKNOWN_OPCODE;
    else if ((g->word_count != 0 && wc != g->word_count) || (g->word_count == 0 && wc < 2 + fixed_operands(g)))
      code = ORC_BAD_WORD_COUNT;
    else if (g->word_count == 0 && !string_ok(w + p + 1 + fixed_operands(g), wc - 1 - fixed_operands(g)))
      code = ORC_BAD_STRING;
    if (code != ORC_OK) {
      r->code = code;
      r->err_word = (uint32_t)p;
      r->n_inst = (uint32_t)k;
      return 0;
    }
    if (idx_off) idx_off[k] = (uint32_t)p;
    if (idx_op) idx_op[k] = (uint16_t)op;
    ++k;
    p += wc;
  }
  r->n_inst = (uint32_t)k;
  if (!semantic) return 0;

  /* 3. ID checks over every ID-role word */
  uint64_t cap = n; /* an upper bound on the number of ID words */
  uint32_t *defs = (uint32_t *)malloc((cap + 1) * sizeof(uint32_t));
  uint32_t *uses = (uint32_t *)malloc((cap + 1) * sizeof(uint32_t));
  if (!defs || !uses) {
    free(defs);
    free(uses);
    return -1;
  }
  uint64_t nd = 0, nu = 0;
  int oob = 0;
  p = 5;
  while (p < n) {
    uint32_t wc = w[p] >> 16, op = w[p] & 0xFFFFu;
    const orc_inst *g = lookup(op);
    for (uint32_t s = 0; g->roles[s] != '\0' && g->roles[s] != 'S'; ++s) {
      char role = g->roles[s];
      if (role != 'U' && role != 'D') continue;
      uint32_t v = w[p + 1 + s];
      if (v == 0 || v >= bound) {
        oob = 1;
        continue;
      }
      if (role == 'D') defs[nd++] = v;
      else uses[nu++] = v;
    }
    p += wc;
  }
  qsort(defs, nd, sizeof(uint32_t), cmp_u32);
  int dup = 0, undef = 0;
  for (uint64_t i = 1; i < nd; ++i)
    if (defs[i] == defs[i - 1]) dup = 1;
  for (uint64_t i = 0; i < nu; ++i)
    if (!contains(defs, nd, uses[i])) undef = 1;
  free(defs);
  free(uses);
  uint32_t f_oob = 0xFFFFFFFFu, f_dup = 0xFFFFFFFFu, f_undef = 0xFFFFFFFFu;
  if (opts & (ORC_OPT_OFFSETS | ORC_OPT_BEFORE_USE)) {
    if (semantic_positions(w, n, bound, (opts & ORC_OPT_BEFORE_USE) != 0, &f_oob, &f_dup, &f_undef) != 0) return -1;
    if (opts & ORC_OPT_BEFORE_USE) undef = f_undef != 0xFFFFFFFFu;
  }
  r->sem_mask = (oob ? 1u : 0u) | (dup ? 2u : 0u) | (undef ? 4u : 0u);
  if (oob) r->code = ORC_ID_OUT_OF_BOUND;
  else if (dup) r->code = ORC_DUPLICATE_ID;
  else if (undef) r->code = ORC_UNDEFINED_ID;
  if (opts & ORC_OPT_OFFSETS) {
    if (r->code == ORC_ID_OUT_OF_BOUND) r->err_word = f_oob;
    else if (r->code == ORC_DUPLICATE_ID) r->err_word = f_dup;
    else if (r->code == ORC_UNDEFINED_ID) r->err_word = f_undef;
  }
  if (rules && r->code == ORC_OK) {
    r->sem_mask = missing_rules(w, n);
    if (r->sem_mask) r->code = ORC_MODULE_RULES;
  }
  return 0;
}

/* Batched entry points over CSR-packed modules: module m is
 * words[mod_off[m] .. mod_off[m+1]).  Index arrays, when given, are gapped
 * CSR: module m's instruction j is at idx_off[mod_off[m] + j] (a word offset
 * within the module) and idx_op[mod_off[m] + j].  Returns 0 or -1. */
int oracle_validate(const uint32_t *words, const int64_t *mod_off, int64_t n_modules, int semantic, int opts,
                    uint32_t *idx_off, uint16_t *idx_op, orc_result *results) {
  for (int64_t m = 0; m < n_modules; ++m) {
    int64_t b = mod_off[m], e = mod_off[m + 1];
    if (e < b) return -1;
    if (check_module(words + b, (uint64_t)(e - b), semantic, opts, idx_off ? idx_off + b : NULL,
                     idx_op ? idx_op + b : NULL, &results[m]) != 0)
      return -1;
  }
  return 0;
}

/* Records mode of the disassembler: for each instruction of the valid prefix
 * of each module (none when the header check failed; the instructions before
 * the failing one when the parse stage failed; all of them otherwise), its
 * opcode, its non-string operand words and the bytes of its string
 * (excluding the NUL).  Output arrays are sized by the caller for
 * the whole batch (n_words entries each is always enough); rec_mod_off gets
 * the record CSR (n_modules+1).  Returns 0, or -1 on bad offsets. */
int oracle_records(const uint32_t *words, const int64_t *mod_off, int64_t n_modules, uint16_t *op_out,
                   int32_t *opnd_off, uint32_t *opnd, int32_t *str_off, uint8_t *chars, int64_t *rec_mod_off) {
  int64_t nr = 0, no = 0, nc = 0;
  opnd_off[0] = 0;
  str_off[0] = 0;
  rec_mod_off[0] = 0;
  for (int64_t m = 0; m < n_modules; ++m) {
    int64_t b = mod_off[m], e = mod_off[m + 1];
    if (e < b) return -1;
    const uint32_t *w = words + b;
    uint64_t n = (uint64_t)(e - b);
    orc_result r;
    check_module(w, n, 0, 0, NULL, NULL, &r);
    if (r.code == ORC_OK || r.code >= ORC_BAD_WORD_COUNT) {
      uint64_t p = 5;
      for (uint32_t j = 0; j < r.n_inst; ++j) {
        uint32_t wc = w[p] >> 16, op = w[p] & 0xFFFFu;
        const orc_inst *g = lookup(op);
        op_out[nr] = (uint16_t)op;
        if (g != NULL && g->word_count == 0) {
          uint32_t k = fixed_operands(g);
          for (uint32_t s = 1; s <= k; ++s) opnd[no++] = w[p + s];
          const uint8_t *bytes = (const uint8_t *)(w + p + 1 + k);
          for (uint64_t i = 0; bytes[i] != 0; ++i) chars[nc++] = bytes[i];
        } else {
          for (uint32_t s = 1; s < wc; ++s) opnd[no++] = w[p + s];
        }
        ++nr;
        opnd_off[nr] = (int32_t)no;
        str_off[nr] = (int32_t)nc;
        p += wc;
      }
    }
    rec_mod_off[m + 1] = nr;
  }
  return 0;
}

/* Upper bound on encoder output: every module valid. */
int64_t oracle_encode_bound(int64_t n_modules, int64_t n_records, int64_t n_opnd, int64_t n_chars) {
  return 5 * n_modules + n_records + n_opnd + n_records + n_chars / 4;
}

/* Encode every module's records to SPIR-V words (the library's write step,
 * bound recomputed as 1 + the largest ID operand, or 1 when there is none).
 * A module with a failing record produces no words at all; enc_code[m] and
 * enc_bad_record[m] (module-relative record index, -1 if none) say why.
 * word_mod_off (n_modules+1) is the dense CSR of the output.  Returns the
 * number of words written, or -1 if words_cap is too small. */
int64_t oracle_encode(const uint16_t *op, const int32_t *opnd_off, const uint32_t *opnd, const int32_t *str_off,
                      const uint8_t *chars, const int64_t *rec_mod_off, int64_t n_modules, uint32_t version_word,
                      uint32_t generator_word, uint32_t *words_out, int64_t *word_mod_off, int64_t words_cap,
                      uint32_t *enc_code, int64_t *enc_bad_record) {
  int64_t out = 0;
  word_mod_off[0] = 0;
  for (int64_t m = 0; m < n_modules; ++m) {
    int64_t r0 = rec_mod_off[m], r1 = rec_mod_off[m + 1];
    uint32_t code = ORC_ENC_OK;
    int64_t bad = -1;
    uint64_t max_id = 0;
    int any_id = 0;
    uint64_t total = 5;
    /* checks first: a failing module writes nothing */
    for (int64_t j = r0; j < r1 && code == ORC_ENC_OK; ++j) {
      const orc_inst *g = lookup(op[j]);
      int64_t n_ops = opnd_off[j + 1] - opnd_off[j];
      int64_t n_chars = str_off[j + 1] - str_off[j];
      uint64_t wc = 0;
      if (g == NULL) code = ORC_ENC_UNKNOWN_OPCODE;
      else if ((g->word_count == 0 && n_ops != (int64_t)fixed_operands(g)) ||
               (g->word_count != 0 && n_ops != g->word_count - 1))
        code = ORC_ENC_OPERAND_COUNT;
      else if (g->word_count != 0 && n_chars != 0) code = ORC_ENC_BAD_STRING;
      else if (g->word_count == 0 && memchr(chars + str_off[j], 0, (size_t)n_chars) != NULL)
        code = ORC_ENC_BAD_STRING;
      else {
        wc = 1 + (uint64_t)n_ops + (g->word_count == 0 ? (uint64_t)n_chars / 4 + 1 : 0);
        if (wc > 65535) code = ORC_ENC_TOO_LONG;
      }
      if (code == ORC_ENC_OK) {
        for (int64_t s = 0; s < n_ops; ++s) {
          char role = g->roles[s];
          if (role != 'U' && role != 'D') continue;
          uint32_t v = opnd[opnd_off[j] + s];
          if (v == 0xFFFFFFFFu) {
            code = ORC_ENC_BAD_ID;
            break;
          }
          if (!any_id || v > max_id) max_id = v;
          any_id = 1;
        }
      }
      if (code != ORC_ENC_OK) bad = j - r0;
      total += wc;
    }
    enc_code[m] = code;
    enc_bad_record[m] = bad;
    if (code != ORC_ENC_OK) {
      word_mod_off[m + 1] = out;
      continue;
    }
    if (out + (int64_t)total > words_cap) return -1;
    uint32_t *w = words_out + out;
    w[0] = ORC_MAGIC;
    w[1] = version_word;
    w[2] = generator_word;
    w[3] = any_id ? (uint32_t)(max_id + 1) : 1u;
    w[4] = 0;
    uint64_t p = 5;
    for (int64_t j = r0; j < r1; ++j) {
      const orc_inst *g = lookup(op[j]);
      int64_t n_ops = opnd_off[j + 1] - opnd_off[j];
      int64_t n_chars = str_off[j + 1] - str_off[j];
      uint64_t str_words = g->word_count == 0 ? (uint64_t)n_chars / 4 + 1 : 0;
      uint64_t wc = 1 + (uint64_t)n_ops + str_words;
      w[p] = (uint32_t)((wc << 16) | op[j]);
      for (int64_t s = 0; s < n_ops; ++s) w[p + 1 + s] = opnd[opnd_off[j] + s];
      for (uint64_t s = 0; s < str_words; ++s) {
        uint32_t word = 0;
        for (uint64_t b = 0; b < 4; ++b) {
          int64_t ci = 4 * (int64_t)s + (int64_t)b;
          uint32_t byte = ci < n_chars ? chars[str_off[j] + ci] : 0u;
          word |= byte << (8 * b);
        }
        w[p + 1 + n_ops + s] = word;
      }
      p += wc;
    }
    out += (int64_t)total;
    word_mod_off[m + 1] = out;
  }
  return out;
}

/* ------------------------------------------------------------------------
 * Disassembly to text (section "Dis/Assembler": the disassembler maps each
 * opcode and operand of the binary back to text; its options listing names
 * five switches, taken here in the listing's order as option bits
 *   1 syntax highlight, 2 inline names, 4 no indentation, 8 grouping,
 *   16 no header).
 * The paper prints no text format beyond the disassembly of its capabilities
 * example (one "OpCapability <name>" line per instruction), so the format
 * below is this oracle's reading, written down in full:
 *   - a module whose header check failed gives no text; otherwise the text
 *     covers the instructions of its valid prefix (as decode's records);
 *   - unless bit 16, five comment lines first: "; SPIR-V", "; Version: M.m",
 *     "; Generator: g", "; Bound: b", "; Schema: 0" (decimal numbers);
 *   - one line per instruction: [indent][%r = ]OpName[ operand]...\n where
 *     the result ID (if the instruction has one) moves to the left of " = "
 *     and the other operands keep their order; unless bit 4 the line is
 *     padded on the left with spaces so that the opcode name starts at
 *     column 15 (no padding if the "%r = " part is 15 characters or more);
 *   - an ID prints as %<decimal>, or with bit 2 as %<name> when the first
 *     OpName of the module that targets it carries a usable name (non-empty,
 *     only [A-Za-z0-9_], not starting with a digit); names are not made
 *     unique;
 *   - a literal prints in decimal, or as its enumerant name where the operand
 *     is an enumerant the table below knows (capability, addressing model,
 *     memory model, execution model; function control as None or its bits
 *     joined by '|'); an unknown value prints in decimal;
 *   - a string prints between double quotes, with '"' and '\' escaped by a
 *     backslash and every other byte as it is;
 *   - bit 8 puts an empty line before every OpFunction and OpLabel;
 *   - bit 1 wraps each opcode name, ID, literal and string token in an ANSI
 *     colour (ESC[36m, ESC[33m, ESC[34m, ESC[32m) and ESC[0m; the padding is
 *     counted without these codes.
 * ------------------------------------------------------------------------ */

enum { DIS_HIGHLIGHT = 1, DIS_INLINE_NAMES = 2, DIS_NO_INDENT = 4, DIS_GROUP = 8, DIS_NO_HEADER = 16 };

typedef struct {
  char *text;
  int64_t cap, pos;
} orc_out;

static void put_byte(orc_out *o, char c) {
  if (o->pos < o->cap) o->text[o->pos] = c;
  ++o->pos;
}

static void put_str(orc_out *o, const char *s) {
  while (*s) put_byte(o, *s++);
}

static void put_dec(orc_out *o, uint32_t v) {
  char buf[12];
  int k = 0;
  do {
    buf[k++] = (char)('0' + v % 10u);
    v /= 10u;
  } while (v);
  while (k) put_byte(o, buf[--k]);
}

static const char *opcode_name(uint32_t op) {
  switch (op) {
    case 5: return "OpName";
    case 14: return "OpMemoryModel";
    case 15: return "OpEntryPoint";
    case 17: return "OpCapability";
    case 21: return "OpTypeInt";
    case 43: return "OpConstant";
    case 54: return "OpFunction";
    case 56: return "OpFunctionEnd";
    case 61: return "OpLoad";
    case 62: return "OpStore";
    case 128: return "OpIAdd";
    case 248: return "OpLabel";
    case 253: return "OpReturn";
  }
  return NULL;
}

/* Enumerant names of the SPIR-V specification for the literal operands of
 * this grammar; NULL where the value is not in the table. */
static const char *capability_name(uint32_t v) {
  static const char *const names[] = {"Matrix",  "Shader",        "Geometry", "Tessellation", "Addresses",
                                      "Linkage", "Kernel",        "Vector16", "Float16Buffer", "Float16",
                                      "Float64", "Int64",         "Int64Atomics"};
  if (v < sizeof(names) / sizeof(names[0])) return names[v];
  if (v == 22) return "Int16";
  if (v == 39) return "Int8";
  return NULL;
}

static const char *addressing_name(uint32_t v) {
  static const char *const names[] = {"Logical", "Physical32", "Physical64"};
  return v < 3 ? names[v] : NULL;
}

static const char *memory_model_name(uint32_t v) {
  static const char *const names[] = {"Simple", "GLSL450", "OpenCL", "Vulkan"};
  return v < 4 ? names[v] : NULL;
}

static const char *execution_model_name(uint32_t v) {
  static const char *const names[] = {"Vertex",   "TessellationControl", "TessellationEvaluation", "Geometry",
                                      "Fragment", "GLCompute",           "Kernel"};
  return v < 7 ? names[v] : NULL;
}

static void color_on(orc_out *o, uint32_t options, const char *code) {
  if (options & DIS_HIGHLIGHT) {
    put_byte(o, '\x1b');
    put_byte(o, '[');
    put_str(o, code);
    put_byte(o, 'm');
  }
}

static void color_off(orc_out *o, uint32_t options) {
  if (options & DIS_HIGHLIGHT) put_str(o, "\x1b[0m");
}

/* The literal at operand slot s of opcode op. */
static void put_literal(orc_out *o, uint32_t options, uint32_t op, uint32_t s, uint32_t v) {
  const char *name = NULL;
  if (op == 17) name = capability_name(v);
  else if (op == 14) name = s == 0 ? addressing_name(v) : memory_model_name(v);
  else if (op == 15) name = execution_model_name(v);
  color_on(o, options, "34");
  if (op == 54) { /* function control: a bit mask */
    static const char *const bits[] = {"Inline", "DontInline", "Pure", "Const"};
    if (v == 0) put_str(o, "None");
    else if (v & ~0xFu) put_dec(o, v);
    else {
      int first = 1;
      for (int b = 0; b < 4; ++b)
        if (v & (1u << b)) {
          if (!first) put_byte(o, '|');
          put_str(o, bits[b]);
          first = 0;
        }
    }
  } else if (name) put_str(o, name);
  else put_dec(o, v);
  color_off(o, options);
}

/* A module's inline names: for each ID that some OpName targets, the first
 * such OpName's string (module order). */
typedef struct {
  uint32_t id, order;
  const uint8_t *name;
} orc_name;

static int cmp_name(const void *a, const void *b) {
  const orc_name *x = (const orc_name *)a, *y = (const orc_name *)b;
  if (x->id != y->id) return (x->id > y->id) - (x->id < y->id);
  return (x->order > y->order) - (x->order < y->order);
}

static int usable_name(const uint8_t *s) {
  if (s[0] == 0 || (s[0] >= '0' && s[0] <= '9')) return 0;
  for (; *s; ++s)
    if (!((*s >= 'a' && *s <= 'z') || (*s >= 'A' && *s <= 'Z') || (*s >= '0' && *s <= '9') || *s == '_'))
      return 0;
  return 1;
}

static const uint8_t *find_name(const orc_name *names, uint64_t n, uint32_t id) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (names[mid].id < id) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && names[lo].id == id) ? names[lo].name : NULL;
}

static void put_id(orc_out *o, uint32_t options, const orc_name *names, uint64_t n_names, uint32_t v) {
  const uint8_t *name = (options & DIS_INLINE_NAMES) ? find_name(names, n_names, v) : NULL;
  color_on(o, options, "33");
  put_byte(o, '%');
  if (name && usable_name(name)) put_str(o, (const char *)name);
  else put_dec(o, v);
  color_off(o, options);
}

/* Width of "%<token> = " without colour codes. */
static int64_t lhs_width(uint32_t options, const orc_name *names, uint64_t n_names, uint32_t v) {
  orc_out probe = {NULL, 0, 0};
  put_id(&probe, options & ~(uint32_t)DIS_HIGHLIGHT, names, n_names, v);
  return probe.pos + 3;
}

/* Text of every module of a CSR batch.  text receives the first
 * min(total, text_cap) bytes of the whole text; text_mod_off (n_modules+1)
 * the byte offsets where each module's text starts in it.  Returns the total
 * number of bytes, or -1 on bad offsets or when memory for the names could
 * not be had. */
int64_t oracle_disassemble(const uint32_t *words, const int64_t *mod_off, int64_t n_modules, uint32_t options,
                           char *text, int64_t text_cap, int64_t *text_mod_off) {
  orc_out o = {text, text_cap, 0};
  text_mod_off[0] = 0;
  for (int64_t m = 0; m < n_modules; ++m) {
    int64_t b = mod_off[m], e = mod_off[m + 1];
    if (e < b) return -1;
    const uint32_t *w = words + b;
    uint64_t n = (uint64_t)(e - b);
    orc_result r;
    check_module(w, n, 0, 0, NULL, NULL, &r);
    if (r.code != ORC_OK && r.code < ORC_BAD_WORD_COUNT) { /* header failed: no text */
      text_mod_off[m + 1] = o.pos;
      continue;
    }
    if (!(options & DIS_NO_HEADER)) {
      put_str(&o, "; SPIR-V\n; Version: ");
      put_dec(&o, (w[1] >> 16) & 0xFFu);
      put_byte(&o, '.');
      put_dec(&o, (w[1] >> 8) & 0xFFu);
      put_str(&o, "\n; Generator: ");
      put_dec(&o, w[2]);
      put_str(&o, "\n; Bound: ");
      put_dec(&o, w[3]);
      put_str(&o, "\n; Schema: ");
      put_dec(&o, w[4]);
      put_byte(&o, '\n');
    }
    /* the names, first OpName per target */
    orc_name *names = NULL;
    uint64_t n_names = 0;
    if (options & DIS_INLINE_NAMES) {
      names = (orc_name *)malloc((r.n_inst + 1) * sizeof(orc_name));
      if (!names) return -1;
      uint64_t p = 5;
      for (uint32_t j = 0; j < r.n_inst; ++j) {
        if ((w[p] & 0xFFFFu) == 5) {
          names[n_names].id = w[p + 1];
          names[n_names].order = j;
          names[n_names].name = (const uint8_t *)(w + p + 2);
          ++n_names;
        }
        p += w[p] >> 16;
      }
      qsort(names, n_names, sizeof(orc_name), cmp_name);
      uint64_t k = 0; /* keep the first of each id */
      for (uint64_t i = 0; i < n_names; ++i)
        if (k == 0 || names[k - 1].id != names[i].id) names[k++] = names[i];
      n_names = k;
    }
    uint64_t p = 5;
    for (uint32_t j = 0; j < r.n_inst; ++j) {
      uint32_t wc = w[p] >> 16, op = w[p] & 0xFFFFu;
      const orc_inst *g = lookup(op);
      if (g == NULL || wc == 0 || p + wc > n) break; /* cannot happen inside the valid prefix */
      uint32_t nfix = g->word_count == 0 ? fixed_operands(g) : wc - 1;
      int has_result = 0;
      uint32_t result = 0;
      for (uint32_t s = 0; s < nfix; ++s)
        if (g->roles[s] == 'D') {
          has_result = 1;
          result = w[p + 1 + s];
        }
      if ((options & DIS_GROUP) && (op == 54 || op == 248)) put_byte(&o, '\n');
      if (!(options & DIS_NO_INDENT)) {
        int64_t width = has_result ? lhs_width(options, names, n_names, result) : 0;
        for (int64_t c = width; c < 15; ++c) put_byte(&o, ' ');
      }
      if (has_result) {
        put_id(&o, options, names, n_names, result);
        put_str(&o, " = ");
      }
      color_on(&o, options, "36");
      put_str(&o, opcode_name(op));
      color_off(&o, options);
      for (uint32_t s = 0; s < nfix; ++s) {
        char role = g->roles[s];
        uint32_t v = w[p + 1 + s];
        if (role == 'D') continue;
        put_byte(&o, ' ');
        if (role == 'U') put_id(&o, options, names, n_names, v);
        else put_literal(&o, options, op, s, v);
      }
      if (g->word_count == 0) { /* the string, validated by the parse stage */
        const uint8_t *s = (const uint8_t *)(w + p + 1 + nfix);
        put_byte(&o, ' ');
        color_on(&o, options, "32");
        put_byte(&o, '"');
        for (; *s; ++s) {
          if (*s == '"' || *s == '\\') put_byte(&o, '\\');
          put_byte(&o, (char)*s);
        }
        put_byte(&o, '"');
        color_off(&o, options);
      }
      put_byte(&o, '\n');
      p += wc;
    }
    free(names);
    text_mod_off[m + 1] = o.pos;
  }
  return o.pos;
}
