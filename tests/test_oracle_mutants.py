"""Mutation check of the oracle's pins: each mutant of oracle.c plants one
plausible mistake (a dropped check, an off-by-one, a wrong index, a
transposed role, a wrong constant) and must make at least one pin fail.
Everything runs on the CPU; the mutants are built with gcc into a temporary
directory and swapped in for the real oracle only inside this test."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import test_oracle_bruteforce as brute
import test_oracle_pins as pins
import test_oracle_rules as rules
from conftest import parse_golden, ROOT

SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("overrun off by one", "if (wc == 0 || p + wc > n) code", "if (wc == 0 || p + wc >= n) code"),
    ("magic not checked", "if (w[0] != ORC_MAGIC) {", "if (0) {"),
    ("minor version limit", "|| minor > 6)", "|| minor > 7)"),
    ("schema not checked", "if (w[4] != 0) {", "if (0) {"),
    ("duplicate ignored", "if (defs[i] == defs[i - 1]) dup = 1;", ";"),
    ("ID 0 allowed", "if (v == 0 || v >= bound) {\n        oob = 1;", "if (v >= bound) {\n        oob = 1;"),
    ("bound inclusive", "if (v == 0 || v >= bound) {\n        oob = 1;", "if (v == 0 || v > bound) {\n        oob = 1;"),
    ("position pass: ID 0 allowed", "if (v == 0 || v >= bound) {\n        if (*f_oob", "if (v >= bound) {\n        if (*f_oob"),
    ("priority DUP over OOB", "if (oob) r->code = ORC_ID_OUT_OF_BOUND;\n  else if (dup)",
     "if (dup) r->code = ORC_DUPLICATE_ID;\n  else if (oob)"),
    ("NUL anywhere accepted", "if (first_nul / 4 != n_words - 1) return 0;", ";"),
    ("padding not checked", "if (((w[b / 4] >> (8 * (b % 4))) & 0xFFu) != 0) return 0;", ";"),
    ("OpLoad roles transposed", '{61, 4, "UDU"}', '{61, 4, "UUD"}'),
    ("OpIAdd result slot", '{128, 5, "UDUU"}', '{128, 5, "DUUU"}'),
    ("string minimum count", "(g->word_count == 0 && wc < 2 + fixed_operands(g))",
     "(g->word_count == 0 && wc < 1 + fixed_operands(g))"),
    ("string always after word 2", "!string_ok(w + p + 1 + fixed_operands(g), wc - 1 - fixed_operands(g))",
     "!string_ok(w + p + 2, wc - 2)"),
    ("OpEntryPoint function not an ID", '{15, 0, "LUS"}', '{15, 0, "LLS"}'),
    ("entry-point rule dropped", "if (op == 15) entry_point = 1;", "entry_point = 1;"),
    ("function rule reads the memory model", "if (op == 54) function = 1;", "if (op == 14) function = 1;"),
    ("records include the failing instruction", "for (uint32_t j = 0; j < r.n_inst; ++j) {",
     "for (uint32_t j = 0; j < r.n_inst + (r.code >= ORC_BAD_WORD_COUNT && r.code <= ORC_BAD_STRING); ++j) {"),
    ("records of header failures", "if (r.code == ORC_OK || r.code >= ORC_BAD_WORD_COUNT) {",
     "if (r.code == ORC_OK || r.code >= ORC_BAD_WORD_COUNT || r.code == ORC_BAD_VERSION) {\n      if (r.code == ORC_BAD_VERSION) r.n_inst = 1;"),
    ("index off by one", "if (idx_off) idx_off[k] = (uint32_t)p;", "if (idx_off) idx_off[k] = (uint32_t)p + 1;"),
    ("n_inst at error", "r->err_word = (uint32_t)p;\n      r->n_inst = (uint32_t)k;",
     "r->err_word = (uint32_t)p;\n      r->n_inst = (uint32_t)k + 1;"),
    ("encode bound = max id", "w[3] = any_id ? (uint32_t)(max_id + 1) : 1u;", "w[3] = any_id ? (uint32_t)max_id : 1u;"),
    ("encode string words rounded", "uint64_t str_words = g->word_count == 0 ? (uint64_t)n_chars / 4 + 1 : 0;",
     "uint64_t str_words = g->word_count == 0 ? ((uint64_t)n_chars + 3) / 4 : 0;"),
    ("encode word count without first word", "wc = 1 + (uint64_t)n_ops + (g->word_count == 0 ?",
     "wc = (uint64_t)n_ops + (g->word_count == 0 ?"),
    ("encode little-endian swapped", "word |= byte << (8 * b);", "word |= byte << (8 * (3 - b));"),
    ("encode failed module keeps its header", "    if (code != ORC_ENC_OK) {\n      word_mod_off[m + 1] = out;",
     "    if (code != ORC_ENC_OK) {\n      word_mod_off[m + 1] = out + 5;"),
    ("first duplicate taken as the first definition",
     "if (defs[i].v == defs[i - 1].v && defs[i].pos < *f_dup) *f_dup = defs[i].pos;",
     "if (defs[i].v == defs[i - 1].v && defs[i].pos < *f_dup) *f_dup = defs[i - 1].pos;"),
    ("a use at its own definition counts as defined", "!forward_use_ok(op, s) && d >= p)", "!forward_use_ok(op, s) && d > p)"),
    ("no forward uses allowed", "(before_use && !forward_use_ok(op, s) && d >= p)", "(before_use && d >= p)"),
    ("offset of the wrong class", "if (r->code == ORC_ID_OUT_OF_BOUND) r->err_word = f_oob;",
     "if (r->code == ORC_ID_OUT_OF_BOUND) r->err_word = f_dup;"),
    ("defined-before-use ignored", "if (opts & ORC_OPT_BEFORE_USE) undef = f_undef != 0xFFFFFFFFu;", ";"),
    ("text: opcode column 14", "for (int64_t c = width; c < 15; ++c)", "for (int64_t c = width; c < 14; ++c)"),
    ("text: last OpName wins", "if (k == 0 || names[k - 1].id != names[i].id) names[k++] = names[i];",
     "if (k > 0 && names[k - 1].id == names[i].id) names[k - 1] = names[i];\n        else names[k++] = names[i];"),
    ("text: digit-led names inlined", "if (s[0] == 0 || (s[0] >= '0' && s[0] <= '9')) return 0;",
     "if (s[0] == 0) return 0;"),
    ("text: quote not escaped", "if (*s == '\"' || *s == '\\\\') put_byte(&o, '\\\\');",
     "if (*s == '\\\\') put_byte(&o, '\\\\');"),
    ("text: no group line before OpLabel", "(op == 54 || op == 248)) put_byte(&o, '\\n');",
     "(op == 54)) put_byte(&o, '\\n');"),
    ("text: version fields swapped", "put_dec(&o, (w[1] >> 16) & 0xFFu);", "put_dec(&o, (w[1] >> 8) & 0xFFu);"),
    ("text: memory model operands swapped", "name = s == 0 ? addressing_name(v) : memory_model_name(v);",
     "name = s == 0 ? memory_model_name(v) : addressing_name(v);"),
    ("text: padding counts colour codes", "put_id(&probe, options & ~(uint32_t)DIS_HIGHLIGHT,",
     "put_id(&probe, options,"),
    ("text: result kept among the operands", "if (role == 'D') continue;", "if (0) continue;"),
    ("text: function control bits reversed", "if (v & (1u << b)) {", "if (v & (8u >> b)) {"),
]


def _battery():
    """Run the pins against whatever library oracle._lib points to; return
    the names of the pins that fail."""
    failed = []
    cases = parse_golden(os.path.join(ROOT, "tests", "golden", "paper_examples.txt"))
    checks = [
        ("paper encode", lambda: pins.test_paper_examples_encode(cases)),
        ("paper decode", lambda: pins.test_paper_examples_decode(cases)),
        ("layout", pins.test_generator_layout_pins_index),
        ("faults", pins.test_injected_faults_known_by_construction),
        ("numpy sets", pins.test_semantic_against_numpy_sets),
        ("round trip", pins.test_round_trip_identity),
        ("encode sizes", pins.test_encode_sizes),
        ("brute force", brute.test_bruteforce_small_modules),
        ("brute encode", brute.test_bruteforce_encode),
        ("brute rules", brute.test_bruteforce_module_rules),
        ("records of failing modules", pins.test_records_of_failing_modules),
        ("rules: earlier stages", rules.test_earlier_stages_win),
    ]
    import inspect
    rule_cases = [m.args for m in pins.test_rules.pytestmark if m.name == "parametrize"][0][1]
    for words, expect in rule_cases:
        checks.append((f"rule {words[:6]}", lambda w=words, e=expect: pins.test_rules(w, e)))
    for rec, code in [m.args for m in pins.test_encode_failures.pytestmark if m.name == "parametrize"][0][1]:
        checks.append((f"enc {rec[0]}", lambda r=rec, c=code: pins.test_encode_failures(r, c)))
    for parts, expect in [m.args for m in rules.test_rules_on_valid_modules.pytestmark
                          if m.name == "parametrize"][0][1]:
        checks.append((f"rules {len(parts)}", lambda p=parts, e=expect: rules.test_rules_on_valid_modules(p, e)))
    for ent, expect in [m.args for m in rules.test_entry_point_forms.pytestmark if m.name == "parametrize"][0][1]:
        checks.append((f"entry {ent[0]:#x}", lambda a=ent, e=expect: rules.test_entry_point_forms(a, e)))
    import test_oracle_disasm as dis
    for case in dis.CASES:
        checks.append((f"text {case['name']}", lambda c=case: dis.test_golden_disassembly(c)))
    checks.append(("text random", dis.test_random_tiny_modules_agree_with_second_statement))
    import test_oracle_positions as posn
    for case in posn.CASES:
        checks.append((f"positions {case[0]}", lambda c=case: posn.test_hand_written_positions(*c)))
    checks.append(("positions and rules", posn.test_rules_follow_the_before_use_stage))
    checks.append(("text batch", dis.test_batch_offsets_and_truncation))
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, RuntimeError):
            failed.append(name)
    return failed


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert old in src, f"mutation site not found: {name}"
    mutated = src.replace(old, new, 1)
    c = tmp_path / "oracle_mutant.c"
    so = tmp_path / "liboracle_mutant.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-w", "-o", str(so), str(c)])
    import ctypes
    real = oracle._load()
    mut = ctypes.CDLL(str(so))
    for fn in ("oracle_validate", "oracle_records", "oracle_encode_bound", "oracle_encode", "oracle_disassemble"):
        getattr(mut, fn).argtypes = getattr(real, fn).argtypes
        getattr(mut, fn).restype = getattr(real, fn).restype
    try:
        oracle._lib = mut
        failed = _battery()
    finally:
        oracle._lib = real
    assert failed, f"mutant '{name}' passed every pin"


def test_real_oracle_passes_the_battery():
    assert _battery() == []
