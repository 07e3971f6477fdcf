"""Independent definitional checker for tiny modules (test infrastructure).

A second, deliberately different statement of the validator contract used by
the brute-force tests to cross-check ``oracle.c``: it reads the module as a
little-endian byte string, describes each instruction by its operand kinds and
uses Python sets for the ID rules.  Sources: SPIR-V module layout as the
toolkit writes it (section "SPIR-V Library": header listing, bound recomputed
at write; section "Parsing Operand Kinds": operand words and word counts), the
SSA single-assignment rule (section "Enabling Function Composition") and the
validation stage (section "Validation Rules").  Slow; only for small inputs.
"""
from __future__ import annotations

import struct
from collections import Counter

# opcode -> (operand kinds after the first word); "str" marks a literal string
# running to the end of the instruction.  Fixed-size instructions have exactly
# len(kinds) operand words.  OpEntryPoint's name is its last operand here: the
# interface IDs SPIR-V allows after it are outside this contract.
KINDS = {
    5: ("id", "str"),                       # OpName target, name
    14: ("lit", "lit"),                     # OpMemoryModel addressing, memory
    15: ("lit", "id", "str"),               # OpEntryPoint model, function, name
    17: ("lit",),                           # OpCapability
    21: ("result", "lit", "lit"),           # OpTypeInt result, width, signedness
    43: ("id", "result", "lit"),            # OpConstant type, result, value
    54: ("id", "result", "lit", "id"),      # OpFunction type, result, control, fn type
    56: (),                                 # OpFunctionEnd
    61: ("id", "result", "id"),             # OpLoad type, result, pointer
    62: ("id", "id"),                       # OpStore pointer, object
    128: ("id", "result", "id", "id"),      # OpIAdd type, result, a, b
    248: ("result",),                       # OpLabel
    253: (),                                # OpReturn
}


def _string_words_ok(raw: bytes) -> bool:
    # the literal ends at its first NUL; the NUL must sit in the final word and
    # the rest of that word must be NUL padding
    nul = raw.find(b"\x00")
    if nul < 0:
        return False
    return nul >= len(raw) - 4 and raw[nul:] == b"\x00" * (len(raw) - nul)


# module-level rules (section "Validation Rules"): mask bit of each rule ->
# the opcodes that satisfy it
RULES = {8: {17}, 16: {14}, 32: {54}, 64: {15}}   # capability, memory model, function, entry point


# ID uses that may name a later definition: OpName's target, OpEntryPoint's
# function (opcode, operand slot)
FORWARD_USES = {(5, 0), (15, 1)}


def check(words, semantic: bool = True, rules: bool = False, offsets: bool = False, before_use: bool = False):
    """(code, sem_mask, err_word, n_inst, [(offset, opcode), ...]).

    before_use: a use counts as undefined unless an earlier instruction
    defines its ID (FORWARD_USES aside); offsets: err_word of a semantic
    failure is the offset of the first instruction of the primary class."""
    w = [int(x) & 0xFFFFFFFF for x in words]
    n = len(w)
    raw = struct.pack("<%dI" % n, *w)
    if n < 5:
        return (1, 0, n, 0, [])
    if raw[0:4] != bytes([0x03, 0x02, 0x23, 0x07]):
        return (2, 0, 0, 0, [])
    ver = raw[4:8]  # bytes: reserved, minor, major, reserved
    if ver[0] != 0 or ver[3] != 0 or ver[2] != 1 or ver[1] > 6:
        return (3, 0, 1, 0, [])
    if w[4] != 0:
        return (4, 0, 4, 0, [])
    bound = w[3]
    insts = []
    pos = 5
    while pos < n:
        count, opcode = divmod(w[pos], 1 << 16)
        end = pos + count
        if count == 0 or end > n:
            return (5, 0, pos, len(insts), insts)
        if opcode not in KINDS:
            return (6, 0, pos, len(insts), insts)
        kinds = KINDS[opcode]
        if "str" in kinds:
            head = kinds.index("str")  # operand words before the string
            if count < 1 + head + 1:
                return (5, 0, pos, len(insts), insts)
            if not _string_words_ok(raw[4 * (pos + 1 + head):4 * end]):
                return (7, 0, pos, len(insts), insts)
        elif count != 1 + len(kinds):
            return (5, 0, pos, len(insts), insts)
        insts.append((pos, opcode))
        pos = end
    if not semantic:
        return (0, 0, 0xFFFFFFFF, len(insts), insts)
    defined = Counter()
    used = set()
    out_of_bound = False
    for pos, opcode in insts:
        for slot, kind in enumerate(KINDS[opcode]):
            if kind not in ("id", "result"):
                continue
            v = w[pos + 1 + slot]
            if not (0 < v < bound):
                out_of_bound = True
            elif kind == "result":
                defined[v] += 1
            else:
                used.add(v)
    dup = any(c > 1 for c in defined.values())
    undef = bool(used - set(defined))
    # the same walk again, in module order, for the first offenders: an
    # instruction is the first of its class when no earlier one is
    seen = set()
    first = {}
    for pos, opcode in insts:
        for slot, kind in enumerate(KINDS[opcode]):
            if kind not in ("id", "result"):
                continue
            v = w[pos + 1 + slot]
            if not (0 < v < bound):
                first.setdefault("oob", pos)
            elif kind == "result":
                if v in seen:
                    first.setdefault("dup", pos)
        for slot, kind in enumerate(KINDS[opcode]):
            v = w[pos + 1 + slot] if kind != "str" else None
            if kind == "id" and 0 < v < bound:
                late = before_use and (opcode, slot) not in FORWARD_USES and v not in seen
                if v not in defined or late:
                    first.setdefault("undef", pos)
        for slot, kind in enumerate(KINDS[opcode]):
            if kind == "result":
                seen.add(w[pos + 1 + slot])
    if before_use:
        undef = "undef" in first
    mask = (1 if out_of_bound else 0) | (2 if dup else 0) | (4 if undef else 0)
    code = 8 if out_of_bound else 9 if dup else 10 if undef else 0
    err = 0xFFFFFFFF
    if offsets and code:
        err = first[{8: "oob", 9: "dup", 10: "undef"}[code]]
    if rules and code == 0:
        present = Counter(opcode for _, opcode in insts)
        mask = sum(bit for bit, ops in RULES.items() if not any(present[o] for o in ops))
        code = 11 if mask else 0
    return (code, mask, err, len(insts), insts)


def encode_module(records, version_word=0x00010600, generator_word=0):
    """Words of one module from records [(opcode, [operands], name_bytes)],
    or (code, bad_index) when a record cannot be encoded."""
    body = []
    ids = []
    for j, (opcode, operands, name) in enumerate(records):
        if opcode not in KINDS:
            return (1, j)
        kinds = KINDS[opcode]
        is_name = "str" in kinds
        want = kinds.index("str") if is_name else len(kinds)
        if len(operands) != want:
            return (2, j)
        if (not is_name and len(name) > 0) or (is_name and b"\x00" in name):
            return (3, j)
        sw = b""
        if is_name:
            padded = name + b"\x00"
            padded += b"\x00" * (-len(padded) % 4)
            sw = padded
        count = 1 + len(operands) + len(sw) // 4
        if count >= 1 << 16:
            return (4, j)
        for kind, v in zip(kinds, operands):
            if kind in ("id", "result"):
                if v == 0xFFFFFFFF:
                    return (5, j)
                ids.append(v)
        body.append(count << 16 | opcode)
        body.extend(operands)
        body.extend(struct.unpack("<%dI" % (len(sw) // 4), sw))
    bound = max(ids) + 1 if ids else 1
    return [0x07230203, version_word, generator_word, bound, 0] + body


# --- disassembly to text (section "Dis/Assembler"; the options listing's
# five switches as bits 1 highlight, 2 inline names, 4 no indentation,
# 8 grouping, 16 no header).  A second statement of the text format of
# oracle.c, built from token lists instead of a byte writer.

NAMES = {5: "OpName", 14: "OpMemoryModel", 15: "OpEntryPoint", 17: "OpCapability", 21: "OpTypeInt",
         43: "OpConstant", 54: "OpFunction", 56: "OpFunctionEnd", 61: "OpLoad", 62: "OpStore", 128: "OpIAdd",
         248: "OpLabel", 253: "OpReturn"}
# enumerants (SPIR-V specification) of the literal operands, by (opcode, operand slot)
ENUMS = {
    (17, 0): {0: "Matrix", 1: "Shader", 2: "Geometry", 3: "Tessellation", 4: "Addresses", 5: "Linkage",
              6: "Kernel", 7: "Vector16", 8: "Float16Buffer", 9: "Float16", 10: "Float64", 11: "Int64",
              12: "Int64Atomics", 22: "Int16", 39: "Int8"},
    (14, 0): {0: "Logical", 1: "Physical32", 2: "Physical64"},
    (14, 1): {0: "Simple", 1: "GLSL450", 2: "OpenCL", 3: "Vulkan"},
    (15, 0): {0: "Vertex", 1: "TessellationControl", 2: "TessellationEvaluation", 3: "Geometry",
              4: "Fragment", 5: "GLCompute", 6: "Kernel"},
}
COLOR = {"op": 36, "id": 33, "lit": 34, "str": 32}


def _function_control(v):
    if v == 0:
        return "None"
    if v >> 4:
        return str(v)
    return "|".join(n for b, n in enumerate(("Inline", "DontInline", "Pure", "Const")) if v >> b & 1)


def _name_ok(name: bytes) -> bool:
    return bool(name) and not name[:1].isdigit() and all(
        c in b"abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ0123456789_" for c in name)


def disassemble_module(words, options: int = 0) -> bytes:
    """Text of one module (bytes); empty when its header check fails."""
    w = [int(x) & 0xFFFFFFFF for x in words]
    code, _, _, _, insts = check(w, semantic=False)
    if 1 <= code <= 4:
        return b""
    raw = struct.pack("<%dI" % len(w), *w)

    def string_at(word_pos):
        b = raw[4 * word_pos:]
        return b[:b.index(b"\x00")]

    names = {}
    if options & 2:
        for pos, opcode in insts:
            if opcode == 5:
                names.setdefault(w[pos + 1], string_at(pos + 2))

    def tok(kind, text):
        return (kind, text)

    def id_tok(v):
        nm = names.get(v)
        return tok("id", "%" + (nm.decode() if nm is not None and _name_ok(nm) else str(v)))

    lines = []
    if not options & 16:
        lines.append([tok(None, "; SPIR-V")])
        lines.append([tok(None, "; Version: %d.%d" % (raw[6], raw[5]))])
        lines.append([tok(None, "; Generator: %d" % w[2])])
        lines.append([tok(None, "; Bound: %d" % w[3])])
        lines.append([tok(None, "; Schema: %d" % w[4])])
    for pos, opcode in insts:
        kinds = KINDS[opcode]
        left, right = [], []
        for slot, kind in enumerate(kinds):
            if kind == "str":
                s = string_at(pos + 1 + slot).decode("latin-1")
                s = s.replace("\\", "\\\\").replace('"', '\\"')
                right.append(tok("str", '"' + s + '"'))
                continue
            v = w[pos + 1 + slot]
            if kind == "result":
                left = [id_tok(v), tok(None, " = ")]
            elif kind == "id":
                right.append(id_tok(v))
            elif opcode == 54:
                right.append(tok("lit", _function_control(v)))
            else:
                right.append(tok("lit", ENUMS.get((opcode, slot), {}).get(v, str(v))))
        if options & 8 and opcode in (54, 248):
            lines.append([])
        line = []
        if not options & 4:
            width = sum(len(t) for _, t in left)
            line.append(tok(None, " " * max(0, 15 - width)))
        line += left + [tok("op", NAMES[opcode])]
        for t in right:
            line += [tok(None, " "), t]
        lines.append(line)
    out = []
    for line in lines:
        for kind, text in line:
            if kind is not None and options & 1:
                text = "\x1b[%dm%s\x1b[0m" % (COLOR[kind], text)
            out.append(text)
        out.append("\n")
    return "".join(out).encode("latin-1")
