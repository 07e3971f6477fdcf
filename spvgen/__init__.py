"""Seeded synthetic SPIR-V workloads (input recipe only).

This package builds the inputs that the tests, the benchmark and the serving
demo feed to both the CPU oracle and the GPU library.  It holds the opcode mix,
the ID / literal / string draws and the fault injection of the synthetic
workloads, nothing else: it computes no decode, validate or encode result.

SPIR-V facts used here (section "SPIR-V Library", header listing, and the
binary layout the toolkit writes): a module is a stream of 32-bit words; a
5-word header (magic 0x07230203, version word 0x00MMmm00, generator, bound,
schema 0) is followed by instructions whose first word carries the word count
in its high 16 bits and the opcode in its low 16 bits.  Result IDs are handed
out once per module, sequentially, as the paper's module-level ID allocation
does (section "Enabling Function Composition", SSA paragraph).

Module recipe (every draw from ``numpy.random.default_rng(seed)``, PCG64):
  * prologue: OpCapability Kernel(6); OpMemoryModel 2 2; OpEntryPoint
    Kernel(6) %2 "main"; OpTypeInt %1 32 0; OpFunction %1 %2 0 %1 (so every
    module meets the four module-level rules: a capability, the memory model,
    a function and an entry point; the entry point names the function that
    the prologue defines next);
  * then i.i.d. opcodes from MIX (percent); a U (ID-use) slot draws uniformly
    from the results defined so far; D (result) slots are sequential from 1;
  * literals: OpCapability in {4,5,6,11,39}, OpMemoryModel (2,2), OpTypeInt
    (32, {0,1}), OpConstant uniform uint32, OpFunction control 0;
  * OpName: length 4..24 uniform, chars uniform over [a-z0-9_], packed
    little-endian into floor(L/4)+1 words, zero padded;
  * header bound = results + 1.
Draw order (fixed): opcodes, OpName lengths, U slots (table order, slot order),
OpCapability literals, OpTypeInt signedness, OpConstant values, name chars.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

MAGIC = 0x07230203
VERSION_1_6 = 0x00010600

# name, opcode, fixed word count (0: variable, the operands before S and then
# the string words), operand roles after the first word (U: ID use, D: result
# ID, L: literal, S: string words), mix percent.
OPS = [
    ("OpCapability", 17, 2, "L", 1),
    ("OpMemoryModel", 14, 3, "LL", 1),
    ("OpName", 5, 0, "US", 10),
    ("OpTypeInt", 21, 4, "DLL", 4),
    ("OpConstant", 43, 4, "UDL", 10),
    ("OpFunction", 54, 5, "UDLU", 3),
    ("OpLabel", 248, 2, "D", 6),
    ("OpLoad", 61, 4, "UDU", 20),
    ("OpStore", 62, 3, "UU", 12),
    ("OpIAdd", 128, 5, "UDUU", 27),
    ("OpReturn", 253, 1, "", 3),
    ("OpFunctionEnd", 56, 1, "", 3),
    # prologue only (weight 0): execution model, entry function, name
    ("OpEntryPoint", 15, 0, "LUS", 0),
]
(K_CAP, K_MEM, K_NAME, K_TYPEINT, K_CONST, K_FUNC, K_LABEL, K_LOAD, K_STORE, K_IADD, K_RET, K_FEND,
 K_ENTRY) = range(13)
PROLOGUE = (K_CAP, K_MEM, K_ENTRY, K_TYPEINT, K_FUNC)
N_PROLOGUE = len(PROLOGUE)
ENTRY_NAME = b"main"
OPCODE = np.array([o[1] for o in OPS], dtype=np.int64)
FIXED_WC = np.array([o[2] for o in OPS], dtype=np.int64)
ROLES = [o[3] for o in OPS]
MIX = np.array([o[4] for o in OPS], dtype=np.float64) / 100.0
HAS_DEF = np.array(["D" in r for r in ROLES])
CAPABILITIES = np.array([4, 5, 6, 11, 39], dtype=np.uint32)
NAME_CHARS = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789_", dtype=np.uint8)

# error codes of the validator contract (kept here only to state what an
# injected fault is expected to produce; the generator never validates)
E_BAD_WORD_COUNT = 5
E_DUPLICATE_ID = 9
E_UNDEFINED_ID = 10


@dataclasses.dataclass
class Module:
    """One generated module plus what the generator knows by construction."""
    words: np.ndarray          # uint32 [n_words]
    kind: np.ndarray           # int8 index into OPS, per instruction
    wc: np.ndarray             # int64 word count per instruction
    starts: np.ndarray         # int64 word offset of each instruction (generator layout)
    n_results: int
    bound: int
    # records (encoder input) of the same instructions
    rec_op: np.ndarray         # uint16 [n_inst]
    rec_opnd_off: np.ndarray   # int32 [n_inst+1]
    rec_opnd: np.ndarray       # uint32
    rec_str_off: np.ndarray    # int32 [n_inst+1]
    rec_chars: np.ndarray      # uint8
    expect: Optional[dict] = None   # set by fault injection

    @property
    def n_inst(self) -> int:
        return int(self.kind.shape[0])

    @property
    def opcodes(self) -> np.ndarray:
        return OPCODE[self.kind]


def _segment_arange(lengths: np.ndarray) -> np.ndarray:
    """Concatenation of arange(l) for each l in lengths."""
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    ends = np.cumsum(lengths)
    starts = ends - lengths
    return np.arange(total, dtype=np.int64) - np.repeat(starts, lengths)


def gen_module(seed, n_inst: int) -> Module:
    """Generate one module of ``n_inst`` (>= 5) instructions."""
    if n_inst < N_PROLOGUE:
        raise ValueError(f"a generated module has at least the {N_PROLOGUE} prologue instructions")
    rng = np.random.default_rng(seed)
    n = int(n_inst)
    kind = np.empty(n, dtype=np.int8)
    kind[:N_PROLOGUE] = PROLOGUE
    kind[N_PROLOGUE:] = rng.choice(len(OPS), size=n - N_PROLOGUE, p=MIX)

    is_name = kind == K_NAME
    n_names = int(is_name.sum())
    name_len = rng.integers(4, 25, size=n_names)
    wc = FIXED_WC[kind].copy()
    wc[is_name] = 2 + name_len // 4 + 1
    entry = 2  # index of the prologue's OpEntryPoint
    wc[entry] = 3 + len(ENTRY_NAME) // 4 + 1

    has_def = HAS_DEF[kind]
    defs_incl = np.cumsum(has_def, dtype=np.int64)
    results_before = defs_incl - has_def
    n_results = int(defs_incl[-1])
    bound = n_results + 1

    starts = 5 + np.concatenate([[0], np.cumsum(wc)[:-1]]).astype(np.int64)
    total = 5 + int(wc.sum())
    words = np.zeros(total, dtype=np.uint32)
    words[0:5] = [MAGIC, VERSION_1_6, 0, bound, 0]
    words[starts] = ((wc << 16) | OPCODE[kind]).astype(np.uint32)

    # result IDs
    for k in range(len(OPS)):
        r = ROLES[k]
        if "D" not in r:
            continue
        idx = np.nonzero(kind == k)[0]
        words[starts[idx] + 1 + r.index("D")] = defs_incl[idx].astype(np.uint32)
    # ID uses: uniform over earlier results (the entry point's function is
    # the prologue's OpFunction, %2, defined after it)
    for k in range(len(OPS)):
        if k == K_ENTRY:
            continue
        for s, role in enumerate(ROLES[k]):
            if role != "U":
                continue
            idx = np.nonzero(kind == k)[0]
            if idx.size == 0:
                continue
            v = rng.integers(1, results_before[idx] + 1)
            words[starts[idx] + 1 + s] = v.astype(np.uint32)
    pe = int(starts[entry])
    words[pe + 1] = 6  # execution model Kernel
    words[pe + 2] = int(defs_incl[4])  # the prologue function's result ID
    words.view(np.uint8)[4 * (pe + 3):4 * (pe + 3) + len(ENTRY_NAME)] = np.frombuffer(ENTRY_NAME, np.uint8)
    # literals
    cap_idx = np.nonzero(kind == K_CAP)[0]
    caps = CAPABILITIES[rng.integers(0, len(CAPABILITIES), size=cap_idx.size)]
    caps[0] = 6  # prologue: Kernel
    words[starts[cap_idx] + 1] = caps
    mem_idx = np.nonzero(kind == K_MEM)[0]
    words[starts[mem_idx] + 1] = 2
    words[starts[mem_idx] + 2] = 2
    ti_idx = np.nonzero(kind == K_TYPEINT)[0]
    sign = rng.integers(0, 2, size=ti_idx.size).astype(np.uint32)
    sign[0] = 0  # prologue: %1 = OpTypeInt 32 0
    words[starts[ti_idx] + 2] = 32
    words[starts[ti_idx] + 3] = sign
    c_idx = np.nonzero(kind == K_CONST)[0]
    words[starts[c_idx] + 3] = rng.integers(0, 1 << 32, size=c_idx.size, dtype=np.uint64).astype(np.uint32)
    f_idx = np.nonzero(kind == K_FUNC)[0]
    words[starts[f_idx] + 3] = 0
    # OpName strings, little-endian bytes, zero padded (buffer starts zeroed)
    n_chars = int(name_len.sum())
    chars = NAME_CHARS[rng.integers(0, len(NAME_CHARS), size=n_chars)]
    name_idx = np.nonzero(is_name)[0]
    byte_pos = np.repeat(4 * (starts[name_idx] + 2), name_len) + _segment_arange(name_len)
    words.view(np.uint8)[byte_pos] = chars

    # records: opcode, non-string operand words, string bytes (the entry
    # point's name comes first: no OpName precedes it)
    n_ops = np.where(is_name, 1, wc - 1).astype(np.int64)
    n_ops[entry] = 2
    opnd_off = np.concatenate([[0], np.cumsum(n_ops)]).astype(np.int32)
    opnd_pos = np.repeat(starts + 1, n_ops) + _segment_arange(n_ops)
    opnd = words[opnd_pos].copy()
    str_len = np.zeros(n, dtype=np.int64)
    str_len[is_name] = name_len
    str_len[entry] = len(ENTRY_NAME)
    str_off = np.concatenate([[0], np.cumsum(str_len)]).astype(np.int32)
    rec_chars = np.concatenate([np.frombuffer(ENTRY_NAME, np.uint8), chars])
    return Module(words=words, kind=kind, wc=wc, starts=starts, n_results=n_results, bound=bound,
                  rec_op=OPCODE[kind].astype(np.uint16), rec_opnd_off=opnd_off, rec_opnd=opnd,
                  rec_str_off=str_off, rec_chars=rec_chars)


# ----------------------------------------------------------------------------
# fault injection (expected outcome known by construction)

def _slot_positions(mod: Module, role: str, post_prologue: bool = True):
    """(instruction index, word position) of every slot with the given role."""
    inst, pos = [], []
    for k in range(len(OPS)):
        for s, r in enumerate(ROLES[k]):
            if r != role:
                continue
            idx = np.nonzero(mod.kind == k)[0]
            if post_prologue:
                idx = idx[idx >= N_PROLOGUE]
            inst.append(idx)
            pos.append(mod.starts[idx] + 1 + s)
    if not inst:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    inst = np.concatenate(inst)
    pos = np.concatenate(pos)
    order = np.argsort(pos, kind="stable")
    return inst[order], pos[order]


def inject_bad_wc(mod: Module, rng) -> Module:
    """A post-prologue fixed-length instruction gets word count +-1."""
    cand = np.nonzero((np.arange(mod.n_inst) >= N_PROLOGUE) & (mod.kind != K_NAME))[0]
    i = int(cand[rng.integers(0, cand.size)])
    delta = 1 if rng.integers(0, 2) else -1
    p = int(mod.starts[i])
    w = mod.words.copy()
    w[p] = np.uint32(((int(mod.wc[i]) + delta) << 16) | int(OPCODE[mod.kind[i]]))
    return dataclasses.replace(mod, words=w, expect=dict(code=E_BAD_WORD_COUNT, sem_mask=0, err_word=p, n_inst=i,
                                                         kind="bad_wc"))


def inject_undef(mod: Module, rng) -> Module:
    """A random ID-use slot refers to the old bound; the header bound grows by one."""
    _, pos = _slot_positions(mod, "U")
    p = int(pos[rng.integers(0, pos.size)])
    w = mod.words.copy()
    w[p] = np.uint32(mod.bound)
    w[3] = np.uint32(mod.bound + 1)
    return dataclasses.replace(mod, words=w, bound=mod.bound + 1,
                               expect=dict(code=E_UNDEFINED_ID, sem_mask=4, err_word=0xFFFFFFFF, n_inst=mod.n_inst,
                                           kind="undef"))


def inject_dup(mod: Module, rng) -> Module:
    """A post-prologue result slot is set to an earlier result ID.

    The displaced ID is then undefined; if some slot uses it, the module is
    also UNDEF (mask 6), which the generator works out from its own slots."""
    _, dpos = _slot_positions(mod, "D")
    p = int(dpos[rng.integers(0, dpos.size)])
    w = mod.words.copy()
    displaced = int(w[p])
    new = int(rng.integers(1, displaced))  # displaced >= 3 after the prologue
    w[p] = np.uint32(new)
    _, upos = _slot_positions(mod, "U", post_prologue=False)
    used = bool(np.any(w[upos] == displaced))
    return dataclasses.replace(mod, words=w, expect=dict(code=E_DUPLICATE_ID, sem_mask=6 if used else 2,
                                                         err_word=0xFFFFFFFF, n_inst=mod.n_inst, kind="dup"))


FAULTS = [inject_bad_wc, inject_undef, inject_dup]


# ----------------------------------------------------------------------------
# batches

@dataclasses.dataclass
class Batch:
    words: np.ndarray      # uint32, CSR-packed modules
    mod_off: np.ndarray    # int64 [M+1]
    modules: List[Module]

    @property
    def n_modules(self) -> int:
        return len(self.modules)


def pack(modules: Sequence[Module]) -> Batch:
    sizes = np.array([m.words.size for m in modules], dtype=np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    words = np.concatenate([m.words for m in modules]) if modules else np.zeros(0, np.uint32)
    return Batch(words=words, mod_off=mod_off, modules=list(modules))


def lognormal_sizes(seed, count: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = np.round(rng.lognormal(np.log(median), sigma, size=count))
    return np.clip(s, lo, hi).astype(np.int64)


def pack_records(modules: Sequence[Module]):
    """Concatenate the encoder records of several modules (CSR by module)."""
    ops = np.concatenate([m.rec_op for m in modules])
    n_rec = np.array([m.n_inst for m in modules], dtype=np.int64)
    rec_mod_off = np.concatenate([[0], np.cumsum(n_rec)]).astype(np.int64)
    opnd_lens = [np.diff(m.rec_opnd_off.astype(np.int64)) for m in modules]
    str_lens = [np.diff(m.rec_str_off.astype(np.int64)) for m in modules]
    opnd_off = np.concatenate([[0], np.cumsum(np.concatenate(opnd_lens))]).astype(np.int32)
    str_off = np.concatenate([[0], np.cumsum(np.concatenate(str_lens))]).astype(np.int32)
    opnd = np.concatenate([m.rec_opnd for m in modules])
    chars = np.concatenate([m.rec_chars for m in modules])
    return dict(op=ops, opnd_off=opnd_off, opnd=opnd, str_off=str_off, chars=chars, rec_mod_off=rec_mod_off)


# ----------------------------------------------------------------------------
# the five workloads

def config1() -> Batch:
    """One module of 10,000 instructions (about 40.6k words), seed 1."""
    return pack([gen_module(1, 10_000)])


def config2(n_inst: int = 16_000_000) -> Batch:
    """One large module, 16M instructions (about 65M words, 260 MB), seed 2."""
    return pack([gen_module(2, n_inst)])


def config3(n_modules: int = 4096, n_faults: Optional[int] = None, median: float = 2000.0,
            lo: int = 200, hi: int = 200_000) -> Batch:
    """Lognormal batch: sizes round(lognormal(ln median, 1.0)) clipped to [lo, hi].

    Module m's content seed is [3, m]; 1% of the modules (chosen without
    replacement with seed [3, 'faults']) carry one fault, kinds cycling
    bad word count / undefined ID / duplicate ID."""
    sizes = lognormal_sizes([3, 0xA11], n_modules, median, 1.0, lo, hi)
    mods = [gen_module([3, m], int(sizes[m])) for m in range(n_modules)]
    if n_faults is None:
        n_faults = max(1, round(0.01 * n_modules))
    frng = np.random.default_rng([3, 0xFA17])
    chosen = np.sort(frng.choice(n_modules, size=min(n_faults, n_modules), replace=False))
    for j, m in enumerate(chosen):
        mods[m] = FAULTS[j % 3](mods[m], frng)
    return pack(mods)


def config4(n_records: int = 10_000_000, n_modules: int = 1024):
    """Encoder input: n_records records split evenly over n_modules modules.

    Module m gets floor((m+1)N/M) - floor(mN/M) records and its own ID space
    (content seed [4, m])."""
    bounds = [(m * n_records) // n_modules for m in range(n_modules + 1)]
    mods = [gen_module([4, m], max(N_PROLOGUE, bounds[m + 1] - bounds[m])) for m in range(n_modules)]
    return mods, pack_records(mods)


def serving_pool(n_pool: int = 8192, median: float = 5000.0, hi: int = 1_000_000, seed: int = 5,
                 lo: int = 200) -> List[Module]:
    """Pool of modules whose sizes follow the serving law (lognormal, sigma 1)."""
    sizes = lognormal_sizes([seed, 0x5], n_pool, median, 1.0, lo, hi)
    return [gen_module([seed, i], int(sizes[i])) for i in range(n_pool)]


def poisson_arrivals(rate: float, duration: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of the given rate."""
    rng = np.random.default_rng([seed, 0xA7])
    n_guess = int(rate * duration * 1.2 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_guess))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n_guess))])
    return t[t < duration]
