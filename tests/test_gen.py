"""Generator invariants: the synthetic modules have the shape the workload
recipe states (word counts per opcode, sequential results, bound, strings)."""
import numpy as np

import spvgen


def test_module_layout_and_mix():
    m = spvgen.gen_module(7, 20_000)
    w = m.words
    assert w[0] == 0x07230203 and w[1] == 0x00010600 and w[2] == 0 and w[4] == 0
    assert int(w[3]) == m.bound == m.n_results + 1
    # starts follow the word counts from the first word after the header
    assert m.starts[0] == 5
    assert np.array_equal(np.diff(m.starts), m.wc[:-1])
    assert m.starts[-1] + m.wc[-1] == w.size
    # first words carry (wc << 16) | opcode
    assert np.array_equal(w[m.starts] >> 16, m.wc)
    assert np.array_equal(w[m.starts] & 0xFFFF, m.opcodes)
    # the fixed-size opcodes have their table sizes; OpName is 2 + floor(L/4) + 1
    fixed = spvgen.FIXED_WC[m.kind]
    assert np.all((fixed == 0) | (m.wc == fixed))
    name = m.kind == spvgen.K_NAME
    L = np.diff(m.rec_str_off.astype(np.int64))[name]
    assert np.all((L >= 4) & (L <= 24))
    assert np.array_equal(m.wc[name], 2 + L // 4 + 1)
    # words per instruction close to the stated 4.064
    assert abs(w.size / m.n_inst - 4.064) < 0.03


def test_sequential_results_and_backward_uses():
    m = spvgen.gen_module(11, 5_000)
    defs, uses = [], []
    for i in range(m.n_inst):
        r = spvgen.ROLES[m.kind[i]]
        for s, role in enumerate(r):
            if role == "D":
                defs.append(int(m.words[m.starts[i] + 1 + s]))
            elif role == "U":
                v = int(m.words[m.starts[i] + 1 + s])
                if m.kind[i] == spvgen.K_ENTRY:
                    assert v == 2  # the prologue's function, defined right after
                else:
                    assert 1 <= v <= len(defs)  # refers to an earlier result
                uses.append(v)
    assert defs == list(range(1, len(defs) + 1))
    assert m.n_results == len(defs)


def test_prologue():
    """Capability, memory model, entry point naming the function %2, %1 =
    OpTypeInt 32 0, %2 = OpFunction %1 None %1."""
    m = spvgen.gen_module(12, 50)
    w = [int(x) for x in m.words[5:5 + 2 + 3 + 5 + 4 + 5]]
    assert w == [0x00020011, 6, 0x0003000E, 2, 2, 0x0005000F, 6, 2, 0x6E69616D, 0,
                 0x00040015, 1, 32, 0, 0x00050036, 1, 2, 0, 1]
    assert list(m.rec_op[:5]) == [17, 14, 15, 21, 54]
    assert bytes(m.rec_chars[:4]) == b"main" and m.rec_str_off[3] == 4


def test_strings_nul_terminated_and_padded():
    m = spvgen.gen_module(3, 2_000)
    bytes_ = m.words.view(np.uint8)
    for i in np.nonzero(m.kind == spvgen.K_NAME)[0][:200]:
        b = bytes_[4 * (m.starts[i] + 2): 4 * (m.starts[i] + m.wc[i])]
        nul = int(np.argmax(b == 0))
        assert b[nul] == 0 and np.all(b[nul:] == 0) and nul >= b.size - 4
        assert np.all(b[:nul] != 0)


def test_determinism():
    a = spvgen.gen_module([3, 17], 3_000)
    b = spvgen.gen_module([3, 17], 3_000)
    assert np.array_equal(a.words, b.words)


def test_lognormal_batch_shape():
    b = spvgen.config3(n_modules=64, n_faults=3)
    assert b.mod_off[0] == 0 and b.mod_off[-1] == b.words.size
    kinds = [m.expect["kind"] for m in b.modules if m.expect]
    assert kinds == ["bad_wc", "undef", "dup"]
