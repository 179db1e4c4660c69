"""Circuit structure and scheduling, on the CPU.

Structure is pinned by the paper's own counts: the 32-bit Kogge-Stone adder
has o counts 31, 30, 28, 24, 16 per prefix level and the 16-bit one 15, 14,
12, 8 (Sec. 5.2, thread counts of Table 16BitAdderStages / 32BitAdderStages
discussion), depth 2 log2 W + 2 (Sec. 7.1), and subtraction is a + NOT(b) + 1
(Sec. 5.3). Function is pinned by cleartext evaluation against integer
arithmetic, and by one small circuit evaluated gate by gate with the CPU
oracle (toy parameters) and decrypted.
"""
import numpy as np
import pytest

from oracle import circuits as OC
from paper_2101_03403_amd import circuits as C
from paper_2101_03403_amd import workloads as W
import oracle_program as OP
from plainsim import eval_dag, run_program_plain


def test_adder_levels_match_paper_32():
    c = C.adder_instance(32)
    assert c.gate_counts_per_level() == [64, 62, 31, 60, 30, 56, 28, 48, 24, 32, 16, 32]
    assert c.num_gates() == 483
    assert c.depth() == 2 * 5 + 2
    # o counts per prefix level = ORs in the odd levels 3, 5, 7, 9, 11
    ors = [c.gate_counts_per_level()[L] for L in (2, 4, 6, 8, 10)]
    assert ors == [31, 30, 28, 24, 16]


def test_adder_levels_match_paper_16():
    c = C.adder_instance(16)
    assert c.gate_counts_per_level() == [32, 30, 15, 28, 14, 24, 12, 16, 8, 16]
    assert c.depth() == 2 * 4 + 2


@pytest.mark.parametrize("width", [8, 16, 32])
def test_add_sub_cleartext(width):
    rng = np.random.default_rng(width)
    add, sub = C.adder_instance(width), C.sub_instance(width)
    assert sub.num_gates() == add.num_gates() + 1          # carry-in OR
    vals = list(rng.integers(0, 1 << width, (200, 2), dtype=np.uint64)) + [(0, 0), ((1 << width) - 1, 1),
                                                                             (0, (1 << width) - 1)]
    for a, b in vals:
        a, b = int(a), int(b)
        bits = C.int_to_bits(a, width) + C.int_to_bits(b, width)
        assert C.bits_to_int(eval_dag(add, bits)[add.outputs["sum"]]) == (a + b) % (1 << width)
        assert C.bits_to_int(eval_dag(sub, bits)[sub.outputs["diff"]]) == (a - b) % (1 << width)


@pytest.mark.parametrize("kind", W.MIX_KINDS)
@pytest.mark.parametrize("width", [8, 16])
def test_instruction_circuits_cleartext(kind, width):
    rng = np.random.default_rng(hash((kind, width)) % 1000)
    c = C.instruction_circuit(kind, width)
    for _ in range(40):
        a, b = (int(x) for x in rng.integers(0, 1 << width, 2, dtype=np.uint64))
        if kind in ("LT", "EQ") and rng.random() < 0.3:
            b = a
        v = eval_dag(c, C.int_to_bits(a, width) + C.int_to_bits(b, width))
        assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(kind, width, a, b)


def test_program_merges_levels_across_instances():
    cs = [C.adder_instance(32) for _ in range(3)] + [C.sub_instance(16)]
    prog = C.Program(cs)
    widths = prog.level_widths()
    assert sum(widths) == 3 * 483 + 196
    assert widths[0] == 3 * 64 + 32
    assert prog.depth == 12
    # every gate's inputs are produced at an earlier level (or are inputs/consts/NOTs)
    produced = set(prog.input_rows.tolist()) | set(prog.consts[1].tolist())
    for L in prog.levels:
        produced |= set(L.nots[1].tolist())
        assert set(L.ia.tolist()) <= produced and set(L.ib.tolist()) <= produced
        produced |= set(L.io.tolist())


@pytest.mark.parametrize("prefix", ["gates", "mux"])
def test_packed_program_fills_rounds_and_computes_the_same(prefix):
    """Levels reassigned to fill whole launch rounds: same depth and the same
    gates, every level's blind rotations a multiple of the round size until
    the last levels, every input produced before its consumer, and level by
    level cleartext execution gives every instruction's integer result."""
    mix = W.instruction_mix(96, seed=11)
    cs = [C.instruction_circuit(k, w, prefix=prefix) for k, w, _, _ in mix]
    bits = []
    for k, w, a, b in mix:
        bits += C.int_to_bits(a, w) + C.int_to_bits(b, w)
    plain = C.Program(cs)
    R = 64
    packed = C.Program(cs, pack=R)
    assert packed.depth == plain.depth
    assert packed.num_gates() == plain.num_gates() and packed.num_muxes() == plain.num_muxes()
    boot = [w + 2 * m for w, m in zip(packed.level_widths(), packed.level_mux_counts())]
    full = [b % R == 0 for b in boot]
    assert sum(full) >= len(boot) - 3, boot          # only the last levels may be ragged
    produced = set(packed.input_rows.tolist()) | set(packed.consts[1].tolist())
    for L in packed.levels:
        produced |= set(L.nots[1].tolist())
        for x in (L.ia, L.ib) + L.mux[:3]:
            assert set(x.tolist()) <= produced
        produced |= set(L.io.tolist()) | set(L.mux[3].tolist())
    for prog in (plain, packed):
        v = run_program_plain(prog, bits)
        for (k, w, a, b), c, off in zip(mix, cs, prog.offsets):
            got = C.bits_to_int([int(x) for x in v[np.array(c.outputs["out"]) + off]])
            assert got == OC.word_result(k, w, a, b), (k, w, a, b)


def test_mixed_stream_recipe():
    mix = W.instruction_mix(1000, seed=5)
    kinds = [k for k, *_ in mix]
    frac = lambda ks: sum(k in ks for k in kinds) / len(kinds)
    assert abs(frac({"ADD", "SUB"}) - 0.4) < 0.05
    assert abs(frac({"MUL"}) - 0.2) < 0.05
    assert abs(frac({"LT", "EQ"}) - 0.2) < 0.05
    assert all(w in (8, 16) for k, w, *_ in mix if k == "MUL")


def test_small_circuits_under_fhe_with_oracle():
    """8-bit ADD and SUB plus a 4-bit EQ and LT, evaluated homomorphically
    gate by gate with the oracle (toy parameters), then decrypted."""
    from oracle import oracle as O
    okeys = O.keygen(O.TOY, 99)
    cases = [("ADD", 8, 200, 100), ("SUB", 8, 17, 50), ("EQ", 4, 9, 9), ("LT", 4, 3, 12)]
    cs = [C.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = C.Program(cs)
    bits = []
    for k, w, a, b in cases:
        bits += C.int_to_bits(a, w) + C.int_to_bits(b, w)
    pool0 = OP.oracle_pool(okeys, prog, bits, seed=3)
    pool = OP.run_on_oracle(okeys, prog, pool0, range(len(cs)))
    # replaying a subset of the instances writes the same rows
    part = OP.run_on_oracle(okeys, prog, pool0, [1, 3])
    rows = np.flatnonzero(OP.instance_rows(prog, [1, 3]))
    assert np.array_equal(part[rows], pool[rows])
    assert OP.bootstrapped_rows(prog, [1, 3]).size == cs[1].num_gates() + cs[3].num_gates()
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        rows = np.array(c.outputs["out"]) + off
        got = C.bits_to_int(O.decrypt_bits(okeys.lwe_key, pool[rows]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)


# ------------------------------------------------------------------ shifters (Sec. 5.4)
@pytest.mark.parametrize("mode", [C.LLS, C.LRS, C.ARS])
@pytest.mark.parametrize("width", [8, 16, 32])
def test_barrel_shift_cleartext(mode, width):
    rng = np.random.default_rng(width + len(mode))
    c = C.instruction_circuit(mode, width)
    amounts = list(range(width + 3)) + [int(x) for x in rng.integers(0, 1 << width, 8, dtype=np.uint64)]
    for k in amounts:
        a = int(rng.integers(0, 1 << width, dtype=np.uint64))
        if k % 3 == 0:
            a |= 1 << (width - 1)                     # exercise the sign fill of ARS
        v = eval_dag(c, C.int_to_bits(a, width) + C.int_to_bits(k, width))
        assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(mode, width, a, k), (a, k)


def test_barrel_shift_structure_32():
    """32-bit register-mode shifter: 5 stages of 32 MUX selects (the thread
    counts of the 32-bit LLS / LRS / ARS tables), 320 bootstraps."""
    for mode in (C.LLS, C.LRS, C.ARS):
        c = C.instruction_circuit(mode, 32)
        prog = C.Program([c])
        assert prog.depth == 5
        assert prog.level_mux_counts() == [32] * 5
        assert prog.level_widths() == [0] * 5
        assert prog.num_bootstraps() == 320 == c.num_bootstraps()


@pytest.mark.parametrize("mode", [C.LLS, C.LRS, C.ARS])
def test_shift_immediate_cleartext(mode):
    rng = np.random.default_rng(7)
    for k in range(0, 20):
        c = C.Circuit()
        A = c.inputs_word(16)
        out = C.shift_immediate(c, A, k, mode)
        assert c.num_bootstraps() == 0
        a = int(rng.integers(0, 1 << 16)) | (1 << 15) * (k % 2)
        v = eval_dag(c, C.int_to_bits(a, 16))
        assert C.bits_to_int(v[out]) == OC.word_result(mode, 16, a, k)


def test_shifters_under_fhe_with_oracle():
    """8-bit LLS and 4-bit LRS / ARS, register mode, evaluated with the
    oracle's MUX (toy parameters), then decrypted."""
    from oracle import oracle as O
    okeys = O.keygen(O.TOY, 98)
    cases = [(C.LLS, 8, 0b10110101, 3), (C.LRS, 4, 0b1101, 1), (C.ARS, 4, 0b1010, 2)]
    cs = [C.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = C.Program(cs)
    bits = []
    for k, w, a, b in cases:
        bits += C.int_to_bits(a, w) + C.int_to_bits(b, w)
    pool = OP.run_on_oracle(okeys, prog, OP.oracle_pool(okeys, prog, bits, seed=8), range(len(prog.circuits)))
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        rows = np.array(c.outputs["out"]) + off
        got = C.bits_to_int(O.decrypt_bits(okeys.lwe_key, pool[rows]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)


# ------------------------------------------------------------------ multiplier and divider (Sec. 5.5, 5.6)
SEQ_KINDS = ["MULSEQ", "SMULSEQ", "DIV"]


@pytest.mark.parametrize("kind", SEQ_KINDS)
def test_sequential_units_exhaustive_4bit(kind):
    c = C.instruction_circuit(kind, 4)
    for a in range(16):
        for b in range(16):
            v = eval_dag(c, C.int_to_bits(a, 4) + C.int_to_bits(b, 4))
            assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(kind, 4, a, b), (a, b)


@pytest.mark.parametrize("kind", SEQ_KINDS)
@pytest.mark.parametrize("width", [8, 16, 32])
def test_sequential_units_cleartext(kind, width):
    rng = np.random.default_rng(width * 7 + len(kind))
    c = C.instruction_circuit(kind, width)
    m = (1 << width) - 1
    cases = [(m, m), (0, 5), (m, 1), (1 << (width - 1), m), (5, 0)]
    cases += [tuple(int(x) for x in rng.integers(0, 1 << width, 2, dtype=np.uint64)) for _ in range(25)]
    cases += [(int(rng.integers(0, 1 << width, dtype=np.uint64)), int(rng.integers(1, 1 << (width // 2)))) for _ in range(10)]
    for a, b in cases:
        v = eval_dag(c, C.int_to_bits(a, width) + C.int_to_bits(b, width))
        assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(kind, width, a, b), (a, b)


def test_sequential_units_structure():
    """W iterations of one W-bit adder (multiplier) or one (W+1)-bit
    add/subtract (divider): the depth grows linearly in W, the widest level is
    the first (all W^2 row ANDs) for the multiplier and one adder stage for the
    divider."""
    for w, mul_depth, div_depth in [(8, 65, 88), (16, 161, 208), (32, 385, 480)]:
        m = C.instruction_circuit("MULSEQ", w)
        d = C.instruction_circuit("DIV", w)
        assert m.depth() == mul_depth and d.depth() == div_depth
        pm = C.Program([m])
        assert pm.level_widths()[0] == w * w
        assert max(C.Program([d]).level_widths()) <= 2 * w + 2


def test_add_with_carry_wire_cleartext():
    for w in (1, 3, 8, 17):
        c = C.Circuit()
        A, B = c.inputs_word(w), c.inputs_word(w)
        cin = c.input()
        s, cout = C.add_with_carry_wire(c, A, B, cin)
        rng = np.random.default_rng(w)
        for _ in range(40):
            a, b, ci = int(rng.integers(0, 1 << w)), int(rng.integers(0, 1 << w)), int(rng.integers(0, 2))
            v = eval_dag(c, C.int_to_bits(a, w) + C.int_to_bits(b, w) + [ci])
            assert C.bits_to_int(v[s]) + (int(v[cout]) << w) == a + b + ci


def test_sequential_units_under_fhe_with_oracle():
    """4-bit unsigned and signed sequential multiplication and 4-bit division,
    evaluated homomorphically with the oracle (toy parameters), decrypted."""
    from oracle import oracle as O
    okeys = O.keygen(O.TOY, 97)
    cases = [("MULSEQ", 4, 13, 11), ("SMULSEQ", 4, 0b1101, 0b0110), ("DIV", 4, 14, 3)]
    cs = [C.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = C.Program(cs)
    bits = []
    for k, w, a, b in cases:
        bits += C.int_to_bits(a, w) + C.int_to_bits(b, w)
    pool = OP.run_on_oracle(okeys, prog, OP.oracle_pool(okeys, prog, bits, seed=9), range(len(prog.circuits)))
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        rows = np.array(c.outputs["out"]) + off
        got = C.bits_to_int(O.decrypt_bits(okeys.lwe_key, pool[rows]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)



# ------------------------------------------------------------------ MUX form of the prefix stage
MUX_KINDS = ["ADD", "SUB", "LT", "MUL", "MULSEQ", "SMULSEQ", "DIV"]


@pytest.mark.parametrize("width", [1, 2, 3, 4, 5])
def test_mux_prefix_units_exhaustive(width):
    """Every adder-based unit with the MUX prefix form, all operand pairs."""
    cs = {k: C.instruction_circuit(k, width, prefix=C.PREFIX_MUX) for k in MUX_KINDS}
    fl = {k: C.flag_setting_circuit(k, width, prefix=C.PREFIX_MUX) for k in ("ADDS", "SUBS")}
    for a in range(1 << width):
        for b in range(1 << width):
            bits = C.int_to_bits(a, width) + C.int_to_bits(b, width)
            for k, c in cs.items():
                v = eval_dag(c, bits)
                assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(k, width, a, b), (k, a, b)
            for k, c in fl.items():
                v = eval_dag(c, bits)
                assert [int(x) for x in v[c.outputs["nzcv"]]] == OC.nzcv(k, width, a, b), (k, a, b)


@pytest.mark.parametrize("kind", ["ADD", "SUB", "LT", "MULSEQ", "DIV"])
def test_mux_prefix_units_cleartext_32(kind):
    rng = np.random.default_rng(len(kind) * 13)
    c = C.instruction_circuit(kind, 32, prefix=C.PREFIX_MUX)
    m = (1 << 32) - 1
    cases = [(m, m), (0, 0), (m, 1), (1 << 31, 1 << 31), (5, 0)]
    cases += [tuple(int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64)) for _ in range(25)]
    for a, b in cases:
        v = eval_dag(c, C.int_to_bits(a, 32) + C.int_to_bits(b, 32))
        assert C.bits_to_int(v[c.outputs["out"]]) == OC.word_result(kind, 32, a, b), (a, b)


def test_mux_prefix_structure_32():
    """One MUX per o: the MUX counts per prefix level are the paper's o counts
    (31, 30, 28, 24, 16), the propagate ANDs are only those a later level
    reads (positions >= 2d), and the adder is log2 W + 2 = 7 levels deep."""
    for kind in ("ADD", "SUB"):
        p = C.Program([C.instruction_circuit(kind, 32, prefix=C.PREFIX_MUX)])
        assert p.depth == 7
        assert p.level_mux_counts() == [0, 31, 30, 28, 24, 16, 0]
        assert p.level_widths() == [64, 30, 28, 24, 16, 0, 32]
        assert p.num_bootstraps() == 64 + 2 * 129 + 98 + 32
    p16 = C.Program([C.adder_instance(16, prefix=C.PREFIX_MUX)])
    assert p16.depth == 6 and p16.level_mux_counts()[1:5] == [15, 14, 12, 8]
    for w, mul_depth, div_depth in [(8, 41, 56), (32, 225, 288)]:
        assert C.instruction_circuit("MULSEQ", w, prefix=C.PREFIX_MUX).depth() == mul_depth
        assert C.instruction_circuit("DIV", w, prefix=C.PREFIX_MUX).depth() == div_depth
    with pytest.raises(ValueError):
        C.adder_instance(8, prefix="tree")


def test_mux_prefix_add_with_carry_wire_cleartext():
    for w in (1, 3, 8, 17):
        c = C.Circuit()
        A, B = c.inputs_word(w), c.inputs_word(w)
        cin = c.input()
        s, cout = C.add_with_carry_wire(c, A, B, cin, C.PREFIX_MUX)
        rng = np.random.default_rng(w + 100)
        for _ in range(40):
            a, b, ci = int(rng.integers(0, 1 << w)), int(rng.integers(0, 1 << w)), int(rng.integers(0, 2))
            v = eval_dag(c, C.int_to_bits(a, w) + C.int_to_bits(b, w) + [ci])
            assert C.bits_to_int(v[s]) + (int(v[cout]) << w) == a + b + ci


def test_mux_prefix_under_fhe_with_oracle():
    """8-bit ADD and SUB and a 4-bit DIV with the MUX prefix form, evaluated
    with the oracle's gates and MUX (toy parameters, levels that mix both),
    then decrypted."""
    from oracle import oracle as O
    okeys = O.keygen(O.TOY, 96)
    cases = [("ADD", 8, 201, 99), ("SUB", 8, 17, 50), ("DIV", 4, 13, 4)]
    cs = [C.instruction_circuit(k, w, prefix=C.PREFIX_MUX) for k, w, _, _ in cases]
    prog = C.Program(cs)
    assert any(L.ops.shape[0] and L.num_muxes for L in prog.levels)
    bits = []
    for k, w, a, b in cases:
        bits += C.int_to_bits(a, w) + C.int_to_bits(b, w)
    pool = OP.run_on_oracle(okeys, prog, OP.oracle_pool(okeys, prog, bits, seed=10), range(len(prog.circuits)))
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        rows = np.array(c.outputs["out"]) + off
        got = C.bits_to_int(O.decrypt_bits(okeys.lwe_key, pool[rows]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)
