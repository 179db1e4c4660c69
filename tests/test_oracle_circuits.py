"""O16, the oracle's circuit layer (oracle/circuits.py), on the CPU.

The oracle's netlists are pinned to plain integer arithmetic (exhaustively at
small widths, on random and boundary operands at 16 and 32 bits) and to the
paper's own structure counts (Sec. 5.2: (g, p) on every bit, then the scan
levels with 31, 30, 28, 24, 16 o operations for 32 bits and 15, 14, 12, 8
for 16 bits, two gates and an OR each, then one XOR per sum bit; Sec. 5.3:
one extra OR for the carry-in of the subtractor). They are then evaluated
homomorphically with the oracle's gates (toy parameters) and decrypted.
Against them the product's circuits (paper_2101_03403_amd/circuits.py) must
show the same per-level gate counts for ADD / SUB and the same outputs for
every instruction.
"""
import itertools

import numpy as np
import pytest

from oracle import circuits as OC
from paper_2101_03403_amd import circuits as C
from plainsim import eval_dag

WORD_KINDS = ["ADD", "SUB", "LT", "EQ", "AND", "OR", "XOR", "ORN", "MUL", "MULSEQ", "SMULSEQ", "DIV"]
SHIFT_KINDS = ["LLS", "LRS", "ARS"]


def _out(net, a, b, width, name="out"):
    v = net.run_plain(OC.to_bits(a, width) + OC.to_bits(b, width))
    return OC.from_bits([v[w] for w in net.outputs[name]]), v


@pytest.mark.parametrize("width", [1, 2, 3, 4, 5])
def test_oracle_units_exhaustive(width):
    for kind in WORD_KINDS:
        net = OC.instruction(kind, width)
        for a, b in itertools.product(range(1 << width), repeat=2):
            assert _out(net, a, b, width)[0] == OC.word_result(kind, width, a, b), (kind, a, b)
    for kind in ("ADDS", "SUBS", "CMP"):
        net = OC.instruction(kind, width)
        for a, b in itertools.product(range(1 << width), repeat=2):
            got, v = _out(net, a, b, width)
            assert got == OC.word_result(kind, width, a, b)
            assert [v[w] for w in net.outputs["nzcv"]] == OC.nzcv(kind, width, a, b), (kind, a, b)


@pytest.mark.parametrize("width", [2, 4, 8])
def test_oracle_shifters_exhaustive(width):
    for kind in SHIFT_KINDS:
        net = OC.instruction(kind, width)
        for a, b in itertools.product(range(1 << width), repeat=2):
            assert _out(net, a, b, width)[0] == OC.word_result(kind, width, a, b), (kind, a, b)


@pytest.mark.parametrize("width", [16, 32])
def test_oracle_units_random_and_boundaries(width):
    rng = np.random.default_rng(width)
    m = (1 << width) - 1
    pairs = [(0, 0), (m, m), (m, 1), (1, m), (1 << (width - 1), 1 << (width - 1)), (5, 0), (m, 0)]
    pairs += [tuple(int(x) for x in rng.integers(0, 1 << width, 2, dtype=np.uint64)) for _ in range(12)]
    kinds = WORD_KINDS + SHIFT_KINDS
    if width == 32:
        kinds = [k for k in kinds if k not in ("MUL", "SMULSEQ")]   # 32-bit products: the 16-bit ones suffice
    for kind in kinds:
        net = OC.instruction(kind, width)
        for a, b in pairs:
            assert _out(net, a, b, width)[0] == OC.word_result(kind, width, a, b), (kind, a, b)
    for kind in ("ADDS", "SUBS"):
        net = OC.instruction(kind, width)
        for a, b in pairs:
            got, v = _out(net, a, b, width)
            assert [v[w] for w in net.outputs["nzcv"]] == OC.nzcv(kind, width, a, b), (kind, a, b)


def test_word_result_and_flags_definitions():
    """The integer semantics themselves, on values worked by hand."""
    assert OC.word_result("ADD", 32, 0xFFFFFFFF, 1) == 0
    assert OC.word_result("SUB", 8, 3, 5) == 254
    assert OC.word_result("SMULSEQ", 4, 0b1111, 0b1111) == 1            # (-1)(-1)
    assert OC.word_result("SMULSEQ", 4, 0b1000, 0b0111) == 256 - 56      # (-8)(7) mod 2^8
    assert OC.word_result("ARS", 8, 0b10000000, 3) == 0b11110000
    assert OC.word_result("LRS", 8, 0b10000000, 3) == 0b00010000
    assert OC.word_result("LLS", 8, 0b10000001, 9) == 0b00000010        # amount mod 8 = 1
    assert OC.word_result("DIV", 8, 200, 7) == 28 and OC.word_result("DIV", 8, 9, 0) == 255
    assert OC.word_result("ORN", 4, 0b0001, 0b0011) == 0b1101
    assert OC.nzcv("ADDS", 8, 0x7F, 1) == [1, 0, 0, 1]      # signed overflow into the sign bit
    assert OC.nzcv("ADDS", 8, 0xFF, 1) == [0, 1, 1, 0]      # unsigned carry, zero result
    assert OC.nzcv("SUBS", 8, 5, 5) == [0, 1, 1, 0]         # no borrow, zero
    assert OC.nzcv("SUBS", 8, 0x80, 1) == [0, 0, 1, 1]      # -128 - 1 overflows
    for a, b in itertools.product(range(16), repeat=2):
        n, z, c, v = OC.nzcv("CMP", 4, a, b)
        sa, sb = (a - 16 if a > 7 else a), (b - 16 if b > 7 else b)
        assert OC.condition("HI", n, z, c, v) == (a > b) and OC.condition("LS", n, z, c, v) == (a <= b)
        assert OC.condition("GE", n, z, c, v) == (sa >= sb) and OC.condition("LT", n, z, c, v) == (sa < sb)
        assert OC.condition("GT", n, z, c, v) == (sa > sb) and OC.condition("LE", n, z, c, v) == (sa <= sb)
        assert OC.condition("CS", n, z, c, v) == (a >= b) and OC.condition("EQ", n, z, c, v) == (a == b)


def test_oracle_adder_matches_the_papers_counts():
    """Sec. 5.2: 32-bit (g, p) on 32 bits (64 gates), scan levels of 31, 30,
    28, 24, 16 o (62, 60, 56, 48, 32 threads: two ANDs each, then as many
    ORs), 32 sum XORs: 483 gates, depth 2 log2 W + 2. 16 bits: 15, 14, 12, 8
    o (30, 28, 24, 16 threads). Sec. 5.3: the subtractor adds one OR."""
    for W, ops in ((32, [31, 30, 28, 24, 16]), (16, [15, 14, 12, 8])):
        want = [2 * W]
        for o in ops:
            want += [2 * o, o]
        want += [W]
        add = OC.instruction("ADD", W)
        assert add.gates_per_level() == want
        assert add.depth() == 2 * len(ops) + 2
        sub = OC.instruction("SUB", W)
        assert sum(sub.gates_per_level()) == sum(want) + 1
        assert sub.depth() == add.depth()
    assert sum(OC.instruction("ADD", 32).gates_per_level()) == 483


@pytest.mark.parametrize("width", [8, 16, 32])
def test_product_adders_have_the_oracles_level_counts(width):
    assert C.adder_instance(width).gate_counts_per_level() == OC.instruction("ADD", width).gates_per_level()
    assert C.sub_instance(width).gate_counts_per_level() == OC.instruction("SUB", width).gates_per_level()
    assert C.adder_instance(width).depth() == OC.instruction("ADD", width).depth()
    assert C.sub_instance(width).depth() == OC.instruction("SUB", width).depth()


@pytest.mark.parametrize("width", [4, 8, 16])
def test_product_circuits_compute_what_the_oracle_computes(width):
    """Every instruction circuit of the product, in both prefix forms, gives
    the oracle netlist's output on the same operands (and the flags of the
    flag-setting forms)."""
    rng = np.random.default_rng(100 + width)
    m = (1 << width) - 1
    pairs = [(0, 0), (m, m), (m, 1), (1 << (width - 1), m), (7 & m, 0)]
    pairs += [tuple(int(x) for x in rng.integers(0, 1 << width, 2, dtype=np.uint64)) for _ in range(10)]
    kinds = WORD_KINDS + SHIFT_KINDS
    for kind in kinds:
        net = OC.instruction(kind, width)
        for prefix in (C.PREFIX_GATES, C.PREFIX_MUX):
            if prefix == C.PREFIX_MUX and kind not in ("ADD", "SUB", "LT", "MUL", "MULSEQ", "SMULSEQ", "DIV"):
                continue
            c = C.instruction_circuit(kind, width, prefix=prefix)
            for a, b in pairs:
                bits = OC.to_bits(a, width) + OC.to_bits(b, width)
                got = OC.from_bits(eval_dag(c, bits)[c.outputs["out"]])
                assert got == _out(net, a, b, width)[0], (kind, prefix, a, b)
    for kind in ("ADDS", "SUBS"):
        net = OC.instruction(kind, width)
        for prefix in (C.PREFIX_GATES, C.PREFIX_MUX):
            c = C.flag_setting_circuit(kind, width, prefix=prefix)
            for a, b in pairs:
                bits = OC.to_bits(a, width) + OC.to_bits(b, width)
                v = eval_dag(c, bits)
                _, ov = _out(net, a, b, width)
                assert [int(x) for x in v[c.outputs["nzcv"]]] == [ov[w] for w in net.outputs["nzcv"]], (kind, a, b)


def test_oracle_netlists_under_fhe():
    """The oracle's own netlists evaluated homomorphically with its gates and
    MUX at toy parameters, level by level, then decrypted: 8-bit ADD and SUB,
    4-bit LT, EQ, ARS, unsigned and signed sequential MUL, DIV, and the
    flags of a 4-bit SUBS."""
    from oracle import oracle as O
    okeys = O.keygen(O.TOY, 95)
    cases = [("ADD", 8, 200, 100), ("SUB", 8, 17, 50), ("LT", 4, 3, 12), ("EQ", 4, 9, 9), ("ARS", 4, 0b1010, 1),
             ("MULSEQ", 3, 7, 5), ("SMULSEQ", 3, 0b101, 0b011), ("DIV", 3, 7, 2), ("SUBS", 4, 3, 9)]
    for i, (kind, w, a, b) in enumerate(cases):
        net = OC.instruction(kind, w)
        ins = O.encrypt_bits(okeys, np.asarray(OC.to_bits(a, w) + OC.to_bits(b, w), np.uint8), seed=40 + i)
        ct = net.run_encrypted(okeys, ins)
        got = OC.from_bits(O.decrypt_bits(okeys.lwe_key, np.stack([ct[x] for x in net.outputs["out"]])))
        assert got == OC.word_result(kind, w, a, b), (kind, a, b, got)
        if "nzcv" in net.outputs:
            f = O.decrypt_bits(okeys.lwe_key, np.stack([ct[x] for x in net.outputs["nzcv"]]))
            assert [int(x) for x in f] == OC.nzcv(kind, w, a, b)
