"""O16 -- CryptoEmu's functional units as levelled netlists of bootstrapped gates.

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module. It imports
nothing from the product package, and the product package never imports it.

Every unit below is built from the paper's own description of it, not from
the product's circuit builders:

  * the parallel-prefix adder (Sec. 5.2): stage 1 ``get_gp`` (g_i = a_i AND
    b_i, p_i = a_i XOR b_i); stage 2 the parallel scan with the operator
    (g_x, p_x) o (g_y, p_y) = (g_x + p_x g_y, p_x p_y), whose ``get_carry``
    takes two ANDs side by side and then the OR, so each scan level is two
    gate latencies; stage 3 one XOR per sum bit. The paper prints the sum bit
    as p_i XOR G_i; read with the carry INTO bit i, s_i = p_i XOR G_(i-1) with
    G_(-1) = carry-in, which is what makes the sum correct.
  * the subtractor (Sec. 5.3): a + NOT(b) + 1 with NOT unbootstrapped, and
    the carry out of bit 0 re-evaluated with one OR because carry-in is 1.
  * unsigned less-than as the borrow of that subtraction, equality as XNOR
    per bit and an AND reduction, the bitwise units of Sec. 5.7 (one gate per
    bit), and an array multiplier (rows of ANDs summed with the adder above).
  * the register-mode shifters of Sec. 5.4: log2 W stages of MUX selects, the
    k-th on amount bit k, moving by 2^k.
  * the sequential multiplier of Sec. 5.5 (its loop: P = 0; W times
    (P, carry) = P + (B[0] ? A : 0), then [carry, P, B] >>= 1) and, for signed
    operands, the plain sign-extended form that the paper starts from (every
    row sign-extended to 2W bits, the last row subtracted) rather than its
    "magic number" simplification, whose figures are missing.
  * the non-restoring divider of Sec. 5.6 (A = 0; W times shift [A, Q] left,
    add or subtract D by the sign of A, Q[0] = NOT sign(A)), with A two bits
    wider than the operands so that the shifted remainder and its sign are
    representable.
  * the NZCV flags of Sec. 6.1 from their definitions: N the result's sign,
    Z set iff every result bit is clear, C the adder's carry out, V set iff
    both operands of the adder have one sign and the result the other.

A netlist assigns every bootstrapped node a level: one more than its latest
bootstrapped input, or later when the builder places it in a later stage (the
paper runs every o of one scan level in the same OpenMP stage). ``run_plain``
evaluates it on cleartext bits with the gate truth tables of Table
"TFHEbenchmark"; ``run_encrypted`` evaluates it level by level with the
oracle's bootstrapped gates and MUX (``oracle.c``), each level one batch.
``word_result``, ``nzcv`` and ``condition`` give what the units must compute
in plain integer arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

# gate op codes of oracle.c (Table "TFHEbenchmark")
NAND, AND, OR, XOR, XNOR, NOR, ANDNY, ANDYN, ORNY, ORYN = range(10)

# Truth tables, outputs for (a, b) = (0, 0), (0, 1), (1, 0), (1, 1).
# ANDNY = (NOT a) AND b, ANDYN = a AND (NOT b), ORNY = (NOT a) OR b,
# ORYN = a OR (NOT b).
TRUTH = {
    NAND: (1, 1, 1, 0), AND: (0, 0, 0, 1), OR: (0, 1, 1, 1), XOR: (0, 1, 1, 0),
    XNOR: (1, 0, 0, 1), NOR: (1, 0, 0, 0), ANDNY: (0, 1, 0, 0), ANDYN: (0, 0, 1, 0),
    ORNY: (1, 1, 0, 1), ORYN: (1, 0, 1, 1),
}


def gate_plain(op: int, a: int, b: int) -> int:
    return TRUTH[op][2 * int(a) + int(b)]


def lwe_not(ct) -> np.ndarray:
    """NOT without bootstrapping (Table "TFHEbenchmark": NOT): every word of
    the sample negated mod 2^32, which negates the phase, +-1/8 -> -+1/8."""
    return (np.uint32(0) - np.asarray(ct, np.uint32)).astype(np.uint32)


def lwe_constant(bit: int, n: int) -> np.ndarray:
    """CONSTANT (Table "TFHEbenchmark"): the noiseless trivial sample
    (0, ..., 0, +1/8) for true, (0, ..., 0, -1/8) for false."""
    c = np.zeros(n + 1, np.uint32)
    c[n] = np.uint32(0x20000000 if bit else 0xE0000000)
    return c


class Netlist:
    """Nodes: ('in', k) | ('const', bit) | ('not', x) | ('gate', op, x, y) |
    ('mux', s, x, y) with mux = s ? x : y. Inputs and constants sit at level
    0 and a NOT at its input's level (it is not bootstrapped)."""

    def __init__(self):
        self.nodes = []
        self.level = []
        self.n_inputs = 0
        self.outputs = {}

    def _add(self, node, level):
        self.nodes.append(node)
        self.level.append(level)
        return len(self.nodes) - 1

    def inp(self):
        self.n_inputs += 1
        return self._add(("in", self.n_inputs - 1), 0)

    def word(self, width):
        return [self.inp() for _ in range(width)]

    def const(self, bit):
        return self._add(("const", int(bit)), 0)

    def NOT(self, x):
        return self._add(("not", x), self.level[x])

    def gate(self, op, x, y, stage=0):
        return self._add(("gate", op, x, y), max(stage, 1 + max(self.level[x], self.level[y])))

    def mux(self, s, x, y, stage=0):
        return self._add(("mux", s, x, y), max(stage, 1 + max(self.level[s], self.level[x], self.level[y])))

    def depth(self):
        return max([self.level[w] for w, nd in enumerate(self.nodes) if nd[0] in ("gate", "mux")], default=0)

    def gates_per_level(self):
        """Bootstrapped binary gates at levels 1 .. depth (MUXes not counted)."""
        cnt = [0] * (self.depth() + 1)
        for w, nd in enumerate(self.nodes):
            if nd[0] == "gate":
                cnt[self.level[w]] += 1
        return cnt[1:]

    def muxes_per_level(self):
        cnt = [0] * (self.depth() + 1)
        for w, nd in enumerate(self.nodes):
            if nd[0] == "mux":
                cnt[self.level[w]] += 1
        return cnt[1:]

    # ----------------------------------------------------------- evaluation
    def run_plain(self, bits) -> list:
        """Cleartext value of every wire; bits feed the inputs in order."""
        bits = [int(b) for b in bits]
        if len(bits) != self.n_inputs:
            raise ValueError("wrong number of input bits")
        v = [0] * len(self.nodes)
        for w, nd in enumerate(self.nodes):
            kind = nd[0]
            if kind == "in":
                v[w] = bits[nd[1]]
            elif kind == "const":
                v[w] = nd[1]
            elif kind == "not":
                v[w] = 1 - v[nd[1]]
            elif kind == "gate":
                v[w] = gate_plain(nd[1], v[nd[2]], v[nd[3]])
            else:
                v[w] = v[nd[2]] if v[nd[1]] else v[nd[3]]
        return v

    def run_encrypted(self, keys, inputs) -> dict:
        """Ciphertext of every wire, computed level by level with the
        oracle's gates: each level's gates are one ``bootstrap_batch`` and its
        MUXes one ``mux_batch``. NOT negates every word of the sample and a
        constant is the noiseless sample (0, ..., 0, +-1/8) (Table
        "TFHEbenchmark": NOT, CONSTANT, not bootstrapped)."""
        inputs = np.asarray(inputs, np.uint32)
        n = keys.params.n
        ct = {}

        def settle(w):
            # inputs, constants and NOT chains below the current level
            if w in ct:
                return ct[w]
            nd = self.nodes[w]
            if nd[0] == "in":
                ct[w] = inputs[nd[1]].copy()
            elif nd[0] == "const":
                ct[w] = lwe_constant(nd[1], n)
            elif nd[0] == "not":
                ct[w] = lwe_not(settle(nd[1]))
            else:
                raise RuntimeError("bootstrapped node used before its level ran")
            return ct[w]

        for L in range(1, self.depth() + 1):
            gw = [w for w, nd in enumerate(self.nodes) if nd[0] == "gate" and self.level[w] == L]
            mw = [w for w, nd in enumerate(self.nodes) if nd[0] == "mux" and self.level[w] == L]
            if gw:
                ops = np.array([self.nodes[w][1] for w in gw], np.int32)
                c1 = np.stack([settle(self.nodes[w][2]) for w in gw])
                c2 = np.stack([settle(self.nodes[w][3]) for w in gw])
                _, out = O.bootstrap_batch(keys, ops, c1, c2, want_extracted=False)
                for i, w in enumerate(gw):
                    ct[w] = out[i]
            if mw:
                s = np.stack([settle(self.nodes[w][1]) for w in mw])
                c1 = np.stack([settle(self.nodes[w][2]) for w in mw])
                c2 = np.stack([settle(self.nodes[w][3]) for w in mw])
                out = O.mux_batch(keys, s, c1, c2)
                for i, w in enumerate(mw):
                    ct[w] = out[i]
        for ws in self.outputs.values():
            for w in ws:
                settle(w)
        return ct


# ------------------------------------------------------------------ units
def _base(net, wires):
    return max(net.level[w] for w in wires)


def prefix_add(net, A, B, carry_in=0):
    """The parallel-prefix adder of Sec. 5.2 on W-bit words (LSB first),
    carry_in 0 or 1 (a cleartext constant). Returns (sum, carry out)."""
    W = len(A)
    s0 = _base(net, list(A) + list(B))
    # stage 1 (get_gp): every bit's generate and propagate, one stage
    g = [net.gate(AND, A[i], B[i], s0 + 1) for i in range(W)]
    p = [net.gate(XOR, A[i], B[i], s0 + 1) for i in range(W)]
    gp = [(g[i], p[i]) for i in range(W)]
    if carry_in:
        # Sec. 5.3: with carry-in 1 the carry out of bit 0 is g_0 + p_0, one OR
        gp[0] = (net.gate(OR, g[0], p[0], s0 + 2), p[0])

    def odot(x, y, stage):
        # (g_x, p_x) o (g_y, p_y) = (g_x + p_x g_y, p_x p_y): get_carry runs
        # the two ANDs side by side, then the OR
        t = net.gate(AND, x[1], y[0], stage)
        pp = net.gate(AND, x[1], y[1], stage)
        return (net.gate(OR, x[0], t, stage + 1), pp)

    # stage 2: scan level k combines every position i >= d = 2^(k-1) with
    # position i - d; the ANDs of level k run in stage s0 + 2k, the ORs in
    # s0 + 2k + 1
    d, k = 1, 1
    while d < W:
        gp = [gp[i] if i < d else odot(gp[i], gp[i - d], s0 + 2 * k) for i in range(W)]
        d, k = 2 * d, k + 1
    # stage 3: s_i = p_i XOR (carry into bit i); the carry into bit 0 is the
    # carry-in, a constant, still one XOR gate
    last = s0 + 2 * k
    carries = [net.const(carry_in)] + [gp[i][0] for i in range(W - 1)]
    s = [net.gate(XOR, p[i], carries[i], last) for i in range(W)]
    return s, gp[W - 1][0]


def prefix_sub(net, A, B):
    """Sec. 5.3: a + NOT(b) + 1. Returns (difference, carry out); carry out
    1 means no borrow (a >= b unsigned)."""
    return prefix_add(net, A, [net.NOT(b) for b in B], carry_in=1)


def less_than(net, A, B):
    _, c = prefix_sub(net, A, B)
    return net.NOT(c)


def equal(net, A, B):
    bits = [net.gate(XNOR, a, b) for a, b in zip(A, B)]
    while len(bits) > 1:
        pairs = [net.gate(AND, bits[i], bits[i + 1]) for i in range(0, len(bits) - 1, 2)]
        bits = pairs + ([bits[-1]] if len(bits) % 2 else [])
    return bits[0]


def bitwise(net, op, A, B):
    return [net.gate(op, a, b) for a, b in zip(A, B)]


def array_multiply(net, A, B):
    """W x W -> 2W unsigned: row i = (A AND B[i]) << i, rows summed one after
    another with the 2W-bit prefix adder."""
    W = len(A)
    zero = net.const(0)
    acc = None
    for i in range(W):
        row = [zero] * i + [net.gate(AND, A[j], B[i]) for j in range(W)] + [zero] * (W - i)
        acc = row if acc is None else prefix_add(net, acc, row)[0]
    return acc


LLS, LRS, ARS = "LLS", "LRS", "ARS"


def barrel_shift(net, A, S, mode):
    """Sec. 5.4 register mode: stage k (amount bit k) replaces bit i by the
    bit 2^k places away when S[k] is set (MUX), zero-filled for LLS and LRS,
    sign-filled for ARS."""
    W = len(A)
    zero = net.const(0)
    cur = list(A)
    k = 0
    while (1 << k) < W:
        d = 1 << k
        if mode == LLS:
            src = [cur[i - d] if i - d >= 0 else zero for i in range(W)]
        elif mode == LRS:
            src = [cur[i + d] if i + d < W else zero for i in range(W)]
        elif mode == ARS:
            src = [cur[i + d] if i + d < W else cur[W - 1] for i in range(W)]
        else:
            raise ValueError(mode)
        cur = [net.mux(S[k], src[i], cur[i]) for i in range(W)]
        k += 1
    return cur


def sequential_multiply(net, A, B):
    """Sec. 5.5 unsigned: P = 0; W times (P, carry) = P + (B[0] ? A : 0),
    [carry, P, B] >>= 1; the product is [P, B] (2W bits, LSB first)."""
    W = len(A)
    P = [net.const(0) for _ in range(W)]
    Bv = list(B)
    for _ in range(W):
        row = [net.gate(AND, A[j], Bv[0]) for j in range(W)]
        P, carry = prefix_add(net, P, row)
        # shift [carry, P, B] right by one: B loses its bit 0, gains P[0]
        Bv = Bv[1:] + [P[0]]
        P = P[1:] + [carry]
    return Bv + P


def signed_multiply(net, A, B):
    """Signed W x W -> 2W (two's complement) in the sign-extended form the
    paper starts from: partial product i is A sign-extended to 2W bits, ANDed
    with B[i] and shifted by i; rows 0 .. W-2 are added and row W-1 (weight
    -2^(W-1)) is subtracted, all with the 2W-bit prefix adder."""
    W = len(A)
    zero = net.const(0)
    acc = None
    for i in range(W):
        bits = [net.gate(AND, A[j], B[i]) for j in range(W)]
        row = ([zero] * i + bits + [bits[W - 1]] * W)[:2 * W]
        if i < W - 1:
            acc = row if acc is None else prefix_add(net, acc, row)[0]
        else:
            acc = prefix_sub(net, acc if acc is not None else [zero] * (2 * W), row)[0]
    return acc


def nonrestoring_divide(net, Q, D):
    """Sec. 5.6, unsigned W-bit Q / D: A = 0; W times: shift [A, Q] left;
    A = A + D if A < 0 else A - D; Q[0] = 1 if A >= 0. The partial remainder
    stays in [-D, D), so after the shift it lies in [-2D, 2D): A is kept
    W + 2 bits wide, which holds that range, so the sign test after the shift
    is exact as printed. Written with an adder and a subtractor per step and
    a MUX on the sign of A; the remainder is not needed."""
    W = len(Q)
    A = [net.const(0) for _ in range(W + 2)]
    Qv = list(Q)
    Dx = list(D) + [net.const(0), net.const(0)]
    for _ in range(W):
        A = [Qv[W - 1]] + A[:W + 1]      # [A, Q] << 1: A takes Q's MSB
        Qv = [None] + Qv[:W - 1]
        neg = A[W + 1]
        plus, _ = prefix_add(net, A, Dx)
        minus, _ = prefix_sub(net, A, Dx)
        A = [net.mux(neg, plus[i], minus[i]) for i in range(W + 2)]
        Qv[0] = net.NOT(A[W + 1])
    return Qv


def flags(net, result, carry, a_sign, b_sign):
    """Sec. 6.1 NZCV: N = the result's sign; Z = 1 iff every result bit is 0
    (AND reduction of the inverted bits); C = the adder's carry out;
    V = 1 iff the adder's operands share a sign that the result does not
    have: (a XNOR b) AND (a XOR s)."""
    W = len(result)
    s = result[W - 1]
    inv = [net.NOT(r) for r in result]
    while len(inv) > 1:
        inv = [net.gate(AND, inv[i], inv[i + 1]) for i in range(0, len(inv) - 1, 2)] + \
              ([inv[-1]] if len(inv) % 2 else [])
    v = net.gate(AND, net.gate(XNOR, a_sign, b_sign), net.gate(XOR, a_sign, s))
    return [s, inv[0], carry, v]


def instruction(kind: str, width: int) -> Netlist:
    """One instruction as a netlist: inputs a then b (width bits each, LSB
    first), output 'out' (and 'nzcv' for ADDS / SUBS / CMP)."""
    net = Netlist()
    A, B = net.word(width), net.word(width)
    if kind == "ADD":
        out = prefix_add(net, A, B)[0]
    elif kind == "SUB":
        out = prefix_sub(net, A, B)[0]
    elif kind == "LT":
        out = [less_than(net, A, B)]
    elif kind == "EQ":
        out = [equal(net, A, B)]
    elif kind in ("AND", "OR", "XOR", "ORN"):
        out = bitwise(net, {"AND": AND, "OR": OR, "XOR": XOR, "ORN": ORYN}[kind], A, B)
    elif kind == "MUL":
        out = array_multiply(net, A, B)
    elif kind in (LLS, LRS, ARS):
        out = barrel_shift(net, A, B, kind)
    elif kind == "MULSEQ":
        out = sequential_multiply(net, A, B)
    elif kind == "SMULSEQ":
        out = signed_multiply(net, A, B)
    elif kind == "DIV":
        out = nonrestoring_divide(net, A, B)
    elif kind == "ADDS":
        out, c = prefix_add(net, A, B)
        net.outputs["nzcv"] = flags(net, out, c, A[width - 1], B[width - 1])
    elif kind in ("SUBS", "CMP"):
        nb = [net.NOT(b) for b in B]
        out, c = prefix_add(net, A, nb, carry_in=1)
        net.outputs["nzcv"] = flags(net, out, c, A[width - 1], nb[width - 1])
    else:
        raise ValueError(f"unknown instruction {kind}")
    net.outputs["out"] = out
    return net


# ------------------------------------------------------- cleartext results
def to_bits(v: int, width: int) -> list:
    return [(int(v) >> i) & 1 for i in range(width)]


def from_bits(bits) -> int:
    v = 0
    for i, b in enumerate(bits):
        v |= int(b) << i
    return v


def _signed(v: int, width: int) -> int:
    return v - (1 << width) if v & (1 << (width - 1)) else v


def word_result(kind: str, width: int, a: int, b: int) -> int:
    """What instruction ``kind`` computes on W-bit unsigned operands a, b:
    W-bit results wrap; MUL, MULSEQ and SMULSEQ give 2W bits; LT and EQ one
    bit; shifts take the amount b modulo W; DIV by zero gives 2^W - 1 (every
    quotient bit set, which is what the non-restoring loop yields)."""
    M = 1 << width
    a, b = int(a) % M, int(b) % M
    if kind in ("ADD", "ADDS"):
        return (a + b) % M
    if kind in ("SUB", "SUBS", "CMP"):
        return (a - b) % M
    if kind in ("MUL", "MULSEQ"):
        return a * b
    if kind == "SMULSEQ":
        return (_signed(a, width) * _signed(b, width)) % (M * M)
    if kind == "LT":
        return 1 if a < b else 0
    if kind == "EQ":
        return 1 if a == b else 0
    if kind == "AND":
        return a & b
    if kind == "OR":
        return a | b
    if kind == "XOR":
        return a ^ b
    if kind == "ORN":
        return a | (M - 1 - b)
    sh = b % width
    if kind == LLS:
        return (a << sh) % M
    if kind == LRS:
        return a >> sh
    if kind == ARS:
        return (_signed(a, width) >> sh) % M
    if kind == "DIV":
        return a // b if b else M - 1
    raise ValueError(f"unknown instruction {kind}")


def nzcv(kind: str, width: int, a: int, b: int) -> list:
    """ARM flags of ADDS / SUBS / CMP (Sec. 6.1): N the result's sign bit, Z
    the result is zero, C unsigned carry out (for subtraction: no borrow),
    V signed overflow."""
    M = 1 << width
    if kind == "ADDS":
        r = (a + b) % M
        c = 1 if a + b >= M else 0
        exact = _signed(a, width) + _signed(b, width)
    elif kind in ("SUBS", "CMP"):
        r = (a - b) % M
        c = 1 if a >= b else 0
        exact = _signed(a, width) - _signed(b, width)
    else:
        raise ValueError(kind)
    v = 0 if _signed(r, width) == exact else 1
    return [r >> (width - 1), 1 if r == 0 else 0, c, v]


def condition(cond: str, n: int, z: int, c: int, v: int) -> bool:
    """ARM condition codes over the NZCV flags."""
    table = {
        "EQ": z == 1, "NE": z == 0,
        "CS": c == 1, "HS": c == 1, "CC": c == 0, "LO": c == 0,
        "MI": n == 1, "PL": n == 0, "VS": v == 1, "VC": v == 0,
        "HI": c == 1 and z == 0, "LS": not (c == 1 and z == 0),
        "GE": n == v, "LT": n != v,
        "GT": z == 0 and n == v, "LE": not (z == 0 and n == v),
        "AL": True,
    }
    return bool(table[cond])
