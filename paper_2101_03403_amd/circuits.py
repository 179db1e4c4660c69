"""Gate-level circuits of CryptoEmu's functional units and the level scheduler
that runs them on the GPU.

Circuits (built from bootstrapped binary gates plus the free NOT / CONSTANT):
  * ``kogge_stone_add`` -- the parallel-prefix adder of Sec. 5.2: stage 1
    computes (g_i, p_i) = (a_i AND b_i, a_i XOR b_i) (Fig. get_gp); stage 2
    applies the operator (g_x, p_x) o (g_y, p_y) = (g_x + p_x g_y, p_x p_y) in
    log2 W levels, each level at distance d = 1, 2, 4, ... and each o made of
    AND -> OR on the carry and AND on the propagate (Fig. get_carry); stage 3
    sums s_i = p_i XOR G_{i-1} with G_{-1} = carry-in. For W = 32 the levels
    hold [64 | 62, 31 | 60, 30 | 56, 28 | 48, 24 | 32, 16 | 32] gates
    (o counts 31, 30, 28, 24, 16 as in the text of Sec. 5.2), 483 in total,
    depth 2 log2 W + 2 = 12. With ``prefix=PREFIX_MUX`` the carry half of
    every o is one FHE MUX (P_x ? G_y : G_x, exact because a position never
    both generates and propagates), so a prefix level is one level and the
    32-bit adder is 7 levels deep (452 bootstraps); every adder-based unit
    below takes the same option.
  * ``subtract`` -- a + NOT(b) + 1 (Sec. 5.3): unbootstrapped NOT of b, the
    carry-in folded into bit 0 by one OR, and the sum bit 0 by one XOR with a
    constant (the subtractor's two extra bootstrapped gates).
  * ``less_than`` (borrow of a - b), ``equal`` (XNOR + AND tree),
    ``bitwise`` (one gate per bit, Sec. 5.7) and ``array_multiply`` (AND
    partial products accumulated with Kogge-Stone adders) -- the compare,
    bitwise and multiply instructions of the mixed instruction stream.
  * ``sequential_multiply`` (unsigned and signed) and ``nonrestoring_divide``
    -- the paper's multiplier (Sec. 5.5: W iterations of an AND row and a
    W-bit adder) and divider (Sec. 5.6: W iterations of an add/subtract
    adder), long chains of narrow levels.
  * ``barrel_shift`` -- the register-mode shifters LLS / LRS / ARS of
    Sec. 5.4: log2 W stages of W FHE MUX selects each (the MUX of Table
    "TFHEbenchmark", two bootstraps), and ``shift_immediate`` -- the
    immediate mode, which only moves wires and inserts constants.

Execution: ``Program`` takes any number of circuit instances, assigns each
bootstrapped gate to a level (one more than its latest bootstrapped input,
i.e. the paper's stage order), and merges the gates and MUXes of one level
across all instances into a single batched launch (gather from / scatter to
one device ciphertext pool). The launch sequence can be captured once as a
hipGraph and replayed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cemu

NAND, AND, OR, XOR, XNOR, NOR, ANDNY, ANDYN, ORNY, ORYN = range(10)

@dataclass
class Circuit:
    """A DAG over wires. Kinds: 'in', 'gate' (bootstrapped), 'mux' (FHE MUX,
    two bootstraps; node (kind, s, a, b) selects a when s is true), 'not',
    'const'.

    Every wire has a level: 0 for inputs and constants, the input's level for
    NOT, and for a gate the larger of 1 + its inputs' levels and a requested
    level (used to keep the paper's stage structure, where every o of one
    prefix level runs in the same stage)."""
    nodes: list = field(default_factory=list)      # (kind, op, a, b)
    lv: list = field(default_factory=list)         # level of each wire
    inputs: list = field(default_factory=list)     # wire ids fed from outside
    outputs: dict = field(default_factory=dict)    # name -> list of wires

    def _new(self, kind, op=-1, a=-1, b=-1, level=0) -> int:
        self.nodes.append((kind, op, a, b))
        self.lv.append(level)
        return len(self.nodes) - 1

    def input(self) -> int:
        w = self._new("in")
        self.inputs.append(w)
        return w

    def inputs_word(self, width: int) -> list:
        return [self.input() for _ in range(width)]

    def gate(self, op: int, a: int, b: int, level: int = 0) -> int:
        return self._new("gate", op, a, b, max(1 + max(self.lv[a], self.lv[b]), level))

    def mux(self, s: int, a: int, b: int, level: int = 0) -> int:
        """s ? a : b."""
        return self._new("mux", s, a, b, max(1 + max(self.lv[s], self.lv[a], self.lv[b]), level))

    def NOT(self, a: int) -> int:
        return self._new("not", -1, a, -1, self.lv[a])

    def const(self, bit: int) -> int:
        return self._new("const", int(bit))

    def levels(self) -> np.ndarray:
        return np.array(self.lv, dtype=np.int64)

    def gate_counts_per_level(self) -> list:
        """Bootstrapped binary gates per level (MUX nodes not included)."""
        gl = [self.lv[w] for w, n in enumerate(self.nodes) if n[0] == "gate"]
        if not gl:
            return []
        gl = np.array(gl)
        return [int(np.sum(gl == L)) for L in range(1, int(gl.max()) + 1)]

    def depth(self) -> int:
        return max([self.lv[w] for w, n in enumerate(self.nodes) if n[0] in ("gate", "mux")], default=0)

    def num_gates(self) -> int:
        return sum(1 for n in self.nodes if n[0] == "gate")

    def num_muxes(self) -> int:
        return sum(1 for n in self.nodes if n[0] == "mux")

    def num_bootstraps(self) -> int:
        return self.num_gates() + 2 * self.num_muxes()


# ------------------------------------------------------------------ circuits
# Forms of the adders' prefix stage: the paper's o operator as AND -> OR
# gates (two levels per prefix level), or as one FHE MUX per carry (one level
# per prefix level).
PREFIX_GATES, PREFIX_MUX = "gates", "mux"


def _prefix_mux(c: Circuit, G: list, P: list, first: int) -> int:
    """MUX form of the prefix stage, in place on G, P (P[i] None = known 0).

    Because g_i = a_i AND b_i and p_i = a_i XOR b_i never hold together, and
    the o operator keeps that true for every group, the carry half of
    (G_x, P_x) o (G_y, P_y) = (G_x + P_x G_y, P_x P_y) is a selection:
    P_x ? G_y : G_x, one FHE MUX (Table "TFHEbenchmark") instead of AND -> OR.
    Prefix level k (distance d = 2^(k-1)) runs at level first + k, its MUXes
    beside the ANDs of the propagates that a later level still needs
    (positions >= 2d). Returns the number of prefix levels."""
    n = len(G)
    d, k = 1, 1
    while d < n:
        newG = {i: G[i] if P[i] is None else c.mux(P[i], G[i - d], G[i], first + k) for i in range(d, n)}
        newP = {i: None if P[i] is None or P[i - d] is None else c.gate(AND, P[i], P[i - d], first + k)
                for i in range(2 * d, n)}
        for i in range(d, n):
            G[i] = newG[i]
            P[i] = newP.get(i)
        d *= 2
        k += 1
    return k - 1


def kogge_stone_add(c: Circuit, A: list, B: list, carry_in: int | None = None, prefix: str = PREFIX_GATES):
    """Parallel-prefix adder (Sec. 5.2). A, B: wires, LSB first. carry_in:
    None (0) or 1 (constant). Returns (sum wires, carry-out wire).

    prefix = PREFIX_GATES (the paper's structure): stages relative to the
    inputs' level: 1 = (g, p); for prefix level k (distance 2^(k-1)): 2k = the
    two ANDs of every o, 2k+1 = its OR; last = the sum XORs.
    prefix = PREFIX_MUX: every o's carry is one MUX (see _prefix_mux), so a
    W-bit adder is log2 W + 2 levels deep (7 for W = 32 instead of 12); with
    carry-in 1 the carry out of bit 0 is a_0 OR b_0, taken in stage 1."""
    W = len(A)
    base = max(c.lv[w] for w in list(A) + list(B))
    if prefix == PREFIX_MUX:
        p = [c.gate(XOR, A[i], B[i], base + 1) for i in range(W)]
        G = [c.gate(OR if (i == 0 and carry_in == 1) else AND, A[i], B[i], base + 1) for i in range(W)]
        P = list(p)
        last = base + 2 + _prefix_mux(c, G, P, base + 1)
        cin = c.const(1 if carry_in == 1 else 0)
        s = [c.gate(XOR, p[0], cin, last)] + [c.gate(XOR, p[i], G[i - 1], last) for i in range(1, W)]
        return s, G[W - 1]
    if prefix != PREFIX_GATES:
        raise ValueError(f"unknown prefix form {prefix}")
    g = [c.gate(AND, A[i], B[i], base + 1) for i in range(W)]
    p = [c.gate(XOR, A[i], B[i], base + 1) for i in range(W)]
    G = list(g)
    P = list(p)
    if carry_in == 1:
        # carry out of bit 0 with carry-in 1: g_0 + p_0 * 1 (one extra OR)
        G[0] = c.gate(OR, g[0], p[0], base + 2)
    d, k = 1, 1
    while d < W:
        tmp = {i: c.gate(AND, P[i], G[i - d], base + 2 * k) for i in range(d, W)}
        newP = {i: c.gate(AND, P[i], P[i - d], base + 2 * k) for i in range(d, W)}
        newG = {i: c.gate(OR, G[i], tmp[i], base + 2 * k + 1) for i in range(d, W)}
        for i in range(d, W):
            G[i] = newG[i]
            P[i] = newP[i]
        d *= 2
        k += 1
    last = base + 2 * k
    cin = c.const(1 if carry_in == 1 else 0)
    s = [c.gate(XOR, p[0], cin, last)] + [c.gate(XOR, p[i], G[i - 1], last) for i in range(1, W)]
    return s, G[W - 1]


def add_with_carry_wire(c: Circuit, A: list, B: list, cin: int, prefix: str = PREFIX_GATES):
    """Kogge-Stone A + B + cin with an encrypted carry-in wire: the carry is
    prefix position -1 with (G, P) = (cin, 0), so it enters through the same
    o levels as every other position (ceil(log2(W + 1)) prefix levels, each
    two gate levels deep, or one with prefix = PREFIX_MUX).
    Returns (sum wires, carry-out wire)."""
    W = len(A)
    base = max(c.lv[w] for w in list(A) + list(B) + [cin])
    g = [c.gate(AND, A[i], B[i], base + 1) for i in range(W)]
    p = [c.gate(XOR, A[i], B[i], base + 1) for i in range(W)]
    G = [cin] + g                  # index 0 = position -1
    P = [None] + list(p)           # None = known zero
    if prefix == PREFIX_MUX:
        last = base + 2 + _prefix_mux(c, G, P, base + 1)
        s = [c.gate(XOR, p[i], G[i], last) for i in range(W)]
        return s, G[W]
    if prefix != PREFIX_GATES:
        raise ValueError(f"unknown prefix form {prefix}")
    d, k = 1, 1
    while d < W + 1:
        newG, newP = {}, {}
        for i in range(d, W + 1):
            tmp = c.gate(AND, P[i], G[i - d], base + 2 * k)
            newP[i] = None if P[i - d] is None else c.gate(AND, P[i], P[i - d], base + 2 * k)
            newG[i] = c.gate(OR, G[i], tmp, base + 2 * k + 1)
        for i in newG:
            G[i] = newG[i]
            P[i] = newP[i]
        d *= 2
        k += 1
    last = base + 2 * k
    s = [c.gate(XOR, p[i], G[i], last) for i in range(W)]   # G[i] = carry into bit i
    return s, G[W]


def subtract(c: Circuit, A: list, B: list, prefix: str = PREFIX_GATES):
    """a - b = a + NOT(b) + 1 (Sec. 5.3). Returns (difference wires, carry-out
    wire; carry-out 1 means no borrow, i.e. a >= b unsigned)."""
    nb = [c.NOT(b) for b in B]
    return kogge_stone_add(c, A, nb, carry_in=1, prefix=prefix)


def less_than(c: Circuit, A: list, B: list, prefix: str = PREFIX_GATES) -> int:
    """Unsigned a < b: the borrow of a - b, i.e. NOT(carry-out)."""
    _, carry = subtract(c, A, B, prefix)
    return c.NOT(carry)


def equal(c: Circuit, A: list, B: list) -> int:
    """a == b: XNOR per bit, then a balanced AND tree."""
    layer = [c.gate(XNOR, a, b) for a, b in zip(A, B)]
    while len(layer) > 1:
        nxt = [c.gate(AND, layer[i], layer[i + 1]) for i in range(0, len(layer) - 1, 2)]
        if len(layer) % 2:
            nxt.append(layer[-1])
        layer = nxt
    return layer[0]


def bitwise(c: Circuit, op: int, A: list, B: list) -> list:
    """One bootstrapped gate per bit (Sec. 5.7)."""
    return [c.gate(op, a, b) for a, b in zip(A, B)]


def _full_add(c: Circuit, a: int, b: int, cin: int):
    """Full adder of bootstrapped gates: s = a ^ b ^ cin, cout = ab + cin(a ^ b)."""
    t = c.gate(XOR, a, b)
    s = c.gate(XOR, t, cin)
    cout = c.gate(OR, c.gate(AND, a, b), c.gate(AND, t, cin))
    return s, cout


def array_multiply(c: Circuit, A: list, B: list, prefix: str = PREFIX_GATES) -> list:
    """Unsigned W x W -> 2W product as an array multiplier: the W^2 AND partial
    products (one level), rows accumulated in carry-save form with full and
    half adders, and a final Kogge-Stone adder for the sum and carry vectors.
    Known-zero positions are skipped rather than computed."""
    W = len(A)
    ZERO = None
    S = [ZERO] * (2 * W)     # sum vector (None = constant 0)
    Cv = [ZERO] * (2 * W)    # carry vector, already aligned to its weight
    for i in range(W):
        row = [ZERO] * (2 * W)
        for j in range(W):
            row[i + j] = c.gate(AND, A[j], B[i])
        newS, newC = [ZERO] * (2 * W), [ZERO] * (2 * W)
        for k in range(2 * W):
            ins = [w for w in (S[k], Cv[k], row[k]) if w is not None]
            if len(ins) == 0:
                continue
            if len(ins) == 1:
                newS[k] = ins[0]
            elif len(ins) == 2:
                newS[k] = c.gate(XOR, ins[0], ins[1])
                if k + 1 < 2 * W:
                    newC[k + 1] = c.gate(AND, ins[0], ins[1])
            else:
                sk, ck = _full_add(c, *ins)
                newS[k] = sk
                if k + 1 < 2 * W:
                    newC[k + 1] = ck
        S, Cv = newS, newC
    zero = c.const(0)
    Sw = [w if w is not None else zero for w in S]
    Cw = [w if w is not None else zero for w in Cv]
    out, _ = kogge_stone_add(c, Sw, Cw, prefix=prefix)
    return out


LLS, LRS, ARS = "LLS", "LRS", "ARS"


def barrel_shift(c: Circuit, A: list, S: list, mode: str) -> list:
    """Register-mode shifter (Sec. 5.4, figures LLS / LRS): stage k (k = 0 ..
    log2 W - 1, in the order of the shift-amount bits) selects for every bit
    i, with the FHE MUX on amount bit S[k], between the bit 2^k places away
    and bit i itself. LLS takes bit i - 2^k (zero shifted in); LRS takes bit
    i + 2^k (zero shifted in); ARS is LRS with the register's sign bit as the
    shift-in value. W must be a power of two; only the low log2 W amount bits
    are used, so the amount is taken modulo W."""
    W = len(A)
    if W & (W - 1) or W < 2:
        raise ValueError("barrel_shift needs a power-of-two width")
    if mode not in (LLS, LRS, ARS):
        raise ValueError(f"unknown shift mode {mode}")
    zero = c.const(0)
    cur = list(A)
    for k in range(W.bit_length() - 1):
        d = 1 << k
        nxt = []
        for i in range(W):
            if mode == LLS:
                src = cur[i - d] if i >= d else zero
            elif mode == LRS:
                src = cur[i + d] if i + d < W else zero
            else:
                src = cur[i + d] if i + d < W else cur[W - 1]
            nxt.append(c.mux(S[k], src, cur[i]))
        cur = nxt
    return cur


def shift_immediate(c: Circuit, A: list, amount: int, mode: str) -> list:
    """Immediate-mode shift (Sec. 5.4): the amount is cleartext, so the bits
    are only moved (COPY) and the vacated positions take the constant zero
    (LLS, LRS) or the sign bit (ARS); nothing is bootstrapped."""
    W = len(A)
    k = int(amount) % W
    if mode == LLS:
        return [c.const(0) for _ in range(k)] + list(A[:W - k])
    if mode == LRS:
        return list(A[k:]) + [c.const(0) for _ in range(k)]
    if mode == ARS:
        return list(A[k:]) + [A[W - 1]] * k
    raise ValueError(f"unknown shift mode {mode}")


def sequential_multiply(c: Circuit, A: list, B: list, signed: bool = False, prefix: str = PREFIX_GATES) -> list:
    """The paper's sequential (carry-save) multiplier (Sec. 5.5): P = 0; W
    times: (P, carry) = P + (B[i] ? A : 0) with a W-bit Kogge-Stone adder,
    then [carry, P, B] >> 1, so bit i of the product is the low sum bit of
    iteration i and the high word is the final P (2W-bit result). The row
    bits are ANDs of A with one bit of B; they depend only on the inputs, so
    they all land in the first level and each iteration is one adder deep.

    signed: two's-complement operands, sign extension removed by the usual
    constant ("magic number") correction. Row i < W-1 has its MSB inverted
    (NAND instead of AND), the last row (weight -2^(W-1)) has its other bits
    inverted, and the constant 2^(2W-1) + 2^W this leaves is added as P's
    initial value 2^(W-1), a carry-in of 1 on the last iteration (the other
    2^(W-1)), and an unbootstrapped NOT of the product's MSB."""
    W = len(A)
    P = [c.const(0) for _ in range(W - 1)] + [c.const(1 if signed else 0)]
    low = []
    for i in range(W):
        last = i == W - 1
        row = []
        for j in range(W):
            invert = signed and ((j == W - 1) != last)
            row.append(c.gate(NAND if invert else AND, A[j], B[i]))
        S, carry = kogge_stone_add(c, P, row, carry_in=1 if (signed and last) else None, prefix=prefix)
        low.append(S[0])
        P = S[1:] + [carry]
    out = low + P
    if signed:
        out[2 * W - 1] = c.NOT(out[2 * W - 1])
    return out


def nonrestoring_divide(c: Circuit, Q: list, D: list, prefix: str = PREFIX_GATES) -> list:
    """Unsigned non-restoring division (Sec. 5.6): A = 0 (one bit wider than
    the operands, the sign bit), W times: shift [A, Q] left, then A = A - D
    if A was >= 0 before the shift, else A = A + D, and Q[0] = NOT sign(A).
    The add/subtract is one adder whose second operand is D XOR SUB with
    carry-in SUB = NOT sign(A) (the paper's adder with SUB select). The
    remainder is not corrected (the instruction only returns the quotient);
    division by zero returns 2^W - 1."""
    W = len(Q)
    A = [c.const(0) for _ in range(W + 1)]
    Q = list(Q)
    for _ in range(W):
        sub = c.NOT(A[W])
        A = [Q[W - 1]] + A[:W]
        Q = [None] + Q[:W - 1]
        Dx = [c.gate(XOR, D[j], sub) for j in range(W)] + [sub]   # D's top bit is 0
        A, _ = add_with_carry_wire(c, A, Dx, sub, prefix)
        Q[0] = c.NOT(A[W])
    return Q


def or_reduce(c: Circuit, bits: list) -> int:
    """Balanced OR tree (log2 W levels, W/2 gates in the first)."""
    layer = list(bits)
    while len(layer) > 1:
        nxt = [c.gate(OR, layer[i], layer[i + 1]) for i in range(0, len(layer) - 1, 2)]
        if len(layer) % 2:
            nxt.append(layer[-1])
        layer = nxt
    return layer[0]


def nzcv_flags(c: Circuit, result: list, carry: int | None = None, a_msb: int | None = None,
               b_msb: int | None = None) -> list:
    """Conditional flags of Sec. 6.1, as wires [N, Z, C, V]: N = the result's
    MSB (a copy); Z = NOT of the OR reduction of the result; C = the adder's
    carry-out (constant 0 when there is none); V = (NOT a . NOT b . s) +
    (a . b . NOT s) on the sign bits of the adder's two operands and of the
    result (constant 0 without operands). Z and V are the bootstrapped part,
    evaluated side by side."""
    W = len(result)
    s = result[W - 1]
    n_flag = s
    z_flag = c.NOT(or_reduce(c, result))
    c_flag = carry if carry is not None else c.const(0)
    if a_msb is None:
        v_flag = c.const(0)
    else:
        both_clear = c.gate(NOR, a_msb, b_msb)
        both_set = c.gate(AND, a_msb, b_msb)
        v_flag = c.gate(OR, c.gate(AND, both_clear, s), c.gate(ANDYN, both_set, s))
    return [n_flag, z_flag, c_flag, v_flag]


def adder_instance(width: int, prefix: str = PREFIX_GATES):
    """A standalone W-bit ADD circuit: inputs a[0..W), b[0..W); output 'sum'."""
    c = Circuit()
    A = c.inputs_word(width)
    B = c.inputs_word(width)
    s, _ = kogge_stone_add(c, A, B, prefix=prefix)
    c.outputs["sum"] = s
    return c


def sub_instance(width: int, prefix: str = PREFIX_GATES):
    c = Circuit()
    A = c.inputs_word(width)
    B = c.inputs_word(width)
    s, _ = subtract(c, A, B, prefix)
    c.outputs["diff"] = s
    return c


def int_to_bits(v: int, width: int) -> list:
    return [(int(v) >> i) & 1 for i in range(width)]


def bits_to_int(bits) -> int:
    return int(sum(int(b) << i for i, b in enumerate(bits)))


# ------------------------------------------------------------------ scheduler
@dataclass
class Level:
    ops: np.ndarray     # uint8 [G]
    ia: np.ndarray      # int32 [G] pool rows
    ib: np.ndarray
    io: np.ndarray
    nots: tuple         # (src rows, dst rows) executed before the level's gates
    mux: tuple = (np.zeros(0, np.int32),) * 4   # (selector, a, b, out) rows [M]

    @property
    def num_muxes(self) -> int:
        return int(self.mux[0].shape[0])


def pack_levels(circuits: list, round_size: int) -> list:
    """Level assignment for a merged program that fills whole launch rounds.

    Every bootstrapped node (gate: one blind rotation, MUX: two) keeps its
    circuit's level as the earliest it may run and gets a latest level from
    the program's depth D (the depth does not grow). Levels are then filled
    in order: the nodes whose latest level has come must run; the other ready
    nodes, most urgent first, join them until the level's blind rotations
    reach the next multiple of ``round_size`` (one full round of the
    throughput kernel: every workgroup busy), or one round when nothing is
    due. NOT runs at its input's level, inputs and constants at 0. Returns
    one level list per circuit, in the form of ``Circuit.lv``."""
    boot_kinds = ("gate", "mux")
    depth = max((c.depth() for c in circuits), default=0)
    # global ids of bootstrapped nodes; a wire's producer is the bootstrapped
    # node behind it (through NOTs), or -1 for inputs and constants
    gid, lo, hi, cost, preds = [], [], [], [], []
    producer = []
    for c in circuits:
        prod = [-1] * len(c.nodes)
        bound = [depth] * len(c.nodes)
        ids = [-1] * len(c.nodes)
        for w, (kind, op, a, b) in enumerate(c.nodes):
            if kind == "not":
                prod[w] = prod[a]
            elif kind in boot_kinds:
                ids[w] = len(lo)
                prod[w] = ids[w]
                lo.append(c.lv[w])
                hi.append(depth)
                cost.append(1 if kind == "gate" else 2)
                ins = (op, a, b) if kind == "mux" else (a, b)
                preds.append([prod[x] for x in ins])
        # latest levels, in reverse topological order (nodes are stored in
        # creation order, inputs before their consumers)
        for w in range(len(c.nodes) - 1, -1, -1):
            kind, op, a, b = c.nodes[w]
            if kind in boot_kinds:
                h = bound[w]
                hi[ids[w]] = h
                for x in ((op, a, b) if kind == "mux" else (a, b)):
                    bound[x] = min(bound[x], h - 1)
            elif kind == "not":
                bound[a] = min(bound[a], bound[w])
        gid.append(ids)
        producer.append(prod)
    nb = len(lo)
    lo = np.asarray(lo, np.int64)
    hi = np.asarray(hi, np.int64)
    cost = np.asarray(cost, np.int64)
    pm = np.full((nb, 3), -1, np.int64)
    for i, ps in enumerate(preds):
        pm[i, :len(ps)] = ps
    lev = np.zeros(nb + 1, np.int64)          # lev[-1] (no producer) stays 0
    for L in range(1, depth + 1):
        pl = lev[pm]                            # levels of the producers (0: unscheduled or none)
        done = (pl < L) & ((pl > 0) | (pm < 0))
        ready = (lev[:nb] == 0) & (lo <= L) & done.all(axis=1)
        due = ready & (hi == L)
        m = int(cost[due].sum())
        cap = round_size * max(1, -(-m // round_size))
        take = due.copy()
        opt = np.flatnonzero(ready & ~due)
        if opt.size and m < cap:
            opt = opt[np.argsort(hi[opt], kind="stable")]
            room = cap - m
            csum = np.cumsum(cost[opt])
            take[opt[csum <= room]] = True
        lev[:nb][take] = L
    assert nb == 0 or lev[:nb].min() >= 1, "every bootstrapped node gets a level"
    out = []
    for c, ids, prod in zip(circuits, gid, producer):
        lv = [0] * len(c.nodes)
        for w, (kind, op, a, b) in enumerate(c.nodes):
            if kind in boot_kinds:
                lv[w] = int(lev[ids[w]])
            elif kind == "not":
                lv[w] = lv[a]
        out.append(lv)
    return out


class Program:
    """Many circuit instances merged level by level into batched launches.

    Pool layout: every wire of every instance gets one row of a device
    ciphertext pool [rows][n+1]; instance k's wire w is row offset[k] + w.
    With ``pack`` (blind rotations per full launch round) the levels are
    reassigned by :func:`pack_levels`; otherwise each node keeps its
    circuit's level.
    """

    def __init__(self, circuits: list, pack: int | None = None):
        self.circuits = circuits
        self.offsets = np.cumsum([0] + [len(c.nodes) for c in circuits])
        self.rows = int(self.offsets[-1])
        lvs = pack_levels(circuits, pack) if pack else [c.lv for c in circuits]
        per_level = {}
        per_level_mux = {}
        nots = {}
        consts = ([], [])
        for k, c in enumerate(circuits):
            off = int(self.offsets[k])
            for w, (kind, op, a, b) in enumerate(c.nodes):
                L = lvs[k][w]
                if kind == "gate":
                    per_level.setdefault(L, []).append((op, off + a, off + b, off + w))
                elif kind == "mux":
                    per_level_mux.setdefault(L, []).append((off + op, off + a, off + b, off + w))
                elif kind == "not":
                    nots.setdefault(L, []).append((off + a, off + w))
                elif kind == "const":
                    consts[0].append(op)
                    consts[1].append(off + w)
        depth = max(list(per_level) + list(per_level_mux), default=0)
        self.levels = []
        for L in range(1, depth + 1):
            arr = np.array(per_level.get(L, []), dtype=np.int64).reshape(-1, 4)
            mx = np.array(per_level_mux.get(L, []), dtype=np.int64).reshape(-1, 4).astype(np.int32)
            na = np.array(nots.get(L - 1, []), dtype=np.int64).reshape(-1, 2)
            self.levels.append(Level(arr[:, 0].astype(np.uint8), arr[:, 1].astype(np.int32),
                                     arr[:, 2].astype(np.int32), arr[:, 3].astype(np.int32),
                                     (na[:, 0].astype(np.int32), na[:, 1].astype(np.int32)),
                                     (mx[:, 0].copy(), mx[:, 1].copy(), mx[:, 2].copy(), mx[:, 3].copy())))
        # NOTs of the last level's outputs run after the last launch
        tail = np.array(nots.get(depth, []), dtype=np.int64).reshape(-1, 2)
        self.tail_nots = (tail[:, 0].astype(np.int32), tail[:, 1].astype(np.int32))
        self.consts = (np.array(consts[0], np.uint8), np.array(consts[1], np.int32))
        self.input_rows = np.concatenate([np.array(c.inputs, np.int64) + int(self.offsets[k])
                                          for k, c in enumerate(circuits)]).astype(np.int32)
        self._dev = None
        self._graph = None

    @property
    def depth(self) -> int:
        return len(self.levels)

    def level_widths(self) -> list:
        """Bootstrapped binary gates per level."""
        return [int(L.ops.shape[0]) for L in self.levels]

    def level_mux_counts(self) -> list:
        return [L.num_muxes for L in self.levels]

    def num_gates(self) -> int:
        return int(sum(self.level_widths()))

    def num_muxes(self) -> int:
        return int(sum(self.level_mux_counts()))

    def num_bootstraps(self) -> int:
        """Blind rotations per run: one per gate, two per MUX."""
        return self.num_gates() + 2 * self.num_muxes()

    # ------------------------------------------------------------ device side
    def to_device(self, device):
        import torch

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)

        self._dev = {
            "levels": [(t(L.ops), t(L.ia), t(L.ib), t(L.io), t(L.nots[0]), t(L.nots[1])) for L in self.levels],
            "mux": [tuple(t(x) for x in L.mux) for L in self.levels],
            # output rows of a level holding both gates and MUXes: gates first
            "level_io": [t(np.concatenate([L.io, L.mux[3]])) if L.io.shape[0] and L.num_muxes else None
                         for L in self.levels],
            "tail": (t(self.tail_nots[0]), t(self.tail_nots[1])),
            "consts": (t(self.consts[0]), t(self.consts[1])),
        }
        return self

    def run(self, keys, pool, form="fft64", stream=None, profile_levels=None, tuner=None):
        """Enqueue the whole program on `stream`: constants, then per level the
        NOTs it needs and one batched launch of the level's gates and MUXes
        (gather/scatter in `pool`; a level holding both goes through
        cemu_bootstrap_level, so its blind rotations share one launch). With
        an autotuner, each launch's form and tiles are the tuner's choice for
        its number of blind rotations."""
        import torch
        if self._dev is None:
            self.to_device(pool.device)
        d = self._dev
        n = keys.n
        if d["consts"][1].shape[0]:
            cemu.lwe_constant(n, d["consts"][0], pool, d["consts"][1], stream=stream)
        for li, (ops, ia, ib, io, ns, nd) in enumerate(d["levels"]):
            if ns.shape[0]:
                cemu.lwe_not(n, pool, ns, pool, nd, stream=stream)
            ev = None
            if profile_levels is not None:
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                ev[0].record(stream)
            ms, ma, mb, mo = d["mux"][li]
            G, M = int(ops.shape[0]), int(ms.shape[0])
            f = tuner.apply(G + 2 * M) if (tuner is not None and G + M) else form
            if G and M:
                cemu.bootstrap_level(keys, pool, (ops, ia, ib), (ms, ma, mb), pool, io=d["level_io"][li], form=f,
                                     stream=stream)
            elif G:
                cemu.bootstrap_gates(keys, ops, pool, ia, ib, pool, io=io, form=f, stream=stream)
            elif M:
                cemu.mux(keys, pool, ms, ma, mb, pool, io=mo, form=f, stream=stream)
            if ev is not None:
                ev[1].record(stream)
                profile_levels.append(ev)
        if d["tail"][0].shape[0]:
            cemu.lwe_not(n, pool, d["tail"][0], pool, d["tail"][1], stream=stream)

    def capture(self, keys, pool, form="fft64", tuner=None):
        """Capture the level sequence as one hipGraph (after an eager run has
        sized the library's workspaces and, with a tuner, tuned every level
        width). Returns the torch graph object. The graph records the cloud
        key's workspace addresses, so it stays valid only until a call on the
        same key needs a larger batch than this program's widest level."""
        import torch
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(g, stream=stream):
                self.run(keys, pool, form=form, stream=torch.cuda.current_stream(), tuner=tuner)
        torch.cuda.synchronize()
        self._graph = g
        return g


def flag_setting_circuit(kind: str, width: int, prefix: str = PREFIX_GATES) -> Circuit:
    """ADDS / SUBS (and CMP, which is SUBS without a destination): outputs
    'out' (the W-bit result) and 'nzcv' (the four flags, Sec. 6.1). For
    SUBS, C = 1 means no borrow (a >= b unsigned) and V is taken on the
    adder's operands a and NOT b, as in the ARM definition."""
    c = Circuit()
    A = c.inputs_word(width)
    B = c.inputs_word(width)
    if kind == "ADDS":
        out, carry = kogge_stone_add(c, A, B, prefix=prefix)
        b_top = B[width - 1]
    elif kind in ("SUBS", "CMP"):
        out, carry = subtract(c, A, B, prefix)
        b_top = c.NOT(B[width - 1])
    else:
        raise ValueError(f"unknown flag-setting instruction {kind}")
    c.outputs["out"] = out
    c.outputs["nzcv"] = nzcv_flags(c, out, carry, A[width - 1], b_top)
    return c


def instruction_circuit(kind: str, width: int, prefix: str = PREFIX_GATES) -> Circuit:
    """One instruction as a circuit with inputs a, b (width bits each, LSB
    first) and output 'out'. Shifts (LLS / LRS / ARS) are register mode: b is
    the shift-amount register. prefix picks the adders' prefix form."""
    c = Circuit()
    A = c.inputs_word(width)
    B = c.inputs_word(width)
    if kind == "ADD":
        out, _ = kogge_stone_add(c, A, B, prefix=prefix)
    elif kind == "SUB":
        out, _ = subtract(c, A, B, prefix)
    elif kind == "MUL":
        out = array_multiply(c, A, B, prefix)
    elif kind == "LT":
        out = [less_than(c, A, B, prefix)]
    elif kind == "EQ":
        out = [equal(c, A, B)]
    elif kind in ("AND", "OR", "XOR"):
        out = bitwise(c, {"AND": AND, "OR": OR, "XOR": XOR}[kind], A, B)
    elif kind in (LLS, LRS, ARS):
        out = barrel_shift(c, A, B, kind)
    elif kind == "MULSEQ":
        out = sequential_multiply(c, A, B, signed=False, prefix=prefix)
    elif kind == "SMULSEQ":
        out = sequential_multiply(c, A, B, signed=True, prefix=prefix)
    elif kind == "DIV":
        out = nonrestoring_divide(c, A, B, prefix)
    elif kind == "ORN":
        out = bitwise(c, ORYN, A, B)
    else:
        raise ValueError(f"unknown instruction {kind}")
    c.outputs["out"] = out
    return c
