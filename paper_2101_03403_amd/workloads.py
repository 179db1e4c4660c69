"""Seeded synthetic workloads shared by the tests, the benchmark and the
smoke check. Only random choices live here (gate types, plaintext bits,
operands, seeds); no arithmetic of the method.

The gate batch mirrors the throughput workload: independent bootstrapped
gates with the type uniform in {NAND, AND, OR, XOR} and uniform input bits.
"""
from __future__ import annotations

import numpy as np

NAND, AND, OR, XOR = 0, 1, 2, 3
THROUGHPUT_OPS = (NAND, AND, OR, XOR)

KEY_SEED = 0x2101_03403
ENC_SEED = 0xC0FFEE
TUNE_SEED = 0x7E57


def gate_batch(B: int, seed: int, ops=THROUGHPUT_OPS):
    """(ops uint8[B], a bits uint8[B], b bits uint8[B])."""
    rng = np.random.default_rng(seed)
    op = rng.choice(np.asarray(ops, dtype=np.uint8), size=B)
    a = rng.integers(0, 2, B, dtype=np.uint8)
    b = rng.integers(0, 2, B, dtype=np.uint8)
    return op, a, b


def all_gates_rows(reps: int = 1):
    """Every op code 0..9 with every input row (a, b) in {0,1}^2."""
    ops = np.repeat(np.arange(10, dtype=np.uint8), 4 * reps)
    a = np.tile(np.array([0, 1, 0, 1], np.uint8), 10 * reps)
    b = np.tile(np.array([0, 0, 1, 1], np.uint8), 10 * reps)
    return ops, a, b


def uint_operands(count: int, width: int, seed: int):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << width, count, dtype=np.uint64)


def sample_indices(B: int, k: int, seed: int):
    """k distinct gate indices covering the first and last tiles of a batch."""
    rng = np.random.default_rng(seed)
    fixed = [0, 1, 15, 16, B - 1]
    rest = rng.choice(B, size=max(0, k - len(fixed)), replace=False)
    idx = sorted(set([i for i in fixed if 0 <= i < B]) | set(int(x) for x in rest))
    return np.array(idx[:max(k, len(fixed))], dtype=np.int64)


# Mixed instruction stream: 40 % ADD/SUB, 20 % array MUL (8x8 or 16x16),
# 20 % compare (LT/EQ), 20 % bitwise AND/OR/XOR; widths 8/16/32 uniform
# (MUL 8 or 16), operands uniform at the width.
MIX_KINDS = ("ADD", "SUB", "MUL", "LT", "EQ", "AND", "OR", "XOR")


def instruction_mix(count: int, seed: int):
    """[(kind, width, a, b)] for `count` independent instructions."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        u = rng.random()
        if u < 0.4:
            kind = "ADD" if rng.random() < 0.5 else "SUB"
            width = int(rng.choice([8, 16, 32]))
        elif u < 0.6:
            kind = "MUL"
            width = int(rng.choice([8, 16]))
        elif u < 0.8:
            kind = "LT" if rng.random() < 0.5 else "EQ"
            width = int(rng.choice([8, 16, 32]))
        else:
            kind = str(rng.choice(["AND", "OR", "XOR"]))
            width = int(rng.choice([8, 16, 32]))
        a, b = (int(x) for x in rng.integers(0, 1 << width, 2, dtype=np.uint64))
        out.append((kind, width, a, b))
    return out
