"""Run a merged circuit schedule on the CPU oracle (test helper).

The GPU runs a program as one pool of ciphertext rows and one batched launch
per level. To check it gate for gate without ever giving the oracle a
ciphertext the GPU produced, the same schedule is replayed on a host pool
with the oracle's gates: the pool starts from the oracle's own encryptions of
the input bits, and every level reads only what earlier oracle levels wrote.
Only the rows of the chosen instances are evaluated, so a few instances of a
wide program stay cheap. The schedule (which gate reads which rows) is the
product's; the ciphertext arithmetic is entirely the oracle's, and the
circuits themselves are checked separately against the oracle's netlists and
integer results.
"""
from __future__ import annotations

import sys

import numpy as np

from oracle import circuits as OC
from oracle import oracle as O


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def instance_rows(prog, instances) -> np.ndarray:
    """Boolean mask over pool rows of the given instance indices."""
    mask = np.zeros(prog.rows, bool)
    for k in instances:
        mask[int(prog.offsets[k]):int(prog.offsets[k + 1])] = True
    return mask


def oracle_pool(okeys, prog, bits, seed) -> np.ndarray:
    """Host pool [rows][n+1] holding the oracle's encryptions of the input
    bits at the program's input rows (every other row zero)."""
    n = okeys.params.n
    pool = np.zeros((prog.rows, n + 1), np.uint32)
    pool[prog.input_rows] = O.encrypt_bits(okeys, np.asarray(bits, np.uint8), seed=seed)
    return pool


def run_on_oracle(okeys, prog, pool, instances, label="") -> np.ndarray:
    """Replay prog's levels for the rows of `instances` with the oracle's
    gates, MUX, NOT and CONSTANT; returns the updated copy of `pool`."""
    pool = pool.copy()
    n = okeys.params.n
    mask = instance_rows(prog, instances)
    for bit, row in zip(*prog.consts):
        if mask[row]:
            pool[row] = OC.lwe_constant(int(bit), n)
    for li, L in enumerate(prog.levels):
        src, dst = L.nots
        sel = mask[dst]
        pool[dst[sel]] = OC.lwe_not(pool[src[sel]])
        g = np.flatnonzero(mask[L.io])
        if g.size:
            _, out = O.bootstrap_batch(okeys, L.ops[g].astype(np.int32), pool[L.ia[g]], pool[L.ib[g]],
                                       want_extracted=False)
        ms, ma, mb, mo = L.mux
        m = np.flatnonzero(mask[mo])
        if m.size:
            mux_out = O.mux_batch(okeys, pool[ms[m]], pool[ma[m]], pool[mb[m]])
        # a level's outputs are never its own inputs: write after reading
        if g.size:
            pool[L.io[g]] = out
        if m.size:
            pool[mo[m]] = mux_out
        if label and (li % 4 == 3 or li == len(prog.levels) - 1):
            _say(f"[oracle] {label}: level {li + 1}/{len(prog.levels)} done")
    src, dst = prog.tail_nots
    sel = mask[dst]
    pool[dst[sel]] = OC.lwe_not(pool[src[sel]])
    return pool


def bootstrapped_rows(prog, instances) -> np.ndarray:
    """Pool rows written by a gate or MUX of the given instances."""
    mask = instance_rows(prog, instances)
    rows = []
    for L in prog.levels:
        rows.append(L.io[mask[L.io]])
        rows.append(L.mux[3][mask[L.mux[3]]])
    return np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
