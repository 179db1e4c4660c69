"""Cleartext execution of the product's circuit DAGs and level schedules, for
the tests only. Gates take the oracle's truth tables (``oracle.circuits``),
so the product's circuit structure is checked against values that no product
code computes."""
import numpy as np

from oracle import circuits as OC


def eval_dag(c, in_bits) -> np.ndarray:
    """Every wire of a product ``Circuit`` on cleartext input bits."""
    it = iter(int(x) for x in in_bits)
    v = np.zeros(len(c.nodes), np.int64)
    for w, (kind, op, a, b) in enumerate(c.nodes):
        if kind == "in":
            v[w] = next(it)
        elif kind == "gate":
            v[w] = OC.gate_plain(op, v[a], v[b])
        elif kind == "mux":
            v[w] = v[a] if v[op] else v[b]
        elif kind == "not":
            v[w] = 1 - v[a]
        elif kind == "const":
            v[w] = op
        else:
            raise ValueError(kind)
    return v


def run_program_plain(prog, in_bits) -> np.ndarray:
    """Execute a product ``Program`` level by level on cleartext bits, in the
    order the device runs it (NOTs of level L-1, then level L's gates and
    MUXes, then the trailing NOTs). Returns every pool row's bit."""
    v = np.zeros(prog.rows, np.int64)
    v[prog.input_rows] = np.asarray(in_bits, np.int64)
    v[prog.consts[1]] = prog.consts[0]
    for L in prog.levels:
        src, dst = L.nots
        v[dst] = 1 - v[src]
        for op, a, b, o in zip(L.ops, L.ia, L.ib, L.io):
            v[o] = OC.gate_plain(int(op), v[a], v[b])
        ms, ma, mb, mo = L.mux
        v[mo] = np.where(v[ms] == 1, v[ma], v[mb])
    src, dst = prog.tail_nots
    v[dst] = 1 - v[src]
    return v
