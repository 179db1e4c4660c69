"""The allocation-free gate entry point against the allocating one.

cemu_bootstrap_gates_noalloc runs the same kernels as cemu_bootstrap_gates
with its workspace in the library's fixed device scratch array. Called
through the C ABI twice in a row -- the full 4096-gate maximum, then a
smaller batch with other inputs scattered to permuted rows -- its outputs
must equal cemu_bootstrap_gates's on the same inputs word for word, in both
product forms; a batch above the maximum is refused with a range error.
"""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2101_03403_amd import cemu, workloads as W  # noqa: E402

SEED = 20210108


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    say("[noalloc] keygen std")
    return cemu.keygen(cemu.STD, SEED), O.keygen(O.STANDARD, SEED), dev


def _inputs(ok, B, seed, dev):
    ops, a, b = W.gate_batch(B, seed=seed)
    c1 = O.encrypt_bits(ok, a, seed=seed + 1)
    c2 = O.encrypt_bits(ok, b, seed=seed + 1, first_index=B)
    pool = torch.from_numpy(np.concatenate([c1, c2]).view(np.int32)).to(dev)
    ops_t = torch.from_numpy(ops).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    return ops_t, pool, ia, ia + B


@pytest.mark.parametrize("form", ["int8", "fft64"])
def test_noalloc_equals_allocating_entry_point(setup, form):
    lk, ok, dev = setup
    f = cemu.FORMS[form]
    L = cemu.lib()
    n1 = lk.n + 1
    for call, (B, seed, scatter) in enumerate([(cemu.NOALLOC_MAX_GATES, 501, False), (37, 777, True)]):
        say(f"[noalloc] {form} call {call + 1}: B = {B}")
        ops, pool, ia, ib = _inputs(ok, B, seed, dev)
        rows = B + 5
        io = None
        if scatter:
            io = torch.from_numpy(np.random.default_rng(seed).permutation(rows)[:B].astype(np.int32)).to(dev)
        got = torch.zeros((rows, n1), dtype=torch.int32, device=dev)
        want = torch.zeros_like(got)
        rc = L.cemu_bootstrap_gates_noalloc(lk.ck, f, vp(ops), vp(pool), vp(ia), vp(ib), vp(io), vp(got),
                                            C.c_int64(B), None)
        assert rc == 0, cemu.lib().cemu_last_error().decode()
        rc = L.cemu_bootstrap_gates(lk.ck, f, vp(ops), vp(pool), vp(ia), vp(ib), vp(io), vp(want), C.c_int64(B), None)
        assert rc == 0, cemu.lib().cemu_last_error().decode()
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        say(f"[noalloc] {form} call {call + 1}: differing words {int(np.sum(g != w))}/{w.size}")
        assert np.array_equal(g, w)
        out_rows = io.cpu().numpy() if io is not None else np.arange(B)
        bits = lk.decrypt(g[out_rows].view(np.uint32))
        _, a, b = W.gate_batch(B, seed=seed)
        opsh = ops.cpu().numpy()
        truth = np.select([opsh == 0, opsh == 1, opsh == 2, opsh == 3], [1 - (a & b), a & b, a | b, a ^ b])
        assert np.array_equal(bits, truth)


def test_noalloc_refuses_batches_beyond_its_scratch(setup):
    lk, ok, dev = setup
    B = cemu.NOALLOC_MAX_GATES + 1
    ops, pool, ia, ib = _inputs(ok, 8, 11, dev)
    out = torch.zeros((8, lk.n + 1), dtype=torch.int32, device=dev)
    rc = cemu.lib().cemu_bootstrap_gates_noalloc(lk.ck, 0, vp(ops), vp(pool), vp(ia), vp(ib), None, vp(out),
                                                 C.c_int64(B), None)
    assert rc == -8
    assert "scratch" in cemu.lib().cemu_last_error().decode()
    assert cemu.lib().cemu_bootstrap_gates_noalloc(lk.ck, 0, None, None, None, None, None, None, 0, None) == 0
