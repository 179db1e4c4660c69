"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Keys are generated independently on both sides from the same seed (library
host code vs. oracle, each implementing Philox4x32-10 and Box-Muller), so the
first tests check key and encryption parity bit for bit. The int8-MFMA form
must then give bit-identical extracted samples and key-switched outputs.
"""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import circuits as OC  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2101_03403_amd import cemu, workloads as W  # noqa: E402

import oracle_program as OP  # noqa: E402  (tests/ helper)

SEED = 20210108


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def toy(dev):
    say("[gpu] keygen toy (library + oracle)")
    return cemu.keygen(cemu.TOY, SEED), O.keygen(O.TOY, SEED)


@pytest.fixture(scope="module")
def std(dev):
    say("[gpu] keygen std (library + oracle)")
    return cemu.keygen(cemu.STD, SEED), O.keygen(O.STANDARD, SEED)


def to_dev(a, dev):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(dev)


def to_host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def run_gates(keys, ops, c1, c2, dev, form="int8", want_ext=True):
    """Pool = [c1; c2]; gate g reads rows g and B+g. Returns (ext, out)."""
    B = ops.shape[0]
    pool = to_dev(np.concatenate([c1, c2]), dev)
    ops_t = torch.from_numpy(np.ascontiguousarray(ops.astype(np.uint8))).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    ib = ia + B
    out = torch.zeros((B, keys.n + 1), dtype=torch.int32, device=dev)
    ext = None
    if want_ext:
        ext = torch.zeros((B, keys.N + 1), dtype=torch.int32, device=dev)
        cemu.blind_rotate_extract(keys, ops_t, pool, ia, ib, ext, form=form)
    cemu.bootstrap_gates(keys, ops_t, pool, ia, ib, out, form=form)
    torch.cuda.synchronize()
    return (to_host_u32(ext) if want_ext else None), to_host_u32(out)


def test_keys_match_oracle_toy(toy):
    lk, ok = toy
    ex = lk.export()
    assert np.array_equal(ex["lwe_key"], ok.lwe_key)
    assert np.array_equal(ex["tlwe_key"], ok.tlwe_key)
    assert np.array_equal(ex["bk"], ok.bk)
    assert np.array_equal(ex["ksk"], ok.ksk)


def test_keys_match_oracle_std(std):
    lk, ok = std
    ex = lk.export()
    assert np.array_equal(ex["lwe_key"], ok.lwe_key)
    assert np.array_equal(ex["tlwe_key"], ok.tlwe_key)
    assert np.array_equal(ex["bk"], ok.bk)
    assert np.array_equal(ex["ksk"], ok.ksk)


def test_encrypt_matches_oracle(toy):
    lk, ok = toy
    rng = np.random.default_rng(1)
    bits = rng.integers(0, 2, 100).astype(np.uint8)
    a = lk.encrypt(bits, seed=5, first_index=1000)
    b = O.encrypt_bits(ok, bits, seed=5, first_index=1000)
    assert np.array_equal(a, b)
    assert np.array_equal(lk.decrypt(a), bits)


def test_toy_eight_nand_bit_exact(toy, dev):
    """Toy parameters, 8 independent NAND gates on uniform random bits."""
    lk, ok = toy
    say("[gpu] toy 8 NAND")
    ops, a, b = W.gate_batch(8, seed=11, ops=(W.NAND,))
    c1 = O.encrypt_bits(ok, a, seed=21)
    c2 = O.encrypt_bits(ok, b, seed=21, first_index=8)
    ext, out = run_gates(lk, ops, c1, c2, dev)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert np.array_equal(ext, oext)
    assert np.array_equal(out, oout)
    assert np.array_equal(lk.decrypt(out), (~(a & b)) & 1)


def test_toy_all_gates_ragged_bit_exact(toy, dev):
    """All ten gates x four input rows, plus a ragged tail (B = 43)."""
    lk, ok = toy
    say("[gpu] toy all gates ragged")
    ops, a, b = W.all_gates_rows()
    ops = np.concatenate([ops, ops[:3]])
    a = np.concatenate([a, a[:3]])
    b = np.concatenate([b, b[:3]])
    c1 = O.encrypt_bits(ok, a, seed=31)
    c2 = O.encrypt_bits(ok, b, seed=32)
    ext, out = run_gates(lk, ops, c1, c2, dev)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert np.array_equal(ext, oext)
    assert np.array_equal(out, oout)
    truth = [lambda x, y: 1 - (x & y), lambda x, y: x & y, lambda x, y: x | y, lambda x, y: x ^ y,
             lambda x, y: 1 - (x ^ y), lambda x, y: 1 - (x | y), lambda x, y: (1 - x) & y,
             lambda x, y: x & (1 - y), lambda x, y: (1 - x) | y, lambda x, y: x | (1 - y)]
    want = np.array([truth[o](int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    assert np.array_equal(lk.decrypt(out), want)


def test_int8_latency_kernel_toy_bit_exact(toy, dev):
    """The one-gate-per-workgroup int8 kernel (key limbs in the MFMA columns,
    the gate's digit Toeplitz matrix as the other operand) against the exact
    oracle: all ten gates x four input rows plus a ragged tail, both wave
    counts; an empty batch and a single gate."""
    lk, ok = toy
    ops, a, b = W.all_gates_rows()
    ops = np.concatenate([ops, ops[:3]])
    a = np.concatenate([a, a[:3]])
    b = np.concatenate([b, b[:3]])
    c1 = O.encrypt_bits(ok, a, seed=61)
    c2 = O.encrypt_bits(ok, b, seed=62)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    saved = cemu.get_tuning(lk)
    try:
        for waves in (8, 4):
            say(f"[gpu] toy int8 latency kernel, {waves} waves, B = {len(ops)}")
            cemu.set_tuning(lk, int8_waves=waves, int8_gates_per_wg=1)
            ext, out = run_gates(lk, ops, c1, c2, dev, form="int8")
            assert np.array_equal(ext, oext)
            assert np.array_equal(out, oout)
            ext1, out1 = run_gates(lk, ops[:1], c1[:1], c2[:1], dev, form="int8")
            assert np.array_equal(ext1, oext[:1]) and np.array_equal(out1, oout[:1])
            ext0, out0 = run_gates(lk, ops[:0], c1[:0], c2[:0], dev, form="int8")
            assert ext0.shape[0] == 0 and out0.shape[0] == 0
    finally:
        cemu.set_tuning(lk, **saved)


def test_int8_latency_kernel_std_rounds_and_mux(std, dev):
    """Standard parameters: the one-gate-per-workgroup int8 kernel on a batch
    of 300 gates (more workgroups than one per compute unit, so they run in
    rounds) and on a MUX level (two blind rotations per MUX) equals the
    16-gate int8 kernel word for word; decryptions exact; sampled gates and
    every MUX bit-exact against the oracle (all 4096 gates of the benchmark
    batch are compared in test_gpu_full_parity)."""
    lk, ok = std
    B = 300
    ops, a, b = W.gate_batch(B, seed=71)
    c1 = O.encrypt_bits(ok, a, seed=72)
    c2 = O.encrypt_bits(ok, b, seed=72, first_index=B)
    bits, cts = _mux_inputs(ok, 40, 73)
    saved = cemu.get_tuning(lk)
    res = {}
    try:
        for shape in (16, 1):
            say(f"[gpu] std int8, {shape} gate(s) per workgroup, B = {B} gates + 40 MUXes")
            cemu.set_tuning(lk, int8_waves=8, int8_gates_per_wg=shape)
            res[shape] = (run_gates(lk, ops, c1, c2, dev, form="int8"), _run_mux(lk, cts, dev, "int8"))
    finally:
        cemu.set_tuning(lk, **saved)
    (ext16, out16), mux16 = res[16]
    (ext1, out1), mux1 = res[1]
    assert np.array_equal(ext1, ext16) and np.array_equal(out1, out16) and np.array_equal(mux1, mux16)
    truth = {0: lambda x, y: 1 - (x & y), 1: lambda x, y: x & y, 2: lambda x, y: x | y, 3: lambda x, y: x ^ y}
    want = np.array([truth[int(o)](int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    assert np.array_equal(lk.decrypt(out1), want)
    assert np.array_equal(lk.decrypt(mux1), np.where(bits[0] == 1, bits[1], bits[2]))
    idx = W.sample_indices(B, 4, seed=74)
    oext, oout = O.bootstrap_batch(ok, ops[idx].astype(np.int32), c1[idx], c2[idx])
    assert np.array_equal(ext1[idx], oext) and np.array_equal(out1[idx], oout)
    assert np.array_equal(mux1, O.mux_batch(ok, cts[0], cts[1], cts[2]))   # all 40 MUXes


@pytest.mark.parametrize("B", [1, 37, 300, 1600, 4096])
def test_key_switch_alone(std, dev, B):
    """Key switching alone, bit-exact against the oracle, across the launch
    shapes: the K range split over 32 (B = 1, 37, 300), 8 (1600) and 2
    (4096) workgroups per tile with integer-atomic sums. The unsplit launch
    (B >= 6529) is covered at B = 8192 in test_gpu_full_parity."""
    lk, ok = std
    say(f"[gpu] key switch B={B}")
    rng = np.random.default_rng(7 + B)
    ins = rng.integers(0, 1 << 32, (B, lk.N + 1), dtype=np.uint64).astype(np.uint32)
    din = to_dev(ins, dev)
    dout = torch.zeros((B, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.key_switch(lk, din, dout)
    torch.cuda.synchronize()
    assert np.array_equal(to_host_u32(dout), O.key_switch_batch(ok, ins))


def test_gather_scatter_pool(toy, dev):
    """Gates read arbitrary pool rows and write to arbitrary output rows."""
    lk, ok = toy
    rng = np.random.default_rng(8)
    P = 20
    bits = rng.integers(0, 2, P).astype(np.uint8)
    pool = O.encrypt_bits(ok, bits, seed=9)
    B = 17
    ia = rng.integers(0, P, B).astype(np.int32)
    ib = rng.integers(0, P, B).astype(np.int32)
    io = rng.permutation(40)[:B].astype(np.int32)
    ops = rng.integers(0, 10, B).astype(np.uint8)
    dpool = to_dev(pool, dev)
    dout = torch.zeros((40, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.bootstrap_gates(lk, torch.from_numpy(ops).to(dev), dpool, torch.from_numpy(ia).to(dev),
                         torch.from_numpy(ib).to(dev), dout, io=torch.from_numpy(io).to(dev))
    torch.cuda.synchronize()
    out = to_host_u32(dout)
    _, oout = O.bootstrap_batch(ok, ops.astype(np.int32), pool[ia], pool[ib], want_extracted=False)
    assert np.array_equal(out[io], oout)


def test_empty_and_single(toy, dev):
    lk, ok = toy
    z = torch.zeros(0, dtype=torch.int32, device=dev)
    cemu.bootstrap_gates(lk, torch.zeros(0, dtype=torch.uint8, device=dev), z, z, z,
                         torch.zeros((0, lk.n + 1), dtype=torch.int32, device=dev))
    ops = np.array([cemu.XOR], np.uint8)
    c1 = O.encrypt_bits(ok, [1], seed=3)
    c2 = O.encrypt_bits(ok, [1], seed=4)
    ext, out = run_gates(lk, ops, c1, c2, dev)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert np.array_equal(out, oout)
    assert lk.decrypt(out)[0] == 0


def test_not_copy_constant(toy, dev):
    lk, ok = toy
    bits = np.array([0, 1, 1, 0], np.uint8)
    c = O.encrypt_bits(ok, bits, seed=13)
    dpool = to_dev(c, dev)
    idx = torch.arange(4, dtype=torch.int32, device=dev)
    dnot = torch.zeros_like(dpool)
    cemu.lwe_not(lk.n, dpool, idx, dnot, idx)
    dcopy = torch.zeros_like(dpool)
    cemu.lwe_copy(lk.n, dpool, idx, dcopy, idx.flip(0).contiguous())
    dconst = torch.zeros_like(dpool)
    cemu.lwe_constant(lk.n, torch.tensor([1, 0, 1, 1], dtype=torch.uint8, device=dev), dconst, idx)
    torch.cuda.synchronize()
    assert np.array_equal(lk.decrypt(to_host_u32(dnot)), 1 - bits)
    assert np.array_equal(to_host_u32(dcopy), c[::-1])
    assert np.array_equal(lk.decrypt(to_host_u32(dconst)), [1, 0, 1, 1])
    assert np.array_equal(to_host_u32(dnot), (0 - c.astype(np.uint64)).astype(np.uint32))


def test_errors_are_reported(toy, dev):
    lk, ok = toy
    z = torch.zeros(4, dtype=torch.int32, device=dev)
    # the FFT64 form is built for N = 1024 only: the toy set (N = 512) is refused
    ops = torch.zeros(2, dtype=torch.uint8, device=dev)
    pool = torch.zeros((2, lk.n + 1), dtype=torch.int32, device=dev)
    rows = torch.arange(2, dtype=torch.int32, device=dev)
    with pytest.raises(cemu.CemuError) as exc:
        cemu.bootstrap_gates(lk, ops, pool, rows, rows, pool, form="fft64")
    assert exc.value.code == -6            # CEMU_ERR_UNSUPPORTED
    with pytest.raises(cemu.CemuError):
        cemu._check(cemu.lib().cemu_bootstrap_gates(lk.ck, 7, None, None, None, None, None, None, 4, None))
    with pytest.raises(cemu.CemuError):
        cemu._check(cemu.lib().cemu_bootstrap_gates(lk.ck, 0, None, C.c_void_p(z.data_ptr()), None, None, None,
                                                     None, 4, None))


def to_i32(x):
    x = np.asarray(x, dtype=np.uint32)
    return x.astype(np.int64) - ((x >> 31).astype(np.int64) << 32)


@pytest.mark.parametrize("B,fg", [(37, 8), (512, 8), (4096, 8), (37, 1), (300, 1)])
def test_fft_form_decrypts_and_phase_error(std, dev, B, fg):
    """FP64-FFT form (fg = gates per workgroup; 1 is the latency kernel):
    every decryption exact; extracted samples compared with the oracle on
    sampled gates (raw words and decrypted phase). B = 4096 at 8 gates per
    workgroup is the benchmark's batch in its launch shape (two full rounds)."""
    lk, ok = std
    say(f"[gpu] fft64 form B={B} fft_gates_per_wg={fg}")
    ops, a, b = W.gate_batch(B, seed=51 + B)
    c1 = O.encrypt_bits(ok, a, seed=61)
    c2 = O.encrypt_bits(ok, b, seed=61, first_index=B)
    saved = cemu.get_tuning(lk)
    try:
        cemu.set_tuning(lk, fft_gates_per_wg=fg)
        ext, out = run_gates(lk, ops, c1, c2, dev, form="fft64")
    finally:
        cemu.set_tuning(lk, **saved)
    truth = {0: lambda x, y: 1 - (x & y), 1: lambda x, y: x & y, 2: lambda x, y: x | y, 3: lambda x, y: x ^ y}
    want = np.array([truth[int(o)](int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    assert np.array_equal(lk.decrypt(out), want)
    assert np.array_equal(lk.decrypt_extracted(ext), want)
    idx = W.sample_indices(B, 8, seed=B)
    oext, _ = O.bootstrap_batch(ok, ops[idx].astype(np.int32), c1[idx], c2[idx], want_out=False)
    perr = to_i32(lk.phase(ext[idx], extracted=True).astype(np.int64) - lk.phase(oext, extracted=True).astype(np.int64))
    words_diff = int(np.sum(ext[idx] != oext))
    werr = np.abs(to_i32(ext[idx].astype(np.int64) - oext.astype(np.int64))).max()
    say(f"[gpu] fft64 vs oracle: max |phase error| = {np.abs(perr).max()}, differing words = {words_diff}"
        f"/{oext.size}, max |word error| = {werr}")
    # every product is an integer polynomial rounded from double precision:
    # while the transform error stays below one half, the extracted samples
    # are the exact ones
    assert words_diff == 0


def _program_pool(prog, ok, bits, dev, seed=77):
    """Device pool holding the oracle's encryptions of the input bits, and
    its host copy (the starting pool of the oracle's replay)."""
    host0 = OP.oracle_pool(ok, prog, bits, seed)
    return to_dev(host0, dev), host0


def _check_against_oracle_replay(ok, prog, host0, host, instances, label, min_per_level=0):
    """Replay the given instances on the oracle from the same encrypted
    inputs (no GPU ciphertext enters the oracle) and require every row they
    write to equal the GPU's word for word. Returns the per-level number of
    compared blind-rotated outputs."""
    want = OP.run_on_oracle(ok, prog, host0, instances, label=label)
    mask = OP.instance_rows(prog, instances)
    per_level = [int(mask[L.io].sum()) + int(mask[L.mux[3]].sum()) for L in prog.levels]
    for li, L in enumerate(prog.levels):
        width = int(L.io.shape[0]) + L.num_muxes
        assert per_level[li] >= min(min_per_level, width), (li, per_level[li], width)
    rows = np.flatnonzero(mask)
    diff = int(np.sum(host[rows] != want[rows]))
    say(f"[gpu] {label}: {int(sum(per_level))} bootstrapped outputs over {len(per_level)} levels "
        f"(min {min(per_level) if per_level else 0} per level) against the oracle replay, differing words {diff}")
    assert diff == 0
    return per_level


def test_program_add_sub_levels_and_graph(std, dev):
    """16 ADD32 + 16 SUB32 instances merged level by level (FFT64 form):
    decryptions equal uint32 arithmetic; two ADD and two SUB instances (at
    least 64 gates of every level) replayed on the oracle from the same
    encrypted inputs equal the GPU's pool word for word; a captured hipGraph
    replayed 3 times (outputs cleared eagerly in between) reproduces the
    eager pool exactly."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    rng = np.random.default_rng(123)
    cases = [("ADD" if i < 16 else "SUB", 32) + tuple(int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64))
             for i in range(32)]
    cs = [Cc.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = Cc.Program(cs).to_device(dev)
    bits = []
    for k, w, a, b in cases:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    say(f"[gpu] program: {prog.num_gates()} gates in {prog.depth} levels")
    pool, host0 = _program_pool(prog, ok, bits, dev)
    prog.run(lk, pool, form="fft64")
    torch.cuda.synchronize()
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b)
    _check_against_oracle_replay(ok, prog, host0, host, [0, 1, 16, 17], "ADD/SUB replay", min_per_level=64)
    # graph capture and replay
    eager = host.copy()
    g = prog.capture(lk, pool, form="fft64")
    keep = torch.zeros(prog.rows, dtype=torch.bool, device=dev)
    keep[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = True
    for rep in range(3):
        pool[~keep] = 0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(pool), eager), f"graph replay {rep} differs"


def test_program_int8_form_small(std, dev):
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    cases = [("ADD", 8, 250, 9), ("SUB", 8, 3, 200), ("MUL", 8, 201, 77), ("EQ", 8, 5, 5), ("LT", 8, 6, 5),
             ("XOR", 8, 0x5A, 0xFF)]
    cs = [Cc.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = Cc.Program(cs).to_device(dev)
    bits = []
    for k, w, a, b in cases:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    pool, host0 = _program_pool(prog, ok, bits, dev)
    prog.run(lk, pool, form="int8")
    torch.cuda.synchronize()
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)
    _check_against_oracle_replay(ok, prog, host0, host, [1, 3, 4, 5], "small int8 program replay")


@pytest.mark.parametrize("prefix", ["gates", "mux"])
def test_packed_program_equals_earliest_level_schedule(toy, dev, prefix):
    """A mixed stream of 64 instructions with its levels refilled to whole
    rounds of 64 blind rotations (pack_levels) writes, word for word, the same
    ciphertext pool as the earliest-level schedule (a gate's bootstrap does
    not depend on the batch it runs in), and every instruction decrypts to
    its integer result (toy parameters, int8 form)."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = toy
    mix = W.instruction_mix(64, seed=17)
    cs = [Cc.instruction_circuit(k, w, prefix=prefix) for k, w, _, _ in mix]
    bits = []
    for k, w, a, b in mix:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    pools = []
    for pack in (None, 64):
        prog = Cc.Program(cs, pack=pack).to_device(dev)
        say(f"[gpu] mixed {prefix} pack={pack}: {prog.depth} levels, widths {prog.level_widths()[:6]}...")
        pool, _ = _program_pool(prog, ok, bits, dev)
        prog.run(lk, pool, form="int8")
        torch.cuda.synchronize()
        pools.append(to_host_u32(pool))
    assert np.array_equal(pools[0], pools[1])
    for (k, w, a, b), c, off in zip(mix, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(pools[1][np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, w, a, b, got)


def test_mixed_stream_std_oracle_replay(std, dev):
    """A seeded mixed stream of 48 instructions (ADD/SUB, array MUL, LT/EQ,
    bitwise; widths 8/16/32) at standard parameters, merged level by level
    with the levels refilled to whole launch rounds (int8 form): every
    instruction decrypts to its integer result, and one instance of each
    kind (the narrowest available) replayed on the oracle from the same
    encrypted inputs equals the GPU's pool word for word."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    mix = W.instruction_mix(48, seed=29)
    cs = [Cc.instruction_circuit(k, w) for k, w, _, _ in mix]
    bits = []
    for k, w, a, b in mix:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    prog = Cc.Program(cs, pack=256).to_device(dev)
    say(f"[gpu] mixed std: {prog.num_gates()} gates in {prog.depth} levels")
    pool, host0 = _program_pool(prog, ok, bits, dev, seed=91)
    prog.run(lk, pool, form="int8")
    torch.cuda.synchronize()
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(mix, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, w, a, b, got)
    pick = {}
    for i, (k, w, _, _) in enumerate(mix):
        group = "BIT" if k in ("AND", "OR", "XOR") else k
        if group not in pick or w < mix[pick[group]][1]:
            pick[group] = i
    say(f"[gpu] mixed std: replaying {sorted((mix[i][0], mix[i][1]) for i in pick.values())}")
    _check_against_oracle_replay(ok, prog, host0, host, sorted(pick.values()), "mixed-stream replay")


def test_tuning_variants_give_identical_results(std, dev):
    """Every launch configuration the autotuner may pick computes the same
    ciphertexts (ragged batch of 45 gates). The FFT64 latency kernel sums in
    another order; it agrees because the form's error stays below half a
    unit, so every product rounds to the exact integer (checked against the
    oracle below)."""
    lk, ok = std
    B = 45
    ops, a, b = W.gate_batch(B, seed=91)
    c1 = O.encrypt_bits(ok, a, seed=92)
    c2 = O.encrypt_bits(ok, b, seed=92, first_index=B)
    ref = None
    saved = cemu.get_tuning(lk)
    try:
        for form, tun in [("fft64", {"fft_gates_per_wg": 8}), ("fft64", {"fft_gates_per_wg": 4}),
                          ("fft64", {"fft_gates_per_wg": 1}),
                          ("int8", {"int8_waves": 8, "int8_gates_per_wg": 16}),
                          ("int8", {"int8_waves": 4, "int8_gates_per_wg": 16}),
                          ("int8", {"int8_waves": 8, "int8_gates_per_wg": 1}),
                          ("int8", {"int8_waves": 4, "int8_gates_per_wg": 1})]:
            say(f"[gpu] tuning variant {form} {tun}")
            cemu.set_tuning(lk, **tun)
            ext, out = run_gates(lk, ops, c1, c2, dev, form=form)
            if ref is None:
                ref = (ext, out)
            assert np.array_equal(ext, ref[0]) and np.array_equal(out, ref[1]), (form, tun)
        with pytest.raises(cemu.CemuError):
            cemu.set_tuning(lk, int8_waves=6)
        with pytest.raises(cemu.CemuError):
            cemu.set_tuning(lk, fft_gates_per_wg=2)
        with pytest.raises(cemu.CemuError):
            cemu.set_tuning(lk, int8_gates_per_wg=2)
    finally:
        cemu.set_tuning(lk, **saved)
    oext, _ = O.bootstrap_batch(ok, ops[:4].astype(np.int32), c1[:4], c2[:4], want_out=False)
    assert np.array_equal(ref[0][:4], oext)


def test_autotuner_picks_and_caches(std, dev, tmp_path):
    from paper_2101_03403_amd.autotune import CANDIDATES, Autotuner, bucket
    lk, ok = std
    path = str(tmp_path / "tune.json")
    t = Autotuner(lk, cache_path=path, reps=1)
    form, tun = t.best(100)
    assert bucket(100) == 128 and form in ("fft64", "int8")
    assert len(t.measurements[128]) == len(CANDIDATES)
    # restricted to one form, only that form's shapes are measured
    ti = Autotuner(lk, forms=("int8",), reps=1)
    assert ti.best(20)[0] == "int8"
    assert len(ti.measurements[32]) == sum(1 for f, _ in CANDIDATES if f == "int8")
    t2 = Autotuner(lk, cache_path=path)
    assert t2.best(120) == (form, tun)      # same bucket, from the file, no measuring
    assert t2.measurements == {}


# ------------------------------------------------------------------ multiplexer and shifters
def _mux_inputs(ok, B, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, (3, B)).astype(np.uint8)
    bits[:, :8] = np.array([[0, 0, 0, 0, 1, 1, 1, 1], [0, 0, 1, 1, 0, 0, 1, 1], [0, 1, 0, 1, 0, 1, 0, 1]])
    cts = [O.encrypt_bits(ok, bits[r], seed=seed + r) for r in range(3)]
    return bits, cts


def _run_mux(lk, cts, dev, form, io_perm=None):
    """Pool rows: selectors 0..B-1, a B..2B-1, b 2B..3B-1; outputs scattered
    to rows io_perm (or 0..B-1) of a separate pool."""
    B = cts[0].shape[0]
    pool = to_dev(np.concatenate(cts), dev)
    rows = torch.arange(B, dtype=torch.int32, device=dev)
    io = None if io_perm is None else torch.from_numpy(io_perm.astype(np.int32)).to(dev)
    out = torch.zeros((B if io_perm is None else int(io_perm.max()) + 1, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.mux(lk, pool, rows, rows + B, rows + 2 * B, out, io=io, form=form)
    torch.cuda.synchronize()
    host = to_host_u32(out)
    return host if io_perm is None else host[io_perm]


def test_mux_toy_bit_exact(toy, dev):
    """MUX (two bootstraps without key switching, sum + 1/8, one key switch)
    against the oracle's MUX, bit for bit, int8 form; all eight input rows
    plus random ones, ragged batch, outputs scattered to permuted rows."""
    lk, ok = toy
    B = 37
    say(f"[gpu] mux toy B={B}")
    bits, cts = _mux_inputs(ok, B, 71)
    perm = np.random.default_rng(3).permutation(B + 5)[:B]
    got = _run_mux(lk, cts, dev, "int8", io_perm=perm)
    want = O.mux_batch(ok, *cts)
    assert np.array_equal(got, want)
    assert np.array_equal(lk.decrypt(got), np.where(bits[0] == 1, bits[1], bits[2]))


@pytest.mark.parametrize("form", ["int8", "fft64"])
def test_mux_std(std, dev, form):
    """Standard parameters: decryptions exact; all 45 MUXes equal the
    oracle's word for word in both forms (the FFT64 products round to the
    exact integers)."""
    lk, ok = std
    B = 45
    say(f"[gpu] mux std {form} B={B}")
    bits, cts = _mux_inputs(ok, B, 81)
    got = _run_mux(lk, cts, dev, form)
    assert np.array_equal(lk.decrypt(got), np.where(bits[0] == 1, bits[1], bits[2]))
    want = O.mux_batch(ok, cts[0], cts[1], cts[2])
    diff = int(np.sum(got != want))
    say(f"[gpu] mux {form} vs oracle: differing words {diff}/{want.size}")
    assert diff == 0


def test_mux_empty_and_errors(toy, dev):
    lk, ok = toy
    z = torch.zeros(0, dtype=torch.int32, device=dev)
    pool = torch.zeros((1, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.mux(lk, pool, z, z, z, pool)           # B = 0 is a no-op
    p = C.c_void_p(pool.data_ptr())
    codes = {}
    for name, args in {"form": (7, p, p, p, p, None, p, 1), "null": (0, p, None, p, p, None, p, 1),
                       "range": (0, p, p, p, p, None, p, -1)}.items():
        rc = cemu.lib().cemu_mux(lk.ck, *args, None)
        codes[name] = rc
        assert rc != 0, name
    assert len(set(codes.values())) == 3      # three distinct error codes


def test_program_shifters_levels_and_graph(std, dev):
    """32-bit LLS / LRS / ARS register-mode shifters (Sec. 5.4), 4 instances
    each, merged level by level (5 levels of MUX batches, int8 form):
    decryptions equal the cleartext shifts; one instance of each replayed on
    the oracle from the same encrypted inputs (96 MUXes of every level)
    equals the GPU's pool word for word; a captured hipGraph replays the run
    exactly."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    rng = np.random.default_rng(55)
    cases = []
    for mode in (Cc.LLS, Cc.LRS, Cc.ARS):
        for _ in range(4):
            cases.append((mode, 32, int(rng.integers(0, 1 << 32, dtype=np.uint64)), int(rng.integers(0, 64))))
    cs = [Cc.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = Cc.Program(cs).to_device(dev)
    bits = []
    for k, w, a, b in cases:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    say(f"[gpu] shifters: {prog.num_muxes()} MUXes in {prog.depth} levels")
    pool, host0 = _program_pool(prog, ok, bits, dev)
    prog.run(lk, pool, form="int8")
    torch.cuda.synchronize()
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)
    _check_against_oracle_replay(ok, prog, host0, host, [0, 4, 8], "shifter replay", min_per_level=64)
    eager = host.copy()
    g = prog.capture(lk, pool, form="int8")
    keep = torch.zeros(prog.rows, dtype=torch.bool, device=dev)
    keep[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = True
    for rep in range(2):
        pool[~keep] = 0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(pool), eager), f"graph replay {rep} differs"


@pytest.mark.timeout(600)
def test_program_sequential_multiplier_and_divider(std, dev):
    """The paper's sequential multiplier (unsigned and signed) and the
    non-restoring divider (Sec. 5.5, 5.6), 8-bit, three instances each,
    merged level by level (FFT64 form, latency kernel): decryptions equal the
    cleartext results; one signed multiplication and one division replayed
    on the oracle from the same encrypted inputs (every gate of theirs, all
    88 levels) equal the GPU's pool word for word."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    rng = np.random.default_rng(77)
    cases = [(k, 8, int(rng.integers(0, 256)), int(rng.integers(1, 256))) for k in ("MULSEQ", "SMULSEQ", "DIV")
             for _ in range(3)]
    cs = [Cc.instruction_circuit(k, w) for k, w, _, _ in cases]
    prog = Cc.Program(cs).to_device(dev)
    bits = []
    for k, w, a, b in cases:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    say(f"[gpu] sequential units: {prog.num_gates()} gates in {prog.depth} levels")
    pool, host0 = _program_pool(prog, ok, bits, dev)
    saved = cemu.get_tuning(lk)
    try:
        cemu.set_tuning(lk, fft_gates_per_wg=1)
        prog.run(lk, pool, form="fft64")
        torch.cuda.synchronize()
    finally:
        cemu.set_tuning(lk, **saved)
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)
    _check_against_oracle_replay(ok, prog, host0, host, [3, 6], "sequential units replay")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("form", ["int8", "fft64"])
def test_bootstrap_level_matches_separate_calls(std, dev, form):
    """A level of G gates and M MUXes through cemu_bootstrap_level (one
    blind-rotation launch of G + 2M) equals, word for word, cemu_bootstrap_gates
    plus cemu_mux on the same inputs; outputs scattered to permuted distinct
    rows; pure-gate and pure-MUX levels too; decryptions exact; every gate
    and MUX word-equal to the oracle in both forms."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    rng = np.random.default_rng(91)
    R, G, M = 40, 29, 13
    say(f"[gpu] bootstrap_level {form} G={G} M={M}")
    bits = rng.integers(0, 2, R).astype(np.uint8)
    host_in = O.encrypt_bits(ok, bits, seed=W.ENC_SEED + 40)
    pool = to_dev(host_in, dev)
    ops_h = rng.integers(0, 10, G).astype(np.uint8)
    ia_h, ib_h = (rng.integers(0, R, G).astype(np.int32) for _ in range(2))
    ms_h, ma_h, mb_h = (rng.integers(0, R, M).astype(np.int32) for _ in range(3))
    perm = rng.permutation(G + M + 7)[:G + M].astype(np.int32)
    ops, ia, ib, ms, ma, mb, io = (_t(x, dev) for x in (ops_h, ia_h, ib_h, ms_h, ma_h, mb_h, perm))
    out_level = torch.zeros((G + M + 7, lk.n + 1), dtype=torch.int32, device=dev)
    out_sep = torch.zeros_like(out_level)
    cemu.bootstrap_level(lk, pool, (ops, ia, ib), (ms, ma, mb), out_level, io=io, form=form)
    cemu.bootstrap_gates(lk, ops, pool, ia, ib, out_sep, io=_t(perm[:G], dev), form=form)
    cemu.mux(lk, pool, ms, ma, mb, out_sep, io=_t(perm[G:], dev), form=form)
    only_g = torch.zeros((G, lk.n + 1), dtype=torch.int32, device=dev)
    only_g_ref = torch.zeros_like(only_g)
    cemu.bootstrap_level(lk, pool, (ops, ia, ib), None, only_g, form=form)
    cemu.bootstrap_gates(lk, ops, pool, ia, ib, only_g_ref, form=form)
    only_m = torch.zeros((M, lk.n + 1), dtype=torch.int32, device=dev)
    only_m_ref = torch.zeros_like(only_m)
    cemu.bootstrap_level(lk, pool, None, (ms, ma, mb), only_m, form=form)
    cemu.mux(lk, pool, ms, ma, mb, only_m_ref, form=form)
    cemu.bootstrap_level(lk, pool, None, None, only_m, form=form)     # G = M = 0: no-op
    dense = torch.zeros((G + M, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.bootstrap_level(lk, pool, (ops, ia, ib), (ms, ma, mb), dense, form=form)   # io NULL: row k
    torch.cuda.synchronize()
    assert torch.equal(out_level, out_sep)
    assert torch.equal(dense, out_level[_t(perm.astype(np.int64), dev)])
    assert torch.equal(only_g, only_g_ref) and torch.equal(only_m, only_m_ref)
    host = to_host_u32(out_level)
    want_g = np.array([OC.gate_plain(int(o), bits[a], bits[b]) for o, a, b in zip(ops_h, ia_h, ib_h)])
    want_m = np.where(bits[ms_h] == 1, bits[ma_h], bits[mb_h])
    assert np.array_equal(lk.decrypt(host[perm[:G]]), want_g)
    assert np.array_equal(lk.decrypt(host[perm[G:]]), want_m)
    # every gate and every MUX of the level against the oracle, in both forms
    _, og = O.bootstrap_batch(ok, ops_h.astype(np.int32), host_in[ia_h], host_in[ib_h], want_extracted=False)
    assert np.array_equal(host[perm[:G]], og)
    om = O.mux_batch(ok, host_in[ms_h], host_in[ma_h], host_in[mb_h])
    assert np.array_equal(host[perm[G:]], om)
    p = C.c_void_p(pool.data_ptr())
    lib = cemu.lib()
    assert lib.cemu_bootstrap_level(lk.ck, 0, p, p, p, p, -1, None, None, None, 0, None, p, None) == -8
    assert lib.cemu_bootstrap_level(lk.ck, 7, p, p, p, p, 1, None, None, None, 0, None, p, None) != 0
    assert lib.cemu_bootstrap_level(lk.ck, 0, p, p, p, p, 0, None, None, None, 2, None, p, None) != 0


def test_program_mux_prefix_levels_and_graph(std, dev):
    """ADD32, SUB32 and LT32 with the MUX prefix form (7 levels, gates and
    MUXes sharing launches), merged across instances, int8 form: decryptions
    equal uint32 arithmetic; one instance of each replayed on the oracle from
    the same encrypted inputs equals the GPU's pool word for word; a captured
    hipGraph replays the run exactly."""
    from paper_2101_03403_amd import circuits as Cc
    lk, ok = std
    rng = np.random.default_rng(321)
    cases = [(k, 32) + tuple(int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64))
             for k in ("ADD",) * 5 + ("SUB",) * 5 + ("LT",) * 3]
    cs = [Cc.instruction_circuit(k, w, prefix=Cc.PREFIX_MUX) for k, w, _, _ in cases]
    prog = Cc.Program(cs).to_device(dev)
    assert prog.depth == 7
    bits = []
    for k, w, a, b in cases:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    say(f"[gpu] mux-prefix program: {prog.num_bootstraps()} blind rotations in {prog.depth} levels")
    pool, host0 = _program_pool(prog, ok, bits, dev)
    prog.run(lk, pool, form="int8")
    torch.cuda.synchronize()
    host = to_host_u32(pool)
    for (k, w, a, b), c, off in zip(cases, cs, prog.offsets):
        got = Cc.bits_to_int(lk.decrypt(host[np.array(c.outputs["out"]) + off]))
        assert got == OC.word_result(k, w, a, b), (k, a, b, got)
    _check_against_oracle_replay(ok, prog, host0, host, [0, 5, 10], "mux-prefix replay")
    eager = host.copy()
    g = prog.capture(lk, pool, form="int8")
    keep = torch.zeros(prog.rows, dtype=torch.bool, device=dev)
    keep[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = True
    for rep in range(2):
        pool[~keep] = 0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(pool), eager), f"graph replay {rep} differs"


def test_bootstrap_level_toy_bit_exact(toy, dev):
    """Toy parameters (N = 512), int8 form: a level of 9 gates and 7 MUXes
    through cemu_bootstrap_level, every output bit-exact against the
    oracle's gates and MUX."""
    lk, ok = toy
    rng = np.random.default_rng(17)
    R, G, M = 12, 9, 7
    say(f"[gpu] bootstrap_level toy G={G} M={M}")
    bits = rng.integers(0, 2, R).astype(np.uint8)
    host_in = O.encrypt_bits(ok, bits, seed=W.ENC_SEED + 41)
    pool = to_dev(host_in, dev)
    ops_h = rng.integers(0, 10, G).astype(np.uint8)
    ia_h, ib_h = (rng.integers(0, R, G).astype(np.int32) for _ in range(2))
    ms_h, ma_h, mb_h = (rng.integers(0, R, M).astype(np.int32) for _ in range(3))
    perm = rng.permutation(G + M).astype(np.int32)
    out = torch.zeros((G + M, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.bootstrap_level(lk, pool, tuple(_t(x, dev) for x in (ops_h, ia_h, ib_h)),
                         tuple(_t(x, dev) for x in (ms_h, ma_h, mb_h)), out, io=_t(perm, dev), form="int8")
    torch.cuda.synchronize()
    host = to_host_u32(out)
    _, og = O.bootstrap_batch(ok, ops_h.astype(np.int32), host_in[ia_h], host_in[ib_h], want_extracted=False)
    om = O.mux_batch(ok, host_in[ms_h], host_in[ma_h], host_in[mb_h])
    assert np.array_equal(host[perm[:G]], og)
    assert np.array_equal(host[perm[G:]], om)


def _plain_gates(ops, a, b):
    """NAND / AND / OR / XOR (the throughput mix) on plaintext bits, vectorised."""
    a = a.astype(np.uint8)
    b = b.astype(np.uint8)
    r = np.select([ops == cemu.NAND, ops == cemu.AND, ops == cemu.OR, ops == cemu.XOR],
                  [1 - (a & b), a & b, a | b, a ^ b], default=255)
    assert (r != 255).all()
    return r.astype(np.uint8)


def test_batches_beyond_one_grid_pass(std, dev):
    """The element-wise kernels (linear combination, the MUX halves and
    combine, NOT / COPY / CONSTANT) walk their range with a grid stride over
    at most 2^24 threads; batches of more than 2^24 elements take several
    passes. Gates and MUXes: one large call equals, word for word, the same
    work split in two calls that each fit one pass, and every decryption is
    exact. Batches beyond one blind-rotation launch are refused with a range
    error before anything is allocated or launched."""
    lk, ok = std
    row = lk.n + 1
    one_pass = 1 << 24

    # NOT / COPY / CONSTANT on random words
    cnt = 30000
    assert cnt * row > one_pass
    say(f"[gpu] grid stride: NOT / COPY / CONSTANT count={cnt}")
    rng = np.random.default_rng(5)
    host = rng.integers(0, 1 << 32, (cnt, row), dtype=np.uint64).astype(np.uint32)
    src = to_dev(host, dev)
    perm = rng.permutation(cnt).astype(np.int32)
    idx = torch.arange(cnt, dtype=torch.int32, device=dev)
    dst = torch.from_numpy(perm).to(dev)
    dnot = torch.zeros_like(src)
    dcopy = torch.zeros_like(src)
    dconst = torch.zeros_like(src)
    bits = rng.integers(0, 2, cnt).astype(np.uint8)
    cemu.lwe_not(lk.n, src, idx, dnot, dst)
    cemu.lwe_copy(lk.n, src, idx, dcopy, dst)
    cemu.lwe_constant(lk.n, torch.from_numpy(bits).to(dev), dconst, dst)
    torch.cuda.synchronize()
    want_copy = np.empty_like(host)
    want_copy[perm] = host
    assert np.array_equal(to_host_u32(dcopy), want_copy)
    assert np.array_equal(to_host_u32(dnot), (0 - want_copy.astype(np.uint64)).astype(np.uint32))
    want_const = np.zeros_like(host)
    want_const[perm, lk.n] = np.where(bits == 1, 0x20000000, 0xE0000000).astype(np.uint32)
    assert np.array_equal(to_host_u32(dconst), want_const)

    # gates: lincomb over B * (n + 1) > 2^24 elements
    B = 30000
    assert B * row > one_pass and (B // 2) * row <= one_pass
    say(f"[gpu] grid stride: {B} gates, fft64, one call against two")
    ops, a, b = W.gate_batch(B, seed=77)
    c1 = O.encrypt_bits(ok, a, seed=78)
    c2 = O.encrypt_bits(ok, b, seed=78, first_index=B)
    pool = to_dev(np.concatenate([c1, c2]), dev)
    ops_t = torch.from_numpy(np.ascontiguousarray(ops.astype(np.uint8))).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    ib = ia + B
    big = torch.zeros((B, row), dtype=torch.int32, device=dev)
    cemu.bootstrap_gates(lk, ops_t, pool, ia, ib, big, form="fft64")
    halves = torch.zeros_like(big)
    h = B // 2
    cemu.bootstrap_gates(lk, ops_t[:h], pool, ia[:h], ib[:h], halves[:h], form="fft64")
    cemu.bootstrap_gates(lk, ops_t[h:], pool, ia[h:], ib[h:], halves[h:], form="fft64")
    torch.cuda.synchronize()
    got = to_host_u32(big)
    assert np.array_equal(got, to_host_u32(halves))
    assert np.array_equal(lk.decrypt(got), _plain_gates(ops, a, b))

    # MUX: its lincomb covers 2M (n + 1) and its combine M (N + 1) > 2^24 elements
    M = 17000
    assert M * (lk.N + 1) > one_pass and 2 * (M // 2) * row <= one_pass
    say(f"[gpu] grid stride: {M} MUXes, fft64, one call against two")
    mbits, cts = _mux_inputs(ok, M, 93)
    mpool = to_dev(np.concatenate(cts), dev)
    rows = torch.arange(M, dtype=torch.int32, device=dev)
    mbig = torch.zeros((M, row), dtype=torch.int32, device=dev)
    cemu.mux(lk, mpool, rows, rows + M, rows + 2 * M, mbig, form="fft64")
    mhalves = torch.zeros_like(mbig)
    hm = M // 2
    cemu.mux(lk, mpool, rows[:hm], rows[:hm] + M, rows[:hm] + 2 * M, mhalves[:hm], form="fft64")
    cemu.mux(lk, mpool, rows[hm:], rows[hm:] + M, rows[hm:] + 2 * M, mhalves[hm:], form="fft64")
    torch.cuda.synchronize()
    mgot = to_host_u32(mbig)
    assert np.array_equal(mgot, to_host_u32(mhalves))
    assert np.array_equal(lk.decrypt(mgot), np.where(mbits[0] == 1, mbits[1], mbits[2]))

    # range errors, returned before any allocation or launch
    p = C.c_void_p(pool.data_ptr())
    o = C.c_void_p(ops_t.data_ptr())
    rc = cemu.lib().cemu_bootstrap_gates(lk.ck, 1, o, p, p, p, None, p, C.c_int64(1 << 41), None)
    assert rc == cemu.lib().cemu_bootstrap_gates(lk.ck, 1, o, p, p, p, None, p, C.c_int64(-1), None) != 0
    saved = cemu.get_tuning(lk)
    try:
        cemu.set_tuning(lk, fft_gates_per_wg=1)
        too_many = (0xFFFFFFFF // 384) + 1          # one workgroup of 384 threads per gate
        rc2 = cemu.lib().cemu_bootstrap_gates(lk.ck, 1, o, p, p, p, None, p, C.c_int64(too_many), None)
        assert rc2 == rc
        assert "too large" in cemu.lib().cemu_last_error().decode()
    finally:
        cemu.set_tuning(lk, **saved)


def test_int8_round_tail_split(std, dev):
    """The 16-gate int8 kernel also runs in rounds of 16 gates per CU; a short
    tail behind full rounds launches on the one-gate kernel. Batches sized from
    the device's CU count (a small and a long tail, and one just past the
    limit) equal, word for word, the one-gate kernel's output for the whole
    batch; every decryption is exact."""
    lk, ok = std
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    saved = cemu.get_tuning(lk)
    try:
        for B in (16 * cus + 37, 16 * cus + 12 * cus, 16 * cus + 12 * cus + 1):
            say(f"[gpu] int8 tail split: B={B} (CUs {cus})")
            ops, a, b = W.gate_batch(B, seed=400 + B)
            c1 = O.encrypt_bits(ok, a, seed=401)
            c2 = O.encrypt_bits(ok, b, seed=401, first_index=B)
            cemu.set_tuning(lk, int8_waves=8, int8_gates_per_wg=16)
            _, got = run_gates(lk, ops, c1, c2, dev, form="int8", want_ext=False)
            cemu.set_tuning(lk, int8_waves=8, int8_gates_per_wg=1)
            _, ref = run_gates(lk, ops, c1, c2, dev, form="int8", want_ext=False)
            assert np.array_equal(got, ref)
            assert np.array_equal(lk.decrypt(got), _plain_gates(ops, a, b))
    finally:
        cemu.set_tuning(lk, **saved)


def test_fft_round_tail_split(std, dev):
    """Every FFT shape runs one workgroup per CU, so a batch of k full rounds
    plus a short tail launches the tail separately on a smaller shape (the
    latency kernel, or 4 gates per workgroup behind 8-gate rounds). Batches
    sized from the device's CU count take each path; every output equals,
    word for word, the latency kernel's output for the whole batch, and every
    decryption is exact."""
    lk, ok = std
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    saved = cemu.get_tuning(lk)
    try:
        for fg, B in ((8, 8 * cus + cus // 2 + 3), (8, 8 * cus + 3 * cus + cus // 2), (4, 4 * cus + 2 * cus + 1),
                      (8, 16 * cus + 5)):
            say(f"[gpu] fft tail split: fg={fg} B={B} (CUs {cus})")
            ops, a, b = W.gate_batch(B, seed=300 + B)
            c1 = O.encrypt_bits(ok, a, seed=301)
            c2 = O.encrypt_bits(ok, b, seed=301, first_index=B)
            cemu.set_tuning(lk, fft_gates_per_wg=fg)
            _, got = run_gates(lk, ops, c1, c2, dev, form="fft64", want_ext=False)
            cemu.set_tuning(lk, fft_gates_per_wg=1)
            _, ref = run_gates(lk, ops, c1, c2, dev, form="fft64", want_ext=False)
            assert np.array_equal(got, ref)
            assert np.array_equal(lk.decrypt(got), _plain_gates(ops, a, b))
    finally:
        cemu.set_tuning(lk, **saved)
