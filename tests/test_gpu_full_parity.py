"""GPU parity over whole batches and the method's edge cases.

Every input here is the oracle's own encryption (or a ciphertext built word
by word in the test), so no oracle input comes from the GPU.

* The throughput batch (4096 independent NAND/AND/OR/XOR gates, standard
  parameters) in the benchmark's launch shapes: every one of the 4096 int8
  outputs (extracted samples and key-switched ciphertexts) equals the
  oracle's word for word, and so do the FFT64 form's; the same for every
  other launch shape of both forms. The FFT64 claim: each
  product is an integer polynomial computed in double precision, so while the
  transform error stays below one half every coefficient rounds to the exact
  integer and the extracted samples equal the exact ones; the maximum error
  against the oracle is printed.
* The output noise of that batch against the closed form for one fixed key.
* All ten gates at standard parameters, and ciphertexts built to hit the
  method's edge cases: trivial inputs (every rescaled mask coefficient 0,
  so the blind rotation does nothing), b-bar = 0, and rescaled mask
  coefficients at 1, N - 1, N, N + 1, 2N - 1 and at the rounding boundaries
  (ties, and values that round up to 2N and wrap to 0).
* Key switching with the whole batch in one unsplit launch (8192 samples),
  and the full-precision key switch (t = 16) that runs on the VALU kernel.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import circuits as OC  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2101_03403_amd import cemu, workloads as W  # noqa: E402

SEED = 20210108
N_STD, n_STD = 1024, 630
THROUGHPUT_B = 4096


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_i32(x):
    x = np.asarray(x, dtype=np.uint32)
    return x.astype(np.int64) - ((x >> 31).astype(np.int64) << 32)


def to_dev(a, dev):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(dev)


def to_host_u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def std(dev):
    say("[gpu-full] keygen std (library + oracle)")
    lk, ok = cemu.keygen(cemu.STD, SEED), O.keygen(O.STANDARD, SEED)
    ex = lk.export(bk=False, ksk=False)
    assert np.array_equal(ex["lwe_key"], ok.lwe_key) and np.array_equal(ex["tlwe_key"], ok.tlwe_key)
    return lk, ok


def gpu_gates(lk, ops, c1, c2, dev, form):
    """Pool = [c1; c2]; gate g reads rows g and B + g. Returns (ext, out)."""
    B = ops.shape[0]
    pool = to_dev(np.concatenate([c1, c2]), dev)
    ops_t = torch.from_numpy(np.ascontiguousarray(ops.astype(np.uint8))).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    ib = ia + B
    ext = torch.zeros((B, lk.N + 1), dtype=torch.int32, device=dev)
    out = torch.zeros((B, lk.n + 1), dtype=torch.int32, device=dev)
    cemu.blind_rotate_extract(lk, ops_t, pool, ia, ib, ext, form=form)
    cemu.bootstrap_gates(lk, ops_t, pool, ia, ib, out, form=form)
    torch.cuda.synchronize()
    return to_host_u32(ext), to_host_u32(out)


def oracle_gates_chunked(ok, ops, c1, c2, label, chunk=256):
    """The oracle over a batch in chunks, printing progress between them."""
    B = ops.shape[0]
    ext = np.zeros((B, ok.params.N + 1), np.uint32)
    out = np.zeros((B, ok.params.n + 1), np.uint32)
    for s in range(0, B, chunk):
        e = min(B, s + chunk)
        ext[s:e], out[s:e] = O.bootstrap_batch(ok, ops[s:e].astype(np.int32), c1[s:e], c2[s:e])
        say(f"[oracle] {label}: {e}/{B} gates")
    return ext, out


def word_report(label, got, want):
    diff = int(np.sum(got != want))
    err = np.abs(to_i32(got.astype(np.int64) - want.astype(np.int64))).max() if got.size else 0
    say(f"[gpu-full] {label}: differing words {diff}/{want.size}, max |word error| {err}")
    return diff


def truth(ops, a, b):
    return np.array([OC.gate_plain(int(o), int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)


# ------------------------------------------------------------------ the whole throughput batch
# the launch shapes besides the benchmark's (int8: 16 gates per workgroup on
# 8 waves; FFT64: 8 gates per workgroup)
OTHER_SHAPES = [
    ("fft64", {"fft_gates_per_wg": 4}),
    ("fft64", {"fft_gates_per_wg": 1}),
    ("int8", {"int8_waves": 4, "int8_gates_per_wg": 16}),
    ("int8", {"int8_waves": 8, "int8_gates_per_wg": 1}),
    ("int8", {"int8_waves": 4, "int8_gates_per_wg": 1}),
]


@pytest.fixture(scope="module")
def batch4096(std, dev):
    lk, ok = std
    B = THROUGHPUT_B
    ops, a, b = W.gate_batch(B, seed=W.KEY_SEED & 0xFFFF)
    c1 = O.encrypt_bits(ok, a, seed=W.ENC_SEED)
    c2 = O.encrypt_bits(ok, b, seed=W.ENC_SEED, first_index=B)
    res = {}
    saved = cemu.get_tuning(lk)
    try:
        cemu.set_tuning(lk, int8_waves=8, int8_gates_per_wg=16, fft_gates_per_wg=8)
        for form in ("int8", "fft64"):
            say(f"[gpu-full] {form} on {B} gates")
            res[form] = gpu_gates(lk, ops, c1, c2, dev, form)
        # every other launch shape on the same batch
        for form, tun in OTHER_SHAPES:
            say(f"[gpu-full] {form} {tun} on {B} gates")
            cemu.set_tuning(lk, **tun)
            res[(form, tuple(sorted(tun.items())))] = gpu_gates(lk, ops, c1, c2, dev, form)
    finally:
        cemu.set_tuning(lk, **saved)
    say(f"[gpu-full] oracle on all {B} gates ({O.num_threads()} threads)")
    res["oracle"] = oracle_gates_chunked(ok, ops, c1, c2, "4096 batch", chunk=512)
    return ops, a, b, res


@pytest.mark.timeout(900)
def test_full_batch_int8_bit_exact(batch4096):
    """All 4096 gates of the int8-MFMA form equal the exact oracle word for
    word: extracted samples and key-switched outputs."""
    _, _, _, res = batch4096
    (ext, out), (oext, oout) = res["int8"], res["oracle"]
    assert word_report("int8 extracted vs oracle", ext, oext) == 0
    assert word_report("int8 output vs oracle", out, oout) == 0


@pytest.mark.timeout(900)
def test_full_batch_fft64_words_equal(batch4096):
    """The FFT64 form's extracted samples equal the exact ones for all 4096
    gates (every product rounded to its exact integer), and hence so do the
    key-switched outputs."""
    _, _, _, res = batch4096
    (ext, out), (oext, oout) = res["fft64"], res["oracle"]
    assert word_report("fft64 extracted vs oracle", ext, oext) == 0
    assert word_report("fft64 output vs oracle", out, oout) == 0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("form,tun", OTHER_SHAPES, ids=[f"{f}-{'-'.join(f'{k}{v}' for k, v in t.items())}" for f, t in OTHER_SHAPES])
def test_full_batch_every_launch_shape(batch4096, form, tun):
    """The other launch shapes (the FFT64 form at 4 gates per workgroup and
    its one-gate latency kernel; the int8 form on 4 waves and its one-gate
    latency kernel on 8 and 4 waves) give the oracle's words for all 4096
    gates too."""
    _, _, _, res = batch4096
    (ext, out), (oext, oout) = res[(form, tuple(sorted(tun.items())))], res["oracle"]
    assert word_report(f"{form} {tun} extracted vs oracle", ext, oext) == 0
    assert word_report(f"{form} {tun} output vs oracle", out, oout) == 0


@pytest.mark.timeout(900)
def test_full_batch_decryptions(std, batch4096):
    lk, ok = std
    ops, a, b, res = batch4096
    want = truth(ops, a, b)
    for form in ("int8", "fft64"):
        ext, out = res[form]
        assert np.array_equal(O.decrypt_bits(ok.lwe_key, out), want), form
        assert np.array_equal(O.decrypt_bits(ok.tlwe_key, ext), want), form


@pytest.mark.timeout(900)
def test_full_batch_noise_against_closed_form(std, batch4096):
    """Output noise e = phase - mu over the 4096 gates, against the closed
    form for one fixed key set (the sample variance across gates of one key).

    Blind rotation: each of the n steps adds, per output coefficient, the
    2l x N products of digits d with the key noise, so Var_BR =
    n * 2l * N * Var(d) * sigma_bk^2 with d uniform on [-Bg/2, Bg/2):
    Var(d) = (Bg^2 - 1) / 12. Key switching subtracts one key row per nonzero
    digit: for one fixed key the row noises e(v), v = 1..3 (e(0) = 0) are
    fixed numbers, and over a uniform digit the variance of e(d) is
    E[e^2] - E[e]^2, which averages to (3/4 - 3/16) sigma_ks^2 =
    (9/16) sigma_ks^2 over keys (the mean part is a bias common to every gate
    of the key); Var_KS = N * t * (9/16) * sigma_ks^2. The rounding to 16 bits
    adds (N/2) * 2^-32 / 12 (negligible). Asserted within +-10 % (the sample
    variance of 4096 draws has a relative standard error of 2.2 %)."""
    lk, ok = std
    ops, a, b, res = batch4096
    p = ok.params
    mu = np.where(truth(ops, a, b) == 1, 1 << 29, -(1 << 29)).astype(np.int64)
    ext, out = res["int8"]
    ph_ext = np.array([O.lwe_phase(ok.tlwe_key, c) for c in ext], np.uint32)
    ph_out = np.array([O.lwe_phase(ok.lwe_key, c) for c in out], np.uint32)
    e_ext = to_i32((ph_ext.astype(np.int64) - mu) % (1 << 32)) / 2.0 ** 32
    e_out = to_i32((ph_out.astype(np.int64) - mu) % (1 << 32)) / 2.0 ** 32
    bg = 1 << p.bgbit
    var_br = p.n * 2 * p.l * p.N * (bg * bg - 1) / 12.0 * p.sigma_bk ** 2
    var_ks = p.N * p.t * (9.0 / 16.0) * p.sigma_ks ** 2 + (p.N / 2) * 2.0 ** -32 / 12.0
    v_ext, v_out = float(np.var(e_ext)), float(np.var(e_out))
    say(f"[gpu-full] noise: extracted var {v_ext:.4g} (closed form {var_br:.4g}), "
        f"output var {v_out:.4g} (closed form {var_br + var_ks:.4g}), output std 2^{np.log2(np.sqrt(v_out)):.2f}")
    assert abs(v_ext / var_br - 1) < 0.10
    assert abs(v_out / (var_br + var_ks) - 1) < 0.10
    # worst case: digits at +-Bg/2 and every key-switching digit nonzero
    worst = p.n * 2 * p.l * p.N * (bg / 2) ** 2 * p.sigma_bk ** 2 + p.N * p.t * p.sigma_ks ** 2
    assert v_out < worst
    # every output stays far inside the decision region (+-1/8 around mu)
    assert np.abs(e_out).max() < 1.0 / 16


# ------------------------------------------------------------------ all gates, edge cases
FORMS = ("int8", "fft64")


@pytest.mark.parametrize("form", FORMS)
def test_all_ten_gates_std(std, dev, form):
    """The ten gates x four input rows x four repetitions at standard
    parameters: outputs equal the oracle word for word and decrypt to the
    truth tables."""
    lk, ok = std
    ops, a, b = W.all_gates_rows(reps=4)
    c1 = O.encrypt_bits(ok, a, seed=301)
    c2 = O.encrypt_bits(ok, b, seed=302)
    say(f"[gpu-full] ten gates std {form}, B = {ops.shape[0]}")
    ext, out = gpu_gates(lk, ops, c1, c2, dev, form)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert word_report(f"ten gates {form} extracted", ext, oext) == 0
    assert word_report(f"ten gates {form} output", out, oout) == 0
    assert np.array_equal(O.decrypt_bits(ok.lwe_key, out), truth(ops, a, b))


def _edge_inputs(n, N, seed):
    """(ops, c1, c2, trivial_count, want): ciphertexts built word by word.

    Gates 0..39: trivial samples (0, ..., 0, +-1/8) into all ten gates, all
    four input rows (a CONSTANT input: every rescaled mask coefficient is 0,
    so every blind-rotation step is skipped). The rest use AND with a zero
    second input, so the gate's linear combination is c1 + (0, ..., 0, -1/8)
    and its rescaled mask is the rescaled mask of c1:
      - random masks with b chosen so that b-bar = 0;
      - masks whose coefficients sit at the centres of 1, N-1, N, N+1,
        2N-1 (and 0) in one pattern, with random b;
      - every coefficient = N (each step multiplies by X^N = -1), or
        2N - 1, or 1;
      - coefficients at the rounding boundaries: the largest value rounding
        down, the tie (rounds up), and values just below 2^32 that round to
        2N and wrap to 0."""
    rng = np.random.default_rng(seed)
    step = (1 << 32) // (2 * N)
    ops, c1, c2, want = [], [], [], []
    rows = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for op in range(10):
        for x, y in rows:
            t1 = np.zeros(n + 1, np.uint32)
            t2 = np.zeros(n + 1, np.uint32)
            t1[n] = 0x20000000 if x else 0xE0000000
            t2[n] = 0x20000000 if y else 0xE0000000
            ops.append(op)
            c1.append(t1)
            c2.append(t2)
            want.append(OC.gate_plain(op, x, y))
    trivial = len(ops)

    def add_and(mask, b):
        c = np.zeros(n + 1, np.uint32)
        c[:n] = np.asarray(mask, np.uint64).astype(np.uint32)
        c[n] = np.uint32(int(b) & 0xFFFFFFFF)
        ops.append(OC.AND)
        c1.append(c)
        c2.append(np.zeros(n + 1, np.uint32))

    # b-bar = 0: the AND constant -1/8 is cancelled by b = +1/8
    for _ in range(6):
        add_and(rng.integers(0, 1 << 32, n, dtype=np.uint64), 1 << 29)
    # pattern of centres
    pattern = np.array([0, 1, N - 1, N, N + 1, 2 * N - 1], np.uint64)
    for r in range(6):
        vals = np.roll(np.resize(pattern, n), r) * step
        add_and(vals, int(rng.integers(0, 1 << 32, dtype=np.uint64)))
    for v in (N, 2 * N - 1, 1):
        for _ in range(2):
            add_and(np.full(n, v * step, np.uint64), int(rng.integers(0, 1 << 32, dtype=np.uint64)))
    # rounding boundaries around random centres, and the wrap to 2N -> 0
    for _ in range(4):
        centre = rng.integers(0, 2 * N, n).astype(np.uint64) * step
        kind = rng.integers(0, 3, n)
        off = np.where(kind == 0, step // 2 - 1, np.where(kind == 1, step // 2, step // 2 + 1)).astype(np.uint64)
        add_and((centre + off) % (1 << 32), int(rng.integers(0, 1 << 32, dtype=np.uint64)))
    wrap = ((1 << 32) - rng.integers(1, step // 2 + 1, n)).astype(np.uint64)
    add_and(wrap, int(rng.integers(0, 1 << 32, dtype=np.uint64)))
    add_and(wrap, 1 << 29)
    return (np.array(ops, np.uint8), np.stack(c1), np.stack(c2), trivial, np.array(want, np.uint8))


@pytest.mark.parametrize("form", FORMS)
def test_edge_case_ciphertexts_std(std, dev, form):
    """The edge-case ciphertexts above: every extracted sample and output
    equals the oracle's word for word; the trivial-input gates decrypt to
    the truth tables."""
    lk, ok = std
    ops, c1, c2, trivial, want = _edge_inputs(n_STD, N_STD, seed=404)
    # the rescaled masks really hit the intended values (checked with the oracle's mod switch)
    lin = np.stack([O.gate_lincomb(int(o), x, y) for o, x, y in zip(ops, c1, c2)])
    bars = O.modswitch_array(lin.reshape(-1), 2 * N_STD).reshape(lin.shape)
    assert np.all(bars[:trivial, :n_STD] == 0)
    assert np.all(bars[trivial:trivial + 6, n_STD] == 0)
    hit = set(np.unique(bars[trivial:, :n_STD]).tolist())
    assert {0, 1, N_STD - 1, N_STD, N_STD + 1, 2 * N_STD - 1} <= hit
    say(f"[gpu-full] edge cases {form}, B = {ops.shape[0]}")
    ext, out = gpu_gates(lk, ops, c1, c2, dev, form)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert word_report(f"edge cases {form} extracted", ext, oext) == 0
    assert word_report(f"edge cases {form} output", out, oout) == 0
    assert np.array_equal(O.decrypt_bits(ok.lwe_key, out[:trivial]), want)


@pytest.mark.parametrize("form", FORMS)
def test_edge_cases_latency_kernels(std, dev, form):
    """The same edge cases on the one-gate-per-workgroup kernels."""
    lk, ok = std
    ops, c1, c2, _, _ = _edge_inputs(n_STD, N_STD, seed=405)
    saved = cemu.get_tuning(lk)
    try:
        cemu.set_tuning(lk, int8_gates_per_wg=1, fft_gates_per_wg=1)
        say(f"[gpu-full] edge cases {form} latency kernel, B = {ops.shape[0]}")
        ext, out = gpu_gates(lk, ops, c1, c2, dev, form)
    finally:
        cemu.set_tuning(lk, **saved)
    oext, oout = O.bootstrap_batch(ok, ops.astype(np.int32), c1, c2)
    assert word_report(f"edge cases {form} latency extracted", ext, oext) == 0
    assert word_report(f"edge cases {form} latency output", out, oout) == 0


# ------------------------------------------------------------------ key switching
def test_key_switch_unsplit_8192(std, dev):
    """8192 samples: enough tiles that the key switch runs without splitting
    its K range (the path of the widest circuit levels), bit-exact."""
    lk, ok = std
    B = 8192
    rng = np.random.default_rng(8192)
    ins = rng.integers(0, 1 << 32, (B, lk.N + 1), dtype=np.uint64).astype(np.uint32)
    dout = torch.zeros((B, lk.n + 1), dtype=torch.int32, device=dev)
    say("[gpu-full] key switch B = 8192")
    cemu.key_switch(lk, to_dev(ins, dev), dout)
    torch.cuda.synchronize()
    got = to_host_u32(dout)
    say("[oracle] key switch B = 8192")
    want = O.key_switch_batch(ok, ins)
    assert word_report("key switch 8192", got, want) == 0


@pytest.mark.parametrize("which,N,n", [("std", 1024, 630), ("toy", 512, 256)])
def test_key_switch_full_precision_valu(dev, which, N, n):
    """t = 16 (t * basebit = 32: no rounding) runs on the VALU key-switch
    kernel: bit-exact against the oracle on random samples, and with
    noiseless keys the phase is preserved exactly."""
    base = O.STANDARD if which == "std" else O.TOY
    for sigma in (2.0 ** -15, 0.0):
        op = O.Params(n=n, N=N, t=16, sigma_lwe=sigma, sigma_ks=sigma, sigma_bk=base.sigma_bk)
        lp = cemu.params(cemu.STD if which == "std" else cemu.TOY, t=16, sigma_lwe=sigma, sigma_ks=sigma)
        say(f"[gpu-full] full-precision key switch {which}, sigma {sigma}")
        lk, ok = cemu.keygen(lp, 77), O.keygen(op, 77)
        ex = lk.export(bk=False)
        assert np.array_equal(ex["ksk"], ok.ksk)
        for B in (1, 37, 300):
            rng = np.random.default_rng(B)
            ins = rng.integers(0, 1 << 32, (B, N + 1), dtype=np.uint64).astype(np.uint32)
            dout = torch.zeros((B, n + 1), dtype=torch.int32, device=dev)
            cemu.key_switch(lk, to_dev(ins, dev), dout)
            torch.cuda.synchronize()
            got = to_host_u32(dout)
            assert np.array_equal(got, O.key_switch_batch(ok, ins)), (which, sigma, B)
            if sigma == 0.0:
                ph_in = np.array([O.lwe_phase(ok.tlwe_key, c) for c in ins], np.uint32)
                ph_out = np.array([O.lwe_phase(ok.lwe_key, c) for c in got], np.uint32)
                assert np.array_equal(ph_in, ph_out)
        lk.free()
