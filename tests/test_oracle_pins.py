"""Pins of the CPU oracle against facts fixed outside of it.

Each test checks the oracle against something that is not the oracle's own
formula: published known-answer vectors, a library routine on small inputs
(numpy polynomial convolution), brute force, algebraic identities, the exact
noiseless result of bootstrapping, gate truth tables under decryption
(homomorphic correctness f(a,b) = Dec(g(Enc a, Enc b)), Sec. 2; gate list of
Table "TFHEbenchmark"), and the closed-form noise variance.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M32 = 1 << 32


def to_i32(x):
    return np.asarray(x, dtype=np.uint32).astype(np.int64) - ((np.asarray(x, dtype=np.uint32) >> 31).astype(np.int64) << 32)


def negacyclic_ref(P, Q):
    """Product mod X^N+1 from numpy's plain convolution, folded by X^N = -1."""
    P = np.asarray(P, dtype=object)
    Q = np.asarray(Q, dtype=object)
    N = len(P)
    c = np.convolve(P, Q)
    out = [int(c[m]) - (int(c[m + N]) if m + N < len(c) else 0) for m in range(N)]
    return np.array([v % M32 for v in out], dtype=np.uint32)


def monomial(a, N):
    P = np.zeros(N, dtype=np.uint32)
    if a < N:
        P[a] = 1
    else:
        P[a - N] = M32 - 1
    return P


# ------------------------------------------------------------------ Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_gaussian_moments():
    sigma = 2.0 ** -15
    x = O.gauss_array(1234, 400_000, sigma).astype(np.float64) / (sigma * 2.0 ** 32)
    assert abs(x.mean()) < 4.0 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 0.015
    k = ((x - x.mean()) ** 4).mean() / x.var() ** 2
    assert abs(k - 3.0) < 0.1
    # symmetric and unbounded-looking tails
    assert (np.abs(x) > 3).mean() == pytest.approx(0.0027, abs=0.0008)


# ------------------------------------------------------------------ products
@pytest.mark.parametrize("N", [4, 16, 64])
def test_negacyclic_matches_numpy_convolution(N):
    rng = np.random.default_rng(N)
    for _ in range(20):
        P = rng.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        Q = rng.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(O.negacyclic_mul(P, Q), negacyclic_ref(P, Q))


def test_negacyclic_bruteforce_small():
    N = 4
    vals = [0, 1, M32 - 1, 2]
    for P in itertools.product(vals, repeat=N):
        Q = np.array([3, M32 - 5, 7, 1], dtype=np.uint32)
        assert np.array_equal(O.negacyclic_mul(np.array(P, np.uint32), Q), negacyclic_ref(P, Q))


@pytest.mark.parametrize("N", [8, 32])
def test_monomial_identity(N):
    """X^a * X^b = X^((a+b) mod 2N), with X^N = -1."""
    for a in range(2 * N):
        for b in range(0, 2 * N, 3):
            got = O.negacyclic_mul(monomial(a, N), monomial(b, N))
            assert np.array_equal(got, monomial((a + b) % (2 * N), N))


def test_product_linear_and_commutative():
    rng = np.random.default_rng(5)
    N = 128
    P, Q, R = (rng.integers(0, M32, N, dtype=np.uint64).astype(np.uint32) for _ in range(3))
    assert np.array_equal(O.negacyclic_mul(P, Q), O.negacyclic_mul(Q, P))
    lhs = O.negacyclic_mul(P, Q + R)
    rhs = O.negacyclic_mul(P, Q) + O.negacyclic_mul(P, R)
    assert np.array_equal(lhs, rhs)


def test_rotation_is_monomial_product():
    rng = np.random.default_rng(6)
    N = 64
    P = rng.integers(0, M32, N, dtype=np.uint64).astype(np.uint32)
    for a in range(2 * N):
        assert np.array_equal(O.rotate(a, P), negacyclic_ref(monomial(a, N), P))


# ------------------------------------------------------------------ modulus switch
@pytest.mark.parametrize("two_n", [1024, 2048])
def test_modswitch_nearest(two_n):
    """abar is the nearest integer to x*2N/2^32 taken mod 2N; ties go up."""
    step = M32 // two_n
    half = step // 2
    centres = np.arange(two_n, dtype=np.int64) * step + half        # tie points
    near = (centres[:, None] + np.arange(-3, 4)[None, :]).reshape(-1) % M32
    rng = np.random.default_rng(two_n)
    xs = np.concatenate([near, rng.integers(0, M32, 2_000_000), [0, 1, M32 - 1, M32 - half, M32 - half - 1]])
    xs = xs.astype(np.uint32)
    got = O.modswitch_array(xs, two_n).astype(np.int64)
    assert got.min() >= 0 and got.max() < two_n
    x = xs.astype(np.int64)
    # circular distance between x*2N and got*2^32, in units of 2^-32 * (1/2N)
    diff = (x * two_n - got * M32) % (two_n * M32)
    diff = np.where(diff >= two_n * M32 // 2, diff - two_n * M32, diff)
    assert np.all(np.abs(diff) <= M32 // 2)
    ties = np.abs(diff) == M32 // 2
    assert np.all(diff[ties] == -(M32 // 2))          # ties round up


# ------------------------------------------------------------------ decomposition
@pytest.mark.parametrize("l,bgbit", [(3, 7), (4, 8), (2, 10), (1, 7)])
def test_decomposition_range_and_precision(l, bgbit):
    rng = np.random.default_rng(l * 100 + bgbit)
    total = l * bgbit
    xs = rng.integers(0, M32, 300_000).astype(np.uint32)
    if total < 32:
        q = 1 << (32 - total)
        tie = (np.arange(0, 4096, dtype=np.int64) * q * 997 + q // 2) % M32
        xs = np.concatenate([xs, tie.astype(np.uint32), (tie + 1).astype(np.uint32), (tie - 1).astype(np.uint32)])
    d = O.decompose_array(xs, l, bgbit).astype(np.int64)
    bg = 1 << bgbit
    assert d.min() >= -bg // 2 and d.max() < bg // 2
    rec = np.zeros(xs.shape[0], dtype=np.int64)
    for j in range(1, l + 1):
        rec += d[:, j - 1] * (1 << (32 - j * bgbit))
    rec %= M32
    err = (xs.astype(np.int64) - rec) % M32
    err = np.where(err >= M32 // 2, err - M32, err)
    if total >= 32:
        assert np.all(err == 0)
    else:
        half = 1 << (31 - total)
        assert np.all(np.abs(err) <= half)
        assert np.all(err[np.abs(err) == half] == -half)   # ties round up
        assert np.all(rec % (1 << (32 - total)) == 0)


# ------------------------------------------------------------------ exhaustive over all 2^32 words
@pytest.mark.slow
def test_modswitch_and_decomposition_exhaustive(tmp_path):
    """Every uint32 word: the modulus switch (2N = 1024 and 2048) is the
    nearest integer of x * 2N / 2^32 modulo 2N with ties up, and the l = 3,
    Bgbit = 7 decomposition has digits in [-64, 64) recomposing to the nearest
    multiple of 2^11 (ties up). The checks are a small C program
    (tests/exhaustive_pins.c) linked with the oracle's source."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "exhaustive_pins")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", os.path.join(here, "exhaustive_pins.c"),
                           os.path.join(os.path.dirname(here), "oracle", "oracle.c"), "-lm", "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    counts = [int(line.split()[-1]) for line in r.stdout.strip().splitlines()]
    assert len(counts) == 5 and sum(counts) == 0 and r.returncode == 0


def test_decomposition_of_zero_is_zero():
    assert np.all(O.decompose(0, 3, 7) == 0)


# ------------------------------------------------------------------ toy keys
@pytest.fixture(scope="module")
def toy_keys():
    return O.keygen(O.TOY, 2021)


def test_keygen_bk_rows_are_trgsw(toy_keys):
    """Each BK row is a TRLWE sample whose phase is its small noise plus the
    gadget term s_i * 2^(32-(j+1)Bgbit) on the constant coefficient of
    component c (for c = 0 the term enters through -A*S)."""
    k = toy_keys
    p = k.params
    S = k.tlwe_key
    for i in [0, 1, p.n - 1]:
        for r in range(2 * p.l):
            c, j = divmod(r, p.l)
            A, B = k.bk[i, r, 0], k.bk[i, r, 1]
            phase = (B.astype(np.int64) - negacyclic_ref(A, S).astype(np.int64)) % M32
            h = 1 << (32 - (j + 1) * p.bgbit)
            mu = np.zeros(p.N, dtype=object)
            if k.lwe_key[i]:
                if c == 1:
                    mu[0] = h
                else:  # A carries +h on X^0, so phase gets -h*S
                    mu = np.array([-h * int(s) for s in S], dtype=object)
            mu = np.array([int(v) % M32 for v in mu], dtype=np.int64)
            noise = to_i32((phase - mu) % M32)
            assert np.abs(noise).max() < 2 ** 7 * 7          # sigma_bk = 2^-25 -> 128 units


def test_keygen_ksk_rows(toy_keys):
    k = toy_keys
    p = k.params
    for i in [0, 7, p.N - 1]:
        for j in range(p.t):
            for v in range(4):
                row = k.ksk[i, j, v]
                ph = O.lwe_phase(k.lwe_key, row)
                mu = (v * int(k.tlwe_key[i]) << (32 - (j + 1) * p.basebit)) % M32
                e = to_i32((ph - mu) % M32)
                assert abs(int(e)) < 2 ** 17 * 7


def test_encrypt_decrypt_and_fresh_noise(toy_keys):
    k = toy_keys
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 2, 4000).astype(np.uint8)
    cts = O.encrypt_bits(k, bits, seed=99)
    assert np.array_equal(O.decrypt_bits(k.lwe_key, cts), bits)
    ph = np.array([O.lwe_phase(k.lwe_key, c) for c in cts[:2000]], dtype=np.uint32)
    mu = np.where(bits[:2000] == 1, 1 << 29, M32 - (1 << 29))
    e = to_i32((ph.astype(np.int64) - mu) % M32).astype(np.float64)
    assert e.var() == pytest.approx((2.0 ** 17) ** 2, rel=0.1)


def test_gate_lincomb_linear(toy_keys):
    rng = np.random.default_rng(4)
    c1 = rng.integers(0, M32, 257).astype(np.uint32)
    c2 = rng.integers(0, M32, 257).astype(np.uint32)
    consts = {0: (1 << 29, -1, -1), 1: (-(1 << 29), 1, 1), 2: (1 << 29, 1, 1), 3: (1 << 30, 2, 2),
              4: (-(1 << 30), -2, -2), 5: (-(1 << 29), -1, -1), 6: (-(1 << 29), -1, 1),
              7: (-(1 << 29), 1, -1), 8: (1 << 29, -1, 1), 9: (1 << 29, 1, -1)}
    for op, (kap, w1, w2) in consts.items():
        want = [(w1 * int(a) + w2 * int(b)) % M32 for a, b in zip(c1, c2)]
        want[-1] = (want[-1] + kap) % M32
        assert np.array_equal(O.gate_lincomb(op, c1, c2), np.array(want, dtype=np.uint32))
    with pytest.raises(ValueError):
        O.gate_lincomb(10, c1, c2)


TRUTH = {
    0: lambda a, b: not (a and b), 1: lambda a, b: a and b, 2: lambda a, b: a or b,
    3: lambda a, b: a != b, 4: lambda a, b: a == b, 5: lambda a, b: not (a or b),
    6: lambda a, b: (not a) and b, 7: lambda a, b: a and (not b),
    8: lambda a, b: (not a) or b, 9: lambda a, b: a or (not b),
}


def test_gate_truth_tables_toy(toy_keys):
    """All ten bootstrapped gates, all four input rows, under decryption."""
    k = toy_keys
    a = np.array([0, 1, 0, 1] * 10, np.uint8)
    b = np.array([0, 0, 1, 1] * 10, np.uint8)
    ops = np.repeat(np.arange(10), 4).astype(np.int32)
    c1 = O.encrypt_bits(k, a, seed=11)
    c2 = O.encrypt_bits(k, b, seed=12)
    ext, out = O.bootstrap_batch(k, ops, c1, c2)
    want = np.array([TRUTH[int(o)](bool(x), bool(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    assert np.array_equal(O.decrypt_bits(k.tlwe_key, ext), want)
    assert np.array_equal(O.decrypt_bits(k.lwe_key, out), want)
    # output phases sit near +-1/8 with margin
    ph = np.array([O.lwe_phase(k.lwe_key, c) for c in out], dtype=np.uint32)
    mu = np.where(want == 1, 1 << 29, M32 - (1 << 29))
    e = to_i32((ph.astype(np.int64) - mu) % M32)
    assert np.abs(e).max() < (1 << 26)


def test_mux_truth_table_toy(toy_keys):
    """MUX(s, a, b) = s ? a : b for all eight input rows, under decryption,
    with the output phase near +-1/8."""
    k = toy_keys
    rows = np.array(list(itertools.product([0, 1], repeat=3)) * 3, np.uint8)
    s, a, b = rows[:, 0], rows[:, 1], rows[:, 2]
    cs = O.encrypt_bits(k, s, seed=31)
    ca = O.encrypt_bits(k, a, seed=32)
    cb = O.encrypt_bits(k, b, seed=33)
    out = O.mux_batch(k, cs, ca, cb)
    want = np.where(s == 1, a, b).astype(np.uint8)
    assert np.array_equal(O.decrypt_bits(k.lwe_key, out), want)
    ph = np.array([O.lwe_phase(k.lwe_key, c) for c in out], dtype=np.uint32)
    mu = np.where(want == 1, 1 << 29, M32 - (1 << 29))
    assert np.abs(to_i32((ph.astype(np.int64) - mu) % M32)).max() < (1 << 26)


# ------------------------------------------------------------------ noiseless exactness
FULL = O.Params(n=64, N=256, l=4, bgbit=8, t=16, basebit=2, sigma_lwe=0.0, sigma_ks=0.0, sigma_bk=0.0)


@pytest.fixture(scope="module")
def full_keys():
    return O.keygen(FULL, 77)


def clear_rotation_phase(k, bar):
    """phi-bar = b-bar - sum abar_i s_i (mod 2N), then X^{-phi-bar} * v."""
    p = k.params
    n, N = p.n, p.N
    phib = (int(bar[n]) - sum(int(bar[i]) * int(k.lwe_key[i]) for i in range(n))) % (2 * N)
    v = np.full(N, 1 << 29, dtype=np.uint32)
    return negacyclic_ref(monomial((2 * N - phib) % (2 * N), N), v)


def test_blind_rotation_exact_without_noise(full_keys):
    """With sigma = 0 and an exact 32-bit gadget (l*Bgbit = 32) the external
    product is exact, so the final accumulator phase is exactly X^{-phibar} v."""
    k = full_keys
    p = k.params
    rng = np.random.default_rng(8)
    bars = rng.integers(0, 2 * p.N, (6, p.n + 1)).astype(np.int32)
    bars[0, :p.n] = 0                       # only the body: ACC = X^{-b} v
    bars[1, 3] = 0
    accs = O.blind_rotate_batch(k, bars)
    for g in range(bars.shape[0]):
        ph = O.tlwe_phase(k.tlwe_key, accs[g])
        assert np.array_equal(ph, clear_rotation_phase(k, bars[g]))


def test_extraction_exact(full_keys):
    k = full_keys
    rng = np.random.default_rng(9)
    N = k.params.N
    acc = rng.integers(0, M32, (2, N)).astype(np.uint32)
    ext = O.sample_extract(acc)
    ph_acc = (acc[1].astype(np.int64) - negacyclic_ref(acc[0], k.tlwe_key).astype(np.int64)) % M32
    assert O.lwe_phase(k.tlwe_key, ext) == int(ph_acc[0])


def test_key_switch_exact_full_precision(full_keys):
    k = full_keys
    rng = np.random.default_rng(10)
    N = k.params.N
    for _ in range(3):
        ext = rng.integers(0, M32, N + 1).astype(np.uint32)
        out = O.key_switch(k, ext)
        assert O.lwe_phase(k.lwe_key, out) == O.lwe_phase(k.tlwe_key, ext)


def test_whole_gate_exact_without_noise(full_keys):
    """Noiseless, full precision: every output phase is exactly +-1/8."""
    k = full_keys
    a = np.array([0, 1, 0, 1] * 4, np.uint8)
    b = np.array([0, 0, 1, 1] * 4, np.uint8)
    ops = np.array([0] * 4 + [1] * 4 + [2] * 4 + [3] * 4, np.int32)
    c1 = O.encrypt_bits(k, a, seed=1)
    c2 = O.encrypt_bits(k, b, seed=2)
    ext, out = O.bootstrap_batch(k, ops, c1, c2)
    want = np.array([TRUTH[int(o)](bool(x), bool(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    for g in range(16):
        mu = (1 << 29) if want[g] else M32 - (1 << 29)
        assert O.lwe_phase(k.lwe_key, out[g]) == mu
        assert O.lwe_phase(k.tlwe_key, ext[g]) == mu


def test_blind_rotation_within_rounding_bound():
    """sigma = 0 but the standard gadget (l = 3, Bgbit = 7): each step adds at
    most (1 + |S|) * 2^(31 - l*Bgbit) of rounding error."""
    p = O.Params(n=32, N=256, sigma_lwe=0.0, sigma_ks=0.0, sigma_bk=0.0)
    k = O.keygen(p, 5)
    rng = np.random.default_rng(12)
    bars = rng.integers(0, 2 * p.N, (4, p.n + 1)).astype(np.int32)
    accs = O.blind_rotate_batch(k, bars)
    bound = p.n * (1 + int(k.tlwe_key.sum())) * (1 << (31 - p.l * p.bgbit))
    for g in range(4):
        err = to_i32((O.tlwe_phase(k.tlwe_key, accs[g]).astype(np.int64)
                      - clear_rotation_phase(k, bars[g]).astype(np.int64)) % M32)
        assert np.abs(err).max() <= bound
        assert np.abs(err).max() > 0          # the rounding really happens


# ------------------------------------------------------------------ noise vs closed form
def digit_second_moment(bgbit):
    bg = 1 << bgbit
    d = np.arange(-bg // 2, bg // 2, dtype=np.float64)
    return (d ** 2).mean()


def test_blind_rotation_noise_variance(toy_keys):
    """Var of the accumulator phase error per coefficient (units of 2^-32):
    sum over steps of 2 l N E[d^2] sigma_bk^2 + s_i (1+|S|) Var(eps)."""
    k = toy_keys
    p = k.params
    rng = np.random.default_rng(13)
    bars = rng.integers(1, 2 * p.N, (8, p.n + 1)).astype(np.int32)
    accs = O.blind_rotate_batch(k, bars)
    errs = []
    for g in range(bars.shape[0]):
        e = to_i32((O.tlwe_phase(k.tlwe_key, accs[g]).astype(np.int64)
                    - clear_rotation_phase(k, bars[g]).astype(np.int64)) % M32)
        errs.append(e)
    e = np.concatenate(errs).astype(np.float64)
    sig = p.sigma_bk * 2.0 ** 32
    q = 2.0 ** (32 - p.l * p.bgbit)
    var_eps = (q * q - 1) / 12.0
    want = p.n * 2 * p.l * p.N * digit_second_moment(p.bgbit) * sig ** 2 \
        + int(k.lwe_key.sum()) * (1 + int(k.tlwe_key.sum())) * var_eps
    assert e.var() == pytest.approx(want, rel=0.10)
    assert abs(e.mean()) < 5 * np.sqrt(want / e.size)


def test_key_switch_noise_variance(toy_keys):
    """Var of the key-switching error over random inputs, for this fixed key:
    the rounded-off low bits weighted by the key, plus, for every (i, j), the
    variance of the row noise picked by a uniform digit in {0..3} (digit 0
    adds nothing). Averaged over keys this is the usual N t (3/4) sigma^2
    minus the key-dependent mean."""
    k = toy_keys
    p = k.params
    rng = np.random.default_rng(14)
    cnt = 4096
    exts = rng.integers(0, M32, (cnt, p.N + 1)).astype(np.uint32)
    outs = O.key_switch_batch(k, exts)
    sext = k.tlwe_key.astype(np.int64)
    ph_in = (exts[:, p.N].astype(np.int64) - (exts[:, :p.N].astype(np.int64) * sext[None, :]).sum(1)) % M32
    ph_out = (outs[:, p.n].astype(np.int64) - (outs[:, :p.n].astype(np.int64) * k.lwe_key[None, :].astype(np.int64)).sum(1)) % M32
    e = to_i32((ph_out - ph_in) % M32).astype(np.float64)
    # noise of every key-switching row, recovered with the secret key
    ksk = k.ksk.astype(np.int64)
    ph_rows = (ksk[..., p.n] - (ksk[..., :p.n] * k.lwe_key.astype(np.int64)).sum(-1)) % M32
    v = np.arange(1 << p.basebit, dtype=np.int64)
    shift = 32 - (np.arange(p.t, dtype=np.int64) + 1) * p.basebit
    mu = (v[None, None, :] * sext[:, None, None]) << shift[None, :, None]
    row_noise = to_i32((ph_rows - mu) % M32).astype(np.float64)
    row_noise[..., 0] = 0.0                      # digit 0 subtracts nothing
    var_rows = (row_noise ** 2).mean(-1) - row_noise.mean(-1) ** 2
    q = 2.0 ** (32 - p.t * p.basebit)
    want = var_rows.sum() + int(k.tlwe_key.sum()) * (q * q - 1) / 12.0
    assert e.var() == pytest.approx(want, rel=0.10)
    # and the key-averaged closed form is within its own spread
    avg = p.N * p.t * 0.75 * (p.sigma_ks * 2.0 ** 32) ** 2
    assert (row_noise[..., 1:] ** 2).mean() * 0.75 * p.N * p.t == pytest.approx(avg, rel=0.05)


def test_mux_exact_without_noise(full_keys):
    """Noiseless, full precision: the multiplexer's output phase is exactly
    +1/8 for a selected true input and -1/8 otherwise (pins the two gate
    choices and the added 1/8)."""
    k = full_keys
    rows = np.array(list(itertools.product([0, 1], repeat=3)), np.uint8)
    s, a, b = rows[:, 0], rows[:, 1], rows[:, 2]
    out = O.mux_batch(k, O.encrypt_bits(k, s, seed=3), O.encrypt_bits(k, a, seed=4), O.encrypt_bits(k, b, seed=5))
    for g in range(8):
        mu = (1 << 29) if (a[g] if s[g] else b[g]) else M32 - (1 << 29)
        assert O.lwe_phase(k.lwe_key, out[g]) == mu

