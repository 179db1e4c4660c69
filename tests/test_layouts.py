"""Data-layout identities the kernels rely on, checked on the CPU against
plain definitions (no GPU).

* FFT latency kernel: each accumulator component is stored as one record per
  coefficient pair (j, j + N/2) holding (R_j, R_{j+N/2}, ACC_j, ACC_{j+N/2})
  with R = X^a ACC. The update waves place ACC_j and ACC_{j+N/2} in record
  r = (j + a) mod N/2 as (v0, v1), (-v1, v0), (-v0, -v1) or (v1, -v0) by
  quadrant k / (N/2), k = (j + a) mod 2N. Checked against the negacyclic
  rotation X^a P (coefficient m of X^a P is P_{m-a}, negated when the index
  wraps past N).
* Signed digits: with the offset added, a 7-bit field holds d + 64; flipping
  its top bit and reading it as 7-bit two's complement gives d (the FFT
  throughput kernel's sign-extending extract).
"""
import numpy as np
import pytest

M32 = 1 << 32


def negacyclic_rotate(p, a):
    N = len(p)
    out = np.zeros(N, np.uint64)
    for m in range(N):
        t = (m - a) % (2 * N)
        out[m] = p[t] if t < N else (M32 - p[t - N]) % M32
    return out


def records_after_update(acc, a):
    """What the update waves write: record r -> (R_r, R_{r+N/2})."""
    N = len(acc)
    H = N // 2
    rec = {}
    for j in range(H):
        v0, v1 = int(acc[j]), int(acc[j + H])
        k = (j + a) % (2 * N)
        q = k // H
        f, s = {0: (v0, v1), 1: ((M32 - v1) % M32, v0), 2: ((M32 - v0) % M32, (M32 - v1) % M32),
                3: (v1, (M32 - v0) % M32)}[q]
        r = k % H
        assert r not in rec
        rec[r] = (f, s)
    return rec


@pytest.mark.parametrize("N", [8, 64, 1024])
def test_rotated_records_equal_negacyclic_rotation(N):
    rng = np.random.default_rng(N)
    H = N // 2
    for a in list(range(0, 2 * N, max(1, N // 16))) + [1, N - 1, N, N + 1, 2 * N - 1]:
        acc = rng.integers(0, M32, N, dtype=np.uint64)
        rot = negacyclic_rotate(acc, a)
        rec = records_after_update(acc, a)
        assert sorted(rec) == list(range(H))
        for r, (f, s) in rec.items():
            assert (f, s) == (int(rot[r]), int(rot[r + H])), (N, a, r)


def test_rotation_by_zero_and_by_n():
    acc = np.arange(16, dtype=np.uint64) + 5
    assert np.array_equal(negacyclic_rotate(acc, 0), acc)
    assert np.array_equal(negacyclic_rotate(acc, 16), (M32 - acc) % M32)


def test_signed_digit_by_flipped_top_bit():
    offset, flips = 0x81020400, 0x81020000
    rng = np.random.default_rng(0)
    for x in list(rng.integers(0, M32, 20000, dtype=np.uint64)) + [0, M32 - 1, 1 << 31, (1 << 31) - 1]:
        y = (int(x) + offset) % M32
        for sh in (25, 18, 11):
            u = (y >> sh) & 127
            f = ((y ^ flips) >> sh) & 127
            assert (f - 128 if f >= 64 else f) == u - 64
