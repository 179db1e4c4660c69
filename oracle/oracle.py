"""ctypes binding of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module. The product
path (``paper_2101_03403_amd``) never imports it.

The oracle follows the standard TFHE gate-bootstrapping definitions that the
paper (CryptoEmu, arXiv 2101.03403, Sec. 3 and Table "TFHEbenchmark") relies on;
every routine is documented in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("N", C.c_int32), ("k", C.c_int32), ("l", C.c_int32),
                ("bgbit", C.c_int32), ("t", C.c_int32), ("basebit", C.c_int32), ("pad", C.c_int32),
                ("sigma_lwe", C.c_double), ("sigma_ks", C.c_double), ("sigma_bk", C.c_double)]


@dataclass(frozen=True)
class Params:
    n: int
    N: int
    l: int = 3
    bgbit: int = 7
    t: int = 8
    basebit: int = 2
    sigma_lwe: float = 2.0 ** -15
    sigma_ks: float = 2.0 ** -15
    sigma_bk: float = 2.0 ** -25

    def c(self) -> OrParams:
        return OrParams(self.n, self.N, 1, self.l, self.bgbit, self.t, self.basebit, 0,
                        self.sigma_lwe, self.sigma_ks, self.sigma_bk)


STANDARD = Params(n=630, N=1024)
TOY = Params(n=256, N=512)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        pp = C.POINTER(OrParams)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_gauss_from_block.argtypes = [u32p, C.c_double]
        L.or_gauss_from_block.restype = C.c_int64
        L.or_negacyclic_mul.argtypes = [C.c_int32, u32p, u32p, u32p]
        L.or_rotate.argtypes = [C.c_int32, C.c_int32, u32p, u32p]
        L.or_modswitch.argtypes = [C.c_uint32, C.c_int32]
        L.or_modswitch.restype = C.c_int32
        L.or_decompose.argtypes = [C.c_uint32, C.c_int32, C.c_int32, i32p]
        L.or_keygen.argtypes = [pp, C.c_uint64, i32p, i32p, u32p, u32p]
        L.or_lwe_encrypt.argtypes = [C.c_int32, i32p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_double, u32p]
        L.or_encrypt_bits.argtypes = [pp, i32p, C.c_uint64, C.c_uint64, u8p, C.c_int64, u32p]
        L.or_lwe_phase.argtypes = [C.c_int32, i32p, u32p]
        L.or_lwe_phase.restype = C.c_uint32
        L.or_decrypt_bits.argtypes = [C.c_int32, i32p, u32p, C.c_int64, u8p]
        L.or_tlwe_phase.argtypes = [C.c_int32, i32p, u32p, u32p]
        L.or_gate_lincomb.argtypes = [C.c_int32, C.c_int32, u32p, u32p, u32p]
        L.or_gate_lincomb.restype = C.c_int32
        L.or_blind_rotate.argtypes = [pp, u32p, i32p, u32p]
        L.or_sample_extract.argtypes = [C.c_int32, u32p, u32p]
        L.or_key_switch.argtypes = [pp, u32p, u32p, u32p]
        L.or_bootstrap_batch.argtypes = [pp, u32p, u32p, i32p, u32p, u32p, C.c_int64, C.c_void_p, C.c_void_p]
        L.or_bootstrap_batch.restype = C.c_int32
        L.or_blind_rotate_batch.argtypes = [pp, u32p, i32p, C.c_int64, u32p]
        L.or_key_switch_batch.argtypes = [pp, u32p, u32p, C.c_int64, u32p]
        L.or_modswitch_array.argtypes = [u32p, C.c_int64, C.c_int32, i32p]
        L.or_decompose_array.argtypes = [u32p, C.c_int64, C.c_int32, C.c_int32, i32p]
        L.or_gauss_array.argtypes = [C.c_uint64, C.c_int64, C.c_double, i64p]
        L.or_num_threads.restype = C.c_int32
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a).astype(np.uint32, copy=False))


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_u32(ctr), _u32(key), out)
    return out


def negacyclic_mul(P, Q) -> np.ndarray:
    P, Q = _u32(P), _u32(Q)
    out = np.zeros(P.shape[0], np.uint32)
    lib().or_negacyclic_mul(P.shape[0], P, Q, out)
    return out


def rotate(a: int, P) -> np.ndarray:
    P = _u32(P)
    out = np.zeros_like(P)
    lib().or_rotate(P.shape[0], int(a), P, out)
    return out


def modswitch(x: int, two_n: int) -> int:
    return int(lib().or_modswitch(int(x) & 0xFFFFFFFF, int(two_n)))


def modswitch_array(x, two_n: int) -> np.ndarray:
    x = _u32(x)
    out = np.zeros(x.shape[0], np.int32)
    lib().or_modswitch_array(x, x.shape[0], int(two_n), out)
    return out


def decompose(x: int, l: int, bgbit: int) -> np.ndarray:
    d = np.zeros(l, np.int32)
    lib().or_decompose(int(x) & 0xFFFFFFFF, l, bgbit, d)
    return d


def decompose_array(x, l: int, bgbit: int) -> np.ndarray:
    x = _u32(x)
    d = np.zeros((x.shape[0], l), np.int32)
    lib().or_decompose_array(x, x.shape[0], l, bgbit, d)
    return d


def gauss_array(seed: int, count: int, sigma: float) -> np.ndarray:
    out = np.zeros(count, np.int64)
    lib().or_gauss_array(seed, count, sigma, out)
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- keys
@dataclass
class Keys:
    params: Params
    lwe_key: np.ndarray     # [n] int32 in {0,1}
    tlwe_key: np.ndarray    # [N] int32 in {0,1}
    bk: np.ndarray          # [n][2l][2][N] uint32
    ksk: np.ndarray         # [N][t][base][n+1] uint32


def keygen(p: Params, seed: int) -> Keys:
    lwe = np.zeros(p.n, np.int32)
    tlwe = np.zeros(p.N, np.int32)
    bk = np.zeros((p.n, 2 * p.l, 2, p.N), np.uint32)
    ksk = np.zeros((p.N, p.t, 1 << p.basebit, p.n + 1), np.uint32)
    cp = p.c()
    lib().or_keygen(C.byref(cp), seed, lwe, tlwe, bk, ksk)
    return Keys(p, lwe, tlwe, bk, ksk)


def encrypt_bits(keys: Keys, bits, seed: int, first_index: int = 0) -> np.ndarray:
    bits = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    p = keys.params
    out = np.zeros((bits.shape[0], p.n + 1), np.uint32)
    cp = p.c()
    lib().or_encrypt_bits(C.byref(cp), keys.lwe_key, seed, first_index, bits, bits.shape[0], out)
    return out


def lwe_encrypt(key, seed: int, index: int, mu: int, sigma: float) -> np.ndarray:
    key = np.ascontiguousarray(key, dtype=np.int32)
    out = np.zeros(key.shape[0] + 1, np.uint32)
    lib().or_lwe_encrypt(key.shape[0], key, seed, index, int(mu) & 0xFFFFFFFF, sigma, out)
    return out


def lwe_phase(key, ct) -> int:
    key = np.ascontiguousarray(key, dtype=np.int32)
    return int(lib().or_lwe_phase(key.shape[0], key, _u32(ct)))


def decrypt_bits(key, cts) -> np.ndarray:
    key = np.ascontiguousarray(key, dtype=np.int32)
    cts = _u32(cts).reshape(-1, key.shape[0] + 1)
    out = np.zeros(cts.shape[0], np.uint8)
    lib().or_decrypt_bits(key.shape[0], key, cts, cts.shape[0], out)
    return out


def tlwe_phase(tlwe_key, acc) -> np.ndarray:
    acc = _u32(acc).reshape(-1)
    N = acc.shape[0] // 2
    out = np.zeros(N, np.uint32)
    lib().or_tlwe_phase(N, np.ascontiguousarray(tlwe_key, np.int32), acc, out)
    return out


# ---------------------------------------------------------------- gate pieces
def gate_lincomb(op: int, c1, c2) -> np.ndarray:
    c1, c2 = _u32(c1), _u32(c2)
    out = np.zeros_like(c1)
    rc = lib().or_gate_lincomb(c1.shape[0] - 1, int(op), c1, c2, out)
    if rc != 0:
        raise ValueError(f"unknown gate op {op}")
    return out


def blind_rotate(keys: Keys, bar) -> np.ndarray:
    bar = np.ascontiguousarray(bar, dtype=np.int32)
    out = np.zeros((2, keys.params.N), np.uint32)
    cp = keys.params.c()
    lib().or_blind_rotate(C.byref(cp), keys.bk, bar, out)
    return out


def blind_rotate_batch(keys: Keys, bars) -> np.ndarray:
    bars = np.ascontiguousarray(bars, dtype=np.int32)
    out = np.zeros((bars.shape[0], 2, keys.params.N), np.uint32)
    cp = keys.params.c()
    lib().or_blind_rotate_batch(C.byref(cp), keys.bk, bars, bars.shape[0], out)
    return out


def sample_extract(acc) -> np.ndarray:
    acc = _u32(acc).reshape(-1)
    N = acc.shape[0] // 2
    out = np.zeros(N + 1, np.uint32)
    lib().or_sample_extract(N, acc, out)
    return out


def key_switch(keys: Keys, ext) -> np.ndarray:
    out = np.zeros(keys.params.n + 1, np.uint32)
    cp = keys.params.c()
    lib().or_key_switch(C.byref(cp), keys.ksk, _u32(ext), out)
    return out


def key_switch_batch(keys: Keys, exts) -> np.ndarray:
    exts = _u32(exts)
    out = np.zeros((exts.shape[0], keys.params.n + 1), np.uint32)
    cp = keys.params.c()
    lib().or_key_switch_batch(C.byref(cp), keys.ksk, exts, exts.shape[0], out)
    return out


def bootstrap_batch(keys: Keys, ops, c1s, c2s, want_extracted: bool = True, want_out: bool = True):
    """Returns (extracted [B][N+1] or None, out [B][n+1] or None)."""
    ops = np.ascontiguousarray(ops, dtype=np.int32)
    c1s, c2s = _u32(c1s), _u32(c2s)
    B = ops.shape[0]
    p = keys.params
    ext = np.zeros((B, p.N + 1), np.uint32) if want_extracted else None
    out = np.zeros((B, p.n + 1), np.uint32) if want_out else None
    cp = p.c()
    rc = lib().or_bootstrap_batch(C.byref(cp), keys.bk, keys.ksk, ops, c1s, c2s, B,
                                  ext.ctypes.data if ext is not None else None,
                                  out.ctypes.data if out is not None else None)
    if rc != 0:
        raise ValueError("unknown gate op in batch")
    return ext, out


# ---------------------------------------------------------------- multiplexer
OP_AND, OP_ANDNY = 1, 6


def mux_batch(keys: Keys, sel, c1s, c2s) -> np.ndarray:
    """Homomorphic multiplexer out = sel ? c1 : c2 (Table "TFHEbenchmark":
    MUX, two bootstraps; the FHE MUX select of the barrel shifters, Sec. 5.4),
    in TFHE's form: AND(sel, c1) and ANDNY(sel, c2) are bootstrapped without
    key switching; at most one of them is true, so their extracted samples
    plus the trivial sample (0, ..., 0, 1/8) encrypt +1/8 exactly when the
    selected input is true and -1/8 otherwise; one key switch follows.
    Returns [B][n+1]."""
    sel, c1s, c2s = _u32(sel), _u32(c1s), _u32(c2s)
    B = sel.shape[0]
    N = keys.params.N
    e1, _ = bootstrap_batch(keys, np.full(B, OP_AND, np.int32), sel, c1s, want_out=False)
    e2, _ = bootstrap_batch(keys, np.full(B, OP_ANDNY, np.int32), sel, c2s, want_out=False)
    summed = e1 + e2                      # uint32 arithmetic wraps mod 2^32
    summed[:, N] += np.uint32(1 << 29)
    return key_switch_batch(keys, summed)

