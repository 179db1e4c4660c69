"""Python binding of libcemu (argument marshalling only).

Every step of gate bootstrapping runs in the HIP kernels of ``libcemu.so``;
this module only converts arguments and checks return codes. Device buffers
are torch tensors on the GPU that holds the cloud key; torch is used for
device memory and streams only. Torus32 words are carried in ``torch.int32``
tensors (same bits as uint32).

The library must be built (``python -m paper_2101_03403_amd.build``); there is
no fallback: if ``libcemu.so`` is missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CEMU_LIB") or os.path.join(HERE, "libcemu.so")

STD, TOY = 0, 1
FORM_INT8, FORM_FFT64 = 0, 1
FORMS = {"int8": FORM_INT8, "fft64": FORM_FFT64}

NAND, AND, OR, XOR, XNOR, NOR, ANDNY, ANDYN, ORNY, ORYN = range(10)
GATE_NAMES = ["NAND", "AND", "OR", "XOR", "XNOR", "NOR", "ANDNY", "ANDYN", "ORNY", "ORYN"]

TRUE_T32 = 0x20000000
FALSE_T32 = 0xE0000000


class CemuError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cemu error {code}: {msg}")
        self.code = code


class Tuning(C.Structure):
    _fields_ = [("int8_waves", C.c_int32), ("fft_gates_per_wg", C.c_int32), ("int8_gates_per_wg", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class Params(C.Structure):
    _fields_ = [("n", C.c_int32), ("N", C.c_int32), ("k", C.c_int32), ("l", C.c_int32),
                ("bgbit", C.c_int32), ("t", C.c_int32), ("basebit", C.c_int32), ("reserved", C.c_int32),
                ("sigma_lwe", C.c_double), ("sigma_ks", C.c_double), ("sigma_bk", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


EXPORTED = [
    "cemu_params_default", "cemu_keygen", "cemu_secret_params", "cemu_cloud_params", "cemu_encrypt",
    "cemu_decrypt", "cemu_decrypt_extracted", "cemu_phase", "cemu_bootstrap_gates", "cemu_bootstrap_gates_noalloc",
    "cemu_blind_rotate_extract", "cemu_key_switch", "cemu_mux", "cemu_bootstrap_level", "cemu_lwe_not", "cemu_lwe_copy", "cemu_lwe_constant",
    "cemu_export_keys", "cemu_free_secret_key", "cemu_free_cloud_key", "cemu_last_error", "cemu_version",
    "cemu_profile_enable", "cemu_profile_read", "cemu_get_tuning", "cemu_set_tuning",
    "cemu_measure_peaks", "cemu_measure_lds",
]
PROFILE_KINDS = ["lincomb_modswitch", "blind_rotate_int8", "blind_rotate_fft64", "key_switch"]

_lib = None


def lib() -> C.CDLL:
    """Load libcemu.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_03403_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    pp = C.POINTER(Params)
    L.cemu_params_default.argtypes = [pp, C.c_int]
    L.cemu_keygen.argtypes = [pp, C.c_uint64, C.POINTER(vp), C.POINTER(vp)]
    L.cemu_secret_params.argtypes = [vp, pp]
    L.cemu_cloud_params.argtypes = [vp, pp]
    L.cemu_encrypt.argtypes = [vp, vp, i64, C.c_uint64, C.c_uint64, vp]
    L.cemu_decrypt.argtypes = [vp, vp, i64, vp]
    L.cemu_decrypt_extracted.argtypes = [vp, vp, i64, vp]
    L.cemu_phase.argtypes = [vp, C.c_int, vp, i64, vp]
    L.cemu_bootstrap_gates.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, i64, vp]
    L.cemu_bootstrap_gates_noalloc.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, i64, vp]
    L.cemu_measure_peaks.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    L.cemu_measure_lds.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    L.cemu_blind_rotate_extract.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, i64, vp]
    L.cemu_key_switch.argtypes = [vp, vp, vp, i64, vp]
    L.cemu_mux.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, i64, vp]
    L.cemu_bootstrap_level.argtypes = [vp, C.c_int, vp, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
    L.cemu_lwe_not.argtypes = [i32, vp, vp, vp, vp, i64, vp]
    L.cemu_lwe_copy.argtypes = [i32, vp, vp, vp, vp, i64, vp]
    L.cemu_lwe_constant.argtypes = [i32, vp, vp, vp, i64, vp]
    L.cemu_export_keys.argtypes = [vp, vp, vp, vp, vp, vp]
    L.cemu_free_secret_key.argtypes = [vp]
    L.cemu_free_secret_key.restype = None
    L.cemu_free_cloud_key.argtypes = [vp]
    L.cemu_free_cloud_key.restype = None
    L.cemu_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.cemu_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.cemu_profile_enable.argtypes = [vp, C.c_int]
    L.cemu_profile_read.argtypes = [vp, vp, vp]
    L.cemu_last_error.restype = C.c_char_p
    L.cemu_version.restype = C.c_char_p
    for name in EXPORTED:
        getattr(L, name)  # raises AttributeError if a declared entry point is missing
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise CemuError(rc, lib().cemu_last_error().decode())


def params(which=STD, **overrides) -> Params:
    p = Params()
    _check(lib().cemu_params_default(C.byref(p), int(which)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t, what="tensor", kind=None, rows=None, width=None, min_rows=None):
    """Device pointer of a contiguous GPU tensor (or None), after checking what
    the library will read it as: kind "words" (int32 / uint32 ciphertext
    words), "rows" (int32 row indices) or "u8" (op codes, bits); `rows` = the
    exact length of a 1-D array; `width` = the row length of a 2-D array,
    `min_rows` its least number of rows. A mismatch raises instead of letting
    the device read the memory as something else."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if kind is not None:
        import torch
        ok = {"words": (torch.int32, getattr(torch, "uint32", torch.int32)), "rows": (torch.int32,),
              "u8": (torch.uint8,)}[kind]
        if t.dtype not in ok:
            raise TypeError(f"{what}: dtype {t.dtype}, expected {' or '.join(str(d) for d in ok)}")
    if rows is not None and (t.dim() != 1 or t.shape[0] != rows):
        raise ValueError(f"{what}: expected shape [{rows}], got {list(t.shape)}")
    if min_rows is not None and (t.shape[0] if t.dim() else 0) < min_rows:
        raise ValueError(f"{what}: needs at least {min_rows} rows, got shape {list(t.shape)}")
    if width is not None and t.numel() > 0 and (t.dim() != 2 or t.shape[1] != width):
        raise ValueError(f"{what}: expected rows of {width} words, got shape {list(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclass
class Keys:
    """Secret key (host) and cloud key (device) handles."""
    sk: C.c_void_p
    ck: C.c_void_p
    params: Params

    @property
    def n(self) -> int:
        return self.params.n

    @property
    def N(self) -> int:
        return self.params.N

    def free(self):
        if self.sk:
            lib().cemu_free_secret_key(self.sk)
            self.sk = None
        if self.ck:
            lib().cemu_free_cloud_key(self.ck)
            self.ck = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -------------------------------------------------------------- host side
    def encrypt(self, bits, seed: int, first_index: int = 0) -> np.ndarray:
        bits = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
        out = np.zeros((bits.shape[0], self.n + 1), np.uint32)
        _check(lib().cemu_encrypt(self.sk, _np_ptr(bits), bits.shape[0], seed, first_index, _np_ptr(out)))
        return out

    def decrypt(self, cts) -> np.ndarray:
        cts = np.ascontiguousarray(np.asarray(cts).view(np.uint32).reshape(-1, self.n + 1))
        out = np.zeros(cts.shape[0], np.uint8)
        _check(lib().cemu_decrypt(self.sk, _np_ptr(cts), cts.shape[0], _np_ptr(out)))
        return out

    def decrypt_extracted(self, cts) -> np.ndarray:
        cts = np.ascontiguousarray(np.asarray(cts).view(np.uint32).reshape(-1, self.N + 1))
        out = np.zeros(cts.shape[0], np.uint8)
        _check(lib().cemu_decrypt_extracted(self.sk, _np_ptr(cts), cts.shape[0], _np_ptr(out)))
        return out

    def phase(self, cts, extracted: bool = False) -> np.ndarray:
        d = self.N if extracted else self.n
        cts = np.ascontiguousarray(np.asarray(cts).view(np.uint32).reshape(-1, d + 1))
        out = np.zeros(cts.shape[0], np.uint32)
        _check(lib().cemu_phase(self.sk, int(extracted), _np_ptr(cts), cts.shape[0], _np_ptr(out)))
        return out

    def export(self, bk: bool = True, ksk: bool = True) -> dict:
        p = self.params
        lwe = np.zeros(p.n, np.int32)
        tlwe = np.zeros(p.N, np.int32)
        bka = np.zeros((p.n, 2 * p.l, 2, p.N), np.uint32) if bk else None
        ksa = np.zeros((p.N, p.t, 1 << p.basebit, p.n + 1), np.uint32) if ksk else None
        _check(lib().cemu_export_keys(self.sk, self.ck, _np_ptr(lwe), _np_ptr(tlwe),
                                      _np_ptr(bka) if bk else None, _np_ptr(ksa) if ksk else None))
        return {"lwe_key": lwe, "tlwe_key": tlwe, "bk": bka, "ksk": ksa}


def get_tuning(keys: Keys) -> dict:
    t = Tuning()
    _check(lib().cemu_get_tuning(keys.ck, C.byref(t)))
    return {"int8_waves": t.int8_waves, "fft_gates_per_wg": t.fft_gates_per_wg,
            "int8_gates_per_wg": t.int8_gates_per_wg}


def set_tuning(keys: Keys, int8_waves: int | None = None, fft_gates_per_wg: int | None = None,
               int8_gates_per_wg: int | None = None):
    """Change the key's launch shapes; arguments left as None keep their value.
    A tuning dict that names only some fields (as the autotuner's candidates
    do) therefore leaves the others as they were: callers that switch shapes
    pass every field they rely on."""
    cur = get_tuning(keys)
    t = Tuning()
    t.int8_waves = cur["int8_waves"] if int8_waves is None else int8_waves
    t.fft_gates_per_wg = cur["fft_gates_per_wg"] if fft_gates_per_wg is None else fft_gates_per_wg
    t.int8_gates_per_wg = cur["int8_gates_per_wg"] if int8_gates_per_wg is None else int8_gates_per_wg
    _check(lib().cemu_set_tuning(keys.ck, C.byref(t)))


def profile_enable(keys: Keys, enable: bool = True):
    """Bracket every library kernel launch with hipEvents (see include/cemu.h)."""
    _check(lib().cemu_profile_enable(keys.ck, int(enable)))


def profile_read(keys: Keys) -> dict:
    """{kind: (total_ms, launches)} since the last read; waits for the events."""
    ms = np.zeros(len(PROFILE_KINDS), np.float64)
    cnt = np.zeros(len(PROFILE_KINDS), np.int64)
    _check(lib().cemu_profile_read(keys.ck, _np_ptr(ms), _np_ptr(cnt)))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_KINDS)}


def keygen(p=STD, seed: int = 0) -> Keys:
    """Generate keys; the cloud key goes to the current torch/HIP device."""
    if not isinstance(p, Params):
        p = params(p)
    sk, ck = C.c_void_p(), C.c_void_p()
    _check(lib().cemu_keygen(C.byref(p), seed, C.byref(sk), C.byref(ck)))
    return Keys(sk, ck, p)


# ------------------------------------------------------------------ device side
def _gate_args(keys, ops, pool_in, ia, ib, B):
    n1 = keys.n + 1
    return (_dptr(ops, "ops", "u8", rows=B), _dptr(pool_in, "pool_in", "words", width=n1, min_rows=1 if B else None),
            _dptr(ia, "ia", "rows", rows=B), _dptr(ib, "ib", "rows", rows=B))


def bootstrap_gates(keys: Keys, ops, pool_in, ia, ib, pool_out, io=None, form="int8", stream=None):
    """Batched bootstrapped gates; see cemu_bootstrap_gates in include/cemu.h."""
    B = int(ops.shape[0])
    _check(lib().cemu_bootstrap_gates(keys.ck, FORMS[form], *_gate_args(keys, ops, pool_in, ia, ib, B),
                                      _dptr(io, "io", "rows", rows=B),
                                      _dptr(pool_out, "pool_out", "words", width=keys.n + 1,
                                            min_rows=B if io is None else None),
                                      B, _stream(stream)))


def bootstrap_gates_noalloc(keys: Keys, ops, pool_in, ia, ib, pool_out, io=None, form="int8", stream=None):
    """The allocation-free variant (at most NOALLOC_MAX_GATES gates; calls on
    one GPU must not overlap); see cemu_bootstrap_gates_noalloc."""
    B = int(ops.shape[0])
    _check(lib().cemu_bootstrap_gates_noalloc(keys.ck, FORMS[form], *_gate_args(keys, ops, pool_in, ia, ib, B),
                                              _dptr(io, "io", "rows", rows=B),
                                              _dptr(pool_out, "pool_out", "words", width=keys.n + 1,
                                                    min_rows=B if io is None else None),
                                              B, _stream(stream)))


NOALLOC_MAX_GATES = 4096


def blind_rotate_extract(keys: Keys, ops, pool_in, ia, ib, out_N, form="int8", stream=None):
    B = int(ops.shape[0])
    _check(lib().cemu_blind_rotate_extract(keys.ck, FORMS[form], *_gate_args(keys, ops, pool_in, ia, ib, B),
                                           _dptr(out_N, "out_N", "words", width=keys.N + 1, min_rows=B),
                                           B, _stream(stream)))


def key_switch(keys: Keys, in_N, out_n, stream=None):
    B = int(in_N.shape[0])
    _check(lib().cemu_key_switch(keys.ck, _dptr(in_N, "in_N", "words", width=keys.N + 1, min_rows=B),
                                 _dptr(out_n, "out_n", "words", width=keys.n + 1, min_rows=B), B, _stream(stream)))


def mux(keys: Keys, pool_in, isel, ia, ib, pool_out, io=None, form="int8", stream=None):
    """Batched homomorphic MUX (isel ? ia : ib); see cemu_mux in include/cemu.h."""
    B = int(isel.shape[0])
    n1 = keys.n + 1
    _check(lib().cemu_mux(keys.ck, FORMS[form], _dptr(pool_in, "pool_in", "words", width=n1, min_rows=1 if B else None),
                          _dptr(isel, "isel", "rows", rows=B), _dptr(ia, "ia", "rows", rows=B),
                          _dptr(ib, "ib", "rows", rows=B), _dptr(io, "io", "rows", rows=B),
                          _dptr(pool_out, "pool_out", "words", width=n1, min_rows=B if io is None else None),
                          B, _stream(stream)))


def bootstrap_level(keys: Keys, pool_in, gates, muxes, pool_out, io=None, form="int8", stream=None):
    """A circuit level of G gates and M MUXes in one blind-rotation launch;
    gates = (ops, ia, ib) or None, muxes = (isel, ia, ib) or None, io = output
    rows [G + M] (gates first); see cemu_bootstrap_level in include/cemu.h."""
    ops, ia, ib = gates if gates is not None else (None, None, None)
    ms, ma, mb = muxes if muxes is not None else (None, None, None)
    G = int(ops.shape[0]) if ops is not None else 0
    M = int(ms.shape[0]) if ms is not None else 0
    n1 = keys.n + 1
    _check(lib().cemu_bootstrap_level(keys.ck, FORMS[form],
                                      _dptr(pool_in, "pool_in", "words", width=n1, min_rows=1 if G + M else None),
                                      _dptr(ops, "ops", "u8", rows=G), _dptr(ia, "ia", "rows", rows=G),
                                      _dptr(ib, "ib", "rows", rows=G), G,
                                      _dptr(ms, "isel", "rows", rows=M), _dptr(ma, "ma", "rows", rows=M),
                                      _dptr(mb, "mb", "rows", rows=M), M, _dptr(io, "io", "rows", rows=G + M),
                                      _dptr(pool_out, "pool_out", "words", width=n1,
                                            min_rows=G + M if io is None else None),
                                      _stream(stream)))


def _rowwise_args(n, pool_in, src, pool_out, dst):
    cnt = int(src.shape[0])
    return (_dptr(pool_in, "pool_in", "words", width=n + 1, min_rows=1 if cnt else None),
            _dptr(src, "src", "rows", rows=cnt),
            _dptr(pool_out, "pool_out", "words", width=n + 1), _dptr(dst, "dst", "rows", rows=cnt), cnt)


def lwe_not(n: int, pool_in, src, pool_out, dst, stream=None):
    _check(lib().cemu_lwe_not(n, *_rowwise_args(n, pool_in, src, pool_out, dst), _stream(stream)))


def lwe_copy(n: int, pool_in, src, pool_out, dst, stream=None):
    _check(lib().cemu_lwe_copy(n, *_rowwise_args(n, pool_in, src, pool_out, dst), _stream(stream)))


def lwe_constant(n: int, bits, pool_out, dst, stream=None):
    cnt = int(dst.shape[0])
    _check(lib().cemu_lwe_constant(n, _dptr(bits, "bits", "u8", rows=cnt),
                                   _dptr(pool_out, "pool_out", "words", width=n + 1),
                                   _dptr(dst, "dst", "rows", rows=cnt), cnt, _stream(stream)))


def measure_peaks(stream=None) -> dict:
    """FP64 FMA and int8 MFMA peak rates of the current GPU at the throughput
    kernels' occupancy; see cemu_measure_peaks in include/cemu_measure.h."""
    f, i = C.c_double(), C.c_double()
    _check(lib().cemu_measure_peaks(C.byref(f), C.byref(i), _stream(stream)))
    return {"fp64_flops_per_s": f.value, "int8_ops_per_s": i.value}


def measure_lds(stream=None) -> dict:
    """LDS write and read bandwidth of the current GPU (bytes/s, all compute
    units); see cemu_measure_lds in include/cemu_measure.h."""
    w, r = C.c_double(), C.c_double()
    _check(lib().cemu_measure_lds(C.byref(w), C.byref(r), _stream(stream)))
    return {"lds_write_bytes_per_s": w.value, "lds_read_bytes_per_s": r.value}


def version() -> str:
    return lib().cemu_version().decode()
