"""Autotuner for the batched gate launches.

For a cloud key and a batch size it measures every candidate launch
configuration -- product form (FP64-FFT or int8-MFMA) x its tile choice
(FFT: 8 or 4 gates per workgroup, or the one-gate-per-workgroup latency
kernel; int8: 16 gates or one gate per workgroup, 8 or 4 waves) -- on a
seeded batch of that size that looks like real work (random bits encrypted
under the key, gate types uniform over NAND / AND / OR / XOR, so the
rescaled masks and the digits are uniform as in use; an all-zero batch would
skip every blind-rotation step and time nothing), keeps the fastest, and
caches the choice per
(parameter set, batch-size bucket) in memory and optionally in a JSON file.
Kernel timing uses the library's own HIP-event profiling (cemu_profile_*),
so it measures exactly the blind-rotation + key-switch launches. The choice
only affects speed: every configuration computes the same ciphertexts.

Buckets are powers of two (16 .. 4096); batches above 4096 use the 4096
decision since the kernels then run several full waves of workgroups.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import cemu
from . import workloads as W

CANDIDATES = (
    ("fft64", {"fft_gates_per_wg": 8}),
    ("fft64", {"fft_gates_per_wg": 4}),
    ("fft64", {"fft_gates_per_wg": 1}),
    ("int8", {"int8_waves": 8, "int8_gates_per_wg": 16}),
    ("int8", {"int8_waves": 4, "int8_gates_per_wg": 16}),
    ("int8", {"int8_waves": 8, "int8_gates_per_wg": 1}),
    ("int8", {"int8_waves": 4, "int8_gates_per_wg": 1}),
)
MIN_BUCKET, MAX_BUCKET = 16, 4096


def bucket(B: int) -> int:
    b = MIN_BUCKET
    while b < B and b < MAX_BUCKET:
        b *= 2
    return b


class Autotuner:
    def __init__(self, keys: cemu.Keys, cache_path: str | None = None, forms=("fft64", "int8"), reps: int = 2):
        self.keys = keys
        self.cache_path = cache_path
        self.forms = tuple(forms)
        self.reps = reps
        self.table = {}
        self.measurements = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = {int(k): tuple(v) for k, v in json.load(f).get(self._pkey(), {}).items()}

    def _pkey(self) -> str:
        p = self.keys.params
        return f"n{p.n}_N{p.N}_l{p.l}_bg{p.bgbit}_t{p.t}_bb{p.basebit}"

    def _save(self):
        if not self.cache_path:
            return
        data = {}
        if os.path.exists(self.cache_path):
            with open(self.cache_path) as f:
                data = json.load(f)
        data[self._pkey()] = {str(k): list(v) for k, v in self.table.items()}
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, self.cache_path)

    def _measure(self, B: int):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        n = self.keys.n
        ops_h, a, b = W.gate_batch(B, seed=W.TUNE_SEED + B)
        c1 = self.keys.encrypt(a, seed=W.TUNE_SEED)
        c2 = self.keys.encrypt(b, seed=W.TUNE_SEED, first_index=B)
        pool = torch.from_numpy(np.concatenate([c1, c2]).view(np.int32)).to(dev)
        ops = torch.from_numpy(ops_h).to(dev)
        ia = torch.arange(B, dtype=torch.int32, device=dev)
        out = torch.zeros((B, n + 1), dtype=torch.int32, device=dev)
        saved = cemu.get_tuning(self.keys)
        res = {}
        try:
            for form, tun in CANDIDATES:
                if form not in self.forms:
                    continue
                cemu.set_tuning(self.keys, **tun)
                cemu.bootstrap_gates(self.keys, ops, pool, ia, ia + B, out, form=form)   # warm / size workspaces
                torch.cuda.synchronize()
                cemu.profile_read(self.keys)
                cemu.profile_enable(self.keys, True)
                for _ in range(self.reps):
                    cemu.bootstrap_gates(self.keys, ops, pool, ia, ia + B, out, form=form)
                torch.cuda.synchronize()
                cemu.profile_enable(self.keys, False)
                prof = cemu.profile_read(self.keys)
                ms = sum(v[0] for v in prof.values()) / self.reps
                res[(form, json.dumps(tun, sort_keys=True))] = ms
        finally:
            cemu.set_tuning(self.keys, **saved)
        return res

    def best(self, B: int):
        """(form, tuning dict) for a batch of B gates."""
        b = bucket(B)
        if b not in self.table:
            res = self._measure(b)
            self.measurements[b] = {f"{k[0]} {k[1]}": v for k, v in res.items()}
            (form, tun), _ = min(res.items(), key=lambda kv: kv[1])
            self.table[b] = (form, tun)
            self._save()
        form, tun = self.table[b]
        tun = dict(json.loads(tun) if isinstance(tun, str) else tun)
        if form == "int8":
            # a cached choice written before the one-gate shape existed means the 16-gate shape
            tun.setdefault("int8_gates_per_wg", 16)
        return form, tun

    def apply(self, B: int) -> str:
        """Set the key's tuning for a batch of B gates; returns the form."""
        form, tun = self.best(B)
        cemu.set_tuning(self.keys, **tun)
        return form

    def tune(self, sizes) -> dict:
        for B in sizes:
            self.best(B)
        return {b: {"choice": self.table[b], "ms": self.measurements.get(b)} for b in sorted(self.table)}
