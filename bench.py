"""Benchmark: batched TFHE gate bootstrapping on one MI355X.

One step = one pass of the whole hot path over one batch of 4096 independent
bootstrapped gates (type uniform in NAND/AND/OR/XOR, uniform input bits,
fresh encryptions) at the standard parameters n=630, N=1024, k=1, l=3,
Bgbit=7, t=8, basebit=2: gate linear combination + modulus switch, blind
rotation with the int8-MFMA products, sample extraction, key switching.
Inputs (keys, ciphertext pool, gate lists) are resident in HBM before the
timed region. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--form int8|fft64]
                  [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bootstrapped gates/s (N=1024,n=630): int8-MFMA vs FP64-FFT; 32b ADD latency"
BATCH = 4096
# Algorithmic work of the blind rotation with int8 limbs, per gate:
# n steps x (k+1)l digit rows x 2 output polys x N^2 MACs x 4 limbs x 2 ops.
N_, n_, ROWS = 1024, 630, 6
INT8_OPS_PER_GATE = n_ * ROWS * 2 * N_ * N_ * 4 * 2
PEAK_INT8_OPS = 5.0e15          # MI355X dense int8 MFMA, ops/s
PEAK_FP64_FLOPS = 78.6e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="int8", choices=["int8", "fft64"])
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64, help="gates in the oracle CPU sample")
    return ap.parse_args()


def cpu_baseline(keys_seed, ops, c1, c2, gpu_out, sample):
    """The CPU oracle, as it stands, on a bounded sample of the same batch."""
    from oracle import oracle as O
    idx = np.arange(sample)
    t0 = time.time()
    okeys = O.keygen(O.STANDARD, keys_seed)
    t_keygen = time.time() - t0
    t0 = time.time()
    _, oout = O.bootstrap_batch(okeys, ops[idx].astype(np.int32), c1[idx], c2[idx], want_extracted=False)
    dt = time.time() - t0
    cores = O.num_threads()
    match = int(np.sum(np.all(oout == gpu_out[idx], axis=1)))
    return {"value": sample / dt, "unit": "gates/s", "cores": cores, "kind": "oracle",
            "sample": f"first {sample} gates of the same 4096-gate batch, same keys and ciphertexts; "
                      f"exact schoolbook products, OpenMP across gates; {dt:.1f} s "
                      f"(oracle keygen {t_keygen:.1f} s not timed)",
            "bit_exact_vs_gpu": f"{match}/{sample}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2101_03403_amd import cemu, workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    keys = cemu.keygen(cemu.STD, W.KEY_SEED)
    B = args.batch
    ops, a, b = W.gate_batch(B, seed=1)
    c1 = keys.encrypt(a, seed=W.ENC_SEED)
    c2 = keys.encrypt(b, seed=W.ENC_SEED, first_index=B)
    pool = torch.from_numpy(np.concatenate([c1, c2]).view(np.int32)).to(dev)
    ops_t = torch.from_numpy(ops).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    ib = ia + B
    out = torch.zeros((B, keys.n + 1), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        cemu.bootstrap_gates(keys, ops_t, pool, ia, ib, out, form=args.form, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    cemu.profile_read(keys)                       # drop anything recorded so far
    cemu.profile_enable(keys, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cemu.profile_enable(keys, False)
    prof = cemu.profile_read(keys)
    ms_per_step = wall * 1e3 / args.steps
    value = B / (wall / args.steps)

    gpu_out = out.cpu().numpy().view(np.uint32)
    truth = {0: lambda x, y: 1 - (x & y), 1: lambda x, y: x & y, 2: lambda x, y: x | y, 3: lambda x, y: x ^ y}
    want = np.array([truth[int(o)](int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)
    dec_ok = int(np.sum(keys.decrypt(gpu_out) == want))

    br_kind = "blind_rotate_int8" if args.form == "int8" else "blind_rotate_fft64"
    br_ms, br_n = prof[br_kind]
    br_avg_ms = br_ms / max(br_n, 1)
    if args.form == "int8":
        achieved = INT8_OPS_PER_GATE * B / (br_avg_ms * 1e-3)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOP/s",
                "frac": achieved / PEAK_INT8_OPS, "traffic": None,
                "kernel": "br_int8_kernel<1024,8>", "avg_ms": br_avg_ms,
                "algorithmic_ops_per_launch": INT8_OPS_PER_GATE * B}
    else:
        flops = 1.63e8 * B
        achieved = flops / (br_avg_ms * 1e-3)
        roof = {"bound": "fp64", "achieved": achieved / 1e12, "peak": PEAK_FP64_FLOPS / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_FLOPS, "traffic": None, "avg_ms": br_avg_ms}
    kernels = {k: {"avg_ms": (v[0] / v[1] if v[1] else None), "launches": v[1]} for k, v in prof.items()}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W.KEY_SEED, ops, c1, c2, gpu_out, min(args.cpu_sample, B))

    rec = {
        "metric": METRIC, "value": value, "unit": "gates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int8" if args.form == "int8" else "f64", "data": "synthetic",
        "config": {"workload": f"{B} independent bootstrapped gates (NAND/AND/OR/XOR uniform, random bits), "
                               "TFHE n=630 N=1024 k=1 l=3 Bgbit=7 t=8 basebit=2",
                   "form": args.form, "batch": B, "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "kernels": kernels,
        "decrypt_exact": f"{dec_ok}/{B}",
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
