"""Benchmark: batched TFHE gate bootstrapping on one MI355X.

One step = one pass of the whole hot path over one batch of 4096 independent
bootstrapped gates (type uniform in NAND/AND/OR/XOR, uniform input bits,
fresh encryptions) at the standard parameters n=630, N=1024, k=1, l=3,
Bgbit=7, t=8, basebit=2: gate linear combination + modulus switch, blind
rotation, sample extraction, key switching. Both product forms are timed:
the FP64 negacyclic-FFT form (the reported value) and the exact int8-MFMA form.
Inputs (keys, ciphertext pool, gate lists) are resident in HBM before the
timed region. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fft64|int8] [--only]
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
PEAK_FP64_FLOPS = 78.6e12        # MI355X FP64 vector, flop/s
# Beside these published peaks the benchmark reports fractions of the peaks
# measured on the device it runs on (cemu_measure_peaks: independent FP64
# FMA chains and independent int8 MFMA accumulations at the kernels'
# occupancy, two waves per SIMD, one workgroup per compute unit).
# FP64-FFT form per gate: n steps x (8 FFTs of 512 points at 5 n log2 n + twist
# 6 x 512, plus 12 x 512 complex multiply-adds at 8 flop).
FFT_FLOP_PER_GATE = n_ * (8 * (5 * 512 * 9 + 6 * 512) + 12 * 512 * 8)
# LDS bytes of the FFT throughput kernel (br_fft_kernel<8>) per gate and CMux
# step, from its structure: 8 transforms x 2 transposes x 8 slots x 16 B x 64
# lanes written and read; the key spectra of 6 digit rows staged once per
# workgroup of 8 gates (6 x 16 KiB / 8) and read by every gate (6 x 16 x 16 B
# x 64); the rotated and own accumulator words read for the digits (2 x 32 x
# 4 B x 64); the accumulator update (2 x 16 x 4 B x 64 read and written).
FFT_LDS_WRITE_PER_GATE_STEP = 8 * 2 * 8 * 16 * 64 + 6 * 16384 // 8 + 2 * 16 * 4 * 64
FFT_LDS_READ_PER_GATE_STEP = 8 * 2 * 8 * 16 * 64 + 6 * 16 * 16 * 64 + 2 * 32 * 4 * 64 + 2 * 16 * 4 * 64
# Key switch per gate, as the contraction it runs: K = N t base one-hot rows
# x 640 columns (n + 1 padded) x 4 limbs x 2 ops; and the key bytes a gate's
# nonzero digits select (3/4 of the N t digits, n + 1 words each).
KS_T, KS_BASE = 8, 4
KS_OPS_PER_GATE = N_ * KS_T * KS_BASE * 640 * 4 * 2
KS_GATHER_BYTES_PER_GATE = N_ * KS_T * 3 // 4 * (n_ + 1) * 4
PEAK_HBM_BYTES = 8.0e12           # MI355X HBM3E, bytes/s


# HBM bytes per launch of the blind-rotation kernels at B = 4096, from two
# rocprofv3 --pmc runs (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000, scales from a
# plain 1 GiB copy); summary and commands in profiles/. Valid only while the
# kernel's source code is the one profiled (sha256 prefix of the sources with
# comments and whitespace removed, so that comment edits keep it), else
# reported as null.
TRAFFIC = {
    "fft64": {"source": ["paper_2101_03403_amd/csrc/cemu_br_fft.hip", "paper_2101_03403_amd/csrc/cemu_fft.h"],
              "sha256_16": "1e1ade1190a8856e",
              "bytes": 486_913 * 1024 * 2 + 16_400 * 1024, "batch": 4096},
    "int8": {"source": "paper_2101_03403_amd/csrc/cemu_br_int8.hip", "sha256_16": "709541717732388d",
             "bytes": 246_002 * 1024 * 2 + 18_960 * 1024, "batch": 4096},
    # the key switch of a 4096-gate batch: ks_init_kernel + ks_mfma_kernel<1024, true> (2 K splits)
    "ks": {"source": "paper_2101_03403_amd/csrc/cemu_ks.hip", "sha256_16": "8f9eb8b89663227d",
           "bytes": (274 + 383_248) * 1024 * 2 + (10_096 + 29_152) * 1024, "batch": 4096},
}


def code_hash(paths):
    """sha256 prefix of C/C++/HIP sources (one path or a list, in order) with
    comments and whitespace removed."""
    import hashlib
    import re
    parts = []
    for path in ([paths] if isinstance(paths, str) else paths):
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        parts.append(" ".join(text.split()))
    return hashlib.sha256(" ".join(parts).encode()).hexdigest()[:16]


def traffic_bytes(form, B):
    t = TRAFFIC[form]
    try:
        src = t["source"]
        h = code_hash([os.path.join(ROOT, x) for x in src] if isinstance(src, list) else os.path.join(ROOT, src))
    except OSError:
        return None
    return t["bytes"] if (h == t["sha256_16"] and B == t["batch"]) else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="fft64", choices=["int8", "fft64"],
                    help="form whose throughput is the reported value (the other is timed too)")
    ap.add_argument("--only", action="store_true", help="time only --form")
    ap.add_argument("--fft-gates-per-wg", type=int, default=8, choices=[1, 4, 8],
                    help="FFT64 launch shape of the throughput loop (1 = the one-gate-per-workgroup latency kernel)")
    ap.add_argument("--int8-gates-per-wg", type=int, default=16, choices=[1, 16],
                    help="int8 launch shape of the throughput loop (1 = the one-gate-per-workgroup latency kernel)")
    ap.add_argument("--int8-waves", type=int, default=8, choices=[4, 8])
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="gates in the oracle CPU sample (about 10-15 s of CPU work on 16 threads)")
    ap.add_argument("--no-add", action="store_true", help="skip the 32-bit ADD / SUB latency measurements")
    ap.add_argument("--no-shift", action="store_true", help="skip the 32-bit barrel-shifter latency measurement")
    ap.add_argument("--no-emu", action="store_true", help="skip the emulator while-loop run")
    ap.add_argument("--no-seq", action="store_true",
                    help="skip the 32-bit sequential multiplier / divider latency measurement")
    ap.add_argument("--add-instances", type=int, default=256)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed instruction stream")
    ap.add_argument("--no-autotune", action="store_true", help="circuits use --form with default tiles")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the FP64 FMA and int8 MFMA peak rates on this GPU, print them and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times) and exit; "
                         "used to scale HBM byte counters")
    return ap.parse_args()


def expected_word(kind, width, a, b):
    """Integer result an instruction circuit must decrypt to: W-bit wrap for
    ADD / SUB / bitwise / shifts (amount mod W), 2W bits for the multipliers,
    one bit for LT / EQ, 2^W - 1 for a division by zero."""
    M = 1 << width
    sgn = lambda v: v - M if v >> (width - 1) else v  # noqa: E731
    if kind in ("LLS", "LRS", "ARS"):
        k = b % width
        return {"LLS": (a << k) % M, "LRS": a >> k, "ARS": (sgn(a) >> k) % M}[kind]
    if kind == "DIV":
        return a // b if b else M - 1
    if kind == "SMULSEQ":
        return (sgn(a) * sgn(b)) % (M * M)
    return {"ADD": (a + b) % M, "SUB": (a - b) % M, "MUL": a * b, "MULSEQ": a * b, "LT": int(a < b),
            "EQ": int(a == b), "AND": a & b, "OR": a | b, "XOR": a ^ b}[kind]


def cpu_add32_latency(okeys, seed=404):
    """One 32-bit ADD (the paper's AND/OR prefix, 12 levels) as the oracle's
    own netlist of Sec. 5.2 on the oracle's gates, level by level: each
    level's gates in one batch, OpenMP across them (the level structure of the
    paper's own parallel ADD). Returns (seconds, decrypted sum correct)."""
    from oracle import circuits as OC
    from oracle import oracle as O
    rng = np.random.default_rng(seed)
    a, b = (int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64))
    net = OC.instruction("ADD", 32)
    inputs = O.encrypt_bits(okeys, np.asarray(OC.to_bits(a, 32) + OC.to_bits(b, 32), np.uint8), seed=seed)
    t0 = time.time()
    ct = net.run_encrypted(okeys, inputs)
    dt = time.time() - t0
    got = OC.from_bits(O.decrypt_bits(okeys.lwe_key, np.stack([ct[w] for w in net.outputs["out"]])))
    return dt, got == OC.word_result("ADD", 32, a, b)


def cpu_baseline(keys_seed, ops, c1, c2, gpu_out, sample, add32=True):
    """The CPU oracle, as it stands, on a bounded sample of the same batch;
    also one gate alone (one thread works on it) and one 32-bit ADD."""
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
    diff = (gpu_out[idx].astype(np.int64) - oout.astype(np.int64)) % (1 << 32)
    diff = np.where(diff >= 1 << 31, diff - (1 << 32), diff)
    t0 = time.time()
    O.bootstrap_batch(okeys, ops[:1].astype(np.int32), c1[:1], c2[:1], want_extracted=False)
    one_gate = time.time() - t0
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    res = {"value": sample / dt, "unit": "gates/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model,
           "sample": f"first {sample} gates of the same 4096-gate batch, same keys and ciphertexts; "
                     f"exact schoolbook products, OpenMP across gates; {dt:.1f} s "
                     f"(oracle keygen {t_keygen:.1f} s not timed)",
           "bit_exact_vs_gpu": f"{match}/{sample}",
           "max_torus_error_vs_gpu": int(np.abs(diff).max()) if sample else None,
           "one_gate_ms": one_gate * 1e3}
    if add32:
        t_add, ok = cpu_add32_latency(okeys)
        res["add32_latency_ms"] = t_add * 1e3
        res["add32"] = ("one 32-bit ADD, the paper's AND/OR prefix (483 gates, 12 levels), each level's gates "
                        f"across the {cores} threads; decrypted sum {'correct' if ok else 'WRONG'}")
    return res


def host_buffers_rate(keys, form, ops_t, pool, ia, ib, out, steps):
    """The same step for a caller whose ciphertexts live in host memory:
    input pool copied from pinned host memory, the gates, outputs copied back,
    all on one stream and timed together (PCIe included). Not the reported
    value, whose inputs are resident in HBM."""
    import torch
    from paper_2101_03403_amd import cemu
    hpool = torch.empty(pool.shape, dtype=pool.dtype, pin_memory=True)
    hpool.copy_(pool)
    hout = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)

    def step():
        pool.copy_(hpool, non_blocking=True)
        cemu.bootstrap_gates(keys, ops_t, pool, ia, ib, out, form=form)
        hout.copy_(out, non_blocking=True)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B = out.shape[0]
    return {"value": B / (wall / steps), "unit": "gates/s", "ms_per_step": wall * 1e3 / steps,
            "bytes_per_step": int(pool.numel() * 4 + out.numel() * 4),
            "note": "inputs copied from pinned host memory and outputs copied back every step"}


def run_form(keys, form, ops_t, pool, ia, ib, out, stream, steps, warmup):
    """Times `steps` whole-path steps of one product form; returns (seconds, kernel profile)."""
    import torch
    from paper_2101_03403_amd import cemu

    def step():
        cemu.bootstrap_gates(keys, ops_t, pool, ia, ib, out, form=form, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    cemu.profile_read(keys)                       # drop anything recorded so far
    cemu.profile_enable(keys, True)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    events[0].record(stream)
    for k in range(steps):
        step()
        events[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cemu.profile_enable(keys, False)
    per_step = [events[k].elapsed_time(events[k + 1]) for k in range(steps)]
    return wall, cemu.profile_read(keys), per_step


def add32_latency(keys, dev, form, instances=256, reps=10, tuner=None, prefix="gates", kind="ADD"):
    """32-bit Kogge-Stone ADD (Sec. 5.2) or SUB (Sec. 5.3, kind="SUB"):
    `instances` concurrent instructions with all gates of a level in one
    launch, the levels (12 with the paper's AND/OR prefix, 7 with the MUX
    prefix) captured as one hipGraph. Latency = first level launch to last
    level done; also one instance alone."""
    import torch
    from paper_2101_03403_amd import circuits as Cc, workloads as W

    out = {}
    for inst in (instances, 1):
        rng = np.random.default_rng(404 + inst)
        ops = rng.integers(0, 1 << 32, (inst, 2), dtype=np.uint64)
        cs = [(Cc.adder_instance if kind == "ADD" else Cc.sub_instance)(32, prefix=prefix) for _ in range(inst)]
        prog = Cc.Program(cs).to_device(dev)
        bits = []
        for a, b in ops:
            bits += Cc.int_to_bits(int(a), 32) + Cc.int_to_bits(int(b), 32)
        pool = torch.zeros((prog.rows, keys.n + 1), dtype=torch.int32, device=dev)
        enc = keys.encrypt(np.asarray(bits, np.uint8), seed=W.ENC_SEED + inst)
        pool[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = \
            torch.from_numpy(enc.view(np.int32)).to(dev)
        prog.run(keys, pool, form=form, tuner=tuner)    # sizes the workspaces, tunes each width
        torch.cuda.synchronize()
        g = prog.capture(keys, pool, form=form, tuner=tuner)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        host = pool.cpu().numpy().view(np.uint32)
        ok = 0
        for k, (a, b) in enumerate(ops):
            rows = np.array(cs[k].outputs["sum" if kind == "ADD" else "diff"]) + prog.offsets[k]
            ok += int(Cc.bits_to_int(keys.decrypt(host[rows])) == expected_word(kind, 32, int(a), int(b)))
        ms = float(np.median(times))
        key = "batch" if inst == instances else "single"
        out[key] = {"instances": inst, "latency_ms": ms, "amortized_ms_per_instruction": ms / inst,
                    "gates": prog.num_gates(), "muxes": prog.num_muxes(), "bootstraps": prog.num_bootstraps(),
                    "levels": prog.depth, "bootstraps_per_s": prog.num_bootstraps() / (ms * 1e-3),
                    "decrypt_exact": f"{ok}/{inst}", "level_widths": prog.level_widths(),
                    "level_muxes": prog.level_mux_counts()}
    out["prefix"] = {"gates": "the paper's AND/OR o operator", "mux": "one MUX per o carry"}[prefix]
    out["form"] = form if tuner is None else "autotuned per level width"
    out["timing"] = f"hipGraph of the level launches, median of {reps} replays (hip events)"
    return out


def shift32_latency(keys, dev, form, reps=10, tuner=None):
    """32-bit register-mode barrel shifters LLS / LRS / ARS (Sec. 5.4): one
    instance each, 5 levels of 32 FHE MUX selects, captured as a hipGraph;
    latency = median replay. The paper reports 474.7 / 472.9 / 491.8 ms on
    its 48-core node."""
    import torch
    from paper_2101_03403_amd import circuits as Cc, workloads as W

    out = {}
    for mode in (Cc.LLS, Cc.LRS, Cc.ARS):
        rng = np.random.default_rng({"LLS": 11, "LRS": 12, "ARS": 13}[mode])
        a = int(rng.integers(0, 1 << 32, dtype=np.uint64)) | (1 << 31)
        amt = int(rng.integers(1, 32))
        c = Cc.instruction_circuit(mode, 32)
        prog = Cc.Program([c]).to_device(dev)
        pool = torch.zeros((prog.rows, keys.n + 1), dtype=torch.int32, device=dev)
        enc = keys.encrypt(np.asarray(Cc.int_to_bits(a, 32) + Cc.int_to_bits(amt, 32), np.uint8), seed=W.ENC_SEED + 9)
        pool[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = torch.from_numpy(enc.view(np.int32)).to(dev)
        prog.run(keys, pool, form=form, tuner=tuner)
        torch.cuda.synchronize()
        g = prog.capture(keys, pool, form=form, tuner=tuner)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        host = pool.cpu().numpy().view(np.uint32)
        got = Cc.bits_to_int(keys.decrypt(host[np.array(c.outputs["out"])]))
        out[mode] = {"latency_ms": float(np.median(times)), "muxes": prog.num_muxes(),
                     "bootstraps": prog.num_bootstraps(), "levels": prog.depth,
                     "decrypt_exact": int(got == expected_word(mode, 32, a, amt))}
    out["form"] = form if tuner is None else "autotuned per launch width"
    out["timing"] = f"hipGraph of the 5 MUX levels, median of {reps} replays (hip events)"
    return out


def sequential_units(keys, dev, form, width=32, reps=3, tuner=None, prefix="gates"):
    """The paper's sequential multiplier (unsigned and signed) and the
    non-restoring divider (Sec. 5.5, 5.6), one instance each: W iterations
    of a W- or (W+1)-bit adder, hundreds of narrow levels, captured as a
    hipGraph; latency = median replay. The paper reports, for 32 bits on its
    48-core node, 36,929 ms (unsigned), 34,826 ms (signed) and 38,257 ms
    (divider); for 16 bits 11,317 / 13,121 / 11,660 ms."""
    import torch
    from paper_2101_03403_amd import circuits as Cc, workloads as W

    out = {}
    for kind in ("MULSEQ", "SMULSEQ", "DIV"):
        rng = np.random.default_rng({"MULSEQ": 21, "SMULSEQ": 22, "DIV": 23}[kind])
        a = int(rng.integers(0, 1 << width, dtype=np.uint64))
        b = int(rng.integers(1, 1 << width, dtype=np.uint64))
        if kind == "DIV":
            b = int(rng.integers(1, 1 << (width // 2)))
        c = Cc.instruction_circuit(kind, width, prefix=prefix)
        prog = Cc.Program([c]).to_device(dev)
        pool = torch.zeros((prog.rows, keys.n + 1), dtype=torch.int32, device=dev)
        enc = keys.encrypt(np.asarray(Cc.int_to_bits(a, width) + Cc.int_to_bits(b, width), np.uint8),
                           seed=W.ENC_SEED + 10)
        pool[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = torch.from_numpy(enc.view(np.int32)).to(dev)
        prog.run(keys, pool, form=form, tuner=tuner)
        torch.cuda.synchronize()
        g = prog.capture(keys, pool, form=form, tuner=tuner)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        host = pool.cpu().numpy().view(np.uint32)
        got = Cc.bits_to_int(keys.decrypt(host[np.array(c.outputs["out"])]))
        out[kind] = {"latency_ms": float(np.median(times)), "gates": prog.num_gates(), "muxes": prog.num_muxes(),
                     "levels": prog.depth, "decrypt_exact": int(got == expected_word(kind, width, a, b))}
    out["width"] = width
    out["prefix"] = {"gates": "the paper's AND/OR o operator", "mux": "one MUX per o carry"}[prefix]
    out["form"] = form if tuner is None else "autotuned per level width"
    out["timing"] = f"hipGraph of all levels, median of {reps} replays (hip events)"
    return out


def emulator_while_loop(keys, dev, form, count=42, tuner=None, prefix="gates"):
    """The paper's while loop (Sec. 6.1) on the emulator front-end: MOV R0,
    #count; Loop: SUBS R0, R0, #1; B_NE Loop -- count encrypted 32-bit
    subtractions with NZCV flags, each branch resolved by the client (the
    secret-key holder) from the encrypted flags. Wall time of the whole run
    including the client round trips; the paper reports 169.8 ms for the
    32-bit flag unit alone and 1115 ms for a 32-bit SUB."""
    import torch
    from paper_2101_03403_amd import circuits as Cc, emulator as E

    text = f"MOV R0, R0, #{count}\nLoop: SUBS R0, R0, #1\nB_NE Loop\n"
    client = E.make_client(keys)
    warm = E.Machine(keys, width=32, form=form, tuner=tuner, device=dev, prefix=prefix)
    warm.run(text.replace(f"#{count}", "#1"), client)          # builds the units, tunes their widths
    mach = E.Machine(keys, width=32, form=form, tuner=tuner, device=dev, prefix=prefix)
    mach._units = warm._units
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = mach.run(text, client)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r0 = Cc.bits_to_int(keys.decrypt(mach.read_register(0)))
    return {"iterations": count, "wall_ms": wall * 1e3, "ms_per_iteration": wall * 1e3 / count,
            "instructions": stats["instructions"], "branches": stats["branches"],
            "bootstraps": stats["bootstraps"], "levels": stats["levels"], "r0_decrypts_to_zero": int(r0 == 0),
            "prefix": {"gates": "the paper's AND/OR o operator", "mux": "one MUX per o carry"}[prefix],
            "form": form if tuner is None else "autotuned per level width"}


def mixed_stream(keys, dev, form, count=1024, seed=2021, tuner=None, prefix="gates", pack=None):
    """1024 independent instructions (40 % ADD/SUB, 20 % 8x8/16x16 array MUL,
    20 % LT/EQ, 20 % AND/OR/XOR; widths 8/16/32), gates of each level merged
    across instructions into one launch. Makespan of one warm run. With
    ``pack`` the levels are refilled to whole rounds of that many blind
    rotations within each gate's slack (circuits.pack_levels); without it
    every gate runs at its earliest level."""
    import torch
    from paper_2101_03403_amd import circuits as Cc, workloads as W

    mix = W.instruction_mix(count, seed)
    cs = [Cc.instruction_circuit(k, w, prefix=prefix) for k, w, _, _ in mix]
    prog = Cc.Program(cs, pack=pack).to_device(dev)
    bits = []
    for k, w, a, b in mix:
        bits += Cc.int_to_bits(a, w) + Cc.int_to_bits(b, w)
    pool = torch.zeros((prog.rows, keys.n + 1), dtype=torch.int32, device=dev)
    enc = keys.encrypt(np.asarray(bits, np.uint8), seed=W.ENC_SEED + 7)
    pool[torch.from_numpy(prog.input_rows.astype(np.int64)).to(dev)] = torch.from_numpy(enc.view(np.int32)).to(dev)
    prog.run(keys, pool, form=form, tuner=tuner)   # warm-up (sizes workspaces, tunes widths)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    prog.run(keys, pool, form=form, tuner=tuner)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    host = pool.cpu().numpy().view(np.uint32)
    ok = 0
    for (k, w, a, b), c, off in zip(mix, cs, prog.offsets):
        ok += int(Cc.bits_to_int(keys.decrypt(host[np.array(c.outputs["out"]) + off])) ==
                  expected_word(k, w, a, b))
    widths = np.array(prog.level_widths())
    hist = {f"<{lim}": int(np.sum(widths < lim)) for lim in (256, 1024, 4096, 16384)}
    hist[">=16384"] = int(np.sum(widths >= 16384))
    return {"instructions": count, "makespan_ms": ms, "gates": prog.num_gates(), "muxes": prog.num_muxes(),
            "bootstraps": prog.num_bootstraps(), "levels": prog.depth,
            "bootstraps_per_s": prog.num_bootstraps() / (ms * 1e-3), "decrypt_exact": f"{ok}/{count}",
            "level_width_histogram": hist,
            "prefix": {"gates": "the paper's AND/OR o operator", "mux": "one MUX per o carry"}[prefix],
            "form": form if tuner is None else "autotuned per level width",
            "schedule": (f"levels refilled to whole rounds of {pack} blind rotations within each gate's slack"
                         if pack else "every gate at its earliest level")}


def mixed_stream_both(keys, dev, form, tuner=None, prefix="gates"):
    """The mixed stream with levels filled to whole rounds of the throughput
    kernel (8 gates per compute unit), and the earliest-level schedule beside it."""
    import torch
    rnd = 8 * torch.cuda.get_device_properties(dev).multi_processor_count
    rec = mixed_stream(keys, dev, form, tuner=tuner, prefix=prefix, pack=rnd)
    asap = mixed_stream(keys, dev, form, tuner=tuner, prefix=prefix)
    rec["earliest_level_schedule"] = {k: asap[k] for k in ("makespan_ms", "bootstraps_per_s", "levels",
                                                           "decrypt_exact", "level_width_histogram")}
    return rec


FFT_KERNEL = {8: "br_fft_kernel<8>", 4: "br_fft_kernel<4>", 1: "br_fft_lat_kernel"}


def output_noise(keys, out, want):
    """Phase error of the bootstrapped outputs against +-1/8, measured with
    the secret key (in torus units, 1 = 2^32): decryption stays exact while
    |error| < 1/8."""
    ph = keys.phase(out).astype(np.int64)
    mu = np.where(want == 1, 1 << 29, (1 << 32) - (1 << 29))
    e = (ph - mu) % (1 << 32)
    e = np.where(e >= 1 << 31, e - (1 << 32), e) / float(1 << 32)
    # closed form for one fixed key (sample variance over the gates): blind
    # rotation n * 2l * N * (Bg^2 - 1)/12 * sigma_bk^2, key switching
    # N * t * (9/16) * sigma_ks^2 plus its rounding (N/2) * 2^-32 / 12
    var_cf = (n_ * 6 * N_ * (128 ** 2 - 1) / 12.0 * 2.0 ** -50 + N_ * KS_T * (9.0 / 16.0) * 2.0 ** -30
              + (N_ / 2) * 2.0 ** -32 / 12.0)
    return {"std": float(np.std(e)), "max_abs": float(np.max(np.abs(e))), "log2_std": float(np.log2(np.std(e))),
            "margin": 0.125, "variance": float(np.var(e)), "closed_form_variance": var_cf,
            "variance_over_closed_form": float(np.var(e)) / var_cf}


def noise_chain(keys, form, out1, want1, seed=3):
    """Second level of a two-level chain: B gates (NAND/AND/OR/XOR) whose
    inputs are the first level's bootstrapped outputs, in two random
    permutations. Bootstrapping resets the noise, so the second level's output
    noise equals the first level's, whatever the (larger, key-switched) input
    noise was. Returns the second level's output noise and decryptions."""
    import torch
    from paper_2101_03403_amd import cemu, workloads as W

    B = out1.shape[0]
    dev = out1.device
    rng = np.random.default_rng(seed)
    ops2, _, _ = W.gate_batch(B, seed=seed + 100)
    pa, pb = rng.permutation(B).astype(np.int32), rng.permutation(B).astype(np.int32)
    out2 = torch.zeros_like(out1)
    cemu.bootstrap_gates(keys, torch.from_numpy(ops2).to(dev), out1, torch.from_numpy(pa).to(dev),
                         torch.from_numpy(pb).to(dev), out2, form=form)
    torch.cuda.synchronize()
    truth = {0: lambda x, y: 1 - (x & y), 1: lambda x, y: x & y, 2: lambda x, y: x | y, 3: lambda x, y: x ^ y}
    want2 = np.array([truth[int(o)](int(want1[a]), int(want1[b])) for o, a, b in zip(ops2, pa, pb)], np.uint8)
    host2 = out2.cpu().numpy().view(np.uint32)
    return {"decrypt_exact": f"{int(np.sum(keys.decrypt(host2) == want2))}/{B}",
            "output_noise": output_noise(keys, host2, want2),
            "inputs": "the first level's outputs (key-switched, not fresh), two random permutations"}


def roofline(form, prof, B, peaks, fft_gates_per_wg=8, int8_gates_per_wg=16, int8_waves=8):
    if form == "int8":
        if int8_gates_per_wg == 16:
            kname = "br_int8_res_kernel<1024>" if int8_waves == 8 else "br_int8_kernel<1024, 4>"
        else:
            kname = f"br_int8_lat_kernel<1024, {int8_waves}>"
        default_shape = int8_gates_per_wg == 16 and int8_waves == 8
        ms, cnt = prof["blind_rotate_int8"]
        avg = ms / max(cnt, 1)
        ach = INT8_OPS_PER_GATE * B / (avg * 1e-3)
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOP/s",
                "frac": ach / PEAK_INT8_OPS, "traffic": traffic_bytes("int8", B) if default_shape else None,
                "kernel": kname,
                "measured_peak": peaks["int8_ops_per_s"] / 1e12, "frac_measured": ach / peaks["int8_ops_per_s"],
                "avg_ms": avg, "algorithmic_per_launch": INT8_OPS_PER_GATE * B,
                "algorithmic_per_gate": "n*2l*2*N^2*4 limbs*2 = 6.34e10 int8 ops"}
    ms, cnt = prof["blind_rotate_fft64"]
    avg = ms / max(cnt, 1)
    ach = FFT_FLOP_PER_GATE * B / (avg * 1e-3)
    lds = None
    if fft_gates_per_wg == 8 and "lds_write_bytes_per_s" in peaks:
        w = FFT_LDS_WRITE_PER_GATE_STEP * n_ * B
        r = FFT_LDS_READ_PER_GATE_STEP * n_ * B
        t = w / peaks["lds_write_bytes_per_s"] + r / peaks["lds_read_bytes_per_s"]
        lds = {"bytes_written_per_launch": w, "bytes_read_per_launch": r,
               "per_gate_and_step": f"{FFT_LDS_WRITE_PER_GATE_STEP} B written, {FFT_LDS_READ_PER_GATE_STEP} B read",
               "measured_write_TBps": peaks["lds_write_bytes_per_s"] / 1e12,
               "measured_read_TBps": peaks["lds_read_bytes_per_s"] / 1e12,
               "time_at_measured_rates_ms": t * 1e3, "frac_of_kernel_time": t / (avg * 1e-3),
               "note": "writes and reads of the kernel's own structure at the LDS rates measured on this GPU, "
                       "serialised: the share of the kernel's time its LDS traffic needs"}
    return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64_FLOPS / 1e12, "unit": "TFLOP/s", "lds": lds,
            "frac": ach / PEAK_FP64_FLOPS, "traffic": traffic_bytes("fft64", B) if fft_gates_per_wg == 8 else None,
            "kernel": FFT_KERNEL[fft_gates_per_wg],
            "measured_peak": peaks["fp64_flops_per_s"] / 1e12, "frac_measured": ach / peaks["fp64_flops_per_s"],
            "avg_ms": avg, "algorithmic_per_launch": FFT_FLOP_PER_GATE * B,
            "algorithmic_per_gate": "n*(8*(5*512*9 + 6*512) + 12*512*8) = 1.63e8 FP64 flop"}


def key_switch_report(prof, B):
    """The key switch of the same launches: achieved int8 rate of its
    contraction, HBM bytes from the committed counters (while the kernel
    source is the one profiled) over its time, and the key bytes the gates'
    digits select over its time (a rate the batch reaches by reusing each
    key row from L2 / MALL across the gates of a tile)."""
    ms, cnt = prof["key_switch"]
    if not cnt:
        return None
    avg = ms / cnt
    sec = avg * 1e-3
    hbm = traffic_bytes("ks", B)
    return {"kernel": "ks_init_kernel + ks_mfma_kernel<1024, true> (2 K splits)" if B == 4096
            else "ks_mfma_kernel<1024, SPLIT>", "avg_ms": avg,
            "int8_TOPs": KS_OPS_PER_GATE * B / sec / 1e12, "frac_int8_peak": KS_OPS_PER_GATE * B / sec / PEAK_INT8_OPS,
            "hbm_bytes": hbm, "hbm_GBps": hbm / sec / 1e9 if hbm else None,
            "frac_hbm_peak": hbm / sec / PEAK_HBM_BYTES if hbm else None,
            "selected_key_bytes_GBps": KS_GATHER_BYTES_PER_GATE * B / sec / 1e9,
            "per_gate": "contraction 4*N*t*640*4 limbs*2 = 1.68e8 int8 ops; selected key rows "
                        "N*t*3/4*(n+1)*4 B = 15.5 MB"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2101_03403_amd import cemu, workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
        return
    peaks = cemu.measure_peaks()
    peaks.update(cemu.measure_lds())
    peaks["how"] = ("cemu_measure_peaks / cemu_measure_lds on this GPU: independent FP64 FMA chains, int8 MFMA "
                    "accumulations, and conflict-free 16-byte LDS writes / reads at immediate offsets, one workgroup of 8 waves per "
                    "compute unit, fastest of 8 launches")
    if args.peaks:
        print(json.dumps({"measured_peaks": peaks}), flush=True)
        return
    keys = cemu.keygen(cemu.STD, W.KEY_SEED)
    cemu.set_tuning(keys, fft_gates_per_wg=args.fft_gates_per_wg, int8_gates_per_wg=args.int8_gates_per_wg,
                    int8_waves=args.int8_waves)
    B = args.batch
    ops, a, b = W.gate_batch(B, seed=1)
    c1 = keys.encrypt(a, seed=W.ENC_SEED)
    c2 = keys.encrypt(b, seed=W.ENC_SEED, first_index=B)
    pool = torch.from_numpy(np.concatenate([c1, c2]).view(np.int32)).to(dev)
    ops_t = torch.from_numpy(ops).to(dev)
    ia = torch.arange(B, dtype=torch.int32, device=dev)
    ib = ia + B
    stream = torch.cuda.current_stream()
    truth = {0: lambda x, y: 1 - (x & y), 1: lambda x, y: x & y, 2: lambda x, y: x | y, 3: lambda x, y: x ^ y}
    want = np.array([truth[int(o)](int(x), int(y)) for o, x, y in zip(ops, a, b)], np.uint8)

    forms = [args.form] + [f for f in ("fft64", "int8") if f != args.form and not args.only]
    res = {}
    outs = {}
    dev_outs = {}
    for form in forms:
        out = torch.zeros((B, keys.n + 1), dtype=torch.int32, device=dev)
        wall, prof, per_step = run_form(keys, form, ops_t, pool, ia, ib, out, stream, args.steps, args.warmup)
        host = out.cpu().numpy().view(np.uint32)
        outs[form] = host
        dev_outs[form] = out
        res[form] = {
            "value": B / (wall / args.steps), "ms_per_step": wall * 1e3 / args.steps,
            "median_ms_per_step": float(np.median(per_step)), "steps_timed": len(per_step),
            "gates_per_s_at_median_step": B / (float(np.median(per_step)) * 1e-3),
            "roofline": roofline(form, prof, B, peaks, args.fft_gates_per_wg, args.int8_gates_per_wg, args.int8_waves),
            "key_switch": key_switch_report(prof, B),
            "kernels": {k: {"avg_ms": (v[0] / v[1] if v[1] else None), "launches": v[1]} for k, v in prof.items()},
            "decrypt_exact": f"{int(np.sum(keys.decrypt(host) == want))}/{B}",
            "output_noise": output_noise(keys, host, want),
        }
    primary = res[args.form]
    primary["host_buffers"] = host_buffers_rate(keys, args.form, ops_t, pool, ia, ib,
                                                torch.zeros((B, keys.n + 1), dtype=torch.int32, device=dev),
                                                args.steps)
    primary["noise_chain_level2"] = noise_chain(keys, args.form, dev_outs[args.form], want)
    if len(outs) == 2:
        same = int(np.sum(np.all(outs["fft64"] == outs["int8"], axis=1)))
        primary["identical_outputs_fft64_vs_int8"] = f"{same}/{B}"

    tuner = None
    if not args.no_autotune and not (args.no_add and args.no_mixed and args.no_shift and args.no_seq and args.no_emu):
        from paper_2101_03403_amd.autotune import Autotuner
        tuner = Autotuner(keys)
    rec_add = None if args.no_add else add32_latency(keys, dev, args.form, tuner=tuner)
    rec_add_mux = None if args.no_add else add32_latency(keys, dev, args.form, tuner=tuner, prefix="mux")
    # the same ADD with every level on the int8-MFMA form (the two forms' latencies side by side);
    # its launch shape (16 gates or one gate per workgroup) is tuned per level width among int8 shapes only
    tuner_i8 = None
    if tuner is not None and not (args.no_add or args.only):
        from paper_2101_03403_amd.autotune import Autotuner
        tuner_i8 = Autotuner(keys, forms=("int8",))
    rec_add_int8 = None if (args.no_add or args.only) else add32_latency(keys, dev, "int8", reps=3, tuner=tuner_i8)
    if rec_add_int8 is not None and tuner_i8 is not None:
        rec_add_int8["form"] = "int8 only, launch shape autotuned per level width"
        rec_add_int8["autotune"] = {str(b): {"choice": [c[0], c[1]], "ms_per_candidate": tuner_i8.measurements.get(b)}
                                    for b, c in sorted(tuner_i8.table.items())}
    rec_sub = None if args.no_add else add32_latency(keys, dev, args.form, tuner=tuner, kind="SUB")
    rec_sub_mux = None if args.no_add else add32_latency(keys, dev, args.form, tuner=tuner, prefix="mux", kind="SUB")
    rec_mix = None if args.no_mixed else mixed_stream_both(keys, dev, args.form, tuner=tuner)
    rec_mix_mux = None if args.no_mixed else mixed_stream_both(keys, dev, args.form, tuner=tuner, prefix="mux")
    rec_shift = None if args.no_shift else shift32_latency(keys, dev, args.form, tuner=tuner)
    rec_seq = None if args.no_seq else sequential_units(keys, dev, args.form, tuner=tuner)
    rec_seq_mux = None if args.no_seq else sequential_units(keys, dev, args.form, tuner=tuner, prefix="mux")
    rec_emu = None if args.no_emu else emulator_while_loop(keys, dev, args.form, tuner=tuner)
    rec_emu_mux = None if args.no_emu else emulator_while_loop(keys, dev, args.form, tuner=tuner, prefix="mux")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W.KEY_SEED, ops, c1, c2, outs[args.form], min(args.cpu_sample, B), add32=not args.no_add)

    rec = {
        "metric": METRIC, "value": primary["value"], "unit": "gates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": primary["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.form == "fft64" else "int8", "data": "synthetic",
        "config": {"workload": f"{B} independent bootstrapped gates (NAND/AND/OR/XOR uniform, random bits), "
                               "TFHE n=630 N=1024 k=1 l=3 Bgbit=7 t=8 basebit=2, "
                               + ("FP64 negacyclic-FFT products" if args.form == "fft64"
                                  else "int8-limb MFMA products"),
                   "form": args.form, "batch": B, "parallelism": "single GPU"},
        "roofline": primary["roofline"], "cpu_baseline": cpu, "key_switch": primary["key_switch"],
        "kernels": primary["kernels"], "decrypt_exact": primary["decrypt_exact"],
        "output_noise": primary["output_noise"], "noise_chain_level2": primary["noise_chain_level2"],
        "host_buffers": primary["host_buffers"], "measured_peaks": peaks,
        "median_ms_per_step": primary["median_ms_per_step"],
        "forms": {f: {k: v for k, v in r.items() if k != "kernels"} for f, r in res.items()},
    }
    if rec_add is not None:
        rec["add32"] = rec_add
        rec["add32_mux_prefix"] = rec_add_mux
        if rec_add_int8 is not None:
            rec["add32_int8_form"] = rec_add_int8
        rec["sub32"] = rec_sub
        rec["sub32_mux_prefix"] = rec_sub_mux
    if rec_mix is not None:
        rec["mixed_stream"] = rec_mix
        rec["mixed_stream_mux_prefix"] = rec_mix_mux
    if rec_shift is not None:
        rec["shift32"] = rec_shift
    if rec_seq is not None:
        rec["mul_div32"] = rec_seq
        rec["mul_div32_mux_prefix"] = rec_seq_mux
    if rec_emu is not None:
        rec["emulator_while_loop"] = rec_emu
        rec["emulator_while_loop_mux_prefix"] = rec_emu_mux
    if tuner is not None:
        rec["autotune"] = {str(b): {"choice": [c[0], c[1]], "ms_per_candidate": tuner.measurements.get(b)}
                           for b, c in sorted(tuner.table.items())}
    if "identical_outputs_fft64_vs_int8" in primary:
        rec["identical_outputs_fft64_vs_int8"] = primary["identical_outputs_fft64_vs_int8"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
