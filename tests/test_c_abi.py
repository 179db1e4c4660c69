"""The library used from plain C (tests/c_abi_client.c): built with gcc
against include/cemu.h, libcemu.so and the HIP runtime's C API, no Python in
between. On the CPU the client checks argument handling; on the GPU it
bootstraps every gate op on all four input rows (toy parameters, int8 form;
the FFT64 form must be refused for N = 512) and its outputs must equal the
oracle's word for word."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2101_03403_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libcemu.so")):
        pytest.skip("libcemu.so is not built")
    exe = str(tmp_path / "c_abi_client")
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", os.path.join(HERE, "c_abi_client.c"), "-I", os.path.join(ROCM, "include"),
           "-L", PKG, "-lcemu", "-Wl,-rpath," + PKG, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    return exe


def test_c_client_argument_checks(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "0 failed checks" in r.stdout


@pytest.mark.gpu
def test_c_client_gates_equal_oracle(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    exe = _build(tmp_path)
    out_path = str(tmp_path / "out.bin")
    r = subprocess.run([exe, "gpu", out_path], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "0 failed checks" in r.stdout
    ok = O.keygen(O.TOY, 7)
    B = 40
    ops = np.arange(B, dtype=np.int32) // 4
    a = (np.arange(B) & 1).astype(np.uint8)
    b = ((np.arange(B) >> 1) & 1).astype(np.uint8)
    c1 = O.encrypt_bits(ok, a, seed=11)
    c2 = O.encrypt_bits(ok, b, seed=11, first_index=B)
    _, want = O.bootstrap_batch(ok, ops, c1, c2, want_extracted=False)
    got = np.fromfile(out_path, dtype=np.uint32).reshape(B, ok.params.n + 1)
    assert np.array_equal(got, want)
