"""Known-answer pin of the oracle's Philox4x32-10 block function against an
independent implementation: rocRAND's engine (ROCm's own source header,
compiled here for the host).  The JL reading draws P from Philox4x32-10
(Salmon, Moraes, Dror, Shaw, SC'11); a wrong multiplier, Weyl increment or
word order in the oracle fails this test even if the device generator
shared the mistake.  Nothing is stored: both sides are evaluated here."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "philox_rocrand_probe.cpp")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    header = os.path.join(ROCM, "include", "rocrand", "rocrand_philox4x32_10.h")
    if not (os.path.exists(hipcc) or shutil.which("hipcc")) or not os.path.exists(header):
        pytest.skip("hipcc or rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "probe")
    cmd = [hipcc if os.path.exists(hipcc) else "hipcc", "-O1", "-x", "c++", "-I" + os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__", SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def run(ctr, key):
        ctr = np.asarray(ctr, np.uint64).reshape(-1, 4)
        key = np.asarray(key, np.uint64).reshape(-1, 2)
        lines = "".join("%d %d %d %d %d %d\n" % (tuple(int(v) for v in c) + tuple(int(v) for v in k))
                        for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w) for w in l.split()] for l in out.strip().splitlines()], np.uint64)
    return run


def _oracle_blocks(ctr, key):
    return np.stack([oracle.philox4x32_10(c[None, :], (int(k[0]), int(k[1])))[0] for c, k in zip(ctr, key)])


def test_structured_counters_and_keys(probe):
    """All-zero, all-ones and mixed-bit words, and keys that carry into
    every word of the Weyl sequence."""
    m = 0xFFFFFFFF
    ctr = np.array([[0, 0, 0, 0], [m, m, m, m], [1, 0, 0, 0], [0, 0, 0, 1], [0x80000000, 1, 0x7FFFFFFF, m],
                    [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]], np.uint64)
    key = np.array([[0, 0], [m, m], [0, 0], [m, 0], [0x61C88646, 0x44BB67AE],
                    [0xA4093822, 0x299F31D0]], np.uint64)
    np.testing.assert_array_equal(_oracle_blocks(ctr, key), probe(ctr, key))


def test_random_counters_and_keys(probe):
    rng = np.random.default_rng(2004)
    ctr = rng.integers(0, 2 ** 32, (256, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, (256, 2), dtype=np.uint64)
    np.testing.assert_array_equal(_oracle_blocks(ctr, key), probe(ctr, key))


def test_jl_counter_layout(probe):
    """The words behind oracle.philox_normals come from the blocks at
    counter (element // 4, outer, inner, stream) under key (seed lo, seed hi):
    rebuild the normals from rocRAND's words with the Box-Muller map."""
    seed, i, j, stream = 0x0123456789ABCDEF, 3, 7, 5
    count = 64
    ctr = np.array([[b, i, j, stream] for b in range(count // 4)], np.uint64)
    key = np.array([[seed & 0xFFFFFFFF, seed >> 32]] * (count // 4), np.uint64)
    w = probe(ctr, key).astype(np.float64)
    u = (w + 0.5) * 2.0 ** -32
    z = np.empty_like(u)
    for a, b in ((0, 1), (2, 3)):
        R = np.sqrt(-2.0 * np.log(u[:, a]))
        z[:, a] = R * np.cos(2.0 * np.pi * u[:, b])
        z[:, b] = R * np.sin(2.0 * np.pi * u[:, b])
    np.testing.assert_array_equal(oracle.philox_normals(count, seed, i, j, stream), z.reshape(-1))
