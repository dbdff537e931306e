"""Pins of the oracle's random stream: Philox4x32-10 words and Box-Muller normals."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x32_10, uniform_fp64, box_muller, normals_for_draw, seed_key

HERE = os.path.dirname(os.path.abspath(__file__))


def test_known_answer_vectors():
    """Published Random123 known-answer vectors (tests/golden/philox4x32_10_kat.txt)."""
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(o) for o in out] == r[6:10]


def _torch_include():
    try:
        import torch
    except ImportError:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) else None


@pytest.mark.skipif(shutil.which("g++") is None or _torch_include() is None,
                    reason="needs g++ and PyTorch's C++ headers")
def test_against_torch_engine(tmp_path):
    """Random counters/keys against PyTorch's independent C++ Philox engine."""
    exe = tmp_path / "philox_torch"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", _torch_include(),
                    os.path.join(HERE, "golden", "philox_torch_engine.cpp"), "-o", str(exe)],
                   check=True)
    rng = np.random.Generator(np.random.PCG64(1234))
    cases = rng.integers(0, 2 ** 63, size=(40, 3), dtype=np.int64).astype(np.uint64)
    cases[:, 0] ^= np.uint64(1) << np.uint64(63)
    args = [str(int(v)) for v in cases.ravel()]
    out = subprocess.run([str(exe)] + args, check=True, capture_output=True, text=True).stdout
    got = np.array([[int(t) for t in l.split()] for l in out.strip().splitlines()], dtype=np.uint64)
    seed, sub, off = (int(c) for c in cases[:, 0]), cases[:, 1], cases[:, 2]
    k = np.array([seed_key(int(s)) for s in cases[:, 0]])
    mask = np.uint64(0xFFFFFFFF)
    for i in range(cases.shape[0]):
        mine = philox4x32_10(off[i] & mask, off[i] >> np.uint64(32), sub[i] & mask,
                             sub[i] >> np.uint64(32), int(k[i, 0]), int(k[i, 1]))
        assert [int(v) for v in mine] == [int(v) for v in got[i]]


def test_uniform_open_interval():
    u = uniform_fp64(np.array([0, 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64))
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 2.0 ** -33 and u[-1] == 1.0 - 2.0 ** -33


def test_box_muller_distribution():
    n = 400_000
    p = np.arange(n, dtype=np.uint64)
    (ax, ay), (bx, by) = normals_for_draw(3, p, 17, 2, seed=99)
    z = np.concatenate([ax, ay, bx, by])
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # components of one draw are independent
    assert abs(np.corrcoef(ax, ay)[0, 1]) < 5.0 / np.sqrt(n)
    assert abs(np.corrcoef(ax, bx)[0, 1]) < 5.0 / np.sqrt(n)
    # fourth moment of a standard normal is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_box_muller_closed_form():
    """u0 = e^-1/2, u1 = 1/8: rho = 1, theta = pi/4."""
    c, s = box_muller(np.array([np.exp(-0.5)]), np.array([0.125]))
    assert np.allclose([c[0], s[0]], [np.sqrt(0.5), np.sqrt(0.5)], rtol=1e-14)


def test_stream_keys_distinct():
    """Different knots, paths, draws or instances give different words."""
    base = np.array([int(v) for v in philox4x32_10(5, 6, 7, 8, 1, 2)])
    for c in [(6, 6, 7, 8), (5, 7, 7, 8), (5, 6, 8, 8), (5, 6, 7, 9)]:
        other = np.array([int(v) for v in philox4x32_10(*c, 1, 2)])
        assert np.all(other != base)
