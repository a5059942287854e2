"""Pins of the oracle's Philox4x32-10, index sampler and Gaussian noise."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


def test_known_answer_vectors():
    for r in _kat():
        ctr, key, want = r[0:4], r[4:6], tuple(r[6:10])
        assert philox.philox4x32_10_scalar(ctr, key) == want
        got = philox.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
        assert tuple(int(g[0]) for g in got) == want


def test_vector_matches_scalar_random_counters():
    rng = np.random.default_rng(7)
    c = rng.integers(0, 2 ** 32, size=(4, 2000), dtype=np.uint64)
    k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
    vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1])
    for i in range(0, 2000, 37):
        want = philox.philox4x32_10_scalar([int(c[j, i]) for j in range(4)], [int(k[0]), int(k[1])])
        assert tuple(int(v[i]) for v in vec) == want


ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
struct Engine : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
  Engine e;
  unsigned a[6];
  while (scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    uint4 r = e.rounds(uint4{a[0], a[1], a[2], a[3]}, uint2{a[4], a[5]});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def test_matches_rocrand_host_engine():
    """Cross-implementation pin: rocRAND's Philox4x32-10 engine run on the host."""
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "kat.cpp")
        exe = os.path.join(td, "kat")
        with open(src, "w") as f:
            f.write(ROCRAND_SRC)
        subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", src, "-o", exe], check=True,
                       capture_output=True)
        rng = np.random.default_rng(11)
        c = rng.integers(0, 2 ** 32, size=(6, 5000), dtype=np.uint64)
        lines = "\n".join(" ".join("%08x" % int(c[j, i]) for j in range(6)) for i in range(5000))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        got = np.array([[int(t, 16) for t in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
        vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], c[4], c[5])
        for j in range(4):
            np.testing.assert_array_equal(got[:, j], vec[j].astype(np.uint64))


def test_index_sampler_definition_and_range():
    seed, u, size, n = 2, 5, 65536 + 13, 4096
    idx = philox.sample_indices(seed, u, size, n)
    assert idx.min() >= 0 and idx.max() < size
    for b in range(0, n, 97):
        w0 = philox.philox4x32_10_scalar([u, 0, b, 0], [seed & 0xFFFFFFFF, seed >> 32])[0]
        assert idx[b] == (w0 * size) >> 32


def test_index_sampler_uniform_chi2():
    size, n = 64, 200000
    idx = np.concatenate([philox.sample_indices(2, u, size, n // 10) for u in range(10)])
    counts = np.bincount(idx, minlength=size)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4


def test_gaussian_moments_and_ks():
    e = philox.gaussian(2, 3, 1, 200000)
    assert abs(e.mean()) < 0.01 and abs(e.std() - 1.0) < 0.01
    assert stats.kstest(e, "norm").pvalue > 1e-4
    e2 = philox.gaussian(2, 3, 2, 1000)
    assert not np.allclose(e[:1000], e2)


def test_box_muller_closed_form_points():
    # u = ((w >> 9) + 0.5) 2^-23: for w0 >> 9 = 2^22 - 1, u1 = 1/2 - 2^-24;
    # for w1 >> 9 = 2^21 (and low bits set, which are dropped), u2 = 1/4 + 2^-24.
    w0 = np.array([((2 ** 22 - 1) << 9) | 0x1FF], dtype=np.uint32)
    w1 = np.array([(2 ** 21) << 9 | 0x155], dtype=np.uint32)
    u1, u2 = 0.5 - 2.0 ** -24, 0.25 + 2.0 ** -24
    want = np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    assert philox.box_muller(w0, w1)[0] == pytest.approx(want, rel=1e-15)
