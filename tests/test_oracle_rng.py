"""Pins of the oracle's counter-based RNG (Philox-4x32-10, uniforms, normals)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def _kats():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kats())
def test_philox_known_answers(ctr, key, want):
    assert list(O.philox4x32_10(ctr, key)) == want


PROBE = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int i = 1; i + 1 < argc; i += 2) {
    unsigned long long seed = strtoull(argv[i], 0, 0), sub = strtoull(argv[i + 1], 0, 0);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, 0, &st);
    uint4 v = rocrand4(&st);
    printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host_build(tmp_path):
    """rocRAND's philox engine, compiled for the host from its open header:
    rocrand_init(seed, subsequence, 0) starts at counter (0, 0, sub lo, sub hi)
    with key (seed lo, seed hi)."""
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(PROBE)
    subprocess.check_call(["hipcc", "--cuda-host-only", "-x", "hip", str(src), "-o", str(exe)])
    rng = np.random.default_rng(1234)
    pairs = [(0, 0), (2**64 - 1, 0), (0x299F31D0A4093822, 1)]
    pairs += [(int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40))) for _ in range(300)]
    args = [str(v) for p in pairs for v in p]
    out = subprocess.check_output([str(exe)] + args, text=True).split("\n")
    for (seed, sub), line in zip(pairs, out):
        want = [int(x) for x in line.split()]
        ctr = [0, 0, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert list(O.philox4x32_10(ctr, key)) == want


def test_draw_counter_layout():
    """draw() places (t, row, purpose | sub << 8, epoch) in the counter and
    the 64-bit seed in the key."""
    seed = 0x0123456789ABCDEF
    got = O.draw(seed, 7, 11, O.RESET, 3, 5)
    want = O.philox4x32_10([7, 11, 1 | (3 << 8), 5], [0x89ABCDEF, 0x01234567])
    assert list(got) == list(want)


def test_u01_exact_values():
    assert O.u01(0) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2**32, 2000, dtype=np.uint64):
        u = O.u01(int(x))
        m = u * 2**24
        assert 0.0 < u < 1.0
        assert m == int(m) and int(m) % 2 == 1           # odd multiple of 2^-24
        assert float(np.float32(u)) == u                 # exact in FP32
        assert int(m) >> 1 == int(x) >> 9                # top 23 bits


def test_u01_uniform_chi2():
    words = np.concatenate([O.draw(0, t, 0, O.ACTION, 0, 0) for t in range(5000)])
    u = np.array([O.u01(int(w)) for w in words])
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    assert stats.chisquare(hist).pvalue > 1e-4


def test_box_muller_normal():
    rng = np.random.default_rng(3)
    u1 = (2 * rng.integers(0, 2**23, 20000) + 1) * 2.0**-24
    u2 = (2 * rng.integers(0, 2**23, 20000) + 1) * 2.0**-24
    z = np.array([O.box_muller(a, b) for a, b in zip(u1, u2)])
    for col in (0, 1):
        assert stats.kstest(z[:, col], "norm").pvalue > 1e-4
    # the pair is the polar point (r cos, r sin) with r^2 = -2 ln u1
    assert np.allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u1), rtol=1e-12)
    assert np.corrcoef(z[:, 0], z[:, 1])[0, 1] ** 2 < 1e-3
