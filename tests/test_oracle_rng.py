"""Pins for the oracle's random streams: Philox4x32-10, uniforms, normals and
the Feistel minibatch permutation."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import batch, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers():
    for row in _kat():
        out = philox.philox4x32_10(*row[0:4], row[4], row[5])
        assert [int(v) for v in out] == row[6:10]


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Expose : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Expose e; unsigned a[6];
  while (scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    uint4 c = {a[0], a[1], a[2], a[3]}; uint2 k = {a[4], a[5]};
    uint4 r = e.rounds(c, k);
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host_code(tmp_path):
    """Cross-check against rocRAND's own Philox4x32-10 rounds, run on the host."""
    src = tmp_path / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    rng = np.random.default_rng(5)
    words = rng.integers(0, 1 << 32, size=(300, 6), dtype=np.uint64)
    words[0] = 0
    words[1] = 0xFFFFFFFF
    inp = "\n".join(" ".join("%08x" % int(v) for v in row) for row in words) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = np.array([[int(v, 16) for v in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    for r, row in enumerate(words):
        out = philox.philox4x32_10(*[int(v) for v in row[0:4]], int(row[4]), int(row[5]))
        assert [int(v) for v in out] == [int(v) for v in got[r]]


def test_uniform52_range_and_grid():
    assert philox.uniform52(0, 0) == 0.5 / 2.0 ** 52
    top = philox.uniform52(0xFFFFFFFF, 0xFFFFFFFF)
    assert 0.0 < top < 1.0
    assert top == 1.0 - 0.5 / 2.0 ** 52
    # 26 + 26 bits: the grid step is 2^-52, the low 6 bits of each word unused
    assert philox.uniform52(0, 64) - philox.uniform52(0, 0) == 2.0 ** -52
    assert philox.uniform52(0, 63) == philox.uniform52(0, 0)
    assert philox.uniform52(64, 0) - philox.uniform52(0, 0) == 2.0 ** -26
    # symmetric grid: u and 1 - u both occur
    assert philox.uniform52(0, 0) + top == 1.0


def test_normals_are_standard():
    eta = philox.noise(1234, 3, 2, 17, np.arange(50_000))
    flat = eta.reshape(-1)
    assert abs(flat.mean()) < 4 * 1 / np.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 4 * np.sqrt(2.0 / flat.size)
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    # the four components are uncorrelated
    c = np.corrcoef(eta.T)
    assert np.abs(c - np.eye(4)).max() < 0.03


def test_noise_streams_differ_and_repeat():
    a = philox.noise(9, 0, 0, 5, np.arange(100))
    assert np.array_equal(a, philox.noise(9, 0, 0, 5, np.arange(100)))
    for other in [philox.noise(9, 0, 1, 5, np.arange(100)), philox.noise(9, 1, 0, 5, np.arange(100)),
                  philox.noise(9, 0, 0, 6, np.arange(100)), philox.noise(10, 0, 0, 5, np.arange(100))]:
        assert np.abs(a - other).min() > 0.0


@pytest.mark.parametrize("N", [1, 2, 3, 5, 17, 100, 1023, 1024, 1025, 32000, 65536])
def test_feistel_is_a_bijection(N):
    for chain, epoch in [(0, 0), (3, 7)]:
        y = batch.permute(np.arange(N, dtype=np.uint64), N, 42, 1, chain, epoch)
        assert np.array_equal(np.sort(y), np.arange(N))


def test_feistel_raw_network_is_bijective_on_power_of_two():
    N = 1 << 13
    y = batch.feistel(np.arange(N, dtype=np.uint64), N - 3, 7, 0, 0, 0)
    assert np.array_equal(np.sort(y), np.arange(N))


def test_epoch_batches_are_disjoint_and_cover():
    N, n = 32000, 1024
    B = N // n
    seen = np.concatenate([batch.batch_indices(3, 0, 0, t, N, n) for t in range(B)])
    assert len(np.unique(seen)) == B * n
    nxt = batch.batch_indices(3, 0, 0, B, N, n)
    assert not np.array_equal(nxt, seen[:n])
    other_chain = batch.batch_indices(3, 0, 1, 0, N, n)
    assert not np.array_equal(other_chain, seen[:n])


def test_permutation_is_not_trivial():
    N = 4096
    y = batch.permute(np.arange(N, dtype=np.uint64), N, 1, 0, 0, 0)
    # a random permutation has about one fixed point; Spearman correlation ~ 0
    assert (y == np.arange(N)).sum() < 10
    assert abs(stats.spearmanr(y, np.arange(N)).statistic) < 0.1
