"""Pins of the oracle's random-number layer (CPU only).

Philox4x32-10 is pinned to the published known-answer vectors and to an
independent library implementation (rocRAND's header-only round function);
the uniform map and Box-Muller normals are pinned by exact identities and by
goodness-of-fit tests against scipy's distributions.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = orc.philox(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(orc, tmp_path):
    exe = tmp_path / "rp"
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")
    subprocess.check_call(["hipcc", "-O1", "-x", "hip", "--cuda-host-only", src, "-o", str(exe)],
                          cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    words = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    words[0] = 0
    words[1] = 0xFFFFFFFF
    inp = "\n".join(" ".join("%08x" % int(v) for v in row) for row in words) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(v, 16) for v in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(words)
    for row, r in zip(words, ref):
        got = orc.philox([int(v) for v in row[:4]], [int(v) for v in row[4:]])
        assert [int(v) for v in got] == r


def test_key_layout(orc):
    k = orc.key(0x0123456789ABCDEF)
    assert int(k[0]) == 0x89ABCDEF
    assert int(k[1]) == 0x01234567 ^ 0x14078071


def test_u01_exact_and_open_interval(orc):
    lo = orc.u01(0)
    hi = orc.u01(0xFFFFFFFF)
    assert lo == 2.0**-24
    assert hi == 1.0 - 2.0**-24
    # every value is an exact float32
    xs = orc.philox_stream(3, 0, 0, 0, 4096)
    us = np.array([orc.u01(int(x)) for x in xs[:512]])
    assert np.all(us.astype(np.float32).astype(np.float64) == us)
    assert np.all((us > 0) & (us < 1))


def test_uniform_chi2_and_lag1(orc):
    n = 1 << 20
    xs = orc.philox_stream(11, 5, 9, (7 << 24), n)
    u = (2.0 * (xs >> 9).astype(np.float64) + 1.0) * 2.0**-24
    counts, _ = np.histogram(u, bins=1024, range=(0, 1))
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5.0 / np.sqrt(n)
    # the four lanes of one call are uncorrelated with each other
    lanes = u.reshape(-1, 4)
    cm = np.corrcoef(lanes.T)
    assert np.max(np.abs(cm - np.eye(4))) < 5.0 / np.sqrt(lanes.shape[0])


def test_box_muller_identities(orc):
    # z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi): pins the
    # lane pairing and the uniform map of the transform.
    k = orc.key(42)
    for c0 in range(64):
        ctr = [c0, 3, 17, (2 << 24) | 5]
        words = orc.philox(ctr, k)
        z = orc.normals4(ctr, k)
        u = [orc.u01(int(w)) for w in words]
        for a in (0, 2):
            assert z[a] ** 2 + z[a + 1] ** 2 == pytest.approx(-2.0 * np.log(u[a]), rel=1e-12)
            ang = np.arctan2(z[a + 1], z[a]) % (2 * np.pi)
            assert ang == pytest.approx(2 * np.pi * u[a + 1], abs=1e-9)


def test_normals_distribution(orc):
    n = 1 << 19
    z = orc.normal_stream(5, 1, 2, (2 << 24), n)
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
