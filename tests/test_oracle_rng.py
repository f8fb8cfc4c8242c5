"""Pins of the oracle's random-number layer: Philox4x32-10 against rocRAND's
independent implementation, the geometric threshold table, and the
statistics of the candidate history (Sec. IV D: each tree site of each slice
is a candidate independently with probability gamma)."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPER_SRC = os.path.join(ROOT, "tests", "philox_rocrand.cpp")
HELPER_BIN = os.path.join(ROOT, "tests", "_build", "philox_rocrand")


def _rocrand_blocks(rows):
    if not os.path.exists(HELPER_BIN) or os.path.getmtime(HELPER_BIN) < os.path.getmtime(HELPER_SRC):
        os.makedirs(os.path.dirname(HELPER_BIN), exist_ok=True)
        try:
            subprocess.check_call(["hipcc", "-O1", "-o", HELPER_BIN, HELPER_SRC])
        except (OSError, subprocess.CalledProcessError):
            pytest.skip("hipcc/rocRAND headers unavailable")
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([HELPER_BIN], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand(orc):
    rng = np.random.default_rng(12345)
    # rocRAND reaches counter word c1 through a 64-bit offset 4 (c0 | c1 << 32),
    # so c1 stays below 2^30 here
    rows = [[0, 0, 0, 0, 0, 0], [1, 2, 3, 4, 5, 6], [2**32 - 1, 2**30 - 1] + [2**32 - 1] * 4]
    r = rng.integers(0, 2**32, size=(200, 6))
    r[:, 1] %= 2**30
    rows += r.tolist()
    # counters of the shapes the sampler uses: (block, draw, traj, tag)
    rows += [[b, j, t, tag, 880003, 0] for b in (0, 1, 2141) for j in (0, 1) for t in (0, 99999) for tag in (1, 2, 3)]
    ref = _rocrand_blocks(rows)
    for r, want in zip(rows, ref):
        got = orc.philox(r[:4], r[4:])
        assert [int(v) for v in got] == [int(v) for v in want], r


def test_thresholds(orc):
    assert np.all(orc.thresholds(0.0) == 0)
    for g in (1e-5, 1e-3, 0.05, 0.5):
        Gi = orc.thresholds(g)
        assert np.all(Gi[1:] >= Gi[:-1])
        sat = Gi == np.uint64(2**64 - 1)
        assert np.all(Gi[1:][~sat[1:]] > Gi[:-1][~sat[1:]])
        G = Gi.astype(np.float64)
        o = np.arange(64)
        want = (1.0 - (1.0 - g) ** (o + 1)) * 2.0**64
        # relative accuracy limited by 1 - (1-g)^(o+1) in double precision
        assert np.allclose(G, want, rtol=1e-9, atol=2.0**12)


def test_uniform_domain(orc):
    us = np.array([orc.uniform(7, s, 0, t, 2) for s in range(1, 40) for t in range(50)])
    assert np.all((us >= 0.0) & (us < 1.0))
    assert abs(us.mean() - 0.5) < 0.03


@pytest.mark.parametrize("n,k,gamma", [(3, 1, 0.02), (6, 1, 1e-3), (4, 2, 0.1)])
def test_candidate_statistics(orc, n, k, gamma):
    """#candidates ~ Binomial(S, gamma); positions uniform over slices, sites
    and block offsets (no artefact at the 64-site block boundaries)."""
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    S = (T - 1) * M
    ntraj = 3000
    counts = np.zeros(ntraj)
    allL = []
    for t in range(ntraj):
        L = orc.sample(n, k, gamma, 4242, t)
        assert np.all(np.diff(L.astype(np.int64)) > 0), "ascending, no repeats"
        assert np.all(L < S)
        counts[t] = len(L)
        allL.append(L)
    allL = np.concatenate(allL).astype(np.int64)
    mean, var = S * gamma, S * gamma * (1 - gamma)
    se = np.sqrt(var / ntraj)
    assert abs(counts.mean() - mean) < 5 * se
    assert abs(counts.var() / var - 1) < 0.15
    # uniformity of block offsets and of slices: chi-square with generous bound
    off = allL % 64
    last = S % 64
    full_blocks = S // 64
    exp_off = np.full(64, full_blocks, dtype=np.float64)
    if last:
        exp_off[:last] += 1
    exp_off *= gamma * ntraj
    h = np.bincount(off, minlength=64)
    chi = ((h - exp_off) ** 2 / exp_off).sum()
    assert chi < 64 + 6 * np.sqrt(2 * 64)
    sl = allL // M
    h = np.bincount(sl, minlength=T - 1)
    e = gamma * ntraj * M
    chi = ((h - e) ** 2 / e).sum()
    assert chi < (T - 1) + 6 * np.sqrt(2 * (T - 1))


def test_sampler_reproducible(orc):
    a = orc.sample(10, 4, 1e-3, 880003, 17)
    b = orc.sample(10, 4, 1e-3, 880003, 17)
    c = orc.sample(10, 4, 1e-3, 880003, 18)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert len(orc.sample(10, 4, 0.0, 1, 1)) == 0
