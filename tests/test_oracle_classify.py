"""Pins of the marking rule: Eq. (subtree) for the qutrit encoding and
Eq. (badrange) for the qubit encoding, the marking-source count of
Eq. (marksources), and E[B] of Eq. (eb)."""
import numpy as np
import pytest

QUTRIT, QUBIT = 0, 1


def _layer(v):
    return int(np.floor(np.log2(v + 1)))


def subtree_leaves(n, v):
    """Eq. subtree: leaf range [2^{n-l} p, 2^{n-l}(p+1) - 1] of node (l, p)."""
    l = _layer(v)
    p = v + 1 - 2**l
    return set(range(2 ** (n - l) * p, 2 ** (n - l) * (p + 1)))


def bad_set(n, enc, v):
    """Direct recursion of Eq. badrange (qubit) / Eq. subtree (qutrit)."""
    if enc == QUTRIT:
        return subtree_leaves(n, v)
    if v == 0:
        return set(range(2**n))
    if v in (1, 2) or v % 2 == 0:
        return subtree_leaves(n, v)
    return bad_set(n, enc, (v - 1) // 2)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 10])
def test_marking_sources(orc, n):
    """Eq. marksources: sum_v |bad(v)| / 2^n = n + (n-1)(n-2)/4 for the
    family-divergence rule and n for the subtree rule."""
    k = 1
    M = 2 * (2**n - 1)
    tot = {QUBIT: 0, QUTRIT: 0}
    for enc in (QUBIT, QUTRIT):
        for v in range(2**n - 1):
            bad = orc.classify(n, k, enc, [2 * v])
            tot[enc] += int(bad.sum())
            if n <= 6:
                assert set(np.nonzero(bad)[0]) == bad_set(n, enc, v)
            # both sites of the node mark the same range
            assert np.array_equal(bad, orc.classify(n, k, enc, [2 * v + 1 + M]))
    assert tot[QUBIT] / 2**n == n + (n - 1) * (n - 2) / 4
    assert tot[QUTRIT] / 2**n == n


@pytest.mark.parametrize("n,enc", [(3, QUBIT), (4, QUBIT), (5, QUTRIT), (4, QUTRIT)])
def test_union_brute_force(orc, n, enc):
    """The bad set of a candidate list is the union of the per-candidate
    ranges (Alg. 1 step 1), by brute force over random lists."""
    k = 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    rng = np.random.default_rng(n * 3 + enc)
    for _ in range(200):
        L = np.sort(rng.choice((T - 1) * M, size=rng.integers(0, 6), replace=False))
        want = set()
        for Lj in L:
            want |= bad_set(n, enc, int(Lj % M) // 2)
        got = set(np.nonzero(orc.classify(n, k, enc, L))[0])
        assert got == want


@pytest.mark.parametrize("n,k,gamma,enc", [(6, 1, 1e-3, QUBIT), (6, 1, 1e-2, QUTRIT), (4, 2, 5e-3, QUBIT)])
def test_expected_bad_branches(orc, n, k, gamma, enc):
    """Eq. eb: an address with s_i marking-source nodes is bad with
    probability 1 - (1-gamma)^{2 (T-1) s_i}."""
    T = 6 * n + 2 * k
    s_i = np.zeros(2**n)
    for v in range(2**n - 1):
        for i in bad_set(n, enc, v):
            s_i[i] += 1
    EB = np.sum(1 - (1 - gamma) ** (2 * (T - 1) * s_i))
    B = []
    for t in range(4000):
        L = orc.sample(n, k, gamma, 99, t)
        B.append(int(orc.classify(n, k, enc, L).sum()))
    B = np.array(B)
    assert abs(B.mean() - EB) < 5 * B.std() / np.sqrt(len(B)) + 1e-9


@pytest.mark.parametrize("n,k,gamma", [(3, 3, 6e-3), (4, 2, 3e-3), (5, 1, 1.5e-3), (4, 1, 2e-2)])
def test_subtree_marking_exact_under_damping(orc, n, k, gamma):
    """Sec. III B and Sec. VI B: a damping jump needs an excitation and idle
    qubits have none, so damping creates no strays and, in the qubit
    encoding, the components a damping jump leaves alive all lie inside the
    candidates' own subtrees (Eq. subtree), a subset of Eq. badrange.
    Pruning with the tighter set is exact when no address outside it
    survives any trajectory in which a jump fired (with no jump, every
    component follows its no-jump orbit).  Checked on the full evolution of
    sampled histories with random auxiliary draws."""
    T = 6 * n + 2 * k
    rng = np.random.default_rng(100 * n + k)
    mem = rng.integers(0, 2**k, size=2**n)
    fired = tighter = 0
    for t in range(400):
        L = orc.sample(n, k, gamma, 4242, t)
        sub = orc.classify(n, k, QUBIT, L, subtree=True).astype(bool)
        wide = orc.classify(n, k, QUBIT, L).astype(bool)
        assert np.all(wide[sub])  # Eq. subtree marks a subset of Eq. badrange
        r = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=L,
                         forced_uaux=rng.random(T), export=True)
        if r["njumps"] == 0:
            continue
        fired += 1
        addrs = r["components"]["addr"]
        assert np.all(sub[addrs]), (t, L)
        tighter += int(np.any(wide & ~sub))
    assert fired >= 20 and tighter >= 5, (fired, tighter)
