"""Pins of the oracle's input classes (Sec. IV D, Sec. VI) and of the
Hamming truncation of the predicted good branches (Sec. V, Theorem 2).

A general input sum_ij c_ij |i>|j> puts any amplitude on every (address, bus
word) pair; the paper's scans draw 500 such branches at random.  Pinned here:
  - against the dense whole-register machine: component by component under
    the oracle's own jump histories, and the trajectory mean against the
    density matrix of the same input;
  - without noise the query is exact (fidelity 1) for any input;
  - an input with one bus word per address gives the same trajectories as
    the (c_i, j_i) form;
  - the reference is the smallest good address holding one bus word;
  - truncation keeps the predicted good branches' output words within wmax
    bit flips of their ideal word: recomputed from the exported state, and
    the dropped share of a good branch equals Theorem 2's tail."""
from math import comb

import numpy as np
import pytest

from oracle import dense as Dn

QUTRIT, QUBIT = 0, 1


def random_cab(n, k, seed, frac=0.5, single_frac=0.0):
    """Complex c_ij with about `frac` of the pairs present; with
    single_frac, that share of the addresses holds exactly one bus word."""
    rng = np.random.default_rng(seed)
    D, K = 1 << n, 1 << k
    c = (rng.normal(size=(D, K)) + 1j * rng.normal(size=(D, K))) * (rng.uniform(size=(D, K)) < frac)
    for i in range(D):
        if rng.uniform() < single_frac:
            j = rng.integers(K)
            v = c[i, j] if c[i, j] != 0 else 0.6 - 0.3j
            c[i] = 0.0
            c[i, j] = v
    c[0, 0] = 0.4 + 0.1j  # never empty
    return c


@pytest.mark.parametrize("n,k,enc,gamma,eps", [
    (2, 1, QUBIT, 0.12, 0.0), (2, 2, QUBIT, 0.08, 0.03), (3, 1, QUBIT, 0.06, 0.0),
    (2, 1, QUTRIT, 0.12, 0.02), (2, 2, QUTRIT, 0.1, 0.0)])
def test_ab_sparse_matches_dense_forced(orc, n, k, enc, gamma, eps):
    """The whole-register state vector from the same c_ij input, evolved
    through the oracle's own jumps and faults, equals the oracle's sparse
    state component by component (before the second wall)."""
    rng = np.random.default_rng(n * 100 + k * 10 + enc)
    mem = rng.integers(0, 2**k, size=2**n)
    cab = random_cab(n, k, 40 + n + k + enc)
    machine = Dn.Machine(n, k, enc, mem)
    seen_jump = 0
    for traj in range(8):
        r = orc.run_traj(n, k, enc, gamma, mem, seed=77, traj=traj, export=True, check_counts=True, eps=eps, cab=cab)
        assert r["max_exc"] < 1 << 20
        faults = []
        if eps > 0:
            L, ty = orc.sample_depol(n, k, enc, eps, 77, traj)
            act = orc.depol_active(n, k)
            off = np.concatenate([[0, 0], np.cumsum(act[1:])])
            for x, t in zip(L, ty):
                s = int(np.searchsorted(off, x, side="right") - 1)
                faults.append((s, int(x - off[s]), int(t) & 3, int(t) >> 2))
        m, psi = Dn.forced_evolution(n, k, enc, mem, gamma, r["jumps"], machine=machine, faults=faults, cab=cab)
        comp = r["components"]
        dig = np.zeros((len(comp["addr"]), m.ndig), dtype=np.int64)
        for x in range(len(comp["addr"])):
            for t in range(n):
                dig[x, m.A(t)] = (int(comp["addr"][x]) >> (n - 1 - t)) & 1
            for b in range(k):
                dig[x, m.B(b)] = (int(comp["bus"][x]) >> b) & 1
            dig[x, n + k:] = comp["tree"][x]
        idx = m.index(dig)
        assert len(np.unique(idx)) == len(idx)
        sparse = np.zeros(m.N, dtype=complex)
        sparse[idx] = comp["amp"]
        assert np.abs(sparse - psi).max() <= 1e-13 * np.abs(psi).max()
        seen_jump += r["njumps"] > 0
    assert seen_jump > 0


@pytest.mark.parametrize("enc,k,gamma,eps", [(QUBIT, 1, 0.05, 0.0), (QUBIT, 2, 0.04, 0.02), (QUTRIT, 2, 0.05, 0.02)])
def test_ab_trajectory_mean_matches_density(orc, enc, k, gamma, eps):
    n = 2
    rng = np.random.default_rng(11 + enc + k)
    mem = rng.integers(0, 2**k, size=4)
    cab = random_cab(n, k, 90 + enc + k, frac=0.6)
    F_rho, tr = Dn.density_fidelity(n, k, enc, mem, gamma, eps, cab=cab)
    assert abs(tr - 1.0) < 1e-12
    fid, fpre, _, _ = orc.run_many(n, k, enc, gamma, mem, 5150, 0, 20000, eps=eps, cab=cab)
    for f in (fid, fpre):
        se = f.std() / np.sqrt(len(f))
        assert abs(f.mean() - F_rho) < 4.5 * se + 1e-12, (f.mean(), F_rho, se)


@pytest.mark.parametrize("n,k,enc", [(3, 2, QUBIT), (4, 3, QUBIT), (3, 2, QUTRIT), (4, 3, QUTRIT)])
def test_ab_noise_free_exact(orc, n, k, enc):
    rng = np.random.default_rng(n + k + enc)
    mem = rng.integers(0, 2**k, size=2**n)
    cab = random_cab(n, k, 5 + n, frac=0.4)
    fid, fpre, st, _ = orc.run_many(n, k, enc, 0.0, mem, 1, 0, 4, cab=cab)
    assert np.allclose(fid, 1.0, atol=1e-12) and np.allclose(fpre, 1.0, atol=1e-12)
    assert np.all(st[:, 3] == (1 << n) << k)  # components: every (address, bus word) label


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_ab_single_bus_equals_cj_form(orc, enc):
    n, k, gamma, eps = 4, 2, 0.03, 0.01
    rng = np.random.default_rng(3 + enc)
    mem = rng.integers(0, 2**k, size=2**n)
    cin = rng.normal(size=2**n) + 1j * rng.normal(size=2**n)
    cin[[3, 9]] = 0.0
    jin = rng.integers(0, 2**k, size=2**n)
    cab = np.zeros((2**n, 2**k), dtype=complex)
    cab[np.arange(2**n), jin] = cin
    a = orc.run_many(n, k, enc, gamma, mem, 99, 0, 300, eps=eps, cin=cin, jin=jin)
    b = orc.run_many(n, k, enc, gamma, mem, 99, 0, 300, eps=eps, cab=cab)
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-14) and np.allclose(a[1], b[1], rtol=1e-12, atol=1e-14)
    cols = [0, 1, 2, 4, 5, 6, 7, 9]  # every statistic but the component count
    assert np.array_equal(a[2][:, cols], b[2][:, cols])


def test_ab_reference_rule(orc):
    """With a c_ij input the reference is the smallest good address that
    holds exactly one bus word (one branch)."""
    n, k = 5, 2
    mem = np.arange(2**n) % 4
    cab = random_cab(n, k, 17, frac=0.7, single_frac=0.3)
    single = (cab != 0).sum(axis=1) == 1
    _, _, st, _ = orc.run_many(n, k, QUBIT, 0.02, mem, 5, 0, 200, cab=cab)
    for t in range(200):
        L = orc.sample(n, k, 0.02, 5, t)
        bad = orc.classify(n, k, QUBIT, L)
        good = [i for i in range(2**n) if not bad[i] and single[i]]
        assert st[t, 2] == (good[0] if good else -1), t


def wall(v):
    """Walsh-Hadamard transform of the bus-word axis, normalised."""
    K = v.shape[-1]
    out = v.astype(complex).copy()
    h = 1
    while h < K:
        for b in range(K):
            if not b & h:
                x, y = out[..., b].copy(), out[..., b + h].copy()
                out[..., b], out[..., b + h] = x + y, x - y
        h *= 2
    return out / np.sqrt(K)


@pytest.mark.parametrize("n,k,gamma", [(3, 3, 0.04), (4, 4, 0.02), (3, 2, 0.1)])
def test_truncation_recomputed_from_state(orc, n, k, gamma):
    """No-jump history, one bus word per address: the truncated fidelity
    before the measurement equals the one recomputed from the exported state
    with the good branches' far words dropped; each good branch's dropped
    share is Theorem 2's tail sum_{w > wmax} C(k,w) alpha^2(k-w) beta^2w /
    (alpha^2 + beta^2)^k with alpha, beta = (1 +- a^(2n)) / 2."""
    rng = np.random.default_rng(n * 7 + k)
    D, K = 2**n, 2**k
    mem = rng.integers(0, K, size=D)
    cin = rng.normal(size=D) + 1j * rng.normal(size=D)
    cin[1] = 0.0
    jin = rng.integers(0, K, size=D)
    T = 6 * n + 2 * k
    ua = np.full(T, 0.5)
    ex = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=ua, forced_ufin=0.2, export=True,
                      cin=cin, jin=jin)
    comp = ex["components"]
    amp = np.zeros((D, K), dtype=complex)
    for x, a_, b_, v in zip(comp["label"], comp["addr"], comp["bus"], comp["amp"]):
        assert not comp["tree"][list(comp["label"]).index(x)].any()  # no jump: ground tree
        amp[a_, b_] += v
    out = wall(amp)  # [address, output word]
    cn = cin / np.linalg.norm(cin)
    want = (jin ^ mem) & (K - 1)
    ref = ex["ref"]
    assert ref == 0
    a = np.sqrt(1 - gamma)
    al, be = (1 + a ** (2 * n)) / 2, (1 - a ** (2 * n)) / 2
    ov = sum(np.conj(cn[i]) * out[i, want[i]] for i in range(D))
    ham = np.array([[bin(c ^ want[i]).count("1") for c in range(K)] for i in range(D)])
    for wmax in range(k + 1):
        r = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=ua, forced_ufin=0.2, cin=cin, jin=jin,
                         wmax=wmax)
        keep = np.ones((D, K), dtype=bool)
        for i in range(D):
            if i != ref and cn[i] != 0:
                keep[i] = ham[i] <= wmax
        wg = (np.abs(out) ** 2 * keep).sum()
        assert abs(r["fid_pre"] - abs(ov) ** 2 / wg) <= 1e-12 * r["fid_pre"], (wmax, r["fid_pre"], abs(ov) ** 2 / wg)
        tail = sum(comb(k, w) * al ** (2 * (k - w)) * be ** (2 * w) for w in range(wmax + 1, k + 1))
        for i in range(2, D):
            full = (np.abs(out[i]) ** 2).sum()
            dropped = (np.abs(out[i]) ** 2 * ~keep[i]).sum()
            assert abs(dropped / full - tail / (al ** 2 + be ** 2) ** k) <= 1e-12, (wmax, i)
    r = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=ua, forced_ufin=0.2, cin=cin, jin=jin,
                     wmax=k)
    assert r["fid_pre"] == orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=ua, forced_ufin=0.2,
                                        cin=cin, jin=jin)["fid_pre"]


def test_truncation_needs_one_bus_word(orc):
    n, k = 3, 2
    mem = np.arange(8) % 4
    cab = random_cab(n, k, 3, frac=0.8)
    assert ((cab != 0).sum(axis=1) > 1).any()
    with pytest.raises(ValueError):
        orc.run_many(n, k, QUBIT, 0.01, mem, 1, 0, 2, cab=cab, wmax=1)
    orc.run_many(n, k, QUBIT, 0.01, mem, 1, 0, 2, cab=cab, wmax=k)  # (no truncation)
