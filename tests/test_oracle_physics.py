"""Pins of the oracle's evolution, joint sampler and fidelity against what
the paper fixes: the density-matrix cross-check of App. C (Table 4), the
exactness of the joint damping sampler (Theorem 4), the closed forms of
Lemma 1 / Theorem 2 / Eq. caddr / Theorem 3 (qubit) and Proposition 1
(qutrit), the leakage law of Sec. IV E, and brute-force dense evolution."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import dense as Dn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
QUTRIT, QUBIT = 0, 1


def test_table4_density_matrix():
    """App. C, Table 4: F_rho = 0.5759 (gamma = 0.05), 0.1676 (gamma = 0.2)
    for the qubit encoding at n = 2, k = 1, memory 0110.  The dense checker
    applies the schedule gates then the damping channel on every tree qubit
    in each slice; the printed four digits pin that placement."""
    g = json.load(open(os.path.join(GOLDEN, "table4_damping.json")))
    for row in g["rows"]:
        F, tr = Dn.density_fidelity(g["n"], g["k"], QUBIT, g["memory_cells"], row["gamma"])
        assert abs(tr - 1.0) < 1e-12
        assert round(F, 4) == row["F_rho"], (row, F)


@pytest.mark.parametrize("enc,gamma,mem", [
    (QUBIT, 0.05, [0, 1, 1, 0]), (QUBIT, 0.2, [0, 1, 1, 0]), (QUTRIT, 0.05, [0, 1, 1, 0]),
    (QUBIT, 0.1, [1, 1, 0, 1]), (QUTRIT, 0.2, [1, 0, 0, 1])])
def test_trajectory_mean_matches_density(orc, enc, gamma, mem):
    """The trajectory ensemble reproduces the channel (Theorem 4): the mean
    post-measurement fidelity equals F_rho within Monte Carlo error, and the
    pre-measurement fidelity, whose mean is the same quantity, too."""
    F_rho, _ = Dn.density_fidelity(2, 1, enc, mem, gamma)
    fid, fpre, st, _ = orc.run_batch(2, 1, enc, gamma, mem, 880000 + int(gamma * 1000), 0, 40000)
    for f in (fid, fpre):
        se = f.std() / np.sqrt(len(f))
        assert abs(f.mean() - F_rho) < 4.5 * se + 1e-12, (f.mean(), F_rho, se)


@pytest.mark.parametrize("n,k,enc,gamma", [
    (2, 1, QUBIT, 0.15), (2, 2, QUBIT, 0.1), (3, 1, QUBIT, 0.06),
    (2, 1, QUTRIT, 0.15), (2, 2, QUTRIT, 0.1), (2, 2, QUTRIT, 0.3)])
def test_sparse_matches_dense_forced(orc, n, k, enc, gamma):
    """Brute force: the whole-register state vector, evolved through the
    oracle's own sequence of joint outcomes, equals the oracle's sparse state
    component by component (before the second wall)."""
    rng = np.random.default_rng(n * 100 + k * 10 + enc)
    mem = rng.integers(0, 2**k, size=2**n)
    seen_jump = 0
    machine = Dn.Machine(n, k, enc, mem)
    for traj in range(8):
        r = orc.run_traj(n, k, enc, gamma, mem, seed=31, traj=traj, export=True, check_counts=True)
        assert r["max_exc"] < 1 << 20, "excitation bookkeeping"
        m, psi = Dn.forced_evolution(n, k, enc, mem, gamma, r["jumps"], machine=machine)
        comp = r["components"]
        dig = np.zeros((len(comp["addr"]), m.ndig), dtype=np.int64)
        for x in range(len(comp["addr"])):
            for t in range(n):
                dig[x, m.A(t)] = (int(comp["addr"][x]) >> (n - 1 - t)) & 1
            for b in range(k):
                dig[x, m.B(b)] = (int(comp["bus"][x]) >> b) & 1
            dig[x, n + k:] = comp["tree"][x]
        idx = m.index(dig)
        assert len(np.unique(idx)) == len(idx), "components are distinct basis states"
        sparse = np.zeros(m.N, dtype=complex)
        sparse[idx] = comp["amp"]
        scale = np.abs(psi).max()
        assert np.abs(sparse - psi).max() <= 1e-13 * scale
        seen_jump += r["njumps"] > 0
    assert seen_jump > 0


def _subsets(M):
    for r in range(M + 1):
        for C in itertools.combinations(range(M), r):
            yield C


@pytest.mark.parametrize("enc,s,hist", [
    (QUBIT, 6, []), (QUBIT, 9, [(4, 1)]), (QUTRIT, 6, []), (QUTRIT, 10, [(5, 0)])])
def test_joint_sampler_exact(orc, enc, s, hist):
    """Theorem 4: averaging the mask weights w_C(J)/W (Eq. maskweight) over
    the state-independent candidate draw C gives <psi|K_J^+ K_J|psi>/<psi|psi>
    for every joint outcome J, computed here on the dense state."""
    n, k, gamma = 2, 1, 0.3
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = [0, 1, 1, 0]
    # a forced earlier history: candidates hist=(slice, site) with u=1-eps
    L = sorted((ss - 1) * M + q for ss, q in hist)
    ua = np.full(T, 1.0 - 1e-15)
    pre = orc.run_traj(n, k, enc, gamma, mem, forced_L=L, forced_uaux=ua)
    jumps = [j for j in pre["jumps"] if j[0] < s]
    m, psi = Dn.layer_state(n, k, enc, mem, gamma, jumps, s)
    norm = np.vdot(psi, psi).real
    # distribution from the sampler
    P = {}
    for C in _subsets(M):
        pC = gamma ** len(C) * (1 - gamma) ** (M - len(C))
        masks, we = orc.layer_masks(n, k, enc, gamma, mem, L, ua, s, list(C))
        W = we + sum(masks.values())
        P[()] = P.get((), 0.0) + pC * we / W
        for mask, w in masks.items():
            J = tuple((C[j], lev) for j, lev in enumerate(mask) if lev)
            P[J] = P.get(J, 0.0) + pC * w / W
    # exact outcome probabilities of the layer Kraus operators
    tree = m.digits[:, n + k:]
    nexc = (tree != 0).sum(axis=1)
    pw = np.abs(psi) ** 2 / norm
    exact = {}
    for x in np.nonzero(pw > 0)[0]:
        exc = [(q, int(tree[x, q])) for q in range(M) if tree[x, q]]
        for r in range(len(exc) + 1):
            for J in itertools.combinations(exc, r):
                pj = gamma ** len(J) * (1 - gamma) ** (nexc[x] - len(J))
                exact[J] = exact.get(J, 0.0) + pw[x] * pj
    keys = set(P) | set(exact)
    assert abs(sum(P.values()) - 1) < 1e-12 and abs(sum(exact.values()) - 1) < 1e-12
    for J in keys:
        assert abs(P.get(J, 0.0) - exact.get(J, 0.0)) < 1e-12, J
    assert len(exact) > 1


def c_addr(n, k, i):
    """Eq. caddr: sum over address bits t with i_t = 1 of T - 4t - 2."""
    T = 6 * n + 2 * k
    return sum(T - 4 * t - 2 for t in range(n) if (i >> (n - 1 - t)) & 1)


def _wht(vec, k):
    out = np.zeros(2**k, dtype=complex)
    for c in range(2**k):
        for b in range(2**k):
            out[c] += (-1) ** bin(b & c).count("1") * vec[b]
    return out / np.sqrt(2**k)


@pytest.mark.parametrize("n,k,gamma", [
    (2, 1, 1e-5), (2, 2, 3e-2), (3, 3, 1e-3), (4, 2, 1e-2), (5, 1, 3e-2), (6, 3, 1e-4), (8, 1, 1e-3)])
def test_qubit_good_branch_closed_form(orc, n, k, gamma):
    """No-jump qubit trajectory: after the second wall each address i holds
    a^{c_addr(i)} c_i alpha^{k-w} beta^w at word c, w = Ham(c xor d_i)
    (Lemma 1, Theorem 2, Eq. caddr, Theorem 3), with the tree in its ground
    state; normalised word probabilities follow Fig. 4a."""
    T = 6 * n + 2 * k
    rng = np.random.default_rng(n + 17 * k)
    mem = rng.integers(0, 2**k, size=2**n)
    r = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=np.zeros(T), export=True)
    comp = r["components"]
    assert np.all(comp["tree"] == 0)
    a = np.sqrt(1 - gamma)
    al, be = (1 + a ** (2 * n)) / 2, (1 - a ** (2 * n)) / 2
    ci = 1 / np.sqrt(2**n)
    for i in range(2**n):
        sel = comp["addr"] == i
        vec = np.zeros(2**k, dtype=complex)
        vec[comp["bus"][sel]] = comp["amp"][sel]
        out = _wht(vec, k)
        for c in range(2**k):
            w = bin(c ^ int(mem[i])).count("1")
            want = ci * a ** c_addr(n, k, i) * al ** (k - w) * be**w
            assert abs(out[c] - want) <= 1e-14 * abs(ci), (i, c)
        p = np.abs(out) ** 2 / np.sum(np.abs(out) ** 2)
        for c in range(2**k):
            w = bin(c ^ int(mem[i])).count("1")
            want = al ** (2 * (k - w)) * be ** (2 * w) / (al**2 + be**2) ** k
            # the small amplitude beta comes out of the wall as a difference of
            # O(1) terms, so its error is absolute (a few ulp of the total)
            assert abs(p[c] - want) <= 1e-12 * want + 1e-15


def no_jump_fidelity_qubit(n, k, gamma):
    """Closed form of the no-jump fidelity for the data-loading input:
    prod_t g(a^{T-4t-2}) g(a^{2n})^k with g(u) = (1+u)^2 / (2(1+u^2))."""
    T = 6 * n + 2 * k
    a = np.sqrt(1 - gamma)
    g = lambda u: (1 + u) ** 2 / (2 * (1 + u * u))
    F = g(a ** (2 * n)) ** k
    for t in range(n):
        F *= g(a ** (T - 4 * t - 2))
    return F


@pytest.mark.parametrize("n,k,gamma", [(6, 1, 1e-4), (6, 1, 1e-3), (6, 1, 1e-2), (4, 3, 1e-3), (8, 2, 1e-5)])
def test_qubit_no_jump_fidelity(orc, n, k, gamma):
    T = 6 * n + 2 * k
    mem = np.random.default_rng(3).integers(0, 2**k, size=2**n)
    r = orc.run_traj(n, k, QUBIT, gamma, mem, forced_L=[], forced_uaux=np.zeros(T), forced_ufin=0.5)
    assert r["q_ground"] == 1
    assert abs(r["fid"] - no_jump_fidelity_qubit(n, k, gamma)) < 1e-13


def qutrit_exposure(n, k, i, d):
    """Exposure count c(i) of Proposition 1 for the qutrit circuit with bus
    input 0: every stored router is excited from its store to its unstore
    (T - 6t - 4 slices), an address bit with i_t = 1 is excited in transit
    for 2(t+1) slices, and a data bit is excited for the n slices after its
    fetch when d_b = 1."""
    T = 6 * n + 2 * k
    c = sum(T - 6 * t - 4 for t in range(n))
    c += sum(2 * (t + 1) for t in range(n) if (i >> (n - 1 - t)) & 1)
    c += n * bin(int(d)).count("1")
    return c


@pytest.mark.parametrize("n,k,gamma", [(2, 1, 1e-3), (3, 2, 3e-2), (5, 3, 1e-2), (7, 1, 1e-4)])
def test_qutrit_proposition1(orc, n, k, gamma):
    """Proposition 1: a no-jump qutrit branch ends as a^{c(i)} |i>|d_i>|Q0>
    with the all-W tree; relative weights are (1-gamma)^{Delta c} (Fig. 4b)."""
    T = 6 * n + 2 * k
    mem = np.random.default_rng(n * 7 + k).integers(0, 2**k, size=2**n)
    r = orc.run_traj(n, k, QUTRIT, gamma, mem, forced_L=[], forced_uaux=np.zeros(T), export=True, forced_ufin=0.1)
    comp = r["components"]
    assert len(comp["addr"]) == 2**n
    assert np.all(comp["tree"] == 0)
    a = np.sqrt(1 - gamma)
    ci = 1 / np.sqrt(2**n)
    for x in range(2**n):
        i = int(comp["addr"][x])
        assert comp["bus"][x] == mem[i]
        assert abs(comp["amp"][x] - ci * a ** qutrit_exposure(n, k, i, mem[i])) <= 1e-14 * ci
    assert abs(r["fid"] - r["fid_pre"]) < 1e-15
    # closed form of the no-jump fidelity
    e = np.array([qutrit_exposure(n, k, i, mem[i]) for i in range(2**n)], dtype=float)
    F = np.sum(a**e) ** 2 / (2**n * np.sum(a ** (2 * e)))
    assert abs(r["fid"] - F) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_coherent_leakage(orc, n):
    """Sec. IV E: conditional on no jump, a data qubit is wrong with
    probability beta^2/(alpha^2+beta^2) = n^2 gamma^2/4 + O(gamma^3); log-log
    slope 2 and prefactor ratio -> 1 (Fig. 5a)."""
    k = 1
    T = 6 * n + 2 * k
    mem = np.random.default_rng(n).integers(0, 2, size=2**n)
    gs = np.array([1e-6, 1e-5, 1e-4])
    err = []
    for g in gs:
        r = orc.run_traj(n, k, QUBIT, g, mem, forced_L=[], forced_uaux=np.zeros(T), export=True)
        comp = r["components"]
        sel = comp["addr"] == 0
        vec = np.zeros(2, dtype=complex)
        vec[comp["bus"][sel]] = comp["amp"][sel]
        out = _wht(vec, 1)
        p = np.abs(out) ** 2 / np.sum(np.abs(out) ** 2)
        e = p[1 - int(mem[0])]
        a = np.sqrt(1 - g)
        al, be = (1 + a ** (2 * n)) / 2, (1 - a ** (2 * n)) / 2
        assert abs(e - be**2 / (al**2 + be**2)) <= 1e-9 * e
        err.append(e)
    err = np.array(err)
    slope = np.polyfit(np.log(gs), np.log(err), 1)[0]
    assert abs(slope - 2.0) < 5e-3
    assert abs(err[0] / (n * n * gs[0] ** 2 / 4) - 1) < 1e-4


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_gamma_zero(orc, enc):
    mem = np.random.default_rng(0).integers(0, 2**3, size=2**5)
    fid, fpre, st, _ = orc.run_batch(5, 3, enc, 0.0, mem, 1, 0, 20)
    assert np.allclose(fid, 1.0, atol=1e-14) and np.allclose(fpre, 1.0, atol=1e-14)
    assert np.all(st[:, 0] == 0) and np.all(st[:, 1] == 0)


def test_norm_loss_decomposition():
    """Sec. IV E: the per-qubit no-jump norm (1 + a^{4n})/2 and the exact
    split (1 - a^{2n})/2 = (1 - a^{4n})/4 + (1 - a^{2n})^2/4, evaluated on the
    oracle-independent closed forms used by the pins above."""
    for n in (2, 6, 10):
        for g in (1e-5, 1e-3, 0.1):
            a = np.sqrt(1 - g)
            al, be = (1 + a ** (2 * n)) / 2, (1 - a ** (2 * n)) / 2
            assert abs(al**2 + be**2 - (1 + a ** (4 * n)) / 2) < 1e-15
            assert abs((1 - a ** (2 * n)) / 2 - ((1 - a ** (4 * n)) / 4 + (1 - a ** (2 * n)) ** 2 / 4)) < 1e-15
