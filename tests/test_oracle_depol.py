"""Pins of the oracle's depolarizing noise (Sec. II B, Sec. III B, App. C)
and of its general input class (Sec. IV D).

- Table 4's Pauli (p = 0.02: F_rho 0.7263) and Mixed (p = gamma = 0.02:
  0.5841) rows through the dense density matrix: they fix the channel
  placement (active positions), the {X, Z, ZX} mixture and the order within a
  slice (gates, depolarizing, damping).
- The oracle's trajectory mean equals the density-matrix value within Monte
  Carlo error (the fault draw and the joint damping sampler reproduce the
  channel), in both encodings.
- The sparse oracle equals a dense state vector under forced histories of
  faults of every type on any site, with damping jumps.
- The X half of the exhaustive single-fault injection at n = 3, k = 3: no
  wrong bus word outside the fault's subtree, no divergent tree
  configuration outside Eq. badrange, and the union over slices and slots
  reaches Eq. badrange exactly (Sec. VI B).
- General inputs: the trajectory mean equals the density matrix of the
  general input state.
"""
import json
import os

import numpy as np
import pytest

from oracle import dense as Dn

QUTRIT, QUBIT = 0, 1
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table4_depolarizing_rows():
    g = json.load(open(os.path.join(GOLDEN, "table4_depolarizing.json")))
    for row in g["rows"]:
        F, tr = Dn.density_fidelity(g["n"], g["k"], QUBIT, g["memory_cells"], row["gamma"], row["eps"])
        assert abs(tr - 1.0) < 1e-12
        assert round(F, 4) == row["F_rho"], (row, F)


def test_table4_order_and_placement_discriminate():
    """The pins fail for the nearest other readings: damping before the
    faults, or faults on every tree site."""
    m = Dn.Machine(2, 1, QUBIT, [0, 1, 1, 0])
    psi = m.wall(m.input_state())

    def run(order, sites):
        rho = np.outer(psi, psi.conj())
        for s in range(1, m.T):
            rho = m.gates_rho(rho, s)
            if order == "damp":
                rho = m.damp_rho(rho, 0.02)
            for q in sites(s):
                ops = m.fault_ops(q)
                new = 0.98 * rho
                for a, b in ops:
                    dest, ph = m._fault_map(q, a, b)
                    r = np.zeros_like(rho)
                    r[np.ix_(dest, dest)] = (ph[:, None] * np.conj(ph)[None, :]) * rho
                    new = new + (0.02 / len(ops)) * r
                rho = new
            if order == "depol":
                rho = m.damp_rho(rho, 0.02)
        rho = m.wall_rho(rho)
        pid = m.ideal_state()
        return float(np.real(pid.conj() @ rho @ pid))

    assert round(run("depol", m.active_sites), 4) == 0.5841
    assert round(run("damp", m.active_sites), 4) != 0.5841
    assert round(run("depol", lambda s: range(m.M)), 4) != 0.5841


def test_active_positions(orc):
    """App. C placement: a prefix of the sites, mirror symmetric in the
    schedule, the root's two sites only at n = 2 (slices 3..11)."""
    a = orc.depol_active(2, 1)
    assert list(a[1:]) == [0, 0, 2, 2, 2, 2, 2, 2, 2, 2, 2, 0, 0]
    for n, k in ((3, 3), (4, 2), (6, 1), (10, 4)):
        a = orc.depol_active(n, k)
        T = 6 * n + 2 * k
        for s in range(1, T):
            assert a[s] == a[T - s]
            l = np.log2(a[s] // 2 + 1)
            assert l == int(l) and l <= n - 1


@pytest.mark.parametrize("enc,gamma,eps,n,k,mem", [
    (QUBIT, 0.0, 0.02, 2, 1, [0, 1, 1, 0]), (QUBIT, 0.02, 0.02, 2, 1, [0, 1, 1, 0]),
    (QUBIT, 0.01, 0.04, 2, 2, [1, 2, 3, 0]),
    (QUTRIT, 0.0, 0.05, 2, 1, [0, 1, 1, 0]), (QUTRIT, 0.05, 0.05, 2, 1, [1, 0, 1, 1]),
    (QUTRIT, 0.02, 0.08, 2, 1, [1, 1, 0, 1])])
def test_depolarizing_trajectory_mean_matches_density(orc, enc, gamma, eps, n, k, mem):
    F_rho, _ = Dn.density_fidelity(n, k, enc, mem, gamma, eps)
    fid, fpre, st, _ = orc.run_many(n, k, enc, gamma, mem, 550000 + n, 0, 25000, eps=eps)
    assert st[:, 9].sum() > 500  # faults were drawn
    for f in (fid, fpre):
        se = f.std() / np.sqrt(len(f))
        assert abs(f.mean() - F_rho) < 4.5 * se + 1e-12, (f.mean(), F_rho, se)


def test_fault_sampler_statistics(orc):
    """Faults are Bernoulli(eps) on the active positions; types are uniform
    over X, Z, ZX on qubits and over the eight Weyl operators on a qutrit
    router."""
    for enc in (QUBIT, QUTRIT):
        n, k, eps = 4, 2, 0.03
        S = int(orc.depol_active(n, k).sum())
        counts, types_d, types_r = [], {}, {}
        for t in range(3000):
            L, ty = orc.sample_depol(n, k, enc, eps, 99, t)
            assert np.all(np.diff(L.astype(np.int64)) > 0) and (len(L) == 0 or L[-1] < S)
            counts.append(len(L))
            for x, y in zip(L, ty):
                # the site of linear index x
                act = orc.depol_active(n, k)
                s = np.searchsorted(np.cumsum(act), x, side="right")
                q = int(x - np.cumsum(act)[s - 1]) if s > 0 else int(x)
                d = types_r if (enc == QUTRIT and q % 2 == 0) else types_d
                d[int(y)] = d.get(int(y), 0) + 1
        c = np.array(counts, dtype=float)
        assert abs(c.mean() - S * eps) < 5 * np.sqrt(S * eps * (1 - eps) / len(c))
        assert abs(c.var() - S * eps * (1 - eps)) < 0.15 * S * eps
        want_d = {1 | 0 << 2, 0 | 1 << 2, 1 | 1 << 2}
        assert set(types_d) == want_d
        tot = sum(types_d.values())
        for v in types_d.values():
            assert abs(v / tot - 1 / 3) < 5 * np.sqrt((1 / 3) * (2 / 3) / tot)
        if enc == QUTRIT:
            assert len(types_r) == 8
            tot = sum(types_r.values())
            for v in types_r.values():
                assert abs(v / tot - 1 / 8) < 5 * np.sqrt((1 / 8) * (7 / 8) / tot)


def _dense_index(m, addr, bus, tree):
    dig = np.zeros(m.ndig, dtype=np.int64)
    for t in range(m.n):
        dig[m.A(t)] = (addr >> (m.n - 1 - t)) & 1
    for b in range(m.k):
        dig[m.B(b)] = (bus >> b) & 1
    for q in range(m.M):
        dig[m.S(q)] = tree[q]
    return m.index(dig)


@pytest.mark.parametrize("n,k,enc,gamma", [(2, 1, QUBIT, 0.1), (3, 1, QUBIT, 0.05), (2, 2, QUTRIT, 0.1),
                                           (2, 1, QUTRIT, 0.2)])
def test_sparse_matches_dense_with_faults(orc, n, k, enc, gamma):
    """Forced histories: random faults of every type on any tree site, the
    oracle's own damping jumps; the oracle's final components equal the dense
    state vector entry by entry."""
    rng = np.random.default_rng(n * 31 + enc)
    mem = rng.integers(0, 2**k, size=2**n)
    m = Dn.Machine(n, k, enc, mem)
    T, M = m.T, m.M
    njumps = 0
    for trial in range(10):
        faults = []
        for _ in range(int(rng.integers(1, 5))):
            s, q = int(rng.integers(1, T)), int(rng.integers(0, M))
            a, b = m.fault_ops(q)[int(rng.integers(0, len(m.fault_ops(q))))]
            faults.append((s, q, a, b))
        faults.sort()
        L = np.sort(rng.choice((T - 1) * M, size=int(rng.integers(0, 6)), replace=False)).astype(np.uint32)
        ua = rng.uniform(0, 1, size=T)
        r = orc.run_traj(n, k, enc, gamma, mem, forced_L=L, forced_uaux=ua, forced_ufin=0.5,
                         forced_dep=faults, export=True, check_counts=True)
        assert r["max_exc"] < 1 << 20
        njumps += r["njumps"]
        _, psi = Dn.forced_evolution(n, k, enc, mem, gamma, r["jumps"], machine=m, faults=faults)
        oc = r["components"]
        dense = psi.copy()
        for addr, bus, amp, tree in zip(oc["addr"], oc["bus"], oc["amp"], oc["tree"]):
            x = _dense_index(m, int(addr), int(bus), tree)
            assert abs(dense[x] - amp) <= 1e-12 * max(1.0, abs(amp)), (trial, addr, bus)
            dense[x] = 0.0
        assert np.abs(dense).max() <= 1e-12, trial  # nothing the oracle lacks
    assert njumps > 0


def test_x_fault_injection_envelope(orc):
    """Sec. III B / Sec. VI B: every X flip at every tree position and event
    slice of the n = 3, k = 3 query (322 cases).  After the second wall,
    address i's branch state should be |d_i> with the tree configuration
    shared by the branches outside the envelope.  Wrong bus words stay inside
    the fault node's subtree, divergent branches inside Eq. badrange, and
    over all slices and slots of a node the divergent branches fill Eq.
    badrange exactly."""
    g = json.load(open(os.path.join(GOLDEN, "single_fault_injection.json")))
    n, k = g["n"], g["k"]
    T, M, D, K2 = 6 * n + 2 * k, 2 * (2**n - 1), 2**n, 2**k
    mem = np.random.default_rng(5).integers(0, K2, size=D).astype(np.uint32)

    def layer_of(v):
        return (v + 1).bit_length() - 1

    def subtree(v):
        l = layer_of(v)
        p = v - (2**l - 1)
        return set(range(p * 2 ** (n - l), (p + 1) * 2 ** (n - l)))

    def supports(r):
        groups = {}
        oc = r["components"]
        for addr, bus, amp, tree in zip(oc["addr"], oc["bus"], oc["amp"], oc["tree"]):
            Q = tuple(np.nonzero(tree)[0])
            v = groups.setdefault((int(addr), Q), np.zeros(K2, complex))
            v[int(bus)] += amp
        sup = {i: set() for i in range(D)}
        H = np.array([[(-1) ** bin(b & c).count("1") for b in range(K2)] for c in range(K2)])
        for (i, Q), v in groups.items():
            out = H @ v
            for c in range(K2):
                if abs(out[c]) > 1e-9:
                    sup[i].add((c, Q))
        return sup

    cases = viol = 0
    union = {}
    for q in range(M):
        v = q >> 1
        bad = subtree(orc.range_node(QUBIT, v))
        for s in range(1, T):
            r = orc.run_traj(n, k, QUBIT, 0.0, mem, forced_L=[], forced_uaux=np.zeros(T), forced_ufin=0.5,
                             forced_dep=[(s, q, 1, 0)], export=True)
            sup = supports(r)
            outside = [i for i in range(D) if i not in bad]
            qref = None
            if outside:  # the configuration the branches outside the envelope share
                qs = {Q for i in outside for (_, Q) in sup[i]}
                assert len(qs) == 1, (q, s, qs)
                qref = qs.pop()
            wrong = {i for i in range(D) if any(c != mem[i] for c, _ in sup[i])}
            diverged = {i for i in range(D) if sup[i] != {(int(mem[i]), qref)}}
            cases += 1
            if not (wrong <= subtree(v) and diverged <= bad):
                viol += 1
            union.setdefault(v, set()).update(diverged)
    assert cases == g["x_cases"]
    assert viol == g["x_violations"]
    for v in range(2**n - 1):
        assert union[v] == subtree(orc.range_node(QUBIT, v)), v


@pytest.mark.parametrize("enc,gamma,eps", [(QUBIT, 0.05, 0.0), (QUBIT, 0.03, 0.03), (QUTRIT, 0.05, 0.02)])
def test_general_input_trajectory_mean(orc, enc, gamma, eps):
    """A general input sum_i c_i |i>|j_i> (complex c_i, one bus word per
    address, some addresses absent): the trajectory mean equals the density
    matrix of that input, whose ideal output is sum_i c_i |i>|j_i xor d_i>."""
    n, k = 2, 1
    rng = np.random.default_rng(7 + enc)
    mem = rng.integers(0, 2, size=4)
    cin = rng.normal(size=4) + 1j * rng.normal(size=4)
    cin[2] = 0.0
    cin /= np.linalg.norm(cin)
    jin = rng.integers(0, 2, size=4)
    m = Dn.Machine(n, k, enc, mem)
    psi = np.zeros(m.N, dtype=complex)
    ideal = np.zeros(m.N, dtype=complex)
    for i in range(4):
        dig = np.zeros(m.ndig, dtype=np.int64)
        for t in range(n):
            dig[m.A(t)] = (i >> (n - 1 - t)) & 1
        dig[m.B(0)] = jin[i]
        psi[m.index(dig)] = cin[i]
        dig[m.B(0)] = jin[i] ^ (mem[i] & 1)
        ideal[m.index(dig)] = cin[i]
    if enc == QUBIT:
        psi = m.wall(psi)
    rho = np.outer(psi, psi.conj())
    for s in range(1, m.T):
        rho = m.gates_rho(rho, s)
        if eps:
            rho = m.depol_rho(rho, s, eps)
        rho = m.damp_rho(rho, gamma)
    if enc == QUBIT:
        rho = m.wall_rho(rho)
    F_rho = float(np.real(ideal.conj() @ rho @ ideal))
    fid, fpre, st, _ = orc.run_many(n, k, enc, gamma, mem, 4040, 0, 25000, eps=eps, cin=cin, jin=jin)
    for f in (fid, fpre):
        se = f.std() / np.sqrt(len(f))
        assert abs(f.mean() - F_rho) < 4.5 * se + 1e-12, (f.mean(), F_rho, se)
    # no noise: the query is exact
    f0, _, _, _ = orc.run_many(n, k, enc, 0.0, mem, 1, 0, 10, cin=cin, jin=jin)
    assert np.allclose(f0, 1.0, atol=1e-12)


def test_invalid_shapes_raise(orc):
    """Shapes outside the schedule's range (k > n, k > 8) are refused with an
    error, on every entry, with and without the depolarizing extras."""
    from paper_2609_34935_amd.inputs import memory_words
    for n, k in [(2, 7), (3, 4), (9, 9)]:
        mem = memory_words(n, min(k, 8), 1)
        with pytest.raises(ValueError):
            orc.run_many(n, k, 1, 0.01, mem, 1, 0, 4)
        with pytest.raises(ValueError):
            orc.run_many(n, k, 0, 0.01, mem, 1, 0, 4, eps=0.01)
        with pytest.raises(ValueError):
            orc.sample_depol(n, k, 1, 0.01, 1, 0)
