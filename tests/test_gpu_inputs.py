"""Inputs with amplitudes on (address, bus word) pairs (Sec. IV D; the random
branch sets of Sec. VI) and the Hamming truncation of the predicted good
branches (Sec. V) on the HIP path, against the oracle.

Every mode runs on the plain engine for these contexts: the full modes
evolve every component; the pruned mode evolves the bad addresses and the
reference (the smallest good address holding one bus word) and predicts the
good ones from it, bus word by bus word for addresses holding several
(Theorem 3).  Checked: fidelities within 1e-12 relative and the integer
statistics identical in every mode, the paper's 500-branch uniform input at
n = 10, k = 3, exported components with their complex amplitudes, and the
truncated fidelities for every w_max."""
import numpy as np
import pytest

from paper_2609_34935_amd.inputs import memory_words

pytestmark = pytest.mark.gpu

QUTRIT, QUBIT = 0, 1
FULL, PRUNED, PLAIN = 0, 1, 2


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_34935_amd as P
    P.load_library()
    return P


def fid_close(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) <= 1e-12 * np.maximum(np.abs(b), 1e-3)


def check(f, st, fo, fpo, so, label):
    bad = np.nonzero(~fid_close(f, fo))[0]
    assert len(bad) == 0, (label, bad[:5], f[bad[:5]], fo[bad[:5]])
    assert np.all(fid_close(st["fid_pre"], fpo)), label
    ref = np.where(so[:, 2] < 0, 0xFFFFFFFF, so[:, 2]).astype(np.uint32)
    assert np.array_equal(st["n_cand"], so[:, 0].astype(np.uint32)), label
    assert np.array_equal(st["n_bad"], so[:, 1].astype(np.uint32)), label
    assert np.array_equal(st["ref_addr"], ref), label
    assert np.array_equal(st["n_jumps"], so[:, 4].astype(np.uint16)), label
    assert np.array_equal(st["first_jump_slice"], so[:, 5].astype(np.uint16)), label
    assert np.array_equal(st["ref_survived"], so[:, 6].astype(np.uint8)), label
    assert np.array_equal(st["q_ground"], so[:, 7].astype(np.uint8)), label


def random_pairs(n, k, seed, frac=0.5, single_frac=0.3):
    rng = np.random.default_rng(seed)
    D, K = 1 << n, 1 << k
    c = (rng.normal(size=(D, K)) + 1j * rng.normal(size=(D, K))) * (rng.uniform(size=(D, K)) < frac)
    for i in range(D):
        if rng.uniform() < single_frac:
            j = rng.integers(K)
            v = c[i, j] if c[i, j] != 0 else 0.5 + 0.5j
            c[i] = 0.0
            c[i, j] = v
    c[0, 0] = 0.3 - 0.2j
    return c


def branch_set(n, k, nb, seed):
    """nb branches drawn without replacement from the 2^(n+k) (address, bus
    word) pairs, uniform weights (the full superposition when 2^(n+k) <= nb)."""
    rng = np.random.default_rng(seed)
    N = (1 << n) << k
    c = np.zeros(N, dtype=complex)
    c[rng.choice(N, size=min(nb, N), replace=False)] = 1.0
    return c.reshape(1 << n, 1 << k)


def run_mode(ctx, mode, seed, t0, nt):
    if mode == PLAIN:
        return ctx.run_plain(seed, t0, nt)
    return (ctx.run_full if mode == FULL else ctx.run_pruned)(seed, t0, nt)


@pytest.mark.parametrize("n,k,enc,gamma,eps,nt", [
    (3, 2, QUBIT, 0.03, 0.0, 300), (4, 2, QUBIT, 0.01, 0.005, 300), (5, 3, QUBIT, 2e-3, 1e-3, 300),
    (6, 2, QUBIT, 1e-3, 0.0, 300),
    (3, 2, QUTRIT, 0.03, 0.0, 300), (4, 2, QUTRIT, 0.01, 0.005, 300), (5, 3, QUTRIT, 2e-3, 1e-3, 300)])
def test_pair_input_every_mode(lib, orc, n, k, enc, gamma, eps, nt):
    mem = memory_words(n, k, 300 + n)
    cab = random_pairs(n, k, 17 + n + 10 * enc)
    fo, fpo, so, _ = orc.run_many(n, k, enc, gamma, mem, 4711, traj0=3, ntraj=nt, eps=eps, cab=cab)
    multi_good_no_jump = 0
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps, input_ab=cab) as ctx:
        for mode in (FULL, PRUNED, PLAIN):
            f, st = run_mode(ctx, mode, 4711, 3, nt)
            check(f, st, fo, fpo, so, (n, k, enc, mode))
            if mode == PRUNED:
                multi_good_no_jump = int(((st["n_jumps"] == 0) & (st["ref_addr"] != 0xFFFFFFFF)).sum())
    assert multi_good_no_jump > 0  # the bus-word-by-bus-word prediction ran


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_branch_set_500_n10(lib, orc, enc):
    """The scans' input: 500 branches with uniform weights drawn from the
    2^(n+k) pairs, n = 10, k = 3, eps = gamma = 1e-3; 4096 trajectories in
    every mode, the first 160 against the oracle, pruned equal to full on all."""
    n, k, gamma, eps, nt, no = 10, 3, 1e-3, 1e-3, 4096, 160
    mem = memory_words(n, k, 510)
    cab = branch_set(n, k, 500, 77 + enc)
    assert ((cab != 0).sum(axis=1) > 1).any()
    fo, fpo, so, _ = orc.run_many(n, k, enc, gamma, mem, 9090, traj0=0, ntraj=no, eps=eps, cab=cab, nthreads=16)
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps, input_ab=cab) as ctx:
        fp, sp = ctx.run_pruned(9090, 0, nt)
        ff, sf = ctx.run_full(9090, 0, nt)
    check(fp[:no], sp[:no], fo, fpo, so, ("500", enc, PRUNED))
    check(ff[:no], sf[:no], fo, fpo, so, ("500", enc, FULL))
    assert np.all(fid_close(fp, ff))
    for fld in ("n_cand", "n_bad", "ref_addr", "n_jumps", "q_ground", "ref_survived"):
        assert np.array_equal(sp[fld], sf[fld]), fld
    assert sp["n_explicit"].mean() < sf["n_explicit"].mean()


@pytest.mark.parametrize("n,k,gamma", [(4, 3, 0.02), (6, 4, 3e-3), (5, 2, 0.01)])
def test_truncation_every_w(lib, orc, n, k, gamma):
    mem = memory_words(n, k, 600 + n)
    rng = np.random.default_rng(n + k)
    cin = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    cin[rng.uniform(size=1 << n) < 0.2] = 0.0
    cin[0] = 0.8
    jin = rng.integers(0, 1 << k, size=1 << n).astype(np.uint32)
    cab = np.zeros((1 << n, 1 << k), dtype=complex)
    cab[np.arange(1 << n), jin] = cin
    nt = 300
    exact = None
    for w in range(k + 1):
        fo, fpo, so, _ = orc.run_many(n, k, QUBIT, gamma, mem, 321, traj0=0, ntraj=nt, cab=cab, wmax=w)
        if w == k:
            exact = fo
        with lib.QramContext(n, k, QUBIT, gamma, mem, input_ab=cab, w_max=w) as ctx:
            for mode in (FULL, PRUNED):
                f, st = run_mode(ctx, mode, 321, 0, nt)
                check(f, st, fo, fpo, so, ("trunc", w, mode))
        with lib.QramContext(n, k, QUBIT, gamma, mem, input_amp=cin, input_bus=jin, w_max=w) as ctx:
            f, st = ctx.run_pruned(321, 0, nt)
            check(f, st, fo, fpo, so, ("trunc c_i", w))
    fo0, _, _, _ = orc.run_many(n, k, QUBIT, gamma, mem, 321, traj0=0, ntraj=nt, cab=cab)
    assert np.array_equal(exact, fo0)


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_export_pair_input(lib, orc, enc):
    n, k, gamma, eps = 3, 2, 0.05, 0.02
    mem = memory_words(n, k, 44)
    cab = random_pairs(n, k, 5 + enc)
    K = 1 << k
    seen_jump = 0
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps, input_ab=cab) as ctx:
        for t in range(40):
            ref = orc.run_traj(n, k, enc, gamma, mem, seed=12, traj=t, export=True, eps=eps, cab=cab)
            seen_jump += ref["njumps"] > 0
            oc = ref["components"]
            want = {int(x): (int(oc["addr"][j]), int(oc["bus"][j]),
                             sorted((q, int(v)) for q, v in enumerate(oc["tree"][j]) if v), oc["amp"][j])
                    for j, x in enumerate(oc["label"])}
            scale = max(np.abs(oc["amp"]).max(), 1e-300)
            for mode in (FULL, PLAIN):
                out = ctx.export_state(mode, 12, t)
                got = {}
                for x, r in enumerate(out["records"]):
                    if (r[0] >> 25) & 1:
                        got[x] = (int(r[0]) & 0xFFFF, (int(r[0]) >> 16) & 0xFF,
                                  sorted((int(v) & 0xFFFF, int(v) >> 16) for v in r[3:3 + int(r[2])]), out["amp"][x])
                assert sorted(got) == sorted(want), (t, mode)
                for x, (a, b, tr, amp) in got.items():
                    wa, wb, wt, wamp = want[x]
                    assert (a, b, tr) == (wa, wb, wt), (t, mode, x)
                    assert x // K == a
                    assert abs(amp - wamp) <= 1e-12 * max(abs(wamp), 1e-3 * scale), (t, mode, x)
                assert abs(out["fid"] - ref["fid"]) <= 1e-12 * max(abs(ref["fid"]), 1e-3)
    assert seen_jump > 0


def test_pair_input_refused_combinations(lib):
    n, k = 3, 2
    mem = memory_words(n, k, 1)
    cab = random_pairs(n, k, 9, single_frac=0.0)
    with pytest.raises(lib.QramError):
        lib.QramContext(n, k, QUBIT, 0.01, mem, input_ab=cab, w_max=1)  # several bus words per address
    with pytest.raises(lib.QramError):
        lib.QramContext(n, k, QUBIT, 0.01, mem, input_ab=cab, input_amp=np.ones(8))
    with pytest.raises(lib.QramError):
        lib.QramContext(n, k, QUBIT, 0.01, mem, w_max=k + 1)
    with lib.QramContext(n, k, QUBIT, 0.01, mem, input_ab=cab, w_max=k) as ctx:  # w_max = k: no truncation
        ctx.run_pruned(1, 0, 10)
