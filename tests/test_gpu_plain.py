"""The plain full evolution (QRAM_MODE_PLAIN: every component of every branch
with its own site list and complex amplitude, slice by slice) against the
oracle: fidelities within 1e-12 relative, integer statistics and jump logs
identical, on small trees with strong damping, the C1/C2 configurations,
sampled C3 trajectories and forced histories; and equal to the pruned mode
on the same trajectories."""
import os

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


def decode_jlog(entries):
    return sorted((int(x) >> 24, int(x) & 0xFFFF, (int(x) >> 16) & 0xFF) for x in entries)


def check_against_oracle(f, st, fo, fpo, so, label):
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
    assert np.all((st["flags"] & 2) == 0), label


@pytest.mark.parametrize("n,k,enc,gamma,ntraj", [
    (1, 1, QUBIT, 0.3, 300), (2, 1, QUBIT, 0.2, 400), (3, 2, QUBIT, 0.08, 300), (4, 4, QUBIT, 0.03, 150),
    (1, 1, QUTRIT, 0.3, 300), (2, 1, QUTRIT, 0.2, 400), (3, 1, QUTRIT, 0.08, 300), (4, 2, QUTRIT, 0.05, 200),
    (5, 3, QUBIT, 0.02, 200), (6, 2, QUTRIT, 0.02, 200)])
def test_plain_small_high_gamma(lib, orc, n, k, enc, gamma, ntraj):
    mem = memory_words(n, k, 77 + n)
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, 12345, 0, ntraj)
    assert so[:, 4].sum() > 0
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        f, st = ctx.run_plain(12345, 0, ntraj)
        fp, sp = ctx.run_pruned(12345, 0, ntraj)
    check_against_oracle(f, st, fo, fpo, so, (n, k, enc, gamma))
    assert np.all(fid_close(f, fp))


def test_plain_config1_all(lib, orc):
    mem = memory_words(3, 1, 1001)
    fo, fpo, so, _ = orc.run_batch(3, 1, QUTRIT, 1e-3, mem, 880001, 0, 1000)
    with lib.QramContext(3, 1, QUTRIT, 1e-3, mem) as ctx:
        f, st = ctx.run_plain(880001, 0, 1000)
    check_against_oracle(f, st, fo, fpo, so, "C1")


@pytest.mark.parametrize("gamma", [1e-4, 1e-3, 1e-2])
def test_plain_config2_all(lib, orc, gamma):
    mem = memory_words(6, 1, 1002)
    fo, fpo, so, _ = orc.run_batch(6, 1, QUBIT, gamma, mem, 880002, 0, 10000)
    with lib.QramContext(6, 1, QUBIT, gamma, mem) as ctx:
        f, st = ctx.run_plain(880002, 0, 10000)
    check_against_oracle(f, st, fo, fpo, so, ("C2", gamma))


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_plain_config3_sampled(lib, orc, enc):
    """n = 10, k = 4, gamma = 1e-3: 4096 trajectories equal the pruned mode;
    the first 160 equal the oracle, jump logs included."""
    n, k, gamma, nt = 10, 4, 1e-3, 4096
    mem = memory_words(n, k, 1003)
    no = 160
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, 880003, 0, no, nthreads=min(16, os.cpu_count() or 1))
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        f, st, jl, njl = ctx.run_jumplog(PLAIN, 880003, 0, nt, 32)
        fp, sp = ctx.run_pruned(880003, 0, nt)
    check_against_oracle(f[:no], st[:no], fo, fpo, so, ("C3", enc))
    assert np.all(fid_close(f, fp))
    for fld in ("n_cand", "n_bad", "n_jumps", "first_jump_slice", "q_ground"):
        assert np.array_equal(st[fld], sp[fld]), fld
    for t in range(no):
        ref = orc.run_traj(n, k, enc, gamma, mem, seed=880003, traj=t)["jumps"] if njl[t] or so[t, 4] else []
        assert decode_jlog(jl[t, :njl[t]]) == sorted(ref), t


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_plain_forced_histories(lib, orc, enc):
    n, k = 4, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 21)
    rng = np.random.default_rng(500 + enc)
    cases = [([], np.full(T, 0.5), 0.3),
             ([(8 - 1) * M + 4, (9 - 1) * M + 5], np.full(T, 0.999999), 0.1),
             ([(2 * n + 1 - 1) * M + 1], np.full(T, 0.9999), 0.2),
             ([(12 - 1) * M + 2, (12 - 1) * M + 6], np.full(T, 0.99999), 0.5)]
    for trial in range(30):
        L = np.sort(rng.choice((T - 1) * M, size=int(rng.integers(1, 16)), replace=False))
        cases.append((L, rng.uniform(0.3, 1.0, size=T), float(rng.uniform())))
    with lib.QramContext(n, k, enc, 0.05, mem) as ctx:
        for L, ua, uf in cases:
            L = np.asarray(L, dtype=np.uint32)
            ref = orc.run_traj(n, k, enc, 0.05, mem, forced_L=L, forced_uaux=ua, forced_ufin=uf)
            f, st = ctx.run_forced(PLAIN, L, ua, uf)
            assert fid_close(f, ref["fid"]), (f, ref["fid"])
            assert fid_close(st["fid_pre"], ref["fid_pre"])
            assert st["n_jumps"] == ref["njumps"] and st["first_jump_slice"] == ref["first_jump"]
            assert st["q_ground"] == ref["q_ground"] and st["ref_survived"] == ref["ref_survived"]


@pytest.mark.parametrize("n,k,enc,gamma,nsample,nt", [
    (15, 1, QUBIT, 1e-3, 2, 64),    # largest qubit tree: 65536 components per trajectory
    (14, 8, QUTRIT, 2e-3, 2, 64),   # largest qutrit tree and data word
    (8, 8, QUBIT, 1e-2, 4, 128)])   # widest qubit bus word (every mode on the plain engine)
def test_plain_maximum_sizes(lib, orc, n, k, enc, gamma, nsample, nt):
    """The plain evolution at the largest trajectories, where its pool's
    pieces lie furthest apart: the first trajectories equal the oracle, all
    of them the pruned mode."""
    mem = memory_words(n, k, 4100 + n + k)
    seed = 991000 + n
    print(f"plain maximum size n={n} k={k} enc={enc}: {nt} trajectories", flush=True)
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, seed, 0, nsample, nthreads=min(16, os.cpu_count() or 1))
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        f, st = ctx.run_plain(seed, 0, nt)
        fp, sp = ctx.run_pruned(seed, 0, nt)
    check_against_oracle(f[:nsample], st[:nsample], fo, fpo, so, ("max", n, k, enc))
    assert np.all(fid_close(f, fp))
    for fld in ("n_cand", "n_jumps", "first_jump_slice", "q_ground"):
        assert np.array_equal(st[fld], sp[fld]), fld


@pytest.mark.parametrize("per_cu,threads", [(1, 0), (2, 256), (4, 128), (8, 64), (32, 64), (3, 128)])
def test_plain_launch_shapes(lib, orc, per_cu, threads):
    n, k, enc, gamma, nt = 5, 3, QUBIT, 0.03, 700
    mem = memory_words(n, k, 55)
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, 99, 3, nt)
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        ctx.set_launch(PLAIN, per_cu, threads)
        got = ctx.get_launch(PLAIN)
        assert got[1] == (threads or got[1]) and 1 <= got[0] <= per_cu
        f, st = ctx.run_plain(99, 3, nt)
    check_against_oracle(f, st, fo, fpo, so, per_cu)


@pytest.mark.parametrize("enc,n,k", [(QUBIT, 5, 3), (QUTRIT, 6, 2)])
def test_plain_register_budgets(lib, orc, enc, n, k):
    """Asking for more workgroups per compute unit than the unconstrained
    build holds selects the kernel's capped register budgets (short records,
    small slabs: registers set the limit); every budget gives the oracle's
    results, and the same fidelities bit for bit."""
    gamma, nt = 0.03, 900
    mem = memory_words(n, k, 57)
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, 98, 0, nt)
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        first = None
        for per_cu in (1, 3, 4, 5, 32):
            ctx.set_launch(PLAIN, per_cu, 256)
            got = ctx.get_launch(PLAIN)
            assert got[1] == 256 and 1 <= got[0] <= per_cu
            f, st = ctx.run_plain(98, 0, nt)
            check_against_oracle(f, st, fo, fpo, so, (enc, per_cu))
            if first is None:
                first = f
            assert np.array_equal(f, first), (enc, per_cu)
        ctx.set_launch(PLAIN, 32, 256)
        assert ctx.get_launch(PLAIN)[0] >= (5 if enc == QUBIT else 4)


def test_plain_engine_shapes_on_depolarizing_context(lib, orc):
    """Both modes of a depolarizing context run on the plain engine; every
    workgroup size gives the oracle's fidelities."""
    n, k, enc, p, nt = 4, 2, QUBIT, 0.01, 600
    mem = memory_words(n, k, 56)
    fo, _, so, _ = orc.run_many(n, k, enc, p, mem, 31, 0, nt, eps=p)
    with lib.QramContext(n, k, enc, p, mem, eps=p) as ctx:
        for mode in (PRUNED, FULL):
            for threads in (64, 128, 256):
                ctx.set_launch(mode, 0, threads)
                assert ctx.get_launch(mode)[1] == threads
                f, st = (ctx.run_pruned if mode == PRUNED else ctx.run_full)(31, 0, nt)
                assert np.all(np.abs(f - fo) <= 1e-12 * np.maximum(np.abs(fo), 1e-3)), (mode, threads)
                assert np.array_equal(st["n_jumps"], so[:, 4].astype(np.uint16))
        with pytest.raises(lib.QramError):
            ctx.set_launch(PRUNED, 0, 96)
        with pytest.raises(lib.QramError):
            ctx.set_launch(FULL, 33, 64)


@pytest.mark.parametrize("n,k,enc,p,threads", [(3, 2, QUBIT, 0.03, 256), (4, 3, QUBIT, 0.01, 64),
                                               (3, 1, QUTRIT, 0.03, 128), (5, 2, QUTRIT, 0.005, 64),
                                               (7, 3, QUBIT, 0.002, 256), (4, 2, QUTRIT, 0.03, 256)])
def test_plain_record_paths(lib, orc, n, k, enc, p, threads):
    """The records staged through shared memory and worked on in device
    memory (QRAM_OPT_TIER2_GLOBAL, or the launch shape's device-memory bit)
    give the oracle's results, with depolarizing strays lengthening the
    lists, in both plain-engine modes.  The slabs cover: whole records;
    records longer than a slab (n = 7 at 256 threads); qutrit lists that
    leave too little room for a slice's growth and stay in device memory
    (n = 3, 4)."""
    nt = 500
    mem = memory_words(n, k, 60 + n)
    fo, fpo, so, _ = orc.run_many(n, k, enc, p, mem, 17, 0, nt, eps=p)
    with lib.QramContext(n, k, enc, p, mem, eps=p) as ctx:
        for glob, sched in ((0, threads), (1, threads), (0, threads + 1)):
            ctx.set_option(lib.qram.QRAM_OPT_TIER2_GLOBAL, glob)
            for mode in (PRUNED, FULL):
                ctx.set_launch(mode, 0, sched)
                assert ctx.get_launch(mode)[1] == threads + (1 if glob or sched & 1 else 0)
                f, st = (ctx.run_pruned if mode == PRUNED else ctx.run_full)(17, 0, nt)
                check_against_oracle(f, st, fo, fpo, so, (glob, sched, mode))


def test_plain_async_device_buffers(lib):
    import torch
    n, k, enc, gamma, nt = 6, 2, QUTRIT, 1e-2, 2000
    mem = memory_words(n, k, 66)
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        f, st = ctx.run_plain(7, 0, nt)
        d = torch.zeros(nt, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        ctx.run_plain_async(7, 0, nt, d, None, s)
        s.synchronize()
        assert np.array_equal(d.cpu().numpy(), f)
