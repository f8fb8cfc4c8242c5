"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: candidate histories and branch classification bit-exact; fidelity within
1e-12 relative per trajectory (absolute 1e-15 when F < 1e-3, the value 0 after
a non-ground tree measurement included); integer statistics identical."""
import numpy as np
import pytest

from paper_2609_34935_amd.inputs import memory_words

pytestmark = pytest.mark.gpu

QUTRIT, QUBIT = 0, 1
FULL, PRUNED = 0, 1


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


def oracle_ref(ri):
    r = ri[:, 2].astype(np.int64)
    return np.where(r < 0, 0xFFFFFFFF, r).astype(np.uint32)


def compare_runs(P, orc, n, k, enc, gamma, mem, seed, traj0, ntraj, threads=None, tier2_global=False):
    fo, fpo, so, _ = orc.run_batch(n, k, enc, gamma, mem, seed, traj0, ntraj)
    with P.QramContext(n, k, enc, gamma, mem) as ctx:
        if tier2_global:
            ctx.set_option(P.qram.QRAM_OPT_TIER2_GLOBAL, 1)
        out = {}
        for mode, fn in ((FULL, ctx.run_full), (PRUNED, ctx.run_pruned)):
            if threads:
                ctx.set_launch(mode, threads[0], threads[1])
            f, st = fn(seed, traj0, ntraj)
            bad = np.nonzero(~fid_close(f, fo))[0]
            assert len(bad) == 0, (mode, bad[:5], f[bad[:5]], fo[bad[:5]], st[bad[:5]])
            assert np.all(fid_close(st["fid_pre"], fpo)), mode
            assert np.array_equal(st["n_cand"], so[:, 0].astype(np.uint32))
            assert np.array_equal(st["n_bad"], so[:, 1].astype(np.uint32))
            assert np.array_equal(st["ref_addr"], oracle_ref(so))
            assert np.array_equal(st["n_jumps"], so[:, 4].astype(np.uint16))
            assert np.array_equal(st["first_jump_slice"], so[:, 5].astype(np.uint16))
            assert np.array_equal(st["ref_survived"], so[:, 6].astype(np.uint8))
            assert np.array_equal(st["q_ground"], so[:, 7].astype(np.uint8))
            out[mode] = (f, st)
    ff, fp = out[FULL][0], out[PRUNED][0]
    assert np.all(fid_close(fp, ff))
    return out, (fo, fpo, so)


# ---------------------------------------------------------------------------
# candidate histories and classification: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,enc,gamma,ntraj", [
    (3, 1, QUTRIT, 1e-3, 300), (3, 1, QUBIT, 0.05, 300), (6, 1, QUBIT, 1e-2, 200),
    (10, 4, QUBIT, 1e-3, 64), (10, 4, QUTRIT, 1e-3, 64), (5, 2, QUTRIT, 0.2, 50), (1, 1, QUBIT, 0.3, 100)])
def test_sampler_and_classifier_bit_exact(lib, orc, n, k, enc, gamma, ntraj):
    mem = memory_words(n, k, 1000 + n)
    seed = 880000 + n
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        out = ctx.sample_faults(seed, 5, ntraj, dump=True)
    for t in range(ntraj):
        L = orc.sample(n, k, gamma, seed, 5 + t)
        assert out["n_cand"][t] == len(L)
        assert np.array_equal(out["cand_L"][t], L), t
        h = 0xcbf29ce484222325
        for x in L.tolist():
            for b in range(4):
                h ^= (x >> (8 * b)) & 0xFF
                h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
        assert int(out["digest"][t]) == h
        bad = orc.classify(n, k, enc, L)
        bits = np.unpackbits(out["bad_bits"][t].view(np.uint8), bitorder="little")[: 1 << n]
        assert np.array_equal(bits, bad), t
        assert out["n_bad"][t] == bad.sum()


def test_sampler_large_history_bit_exact(lib, orc):
    """n = 14 qutrit at gamma = 1e-2: ~27.9k candidates per trajectory."""
    n, k, enc, gamma = 14, 1, QUTRIT, 1e-2
    mem = memory_words(n, k, 1005)
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        out = ctx.sample_faults(880005, 1000, 4, dump=True)
    for t in range(4):
        L = orc.sample(n, k, gamma, 880005, 1000 + t)
        assert np.array_equal(out["cand_L"][t], L)
        bits = np.unpackbits(out["bad_bits"][t].view(np.uint8), bitorder="little")[: 1 << n]
        assert np.array_equal(bits, orc.classify(n, k, enc, L))


# ---------------------------------------------------------------------------
# trajectories: fidelity and statistics against the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,enc,gamma,ntraj", [
    (2, 1, QUBIT, 0.2, 400), (2, 1, QUTRIT, 0.2, 400), (3, 2, QUBIT, 0.08, 300),
    (3, 1, QUTRIT, 0.08, 300), (3, 3, QUBIT, 0.05, 200), (4, 2, QUTRIT, 0.05, 200),
    (1, 1, QUBIT, 0.3, 200), (1, 1, QUTRIT, 0.3, 200), (4, 4, QUBIT, 0.03, 100)])
def test_small_high_gamma(lib, orc, n, k, enc, gamma, ntraj):
    """Small trees with strong damping: many jumps, deviated routing."""
    mem = memory_words(n, k, 77 + n)
    out, (fo, _, so) = compare_runs(lib, orc, n, k, enc, gamma, mem, 12345, 0, ntraj)
    assert so[:, 4].sum() > 0  # jumps happened


@pytest.mark.parametrize("n,k,enc,gamma,ntraj", [
    (3, 2, QUBIT, 0.08, 300), (3, 1, QUTRIT, 0.08, 300), (4, 2, QUTRIT, 0.05, 200), (4, 4, QUBIT, 0.03, 100)])
def test_small_high_gamma_global_lists(lib, orc, n, k, enc, gamma, ntraj):
    """The same trajectories with every explicit site list in global memory."""
    mem = memory_words(n, k, 77 + n)
    compare_runs(lib, orc, n, k, enc, gamma, mem, 12345, 0, ntraj, tier2_global=True)


def test_config1_qutrit_all_trajectories(lib, orc):
    """Qutrit n = 3, k = 1, gamma = 1e-3, 1000 trajectories, both modes."""
    mem = memory_words(3, 1, 1001)
    compare_runs(lib, orc, 3, 1, QUTRIT, 1e-3, mem, 880001, 0, 1000)


@pytest.mark.parametrize("gamma", [1e-4, 1e-3, 1e-2])
def test_config2_qubit_all_trajectories(lib, orc, gamma):
    """Qubit n = 6, k = 1: every one of the 1e4 trajectories per gamma against
    the oracle, both modes."""
    mem = memory_words(6, 1, 1002)
    out, (fo, _, so) = compare_runs(lib, orc, 6, 1, QUBIT, gamma, mem, 880002, 0, 10000)
    assert so[:, 4].sum() > 0


@pytest.mark.parametrize("spt,sched", [(4, 0), (8, 1), (16, 0), (32, 1), (64, 1), (8, 2), (32, 3), (64, 3)])
def test_launch_shapes(lib, orc, spt, sched):
    mem = memory_words(5, 3, 55)
    compare_runs(lib, orc, 5, 3, QUBIT, 0.01, mem, 99, 0, 120, threads=(spt, sched))


@pytest.mark.parametrize("spt,sched", [(4, 1), (8, 1), (16, 3), (32, 1)])
def test_launch_shapes_qutrit(lib, orc, spt, sched):
    """Qutrit workgroups of different sizes (the no-jump walk strides over
    the workgroup's waves)."""
    mem = memory_words(7, 2, 77)
    compare_runs(lib, orc, 7, 2, QUTRIT, 3e-3, mem, 98, 0, 150, threads=(spt, sched))


# ---------------------------------------------------------------------------
# forced histories
# ---------------------------------------------------------------------------
def forced_case(lib, orc, n, k, enc, gamma, mem, L, ua, uf):
    fo = orc.run_traj(n, k, enc, gamma, mem, forced_L=L, forced_uaux=ua, forced_ufin=uf)
    with lib.QramContext(n, k, enc, gamma, mem) as ctx:
        for mode in (FULL, PRUNED):
            f, st = ctx.run_forced(mode, L, ua, uf)
            assert fid_close(f, fo["fid"]), (mode, f, fo["fid"])
            assert fid_close(st["fid_pre"], fo["fid_pre"])
            assert st["n_jumps"] == fo["njumps"] and st["first_jump_slice"] == fo["first_jump"]
            assert st["q_ground"] == fo["q_ground"]
    return fo


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_forced_no_jump(lib, orc, enc):
    n, k = 5, 2
    T = 6 * n + 2 * k
    mem = memory_words(n, k, 3)
    fo = forced_case(lib, orc, n, k, enc, 1e-2, mem, [], np.full(T, 0.5), 0.3)
    assert fo["njumps"] == 0


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_forced_reference_annihilated(lib, orc, enc):
    """A jump on the root router kills every good branch, the reference
    included (Sec. VI A: the annihilation propagates to the predicted groups)."""
    n, k = 4, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 4)
    # router of node 2 (range: its own subtree) at slice 8, a second candidate
    L = [(8 - 1) * M + 4, (9 - 1) * M + 5]
    ua = np.full(T, 0.999999)
    fo = forced_case(lib, orc, n, k, enc, 0.02, mem, L, ua, 0.1)
    assert fo["ref"] == 0 and fo["njumps"] >= 1 and fo["ref_survived"] == 0


def test_forced_data_slot_jump_qubit(lib, orc):
    """A jump on the root data slot while bus bit 0 passes (slice 2n+1)."""
    n, k = 4, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 5)
    L = [(2 * n + 1 - 1) * M + 1]
    fo = forced_case(lib, orc, n, k, QUBIT, 0.02, mem, L, np.full(T, 0.9999), 0.2)
    assert fo["njumps"] == 1


def test_forced_router_jump_qutrit(lib, orc):
    """A qutrit router jump (K1 or K2 by level) below the root."""
    n, k = 4, 1
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 6)
    for site in (2, 4, 6):  # routers of nodes 1, 2, 3
        L = [(12 - 1) * M + site]
        forced_case(lib, orc, n, k, QUTRIT, 0.05, mem, L, np.full(T, 0.99999), 0.5)


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_forced_idle_sites(lib, orc, enc):
    """Candidates on sites no component excites never fire."""
    n, k = 4, 1
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 7)
    # slice 1 excites only the root data slot, slice 2 only the root router,
    # and after the last uncopy (slice T-1) the tree is empty
    L = [0 * M + 5, 0 * M + 29, 1 * M + 7, (T - 2) * M + 0, (T - 2) * M + 1]
    fo = forced_case(lib, orc, n, k, enc, 0.05, mem, L, np.full(T, 0.99999), 0.5)
    assert fo["njumps"] == 0


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_forced_many_candidates_one_slice(lib, orc, enc):
    """More candidates in one slice than the list scan holds (bitmap path)."""
    n, k = 5, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 8)
    rng = np.random.default_rng(enc)
    for trial in range(6):
        s = int(rng.integers(1, T))
        qs = np.sort(rng.choice(M, size=24, replace=False))
        extra = np.sort(rng.choice((T - 1) * M, size=5, replace=False))
        L = np.unique(np.concatenate([(s - 1) * M + qs, extra])).astype(np.uint32)
        ua = rng.uniform(0, 1, size=T)
        ua[s] = rng.uniform(0.5, 1.0)
        forced_case(lib, orc, n, k, enc, 0.05, mem, L, ua, float(rng.uniform()))


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_forced_random_histories(lib, orc, enc):
    n, k = 3, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 9)
    rng = np.random.default_rng(100 + enc)
    for trial in range(40):
        L = np.sort(rng.choice((T - 1) * M, size=int(rng.integers(0, 12)), replace=False)).astype(np.uint32)
        ua = rng.uniform(0, 1, size=T)
        forced_case(lib, orc, n, k, enc, 0.1, mem, L, ua, float(rng.uniform()))


# ---------------------------------------------------------------------------
# determinism, ranges, gamma = 0, async
# ---------------------------------------------------------------------------
def test_deterministic_and_range_split(lib):
    n, k = 6, 2
    mem = memory_words(n, k, 10)
    with lib.QramContext(n, k, QUBIT, 3e-3, mem) as ctx:
        for fn in (ctx.run_full, ctx.run_pruned):
            a, sa = fn(5, 100, 500)
            b, sb = fn(5, 100, 500)
            assert np.array_equal(a, b) and np.array_equal(sa, sb)
            c1, _ = fn(5, 100, 123)
            c2, _ = fn(5, 223, 377)
            assert np.array_equal(np.concatenate([c1, c2]), a)


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_gamma_zero(lib, enc):
    n, k = 8, 2
    mem = memory_words(n, k, 11)
    with lib.QramContext(n, k, enc, 0.0, mem) as ctx:
        f, st = ctx.run_pruned(1, 0, 50)
        assert np.allclose(f, 1.0, atol=1e-13)
        assert np.all(st["n_cand"] == 0) and np.all(st["n_bad"] == 0)
        assert np.all(st["n_explicit"] == (2**k if enc == QUBIT else 1))
        f2, _ = ctx.run_full(1, 0, 50)
        assert np.allclose(f2, 1.0, atol=1e-13)


def test_async_device_buffers(lib):
    import torch
    n, k = 6, 1
    mem = memory_words(n, k, 12)
    with lib.QramContext(n, k, QUBIT, 1e-3, mem) as ctx:
        ref_f, ref_s = ctx.run_pruned(42, 0, 1000)
        d_f = torch.empty(1000, dtype=torch.float64, device="cuda")
        d_s = torch.empty(1000 * 32, dtype=torch.uint8, device="cuda")
        s = torch.cuda.Stream()
        ctx.run_pruned_async(42, 0, 1000, d_f, d_s, stream=s)
        s.synchronize()
        assert np.array_equal(d_f.cpu().numpy(), ref_f)
        st = np.frombuffer(d_s.cpu().numpy().tobytes(), dtype=lib.STATS_DTYPE)
        assert np.array_equal(st, ref_s)


# ---------------------------------------------------------------------------
# graph mode: each batch captured once, updated in place and replayed
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_graph_replays_match_eager(lib, enc):
    import torch
    n, k, gamma = 8, 2, 3e-3
    mem = memory_words(n, k, 13)
    calls = [(7, 0, 600), (7, 600, 600), (8, 0, 600), (7, 0, 600), (9, 17, 250), (9, 17, 250)]
    with lib.QramContext(n, k, enc, gamma, mem) as eager, lib.QramContext(n, k, enc, gamma, mem) as g:
        g.set_option(lib.qram.QRAM_OPT_GRAPH, 1)
        for mode in (FULL, PRUNED):
            for seed, traj0, nt in calls:
                fe, se = (eager.run_pruned if mode else eager.run_full)(seed, traj0, nt)
                # unrelated device work between replays
                x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
                torch.cuda.synchronize()
                fg, sg = (g.run_pruned if mode else g.run_full)(seed, traj0, nt)
                assert float((x * x).sum()) > 0
                assert np.array_equal(fg, fe), (mode, seed, traj0, nt)
                assert np.array_equal(sg, se), (mode, seed, traj0, nt)


def test_graph_async_streams(lib):
    import torch
    n, k = 6, 1
    mem = memory_words(n, k, 14)
    with lib.QramContext(n, k, QUBIT, 1e-3, mem) as ctx:
        ref_f, _ = ctx.run_pruned(42, 0, 1000)
        ctx.set_option(lib.qram.QRAM_OPT_GRAPH, 1)
        for stream in (torch.cuda.Stream(), None, torch.cuda.Stream()):
            d_f = torch.full((1000,), -1.0, dtype=torch.float64, device="cuda")
            ctx.run_pruned_async(42, 0, 1000, d_f, None, stream=stream)
            torch.cuda.synchronize()
            assert np.array_equal(d_f.cpu().numpy(), ref_f)


# ---------------------------------------------------------------------------
# qubit tier 2: lists shared by an address's bus words, and their splits
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,gamma,nt,seed", [
    (6, 4, 1e-2, 3000, 4242),    # many jumps during the data phase
    (6, 6, 1e-2, 1000, 4343),    # 64 bus words per address
    (8, 1, 1e-2, 2000, 4545),    # two bus words per address
    (11, 2, 8e-3, 600, 4646),    # slices with more than 16 candidates (bitmap hits)
    (10, 4, 1e-3, 20000, 4444)])  # the benchmark's tree: splits into classes
def test_qubit_shared_lists_match_component_lists(lib, n, k, gamma, nt, seed):
    """Shared per-address lists, split into classes (default), against one
    global-memory list per component: bitwise equal fidelities and
    statistics."""
    mem = memory_words(n, k, 600 + n + k)
    res = []
    for glob in (0, 1):
        with lib.QramContext(n, k, QUBIT, gamma, mem) as ctx:
            ctx.set_option(lib.qram.QRAM_OPT_TIER2_GLOBAL, glob)
            res.append([fn(seed, 0, nt) for fn in (ctx.run_full, ctx.run_pruned)])
    for (fa, sa), (fb, sb) in zip(res[0], res[1]):
        assert np.array_equal(fa, fb)
        assert np.array_equal(sa, sb)
    js = res[0][0][1]["first_jump_slice"]
    assert np.sum((js > 2 * n) & (js < 4 * n + 2 * k)) > 50


def test_qubit_classes_against_oracle(lib, orc):
    """Strong damping on a tree deep enough for stranded tokens to reach a
    store: the class splits against the oracle trajectory by trajectory."""
    mem = memory_words(5, 3, 5353)
    compare_runs(lib, orc, 5, 3, QUBIT, 0.03, mem, 5353, 0, 300)


@pytest.mark.parametrize("s,site", [(12, 0), (14, 0), (13, 2), (15, 4), (16, 2), (17, 0)])
def test_forced_router_jump_with_data_in_tree_qubit(lib, orc, s, site):
    """A router jump while data tokens are below it: the tokens routed
    through it get stuck, so the bus words of an address stop sharing their
    routing (shared lists split)."""
    n, k = 4, 2
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = memory_words(n, k, 7)
    L = [(s - 1) * M + site]
    forced_case(lib, orc, n, k, QUBIT, 0.05, mem, L, np.full(T, 0.99999), 0.5)


@pytest.mark.parametrize("n,k,gamma,nt,seed", [(6, 6, 3e-2, 1500, 5454), (5, 5, 4e-2, 2000, 5555)])
def test_qubit_many_classes_pre_splits(lib, orc, n, k, gamma, nt, seed):
    """Regression: addresses with many classes whose work-list entries span
    wave boundaries, split again before a store.  One thread per address takes
    the split (the others must not read the split set while it changes).
    Fidelities and statistics against the oracle, and bitwise against one
    global-memory list per component."""
    mem = memory_words(n, k, 700 + n + k)
    out, _ = compare_runs(lib, orc, n, k, QUBIT, gamma, mem, seed, 0, nt)
    with lib.QramContext(n, k, QUBIT, gamma, mem) as ctx:
        ctx.set_option(lib.qram.QRAM_OPT_TIER2_GLOBAL, 1)
        fg, sg = ctx.run_pruned(seed, 0, nt)
    assert np.array_equal(out[PRUNED][0], fg)
    assert np.array_equal(out[PRUNED][1], sg)
