"""Request server (continuous batching) on the GPU: every result equals the
direct run of the same request and the oracle's trajectories (fidelities
within 1e-12 relative), alone or in a mix; admission by footprint; requests
of the serving mix's largest shape (n = 12, k = 4) checked on sampled
trajectories against the oracle."""
import os

import numpy as np
import pytest

from paper_2609_34935_amd.inputs import memory_words, request_mix

pytestmark = pytest.mark.gpu

QUTRIT, QUBIT = 0, 1
FULL, PRUNED = 0, 1


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_34935_amd as P
    P.load_library()
    return P


def small_mix(nreq, seed):
    """The serving mix with n and shots scaled down so the test stays short."""
    out = []
    for r in request_mix(nreq, seed):
        r = dict(r)
        r["n"] = 3 + r["n"] % 6          # 3..8
        r["k"] = min(r["k"], r["n"])
        r["shots"] = 200 + r["shots"] % 1800
        r["mode"] = PRUNED if r["id"] % 3 else FULL
        r["traj0"] = r["id"] * 7
        out.append(r)
    return out


def fid_close(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) <= 1e-12 * np.maximum(np.abs(b), 1e-3)


def oracle_fids(orc, r, idx=None):
    mem = memory_words(r["n"], r["k"], r["mem_seed"])
    nth = min(16, os.cpu_count() or 1)
    if idx is None:
        return orc.run_batch(r["n"], r["k"], r["enc"], r["gamma"], mem, r["seed"], r["traj0"], r["shots"],
                             nthreads=nth)[0]
    return orc.run_indices(r["n"], r["k"], r["enc"], r["gamma"], mem, r["seed"],
                           [r["traj0"] + i for i in idx], nthreads=nth)[0]


def direct(P, r):
    mem = memory_words(r["n"], r["k"], r["mem_seed"])
    with P.QramContext(r["n"], r["k"], r["enc"], r["gamma"], mem) as ctx:
        fn = ctx.run_pruned if r["mode"] == PRUNED else ctx.run_full
        f, _ = fn(r["seed"], r["traj0"], r["shots"])
    return f


def submit(P, srv, r):
    mem = memory_words(r["n"], r["k"], r["mem_seed"])
    return srv.submit(r["n"], r["k"], r["enc"], r["gamma"], mem, r["seed"], r["shots"], r["mode"], r["traj0"])


def test_mix_results_equal_direct_runs(P, orc):
    reqs = small_mix(12, 77)
    with P.QramServer(8 << 30, max_active=4, chunk=300) as srv:
        tickets = [submit(P, srv, r) for r in reqs]
        for r, t in zip(reqs, tickets):
            res = srv.wait(t)
            assert res["state"] == "done", res
            f = srv.fidelities(t, r["shots"])
            ref = direct(P, r)
            assert np.array_equal(f, ref), r
            fo = oracle_fids(orc, r)
            assert np.all(fid_close(f, fo)), r
            m, s = P.qram_fidelity(ref)
            assert res["mean"] == m and res["sem"] == s
            assert res["latency_ms"] >= res["queue_ms"] >= 0.0
            assert res["footprint_bytes"] > 8 * r["shots"]
            srv.release(t)


def test_alone_and_in_mix_identical(P):
    reqs = small_mix(8, 78)
    probe = dict(reqs[0], shots=1500, mode=PRUNED)
    with P.QramServer(8 << 30, max_active=2, chunk=256) as srv:
        t = submit(P, srv, probe)
        assert srv.wait(t)["state"] == "done"
        alone = srv.fidelities(t, probe["shots"])
    with P.QramServer(8 << 30, max_active=6, chunk=128) as srv:
        ts = [submit(P, srv, r) for r in reqs[1:4]]
        t = submit(P, srv, probe)
        ts += [submit(P, srv, r) for r in reqs[4:]]
        assert srv.wait(t)["state"] == "done"
        mixed = srv.fidelities(t, probe["shots"])
        for x in ts:
            assert srv.wait(x)["state"] == "done"
    assert np.array_equal(alone, mixed)


def test_admission_by_footprint(P):
    reqs = small_mix(6, 79)
    mems = [memory_words(r["n"], r["k"], r["mem_seed"]) for r in reqs]
    fps = []
    for r, mem in zip(reqs, mems):
        with P.QramContext(r["n"], r["k"], r["enc"], r["gamma"], mem) as ctx:
            fps.append(ctx.footprint(r["mode"], min(r["shots"], 200)) + 8 * r["shots"])
    budget = max(fps) + 1  # room for one request at a time
    with P.QramServer(budget, max_active=4, chunk=200) as srv:
        tickets = [submit(P, srv, r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        assert all(x["state"] == "done" for x in res), res
        assert [x["footprint_bytes"] for x in res] == fps
        # one at a time: each admission waits for the previous completion
        for a, b in zip(res, res[1:]):
            assert b["queue_ms"] > 0.0
        for r, t in zip(reqs, tickets):
            assert np.array_equal(srv.fidelities(t, r["shots"]), direct(P, r))
    with P.QramServer(1 << 20, max_active=2, chunk=200) as srv:
        big = dict(reqs[0], n=10, k=2, shots=5000)
        t = submit(P, srv, big)
        res = srv.wait(t)
        assert res["state"] == "failed" and res["status"] == "QRAM_E_CAPACITY"


def test_largest_mix_shape_against_oracle(P, orc):
    """Two requests of the mix's largest shape (n = 12, k = 4; both
    encodings, up to 1e5 shots) served among smaller ones: every result equals
    the direct run, and sampled trajectories equal the oracle's."""
    big = [dict(id=900, n=12, k=4, enc=QUBIT, gamma=1e-3, shots=100000, mode=PRUNED, seed=4242900,
                traj0=0, mem_seed=5900),
           dict(id=901, n=12, k=4, enc=QUTRIT, gamma=1e-4, shots=30000, mode=PRUNED, seed=4242901,
                traj0=17, mem_seed=5901)]
    reqs = small_mix(6, 80)
    with P.QramServer(16 << 30, max_active=4, chunk=8192) as srv:
        ts = [submit(P, srv, r) for r in reqs[:3]]
        tb = [submit(P, srv, r) for r in big]
        ts += [submit(P, srv, r) for r in reqs[3:]]
        for r, t in zip(big, tb):
            print(f"request n={r['n']} k={r['k']} enc={r['enc']} shots={r['shots']}", flush=True)
            res = srv.wait(t)
            assert res["state"] == "done", res
            f = srv.fidelities(t, r["shots"])
            assert np.array_equal(f, direct(P, r)), r["id"]
            rng = np.random.default_rng(r["id"])
            idx = sorted(set([0, 1, r["shots"] - 1] + rng.choice(r["shots"], 5, replace=False).tolist()))
            fo = oracle_fids(orc, r, idx)
            assert np.all(fid_close(f[idx], fo)), (r["id"], f[idx], fo)
        for t in ts:
            assert srv.wait(t)["state"] == "done"
