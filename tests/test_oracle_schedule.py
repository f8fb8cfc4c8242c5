"""Pins of the bucket-brigade schedule (Sec. II A, Eq. schedule and
Eq. window; Eq. caddr; the injection counts of Sec. VI B)."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _events(orc, n, k):
    T = 6 * n + 2 * k
    return T, {s: orc.schedule(n, k, s) for s in range(1, T)}


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (3, 3), (4, 2), (6, 1), (10, 4), (14, 1)])
def test_event_times_and_mirror(orc, n, k):
    T, ev = _events(orc, n, k)
    assert T == 6 * n + 2 * k
    for b in range(k):
        assert ("bus", b) in ev[2 * n + 2 * b + 1]          # tau_in
        assert ("fetch", b) in ev[3 * n + 2 * b + 1]        # tau_fetch
        assert ("bus", b) in ev[4 * n + 2 * b + 1]          # tau_out
        assert (4 * n + 2 * b + 1) - (2 * n + 2 * b + 1) == 2 * n  # Eq. window
    # mirror symmetry out(t) = T - t: bus-in of bit b <-> bus-out of bit k-1-b
    for s in range(1, T):
        kinds = sorted(name for name, _ in ev[s])
        mirror = sorted(name for name, _ in ev[T - s])
        assert kinds == mirror, (s, ev[s], ev[T - s])
    for b in range(k):
        assert T - (2 * n + 2 * b + 1) == 4 * n + 2 * (k - 1 - b) + 1


@pytest.mark.parametrize("n,k", [(2, 1), (3, 3), (5, 4), (10, 4)])
def test_slice_ops_disjoint(orc, n, k):
    """Within a slice every operation acts on its own qubits: controlled
    swaps run on layers of one parity, stores and swaps of other layers do
    not touch them."""
    T, ev = _events(orc, n, k)
    for s in range(1, T):
        touched = []
        for name, a in ev[s]:
            if name == "cswap":
                touched.append({("d", a), ("d", a + 1), ("a", a)})
            elif name == "store":
                touched.append({("a", a), ("d", a)})
            elif name in ("copy", "bus"):
                touched.append({("d", 0)})
            elif name == "fetch":
                touched.append({("d", n - 1), ("a", n - 1)})
        writes = []
        for name, a in ev[s]:
            if name == "cswap":
                writes.append({("d", a), ("d", a + 1)})
            elif name == "store":
                writes.append({("a", a), ("d", a)})
            elif name in ("copy", "bus"):
                writes.append({("d", 0)})
            elif name == "fetch":
                writes.append({("d", n - 1)})
        for i in range(len(writes)):
            for j in range(len(touched)):
                if i != j:
                    assert not (writes[i] & touched[j]), (s, ev[s])


def test_worked_example_n2(orc):
    T, ev = _events(orc, 2, 1)
    want = {1: [("copy", 0)], 2: [("store", 0)], 3: [("copy", 1)], 4: [("cswap", 0)],
            5: [("bus", 0), ("store", 1)], 6: [("cswap", 0)], 7: [("fetch", 0)],
            8: [("cswap", 0)], 9: [("bus", 0), ("store", 1)], 10: [("cswap", 0)],
            11: [("copy", 1)], 12: [("store", 0)], 13: [("copy", 0)]}
    for s in range(1, T):
        assert sorted(ev[s]) == sorted(want[s])


def _nonvacuous(orc, n, k, enc, mem):
    """(slice, site) pairs at which some component of the data-loading input
    is excited in the no-jump orbit."""
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    allsites = list(range(M))
    hits = set()
    for s in range(1, T):
        masks, _ = orc.layer_masks(n, k, enc, 0.01, mem, [], np.zeros(T), s, allsites)
        for mask in masks:
            for q, lev in enumerate(mask):
                if lev:
                    hits.add((s, q))
    return hits


def test_injection_counts(orc):
    """Sec. VI B: at n = 3, k = 3 there are 14 positions x 23 slices = 322
    damping cases, of which 178 are vacuous and 144 are not."""
    g = json.load(open(os.path.join(GOLDEN, "single_fault_injection.json")))
    n, k = g["n"], g["k"]
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    assert M == g["injection_positions"] and T - 1 == g["event_slices"]
    assert M * (T - 1) == g["damping_cases"]
    mem = [5, 2, 7, 0, 1, 6, 3, 4]
    hits = _nonvacuous(orc, n, k, 1, mem)
    assert len(hits) == g["nonvacuous_damping_cases"]
    assert M * (T - 1) - len(hits) == g["vacuous_damping_cases"]


def test_injection_containment(orc):
    """A single forced damping jump at (s, q) leaves surviving components only
    inside the subtree of q's node; vacuous positions never fire."""
    n, k = 3, 3
    T, M = 6 * n + 2 * k, 2 * (2**n - 1)
    mem = [5, 2, 7, 0, 1, 6, 3, 4]
    hits = _nonvacuous(orc, n, k, 1, mem)
    ua = np.full(T, 1.0 - 1e-15)
    for s in range(1, T):
        for q in range(M):
            L = [(s - 1) * M + q]
            r = orc.run_traj(n, k, 1, 0.01, mem, forced_L=L, forced_uaux=ua, export=True)
            if (s, q) not in hits:
                assert r["njumps"] == 0
                continue
            assert r["njumps"] == 1 and r["jumps"] == [(s, q, 1)]
            v = q // 2
            layer = int(np.floor(np.log2(v + 1)))
            p = v + 1 - 2**layer
            addrs = r["components"]["addr"]
            assert len(addrs) > 0
            assert np.all((addrs >> (n - layer)) == p)


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2), (4, 3), (5, 1)])
def test_nonvacuous_count_formula(orc, n, k):
    """Count of non-vacuous site-slices equals sum_l 2^l (8n + 4k - 8l - 4):
    per node of layer l the router is excited from its store to its unstore
    and the data slot carries each address bit below it twice and each data
    bit twice."""
    mem = list(np.random.default_rng(n * 10 + k).integers(0, 2**k, size=2**n))
    hits = _nonvacuous(orc, n, k, 1, mem)
    want = sum(2**l * (8 * n + 4 * k - 8 * l - 4) for l in range(n))
    assert len(hits) == want
