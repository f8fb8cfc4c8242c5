"""The GPU dense cross-check service (App. C) against the oracle's dense
machine and the branch simulators.

  - qram_dense_density: F_rho and the trace of the whole query as a density
    matrix (n = 2), both encodings, damping, depolarizing, the outlook
    channels (dephasing, heating) and general / pair inputs, against the
    oracle's dense machine within 1e-12; Table 4's four rows to the printed
    digits.
  - qram_dense_forced: the state vector under the oracle's own sampled
    histories (jumps and faults) against the oracle's dense machine (small
    registers) and against the oracle's sparse export component by
    component (qubit n = 3, k = 3: 2^20 labels; qutrit n = 3, k = 1)."""
import json
import os

import numpy as np
import pytest

from oracle import dense as Dn
from paper_2609_34935_amd.inputs import memory_words

pytestmark = pytest.mark.gpu

QUTRIT, QUBIT = 0, 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_34935_amd as P
    P.load_library()
    return P


def cab_random(n, k, seed):
    rng = np.random.default_rng(seed)
    c = (rng.normal(size=(1 << n, 1 << k)) + 1j * rng.normal(size=(1 << n, 1 << k)))
    c *= rng.uniform(size=c.shape) < 0.6
    c[0, 0] = 0.5
    return c


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
@pytest.mark.parametrize("k,gamma,eps,deph,heat,inp", [
    (1, 0.05, 0.0, 0.0, 0.0, None), (1, 0.02, 0.02, 0.0, 0.0, None), (2, 0.03, 0.01, 0.0, 0.0, "pairs"),
    (1, 0.02, 0.0, 0.03, 0.0, None), (1, 0.0, 0.0, 0.0, 0.02, None), (2, 0.01, 0.01, 0.01, 0.01, "pairs"),
    (1, 0.04, 0.0, 0.0, 0.0, "cj")])
def test_density_against_dense_machine(lib, enc, k, gamma, eps, deph, heat, inp):
    n = 2
    mem = memory_words(n, k, 40 + k)
    kw = {}
    cab = None
    if inp == "pairs":
        cab = cab_random(n, k, 7 + enc + k)
        kw["input_ab"] = cab
    elif inp == "cj":
        rng = np.random.default_rng(5)
        cin = rng.normal(size=4) + 1j * rng.normal(size=4)
        cin[1] = 0.0
        jin = rng.integers(0, 2**k, size=4).astype(np.uint32)
        kw["input_amp"], kw["input_bus"] = cin, jin
        cab = np.zeros((4, 2**k), dtype=complex)
        cab[np.arange(4), jin] = cin
    F_o, tr_o = Dn.density_fidelity(n, k, enc, mem, gamma, eps, cab=cab, dephase=deph, heat=heat)
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps, **kw) as ctx:
        F, tr = ctx.dense_density(deph, heat)
    assert abs(F - F_o) <= 1e-12 * max(abs(F_o), 1e-3), (F, F_o)
    assert abs(tr - 1.0) <= 1e-12 and abs(tr_o - 1.0) <= 1e-12


def test_table4_rows(lib):
    mem = np.array([0, 1, 1, 0], dtype=np.uint32)
    rows = [(0.05, 0.0, 0.5759), (0.2, 0.0, 0.1676)]
    g = json.load(open(os.path.join(GOLDEN, "table4_depolarizing.json")))
    rows += [(r["gamma"], r["eps"], r["F_rho"]) for r in g["rows"]]
    for gamma, eps, want in rows:
        with lib.QramContext(2, 1, QUBIT, gamma, mem, eps=eps) as ctx:
            F, tr = ctx.dense_density()
        assert round(F, 4) == want, (gamma, eps, F, want)
        assert abs(tr - 1.0) < 1e-12


def oracle_faults(orc, n, k, enc, eps, seed, traj):
    L, ty = orc.sample_depol(n, k, enc, eps, seed, traj)
    act = orc.depol_active(n, k)
    off = np.concatenate([[0, 0], np.cumsum(act[1:])])
    out = []
    for x, t in zip(L, ty):
        s = int(np.searchsorted(off, x, side="right") - 1)
        out.append((s, int(x - off[s]), int(t) & 3, int(t) >> 2))
    return out


@pytest.mark.parametrize("n,k,enc,gamma,eps", [
    (3, 1, QUBIT, 0.06, 0.02), (2, 2, QUBIT, 0.1, 0.03), (2, 2, QUTRIT, 0.1, 0.03), (2, 1, QUTRIT, 0.15, 0.0)])
def test_forced_against_dense_machine(lib, orc, n, k, enc, gamma, eps):
    mem = memory_words(n, k, 70 + n + k)
    cab = cab_random(n, k, 3 + enc)
    machine = Dn.Machine(n, k, enc, mem)
    seen = 0
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps, input_ab=cab) as ctx:
        for t in range(6):
            r = orc.run_traj(n, k, enc, gamma, mem, seed=19, traj=t, eps=eps, cab=cab)
            faults = oracle_faults(orc, n, k, enc, eps, 19, t) if eps > 0 else []
            _, want = Dn.forced_evolution(n, k, enc, mem, gamma, r["jumps"], machine=machine, faults=faults,
                                          cab=cab)
            got = ctx.dense_forced(r["jumps"], faults)
            assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), t
            seen += len(r["jumps"]) > 0
    assert seen > 0


@pytest.mark.parametrize("n,k,enc,gamma,eps", [(3, 3, QUBIT, 0.03, 0.01), (3, 1, QUTRIT, 0.04, 0.01)])
def test_forced_against_sparse_export(lib, orc, n, k, enc, gamma, eps):
    """Larger registers than the dense machine holds: the state vector
    against the oracle's exported components (labels are basis states)."""
    mem = memory_words(n, k, 90 + k)
    M = 2 * (2**n - 1)
    rad = [2] * (n + k) + [3 if (enc == QUTRIT and q % 2 == 0) else 2 for q in range(M)]
    pv = np.ones(len(rad), dtype=np.int64)
    for i in range(len(rad) - 2, -1, -1):
        pv[i] = pv[i + 1] * rad[i + 1]
    seen = 0
    with lib.QramContext(n, k, enc, gamma, mem, eps=eps) as ctx:
        for t in range(4):
            r = orc.run_traj(n, k, enc, gamma, mem, seed=23, traj=t, eps=eps, export=True)
            faults = oracle_faults(orc, n, k, enc, eps, 23, t)
            got = ctx.dense_forced(r["jumps"], faults)
            comp = r["components"]
            want = np.zeros_like(got)
            for a, b, tr, amp in zip(comp["addr"], comp["bus"], comp["tree"], comp["amp"]):
                dig = [(int(a) >> (n - 1 - i)) & 1 for i in range(n)] + [(int(b) >> j) & 1 for j in range(k)]
                dig += [int(v) for v in tr]
                want[int(np.dot(dig, pv))] += amp
            assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), t
            seen += len(r["jumps"]) > 0 or len(faults) > 0
    assert seen > 0


def test_dense_limits(lib):
    mem = memory_words(3, 1, 1)
    with lib.QramContext(3, 1, QUBIT, 0.01, mem) as ctx:
        with pytest.raises(lib.QramError):
            ctx.dense_density()  # 2^18 labels: too large for a density matrix
        with pytest.raises(lib.QramError):
            ctx.dense_forced([(99, 0, 1)])  # slice out of range
