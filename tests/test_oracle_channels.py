"""Pins of the dense machine's outlook channels (Sec. VII: dephasing and the
heating channel, both with a diagonal no-jump operator), the test
infrastructure the GPU dense cross-check is compared with.

Each channel is checked on its own against its Kraus form on a single site
(written out here as 2x2 / 3x3 matrices), and on the whole register for
trace preservation, hermiticity and positivity; with both strengths zero
the query's density fidelity is the damping-only one."""
import numpy as np
import pytest

from oracle import dense as Dn

QUTRIT, QUBIT = 0, 1


def kraus_dephase(d, p):
    w = np.exp(2j * np.pi / d)
    Z = np.diag([w**v for v in range(d)])
    ops = [np.sqrt(1 - p) * np.eye(d)]
    ops += [np.sqrt(p / (d - 1)) * np.linalg.matrix_power(Z, m) for m in range(1, d)]
    return ops


def kraus_heat(d, p):
    K0 = np.diag([np.sqrt(1 - p)] + [1.0] * (d - 1))
    ops = [K0]
    for lev in range(1, d):
        K = np.zeros((d, d))
        K[lev, 0] = np.sqrt(p / (d - 1))
        ops.append(K)
    return ops


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", ["dephase", "heat"])
def test_kraus_complete(d, kind):
    ops = (kraus_dephase if kind == "dephase" else kraus_heat)(d, 0.3)
    S = sum(K.conj().T @ K for K in ops)
    assert np.allclose(S, np.eye(d), atol=1e-14)
    if kind == "heat":
        assert np.allclose(ops[0], np.diag(np.diag(ops[0])))  # diagonal no-jump operator


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
@pytest.mark.parametrize("kind", ["dephase", "heat"])
def test_channel_matches_kraus_on_one_site(enc, kind):
    """On a register whose tree is in a random state of site q and ground
    elsewhere, the marginal of site q after the machine's channel (which acts
    on every site) equals sum_K K rho K+ with the channel's Kraus matrices."""
    n, k = 2, 1
    m = Dn.Machine(n, k, enc, [0, 1, 1, 0])
    rng = np.random.default_rng(3 + enc)
    p = 0.23
    for q in (0, 1, 4):
        d = m.levels(q)
        a = rng.normal(size=d) + 1j * rng.normal(size=d)
        a /= np.linalg.norm(a)
        psi = np.zeros(m.N, dtype=complex)
        for v in range(d):
            dig = np.zeros(m.ndig, dtype=np.int64)
            dig[m.S(q)] = v
            psi[m.index(dig)] = a[v]
        rho = np.outer(psi, psi.conj())
        out = m.dephase_rho(rho, p) if kind == "dephase" else m.heat_rho(rho, p)
        assert abs(np.trace(out) - 1) < 1e-13
        # the marginal of site q
        site = m.digits[:, m.S(q)]
        red = np.zeros((d, d), dtype=complex)
        for x in np.nonzero(np.abs(out).sum(axis=1) > 0)[0]:
            for y in np.nonzero(np.abs(out[x]) > 0)[0]:
                rest_x = m.digits[x].copy()
                rest_y = m.digits[y].copy()
                rest_x[m.S(q)] = 0
                rest_y[m.S(q)] = 0
                if np.array_equal(rest_x, rest_y):
                    red[site[x], site[y]] += out[x, y]
        r0 = np.outer(a, a.conj())
        ops = (kraus_dephase if kind == "dephase" else kraus_heat)(d, p)
        want = sum(K @ r0 @ K.conj().T for K in ops)
        assert np.allclose(red, want, atol=1e-13), (enc, kind, q)


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_channels_cptp_on_register(enc):
    n, k = 2, 1
    m = Dn.Machine(n, k, enc, [1, 0, 0, 1])
    rng = np.random.default_rng(9 + enc)
    X = rng.normal(size=(m.N, 6)) + 1j * rng.normal(size=(m.N, 6))
    rho = X @ X.conj().T
    rho /= np.trace(rho)
    for f in (lambda r: m.dephase_rho(r, 0.17), lambda r: m.heat_rho(r, 0.11)):
        out = f(rho)
        assert abs(np.trace(out) - 1) < 1e-12
        assert np.allclose(out, out.conj().T, atol=1e-14)
        assert np.linalg.eigvalsh(out).min() > -1e-12


@pytest.mark.parametrize("enc", [QUBIT, QUTRIT])
def test_zero_strength_is_damping_only(enc):
    mem = [0, 1, 1, 0]
    a = Dn.density_fidelity(2, 1, enc, mem, 0.05, 0.01)
    b = Dn.density_fidelity(2, 1, enc, mem, 0.05, 0.01, dephase=0.0, heat=0.0)
    assert a == b
    c = Dn.density_fidelity(2, 1, enc, mem, 0.05, 0.01, dephase=0.02, heat=0.02)
    assert abs(c[1] - 1) < 1e-12 and c[0] < a[0]
