"""Dense brute-force checkers for tiny QRAM instances (n <= 3).

TEST INFRASTRUCTURE.  This is a second, independent rendering of the same
circuit with a different state representation: every register digit of the
whole machine (address bits, bus bits, every tree site) is an axis of a dense
numpy array, each gate is a permutation of the full basis built by vectorised
digit arithmetic, and noise is either a forced joint Kraus outcome K_J
(Eq. layerkraus) applied to a state vector, or the full amplitude-damping
channel (Eq. kraus, Eq. kraus-tri) applied site by site to a density matrix,
as in the circuit-level cross-check of App. C.  Depolarizing noise (Sec. II
B) is the uniform mixture of X, Z and ZX on a qubit and of the eight
nontrivial Weyl operators Z^b X^a on a qutrit router, on the active positions
of App. C's placement, before the slice's damping.

Register digits, in order: address bit t (t = 0 is the root's bit, the most
significant bit of i), bus bit b, then tree sites q = 2v (router) and
q = 2v+1 (data slot).  Qubit sites have 2 levels; a qutrit router has 3
(W, L, R = 0, 1, 2).
"""
from __future__ import annotations

import numpy as np

QUTRIT, QUBIT = 0, 1


class Machine:
    def __init__(self, n: int, k: int, enc: int, mem):
        self.n, self.k, self.enc = n, k, enc
        self.T = 6 * n + 2 * k
        self.M = 2 * ((1 << n) - 1)
        self.mem = [int(m) & ((1 << k) - 1) for m in mem]
        radix = [2] * (n + k)
        for q in range(self.M):
            radix.append(3 if (enc == QUTRIT and q % 2 == 0) else 2)
        self.radix = np.array(radix, dtype=np.int64)
        self.ndig = len(radix)
        self.N = int(np.prod(self.radix))
        # place values, last digit fastest
        pv = np.ones(self.ndig, dtype=np.int64)
        for d in range(self.ndig - 2, -1, -1):
            pv[d] = pv[d + 1] * self.radix[d + 1]
        self.pv = pv
        idx = np.arange(self.N, dtype=np.int64)
        self.digits = (idx[:, None] // pv[None, :]) % self.radix[None, :]
        self._slice_perm = {}

    # digit positions
    def A(self, t):
        return t

    def B(self, b):
        return self.n + b

    def S(self, q):
        return self.n + self.k + q

    def index(self, dig):
        return dig @ self.pv

    # ---- gates of App. A/C as maps on the digit table ----
    def events(self, s):
        n, k, T = self.n, self.k, self.T
        ev = set()
        for t in range(n):
            if s in (2 * t + 1, T - 2 * t - 1):
                ev.add(("copy", t))
            for l in range(t):
                if s in (2 * t + 2 + l, T - 2 * t - 2 - l):
                    ev.add(("cswap", l))
            if s in (3 * t + 2, T - 3 * t - 2):
                ev.add(("store", t))
        for b in range(k):
            if s in (2 * n + 2 * b + 1, 4 * n + 2 * b + 1):
                ev.add(("bus", b))
            for l in range(n - 1):
                if s in (2 * n + 2 * b + 2 + l, 4 * n + 2 * b - l):
                    ev.add(("cswap", l))
            if s == 3 * n + 2 * b + 1:
                ev.add(("fetch", b))
        return sorted(ev)

    def _apply(self, dig, ph, name, arg):
        d = dig.copy()
        n = self.n
        if name == "copy":
            d[:, self.S(1)] ^= dig[:, self.A(arg)]
        elif name == "bus":
            d[:, self.B(arg)] = dig[:, self.S(1)]
            d[:, self.S(1)] = dig[:, self.B(arg)]
        elif name == "store":
            for v in range(2 ** arg - 1, 2 ** (arg + 1) - 1):
                r, x = dig[:, self.S(2 * v)], dig[:, self.S(2 * v + 1)]
                if self.enc == QUBIT:
                    d[:, self.S(2 * v)], d[:, self.S(2 * v + 1)] = x, r
                else:
                    if v == 0:
                        g = np.ones(len(dig), dtype=bool)
                    else:
                        p = (v - 1) // 2
                        want = 1 if v % 2 == 1 else 2
                        g = dig[:, self.S(2 * p)] == want
                    # (W,0)<->(L,0) and (W,1)<->(R,0)
                    m1 = g & (r == 0)
                    m2 = g & (r != 0) & (x == 0)
                    nr = r.copy()
                    nx = x.copy()
                    nr[m1] = np.where(x[m1] == 1, 2, 1)
                    nx[m1] = 0
                    nr[m2] = 0
                    nx[m2] = np.where(r[m2] == 2, 1, 0)
                    d[:, self.S(2 * v)], d[:, self.S(2 * v + 1)] = nr, nx
        elif name == "cswap":
            for v in range(2 ** arg - 1, 2 ** (arg + 1) - 1):
                r = dig[:, self.S(2 * v)]
                dv = dig[:, self.S(2 * v + 1)]
                dl = dig[:, self.S(2 * (2 * v + 1) + 1)]
                dr = dig[:, self.S(2 * (2 * v + 2) + 1)]
                if self.enc == QUBIT:
                    left, right = r == 0, r == 1
                else:
                    left, right = r == 1, r == 2
                d[:, self.S(2 * v + 1)] = np.where(left, dl, np.where(right, dr, dv))
                d[:, self.S(2 * (2 * v + 1) + 1)] = np.where(left, dv, dl)
                d[:, self.S(2 * (2 * v + 2) + 1)] = np.where(right, dv, dr)
        elif name == "fetch":
            b = arg
            l = n - 1
            for v in range(2 ** l - 1, 2 ** (l + 1) - 1):
                p = v - (2 ** l - 1)
                r = dig[:, self.S(2 * v)]
                x = dig[:, self.S(2 * v + 1)]
                m0 = (self.mem[2 * p] >> b) & 1
                m1 = (self.mem[2 * p + 1] >> b) & 1
                if self.enc == QUBIT:
                    bitv = np.where(r == 1, m1, m0)
                    ph = ph * np.where((x == 1) & (bitv == 1), -1.0, 1.0)
                else:
                    bitv = np.where(r == 2, m1, m0)
                    bitv = np.where(r == 0, 0, bitv)
                    d[:, self.S(2 * v + 1)] = x ^ bitv
        return d, ph

    def slice_perm(self, s):
        """(dest index, phase) of every basis state under the gates of slice s.
        Within a slice the operations touch disjoint digits, so they are
        applied one after the other on the original table."""
        if s not in self._slice_perm:
            dig = self.digits
            ph = np.ones(self.N)
            for name, arg in self.events(s):
                dig, ph = self._apply(dig, ph, name, arg)
            dest = self.index(dig)
            assert len(np.unique(dest)) == self.N, "gates must be a permutation"
            self._slice_perm[s] = (dest, ph)
        return self._slice_perm[s]

    def gates(self, psi, s):
        dest, ph = self.slice_perm(s)
        out = np.zeros_like(psi)
        out[dest] = ph * psi
        return out

    def gates_rho(self, rho, s):
        dest, ph = self.slice_perm(s)
        out = np.zeros_like(rho)
        out[np.ix_(dest, dest)] = (ph[:, None] * ph[None, :]) * rho
        return out

    def wall(self, psi):
        """Hadamard on every bus qubit (qubit encoding only)."""
        shape = tuple(int(r) for r in self.radix)
        x = psi.reshape(shape)
        H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
        for b in range(self.k):
            ax = self.B(b)
            x = np.moveaxis(np.tensordot(H, x, axes=([1], [ax])), 0, ax)
        return x.reshape(self.N)

    def wall_rho(self, rho):
        rho = np.apply_along_axis(self.wall, 0, rho)
        rho = np.apply_along_axis(self.wall, 1, rho.conj()).conj()
        return rho

    # ---- states ----
    def _basis(self, i, j):
        dig = np.zeros(self.ndig, dtype=np.int64)
        for t in range(self.n):
            dig[self.A(t)] = (i >> (self.n - 1 - t)) & 1
        for b in range(self.k):
            dig[self.B(b)] = (j >> b) & 1
        return self.index(dig)

    def input_state(self, cab=None):
        """sum_ij c_ij |i>|j>|ground> (cab[i, j], normalised here); None: the
        data-loading input, uniform over addresses with bus word 0."""
        psi = np.zeros(self.N, dtype=complex)
        if cab is None:
            for i in range(1 << self.n):
                psi[self._basis(i, 0)] = 1.0 / np.sqrt(1 << self.n)
            return psi
        cab = np.asarray(cab, dtype=complex).reshape(1 << self.n, 1 << self.k)
        for i in range(1 << self.n):
            for j in range(1 << self.k):
                psi[self._basis(i, j)] = cab[i, j]
        return psi / np.linalg.norm(psi)

    def ideal_state(self, cab=None):
        """The ideal output sum_ij c_ij |i>|j xor d_i>|ground>."""
        psi = np.zeros(self.N, dtype=complex)
        if cab is None:
            for i in range(1 << self.n):
                psi[self._basis(i, self.mem[i])] = 1.0 / np.sqrt(1 << self.n)
            return psi
        cab = np.asarray(cab, dtype=complex).reshape(1 << self.n, 1 << self.k)
        for i in range(1 << self.n):
            for j in range(1 << self.k):
                psi[self._basis(i, j ^ self.mem[i])] = cab[i, j]
        return psi / np.linalg.norm(psi)

    def excited(self):
        """Boolean table: tree site q excited in basis state x."""
        return self.digits[:, self.n + self.k:] != 0

    # ---- depolarizing faults ----
    def active_sites(self, s):
        """Sites of the layers above the leaf layer whose router holds its
        address bit before and after the gates of slice s (stored at 3t+2,
        unstored at T-3t-2): every site of those layers."""
        l = sum(1 for t in range(self.n - 1) if 3 * t + 2 < s < self.T - 3 * t - 2)
        return list(range(2 * (2 ** l - 1)))

    def levels(self, q):
        return 3 if (self.enc == QUTRIT and q % 2 == 0) else 2

    def fault_ops(self, q):
        """The (a, b) of the depolarizing mixture at site q: Z^b X^a."""
        if self.levels(q) == 2:
            return [(1, 0), (0, 1), (1, 1)]
        return [(a, b) for a in range(3) for b in range(3) if (a, b) != (0, 0)]

    def _fault_map(self, q, a, b):
        d = self.levels(q)
        dig = self.digits.copy()
        new = (dig[:, self.S(q)] + a) % d
        dig[:, self.S(q)] = new
        w = np.exp(2j * np.pi / d)
        return self.index(dig), w ** (b * new)

    def fault(self, psi, q, a, b):
        """Apply Z^b X^a to site q of a state vector."""
        dest, ph = self._fault_map(q, a, b)
        out = np.zeros_like(psi)
        out[dest] = ph * psi
        return out

    def depol_rho(self, rho, s, p):
        """Depolarizing channel of strength p on every active site of slice s."""
        for q in self.active_sites(s):
            ops = self.fault_ops(q)
            new = (1.0 - p) * rho
            for a, b in ops:
                dest, ph = self._fault_map(q, a, b)
                r = np.zeros_like(rho)
                r[np.ix_(dest, dest)] = (ph[:, None] * np.conj(ph)[None, :]) * rho
                new = new + (p / len(ops)) * r
            rho = new
        return rho

    # ---- noise ----
    def kraus_J(self, psi, J, gamma):
        """Apply K_J (Eq. layerkraus) for the joint outcome J = {(site, level)}."""
        a = np.sqrt(1.0 - gamma)
        tree = self.digits[:, self.n + self.k:]
        nexc = (tree != 0).sum(axis=1)
        ok = np.ones(self.N, dtype=bool)
        dig = self.digits.copy()
        for q, lev in J:
            ok &= tree[:, q] == lev
            dig[:, self.S(q)] = 0
        fac = np.sqrt(gamma) ** len(J) * a ** (nexc - len(J))
        out = np.zeros_like(psi)
        src = np.nonzero(ok)[0]
        out[self.index(dig[src])] = fac[src] * psi[src]
        return out

    def dephase_rho(self, rho, p):
        """Dephasing of strength p on every tree site (an outlook channel of
        Sec. VII): (1-p) rho + p Z rho Z+ on a qubit site, (1-p) rho + (p/2)
        (Z rho Z+ + Z^2 rho Z^2+) on a qutrit router, Z = diag(w^v)."""
        for q in range(self.M):
            d = self.levels(q)
            col = self.digits[:, self.S(q)]
            new = (1.0 - p) * rho
            for m in range(1, d):
                z = np.exp(2j * np.pi * m * col / d)
                new = new + (p / (d - 1)) * (z[:, None] * rho * np.conj(z)[None, :])
            rho = new
        return rho

    def heat_rho(self, rho, p):
        """Heating of strength p on every tree site (an outlook channel of
        Sec. VII): level 0 rises with probability p, to 1 on a qubit site and
        to L or R with p/2 each on a qutrit router; the no-jump operator is
        diag(sqrt(1-p), 1, 1)."""
        for q in range(self.M):
            d = self.levels(q)
            col = self.digits[:, self.S(q)]
            k0 = np.where(col == 0, np.sqrt(1.0 - p), 1.0)
            new = (k0[:, None] * k0[None, :]) * rho
            src = np.nonzero(col == 0)[0]
            for lev in range(1, d):
                dig = self.digits[src].copy()
                dig[:, self.S(q)] = lev
                dst = self.index(dig)
                new[np.ix_(dst, dst)] += (p / (d - 1)) * rho[np.ix_(src, src)]
            rho = new
        return rho

    def damp_rho(self, rho, gamma):
        """Amplitude damping on every tree site (Eq. kraus / kraus-tri)."""
        a = np.sqrt(1.0 - gamma)
        for q in range(self.M):
            col = self.digits[:, self.S(q)]
            k0 = np.where(col != 0, a, 1.0)
            new = (k0[:, None] * k0[None, :]) * rho
            for lev in (1, 2):
                if lev == 2 and not (self.enc == QUTRIT and q % 2 == 0):
                    continue
                src = np.nonzero(col == lev)[0]
                if len(src) == 0:
                    continue
                dig = self.digits[src].copy()
                dig[:, self.S(q)] = 0
                dst = self.index(dig)
                new[np.ix_(dst, dst)] += gamma * rho[np.ix_(src, src)]
            rho = new
        return rho


def density_fidelity(n, k, enc, mem, gamma, eps=0.0, cab=None, dephase=0.0, heat=0.0):
    """F_rho = <psi_id| rho |psi_id> of the whole query under damping and
    (eps > 0) depolarizing noise: per slice the gates, then the depolarizing
    channel on the active sites, then damping on every tree site, then
    (dephase, heat > 0) dephasing and heating on every tree site.  cab: a
    general input c_ij (None: the data-loading input)."""
    m = Machine(n, k, enc, mem)
    psi = m.input_state(cab)
    if enc == QUBIT:
        psi = m.wall(psi)
    rho = np.outer(psi, psi.conj())
    for s in range(1, m.T):
        rho = m.gates_rho(rho, s)
        if eps > 0.0:
            rho = m.depol_rho(rho, s, eps)
        if gamma > 0.0:
            rho = m.damp_rho(rho, gamma)
        if dephase > 0.0:
            rho = m.dephase_rho(rho, dephase)
        if heat > 0.0:
            rho = m.heat_rho(rho, heat)
    if enc == QUBIT:
        rho = m.wall_rho(rho)
    pid = m.ideal_state(cab)
    return float(np.real(pid.conj() @ rho @ pid)), float(np.real(np.trace(rho)))


def forced_evolution(n, k, enc, mem, gamma, jumps, stop_before_wall=True, machine=None, faults=(), cab=None):
    """State vector under a forced sequence of joint outcomes.

    jumps: list of (slice, site, level).  Every other layer applies K_empty.
    faults: depolarizing faults (slice, site, a, b), applied after the gates
    of their slice and before its damping layer.  cab: a general input.
    Returns the final state (before the second wall unless told otherwise)."""
    m = machine if machine is not None else Machine(n, k, enc, mem)
    psi = m.input_state(cab)
    if enc == QUBIT:
        psi = m.wall(psi)
    byslice = {}
    for s, q, lev in jumps:
        byslice.setdefault(s, []).append((q, lev))
    fby = {}
    for s, q, a, b in faults:
        fby.setdefault(s, []).append((q, a, b))
    for s in range(1, m.T):
        psi = m.gates(psi, s)
        for q, a, b in fby.get(s, []):
            psi = m.fault(psi, q, a, b)
        psi = m.kraus_J(psi, byslice.get(s, []), gamma)
    if enc == QUBIT and not stop_before_wall:
        psi = m.wall(psi)
    return m, psi


def layer_state(n, k, enc, mem, gamma, jumps, s):
    """State after the damping layers of slices 1..s-1 and the gates of s."""
    m = Machine(n, k, enc, mem)
    psi = m.input_state()
    if enc == QUBIT:
        psi = m.wall(psi)
    byslice = {}
    for ss, q, lev in jumps:
        byslice.setdefault(ss, []).append((q, lev))
    for ss in range(1, s + 1):
        psi = m.gates(psi, ss)
        if ss < s:
            psi = m.kraus_J(psi, byslice.get(ss, []), gamma)
    return m, psi
