"""ctypes front end of the plain CPU oracle (``qram_oracle.c``).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It never imports
the HIP package, and the HIP package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qram_oracle.c")
LIB = os.path.join(HERE, "liborc_qram.so")

QUTRIT = 0
QUBIT = 1
TAG_FAULT, TAG_AUX, TAG_FINAL = 1, 2, 3
EV_NAMES = {1: "copy", 2: "store", 3: "cswap", 4: "bus", 5: "fetch"}
NRD, NRI = 4, 10

_lib = None


def build_lib(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE-exact: no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
             "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build_lib()
        L = C.CDLL(LIB)
        u32p = C.POINTER(C.c_uint32)
        i32p = C.POINTER(C.c_int)
        f64p = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_thresholds.argtypes = [C.c_double, C.POINTER(C.c_uint64)]
        L.orc_schedule.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p]
        L.orc_sample.argtypes = [C.c_int, C.c_int, C.c_double, C.c_uint64, C.c_uint32, u32p, C.c_int]
        L.orc_classify.argtypes = [C.c_int, C.c_int, C.c_int, u32p, C.c_int, u8p]
        L.orc_range_node.argtypes = [C.c_int, C.c_uint32]
        L.orc_run_traj.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, u32p, C.c_uint64, C.c_uint32,
            u32p, C.c_int, f64p, C.c_double, C.c_int, f64p, i32p,
            i32p, i32p, i32p, C.c_int, i32p,
            u32p, u32p, f64p, u8p, u32p, C.c_int]
        L.orc_layer_masks.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, u32p, u32p, C.c_int, f64p,
            C.c_int, i32p, C.c_int, u8p, f64p, C.c_int, f64p]
        L.orc_run_batch.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, u32p, C.c_uint64, C.c_uint32,
            C.c_int, C.c_int, f64p, f64p, i32p]
        L.orc_run_indices.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, u32p, C.c_uint64, u32p,
            C.c_int, C.c_int, f64p, f64p, i32p]
        L.orc_run_traj_ex.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, u32p, f64p, u32p, f64p, C.c_int,
            C.c_uint64, C.c_uint32, u32p, C.c_int, f64p, C.c_double,
            C.c_int, u32p, u32p, u8p, C.c_int, C.c_int, f64p, i32p,
            i32p, i32p, i32p, C.c_int, i32p,
            u32p, u32p, f64p, u8p, u32p, C.c_int]
        L.orc_run_many_ex.argtypes = [
            C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, u32p, f64p, u32p, f64p, C.c_int,
            C.c_uint64, C.c_uint32, u32p, C.c_int, C.c_int, f64p, f64p, i32p]
        L.orc_sample_depol.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint64, C.c_uint32,
                                       u32p, u8p, C.c_int]
        L.orc_depol_active.argtypes = [C.c_int, C.c_int, i32p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def uniform(seed, c0, c1, traj, tag):
    return lib().orc_uniform(seed, c0, c1, traj, tag)


def thresholds(gamma):
    G = np.zeros(64, dtype=np.uint64)
    lib().orc_thresholds(gamma, _p(G, C.c_uint64))
    return G


def schedule(n, k, s):
    t = np.zeros(64, dtype=np.int32)
    a = np.zeros(64, dtype=np.int32)
    m = lib().orc_schedule(n, k, s, _p(t, C.c_int), _p(a, C.c_int))
    if m < 0:
        raise ValueError(f"bad (n,k)=({n},{k})")
    return [(EV_NAMES[int(t[e])], int(a[e])) for e in range(m)]


def sample(n, k, gamma, seed, traj):
    cnt = lib().orc_sample(n, k, gamma, seed, traj, None, 0)
    if cnt < 0:
        raise ValueError("bad parameters")
    L = np.zeros(max(cnt, 1), dtype=np.uint32)
    lib().orc_sample(n, k, gamma, seed, traj, _p(L, C.c_uint32), cnt)
    return L[:cnt]


def classify(n, k, enc, L, subtree=False):
    """Bad-address bitmap of a candidate list.  subtree=True marks every
    candidate's own subtree (Eq. subtree) whatever the encoding: the tighter
    rule for damping candidates of the qubit encoding (Sec. III B: damping
    creates no strays, so its damage stays inside the candidate's subtree)."""
    L = np.ascontiguousarray(L, dtype=np.uint32)
    bad = np.zeros(1 << n, dtype=np.uint8)
    rule = QUTRIT if subtree else enc
    nb = lib().orc_classify(n, k, rule, _p(L, C.c_uint32), len(L), _p(bad, C.c_uint8))
    if nb < 0:
        raise ValueError("bad parameters")
    return bad


def range_node(enc, v):
    return lib().orc_range_node(enc, v)


def _mem(mem):
    return np.ascontiguousarray(mem, dtype=np.uint32)


def _cin(cin, n):
    if cin is None:
        return None
    c = np.asarray(cin, dtype=np.complex128)
    assert c.shape == (1 << n,)
    out = np.empty(2 * len(c))
    out[0::2], out[1::2] = c.real, c.imag
    return out


def _cab(cab, n, k):
    """c_ij of every (address, bus word), address-major, as (re, im) pairs."""
    if cab is None:
        return None
    c = np.asarray(cab, dtype=np.complex128).reshape(-1)
    assert c.shape == ((1 << n) << k,)
    out = np.empty(2 * len(c))
    out[0::2], out[1::2] = c.real, c.imag
    return out


def _jin(jin, n):
    if jin is None:
        return None
    j = np.ascontiguousarray(jin, dtype=np.uint32)
    assert j.shape == (1 << n,)
    return j


def run_traj(n, k, enc, gamma, mem, seed=0, traj=0, forced_L=None,
             forced_uaux=None, forced_ufin=-1.0, check_counts=False,
             export=False, jcap=4096, eps=0.0, cin=None, jin=None, forced_dep=None, cab=None, wmax=-1):
    """One trajectory of the full (unpruned) evolution.

    eps: depolarizing strength; cin / jin: input amplitude and bus word of
    every address (None: uniform, 0); or cab: amplitude c_ij of every
    (address i, bus word j), shape (2^n, 2^k); wmax: Hamming truncation of
    the predicted good branches (-1: none); forced_dep: list of faults (slice,
    site, a, b), the operator Z^b X^a, replacing the depolarizing draws.  Returns a dict with fid, fid_pre, w_ground,
    w_total, ncand, nbad, ref, nexplicit, njumps, first_jump, ref_survived,
    q_ground, max_exc, ndep, the jump log and, if export, the final pre-wall
    components."""
    mem = _mem(mem)
    T = 6 * n + 2 * k
    M = 2 * ((1 << n) - 1)
    E = (1 << n) * ((1 << k) if enc == QUBIT or cab is not None else 1)
    rd = np.zeros(NRD)
    ri = np.zeros(NRI, dtype=np.int32)
    js = np.zeros(jcap, dtype=np.int32)
    jq = np.zeros(jcap, dtype=np.int32)
    jv = np.zeros(jcap, dtype=np.int32)
    njl = np.zeros(1, dtype=np.int32)
    fL = None if forced_L is None else np.ascontiguousarray(forced_L, dtype=np.uint32)
    fU = None
    if forced_uaux is not None:
        fU = np.ascontiguousarray(forced_uaux, dtype=np.float64)
        assert len(fU) >= T
    cap = E if export else 0
    ea = np.zeros(max(cap, 1), dtype=np.uint32)
    eb = np.zeros(max(cap, 1), dtype=np.uint32)
    eamp = np.zeros(2 * max(cap, 1))
    etree = np.zeros(max(cap, 1) * M, dtype=np.uint8)
    elab = np.zeros(max(cap, 1), dtype=np.uint32)
    cinp, jinp, cabp = _cin(cin, n), _jin(jin, n), _cab(cab, n, k)
    dS = dQ = dT = None
    if forced_dep is not None:  # list of (slice, site, a, b), slices ascending
        fd = sorted(forced_dep, key=lambda f: f[0])
        dS = np.array([f[0] for f in fd], dtype=np.uint32)
        dQ = np.array([f[1] for f in fd], dtype=np.uint32)
        dT = np.array([f[2] | (f[3] << 2) for f in fd], dtype=np.uint8)
    ne = lib().orc_run_traj_ex(
        n, k, enc, gamma, eps, _p(mem, C.c_uint32), _p(cinp, C.c_double), _p(jinp, C.c_uint32),
        _p(cabp, C.c_double), int(wmax), seed, traj,
        _p(fL, C.c_uint32) if fL is not None else None,
        len(fL) if fL is not None else 0,
        _p(fU, C.c_double) if fU is not None else None, forced_ufin,
        1 if forced_dep is not None else 0,
        _p(dS, C.c_uint32) if dS is not None and len(dS) else None,
        _p(dQ, C.c_uint32) if dQ is not None and len(dQ) else None,
        _p(dT, C.c_uint8) if dT is not None and len(dT) else None,
        0 if dS is None else len(dS),
        1 if check_counts else 0, _p(rd, C.c_double), _p(ri, C.c_int),
        _p(js, C.c_int), _p(jq, C.c_int), _p(jv, C.c_int), jcap, _p(njl, C.c_int),
        _p(ea, C.c_uint32), _p(eb, C.c_uint32), _p(eamp, C.c_double),
        _p(etree, C.c_uint8), _p(elab, C.c_uint32), cap)
    if ne < 0:
        raise ValueError(f"oracle error {ne}")
    out = dict(fid=rd[0], fid_pre=rd[1], w_ground=rd[2], w_total=rd[3],
               ncand=int(ri[0]), nbad=int(ri[1]), ref=int(ri[2]),
               nexplicit=int(ri[3]), njumps=int(ri[4]), first_jump=int(ri[5]),
               ref_survived=int(ri[6]), q_ground=int(ri[7]), max_exc=int(ri[8]), ndep=int(ri[9]))
    nj = int(njl[0])
    out["jumps"] = [(int(js[j]), int(jq[j]), int(jv[j])) for j in range(min(nj, jcap))]
    if export:
        out["components"] = dict(
            label=elab[:ne].copy(), addr=ea[:ne].copy(), bus=eb[:ne].copy(),
            amp=(eamp[0:2 * ne:2] + 1j * eamp[1:2 * ne:2]).copy(),
            tree=etree[:ne * M].reshape(ne, M).copy())
    return out


def layer_masks(n, k, enc, gamma, mem, forced_L, forced_uaux, s, cand, cap=4096):
    """Mask weights w(J) of the damping layer at slice s (see the C entry)."""
    mem = _mem(mem)
    fL = np.ascontiguousarray(forced_L, dtype=np.uint32)
    fU = np.ascontiguousarray(forced_uaux, dtype=np.float64)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    nc = len(cand)
    masks = np.zeros(cap * max(nc, 1), dtype=np.uint8)
    w = np.zeros(cap)
    we = np.zeros(1)
    nm = lib().orc_layer_masks(
        n, k, enc, gamma, _p(mem, C.c_uint32), _p(fL, C.c_uint32), len(fL),
        _p(fU, C.c_double), s, _p(cand, C.c_int), nc, _p(masks, C.c_uint8),
        _p(w, C.c_double), cap, _p(we, C.c_double))
    if nm < 0:
        raise ValueError("oracle error")
    return {tuple(int(v) for v in masks[m * nc:(m + 1) * nc]): float(w[m])
            for m in range(nm)}, float(we[0])


def run_batch(n, k, enc, gamma, mem, seed, traj0, ntraj, nthreads=0):
    """Trajectories traj0..traj0+ntraj-1; returns (fid, fid_pre, stats, threads)."""
    mem = _mem(mem)
    fid = np.zeros(ntraj)
    fpre = np.zeros(ntraj)
    ri = np.zeros(ntraj * NRI, dtype=np.int32)
    used = lib().orc_run_batch(n, k, enc, gamma, _p(mem, C.c_uint32), seed, traj0,
                               ntraj, nthreads, _p(fid, C.c_double),
                               _p(fpre, C.c_double), _p(ri, C.c_int))
    if used < 0:
        raise ValueError("oracle error")
    return fid, fpre, ri.reshape(ntraj, NRI), used


def run_many(n, k, enc, gamma, mem, seed, traj0=0, ntraj=None, idx=None, nthreads=0, eps=0.0, cin=None,
             jin=None, cab=None, wmax=-1):
    """Trajectories traj0.. (or the listed indices) with depolarizing
    strength eps and a general input (cin/jin, or cab as in run_traj) and
    the truncation wmax; returns (fid, fid_pre, stats, threads)."""
    mem = _mem(mem)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.uint32)
        ntraj = len(idx)
    fid = np.zeros(ntraj)
    fpre = np.zeros(ntraj)
    ri = np.zeros(max(ntraj, 1) * NRI, dtype=np.int32)
    cinp, jinp, cabp = _cin(cin, n), _jin(jin, n), _cab(cab, n, k)
    used = lib().orc_run_many_ex(n, k, enc, gamma, eps, _p(mem, C.c_uint32), _p(cinp, C.c_double),
                                 _p(jinp, C.c_uint32), _p(cabp, C.c_double), int(wmax), seed, traj0,
                                 _p(idx, C.c_uint32), ntraj, nthreads,
                                 _p(fid, C.c_double), _p(fpre, C.c_double), _p(ri, C.c_int))
    if used < 0:
        raise ValueError("oracle error")
    return fid, fpre, ri[:ntraj * NRI].reshape(ntraj, NRI), used


def sample_depol(n, k, enc, eps, seed, traj):
    """Depolarizing faults of one trajectory: (linear indices, types a | b << 2)."""
    cnt = lib().orc_sample_depol(n, k, enc, eps, seed, traj, None, None, 0)
    if cnt < 0:
        raise ValueError("bad parameters")
    L = np.zeros(max(cnt, 1), dtype=np.uint32)
    t = np.zeros(max(cnt, 1), dtype=np.uint8)
    lib().orc_sample_depol(n, k, enc, eps, seed, traj, _p(L, C.c_uint32), _p(t, C.c_uint8), cnt)
    return L[:cnt], t[:cnt]


def depol_active(n, k):
    """Active depolarizing positions of each slice (index = slice)."""
    a = np.zeros(6 * n + 2 * k, dtype=np.int32)
    T = lib().orc_depol_active(n, k, _p(a, C.c_int))
    return a[:T]


def run_indices(n, k, enc, gamma, mem, seed, idx, nthreads=0):
    """The listed trajectory indices; returns (fid, fid_pre, stats, threads)."""
    mem = _mem(mem)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    nt = len(idx)
    fid = np.zeros(nt)
    fpre = np.zeros(nt)
    ri = np.zeros(max(nt, 1) * NRI, dtype=np.int32)
    used = lib().orc_run_indices(n, k, enc, gamma, _p(mem, C.c_uint32), seed, _p(idx, C.c_uint32),
                                 nt, nthreads, _p(fid, C.c_double), _p(fpre, C.c_double), _p(ri, C.c_int))
    if used < 0:
        raise ValueError("oracle error")
    return fid, fpre, ri[:nt * NRI].reshape(nt, NRI), used


STAT_FIELDS = ["ncand", "nbad", "ref", "nexplicit", "njumps", "first_jump",
               "ref_survived", "q_ground", "max_exc", "ndep"]
