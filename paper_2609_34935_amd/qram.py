"""Python binding of the C ABI in include/qram.h (argument marshalling only).

Every step of a trajectory runs in the HIP library ``libqram_hip.so``; this
module loads it with ctypes and fails loudly when it is missing.  PyTorch is
used only for device buffers and streams in the ``*_async`` calls.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqram_hip.so")

QRAM_QUTRIT, QRAM_QUBIT = 0, 1
QRAM_MODE_FULL, QRAM_MODE_PRUNED, QRAM_MODE_PLAIN = 0, 1, 2
STATUS = {0: "QRAM_OK", -1: "QRAM_E_INVAL", -2: "QRAM_E_NOMEM", -3: "QRAM_E_DEVICE",
          -4: "QRAM_E_RANGE", -5: "QRAM_E_CAPACITY"}

STATS_DTYPE = np.dtype([
    ("n_cand", "<u4"), ("n_bad", "<u4"), ("ref_addr", "<u4"), ("n_explicit", "<u4"),
    ("n_jumps", "<u2"), ("first_jump_slice", "<u2"), ("ref_survived", "u1"),
    ("q_ground", "u1"), ("flags", "u1"), ("pad", "u1"), ("fid_pre", "<f8")])
assert STATS_DTYPE.itemsize == 32


class QramRequest(C.Structure):
    _fields_ = [("n_addr", C.c_int), ("k_data", C.c_int), ("enc", C.c_int), ("gamma", C.c_double),
                ("memory_bits", C.POINTER(C.c_uint32)), ("seed", C.c_uint64), ("traj0", C.c_uint64),
                ("shots", C.c_uint32), ("mode", C.c_int)]


class QramParams(C.Structure):
    _fields_ = [("n_addr", C.c_int), ("k_data", C.c_int), ("enc", C.c_int), ("gamma", C.c_double),
                ("eps", C.c_double), ("memory_bits", C.POINTER(C.c_uint32)),
                ("input_amp", C.POINTER(C.c_double)), ("input_bus", C.POINTER(C.c_uint32)),
                ("input_ab", C.POINTER(C.c_double)), ("truncate", C.c_int), ("w_max", C.c_int)]


class QramResult(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("state", C.c_int), ("status", C.c_int), ("mean", C.c_double),
                ("sem", C.c_double), ("shots", C.c_uint32), ("footprint_bytes", C.c_uint64),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double)]

# Every entry point declared in include/qram.h.
EXPORTS = [
    "qram_create", "qram_create_ex", "qram_destroy", "qram_last_error", "qram_sample_faults", "qram_sample_depol",
    "qram_run_full", "qram_run_pruned", "qram_run_full_async", "qram_run_pruned_async",
    "qram_fidelity", "qram_set_launch", "qram_get_launch", "qram_autotune",
    "qram_last_kernel_ms", "qram_set_timing", "qram_stage_times", "qram_stage_launches", "qram_set_option",
    "qram_run_forced", "qram_footprint", "qram_reserve", "qram_errors", "qram_run_pruned_async_noalloc",
    "qram_export_state", "qram_run_jumplog", "qram_run_plain", "qram_run_plain_async", "qram_stage_buckets",
    "qram_dense_dim", "qram_dense_density", "qram_dense_forced",
    "qram_server_create", "qram_server_submit", "qram_server_poll", "qram_server_wait",
    "qram_server_fidelities", "qram_server_release", "qram_server_destroy",
]
QRAM_OPT_TIER2_GLOBAL = 1
QRAM_OPT_GRAPH = 2
QRAM_OPT_SUBTREE_MARKING = 3


class QramError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library not found at {path}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(path)
    vp, u32, u64, f64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_double
    p = C.POINTER
    L.qram_create.argtypes = [C.c_int, C.c_int, C.c_int, f64, p(u32), p(vp)]
    L.qram_create.restype = C.c_int
    L.qram_create_ex.argtypes = [C.POINTER(QramParams), p(vp)]
    L.qram_create_ex.restype = C.c_int
    L.qram_sample_depol.argtypes = [vp, u64, u64, u32, p(u32), p(u32), u64]
    L.qram_dense_dim.argtypes = [vp, p(u64)]
    L.qram_dense_density.argtypes = [vp, f64, f64, p(f64), p(f64)]
    L.qram_dense_forced.argtypes = [vp, p(u32), u32, p(u32), u32, p(f64), u64]
    L.qram_destroy.argtypes = [vp]
    L.qram_destroy.restype = None
    L.qram_server_destroy.restype = None
    L.qram_last_error.argtypes = [vp]
    L.qram_last_error.restype = C.c_char_p
    L.qram_sample_faults.argtypes = [vp, u64, u64, u32, p(u32), p(u64), p(u32), p(u64), p(u32), u64]
    for f in (L.qram_run_full, L.qram_run_pruned, L.qram_run_plain):
        f.argtypes = [vp, u64, u64, u32, p(f64), vp]
    for f in (L.qram_run_full_async, L.qram_run_pruned_async, L.qram_run_pruned_async_noalloc,
              L.qram_run_plain_async):
        f.argtypes = [vp, u64, u64, u32, vp, vp, vp]
    L.qram_fidelity.argtypes = [p(f64), u32, p(f64), p(f64)]
    L.qram_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.qram_get_launch.argtypes = [vp, C.c_int, p(C.c_int), p(C.c_int)]
    L.qram_autotune.argtypes = [vp, C.c_int, u64, u64, u32, p(f64)]
    L.qram_last_kernel_ms.argtypes = [vp, p(f64)]
    L.qram_run_forced.argtypes = [vp, C.c_int, p(u32), u32, p(f64), f64, p(f64), vp]
    L.qram_export_state.argtypes = [vp, C.c_int, u64, u32, p(u32), u32, p(f64), f64, p(u32), u32, p(f64),
                                    p(u32), u32, p(u32), p(f64), vp]
    L.qram_run_jumplog.argtypes = [vp, C.c_int, u64, u64, u32, p(f64), vp, p(u32), u32, p(u32)]
    L.qram_set_timing.argtypes = [vp, C.c_int]
    L.qram_stage_times.argtypes = [vp, p(f64), p(u32)]
    L.qram_stage_launches.argtypes = [vp, p(u32)]
    L.qram_stage_buckets.argtypes = [vp, p(f64), p(u32), p(u32), p(u32), p(C.c_int)]
    L.qram_set_option.argtypes = [vp, C.c_int, C.c_int]
    L.qram_footprint.argtypes = [vp, C.c_int, u32, p(u64)]
    L.qram_reserve.argtypes = [vp, C.c_int, u32]
    L.qram_errors.argtypes = [vp]
    L.qram_server_create.argtypes = [u64, C.c_int, u32, p(vp)]
    L.qram_server_submit.argtypes = [vp, p(QramRequest), p(u64)]
    L.qram_server_poll.argtypes = [vp, u64, p(QramResult)]
    L.qram_server_wait.argtypes = [vp, u64, f64, p(QramResult)]
    L.qram_server_fidelities.argtypes = [vp, u64, p(f64), u32]
    L.qram_server_release.argtypes = [vp, u64]
    L.qram_server_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("qram_destroy", "qram_last_error", "qram_server_destroy"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def qram_fidelity(fid):
    """Mean and standard error of the mean of per-trajectory fidelities."""
    L = load_library()
    f = np.ascontiguousarray(fid, dtype=np.float64)
    m, s = C.c_double(), C.c_double()
    st = L.qram_fidelity(_ptr(f, C.c_double), len(f), C.byref(m), C.byref(s))
    if st:
        raise QramError(st, "qram_fidelity")
    return m.value, s.value


class QramContext:
    """One (n, k, encoding, gamma, memory) simulator context on the current
    HIP device (``qram_create`` ... ``qram_destroy``)."""

    def __init__(self, n_addr, k_data, encoding, gamma, memory_bits, eps=0.0, input_amp=None, input_bus=None,
                 input_ab=None, w_max=None):
        """eps: depolarizing strength; input_amp (complex, 2^n) and input_bus
        (2^n words): a general input sum_i c_i |i>|j_i>; or input_ab
        (complex, 2^n x 2^k): sum_ij c_ij |i>|j>; w_max: Hamming truncation
        of the predicted good branches (``qram_create_ex``)."""
        L = load_library()
        self.n, self.k, self.enc, self.gamma = int(n_addr), int(k_data), int(encoding), float(gamma)
        self.eps = float(eps)
        self.T = 6 * self.n + 2 * self.k
        self.M = 2 * ((1 << self.n) - 1)
        self.D = 1 << self.n
        mem = np.ascontiguousarray(memory_bits, dtype=np.uint32)
        if mem.shape != (self.D,):
            raise ValueError(f"memory_bits must hold 2^n = {self.D} words")
        self.K2 = (1 << self.k) if (self.enc == 1 or input_ab is not None) else 1
        h = C.c_void_p()
        if self.eps == 0.0 and input_amp is None and input_bus is None and input_ab is None and w_max is None:
            st = L.qram_create(self.n, self.k, self.enc, self.gamma, _ptr(mem, C.c_uint32), C.byref(h))
        else:
            amp = bus = None
            if input_amp is not None:
                c = np.asarray(input_amp, dtype=np.complex128)
                if c.shape != (self.D,):
                    raise ValueError(f"input_amp must hold 2^n = {self.D} amplitudes")
                amp = np.empty(2 * self.D)
                amp[0::2], amp[1::2] = c.real, c.imag
            if input_bus is not None:
                bus = np.ascontiguousarray(input_bus, dtype=np.uint32)
                if bus.shape != (self.D,):
                    raise ValueError(f"input_bus must hold 2^n = {self.D} words")
            ab = None
            if input_ab is not None:
                c = np.asarray(input_ab, dtype=np.complex128).reshape(-1)
                if c.shape != (self.D << self.k,):
                    raise ValueError(f"input_ab must hold 2^n * 2^k = {self.D << self.k} amplitudes")
                ab = np.empty(2 * len(c))
                ab[0::2], ab[1::2] = c.real, c.imag
            prm = QramParams(self.n, self.k, self.enc, self.gamma, self.eps, _ptr(mem, C.c_uint32),
                             _ptr(amp, C.c_double), _ptr(bus, C.c_uint32), _ptr(ab, C.c_double),
                             0 if w_max is None else 1, 0 if w_max is None else int(w_max))
            st = L.qram_create_ex(C.byref(prm), C.byref(h))
        if st:
            raise QramError(st, L.qram_last_error(None).decode())
        self._h = h
        self._L = L

    def dense_density(self, dephase=0.0, heat=0.0):
        """qram_dense_density: (F_rho, trace) of the whole query as a density
        matrix under the context's channels plus dephasing / heating."""
        F, tr = C.c_double(), C.c_double()
        self._check(self._L.qram_dense_density(self._h, float(dephase), float(heat), C.byref(F), C.byref(tr)),
                    "qram_dense_density")
        return F.value, tr.value

    def dense_forced(self, jumps=(), faults=()):
        """qram_dense_forced: the state vector (complex, N) before the second
        wall under the given jumps (slice, site, level) and faults (slice,
        site, a, b)."""
        N = C.c_uint64()
        self._check(self._L.qram_dense_dim(self._h, C.byref(N)), "qram_dense_dim")
        js = sorted(jumps)
        fs = sorted(faults, key=lambda f: f[0])
        ja = np.array([q | (lev << 16) | (s << 24) for s, q, lev in js] or [0], dtype=np.uint32)
        fa = np.array([q | (s << 16) | ((a | (b << 2)) << 24) for s, q, a, b in fs] or [0], dtype=np.uint32)
        psi = np.zeros(2 * N.value)
        self._check(self._L.qram_dense_forced(self._h, _ptr(ja, C.c_uint32), len(js), _ptr(fa, C.c_uint32), len(fs),
                                              _ptr(psi, C.c_double), N.value), "qram_dense_forced")
        return psi[0::2] + 1j * psi[1::2]

    def sample_depol(self, seed, traj0, ntraj, cap=None):
        """Depolarizing faults: (counts [ntraj], entries site | slice << 16 |
        type << 24 concatenated in trajectory order)."""
        cnt = np.zeros(ntraj, dtype=np.uint32)
        self._check(self._L.qram_sample_depol(self._h, seed, traj0, ntraj, _ptr(cnt, C.c_uint32), None, 0),
                    "qram_sample_depol")
        tot = int(cnt.sum())
        cap = tot if cap is None else cap
        dep = np.zeros(max(cap, 1), dtype=np.uint32)
        self._check(self._L.qram_sample_depol(self._h, seed, traj0, ntraj, _ptr(cnt, C.c_uint32),
                                              _ptr(dep, C.c_uint32), cap), "qram_sample_depol")
        return cnt, dep[:tot]

    def _check(self, st, what):
        if st:
            raise QramError(st, f"{what}: {self._L.qram_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.qram_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- entry points -------------------------------------------------
    def sample_faults(self, seed, traj0, ntraj, dump=False, dump_cap=None):
        w64 = (self.D + 63) // 64
        n_cand = np.zeros(ntraj, dtype=np.uint32)
        dig = np.zeros(ntraj, dtype=np.uint64)
        n_bad = np.zeros(ntraj, dtype=np.uint32)
        bits = np.zeros(ntraj * w64, dtype=np.uint64)
        cap = 0
        buf = None
        if dump:
            cap = dump_cap if dump_cap is not None else max(1, int(ntraj * (self.M * (self.T - 1) * self.gamma + 64 + 10 * np.sqrt(self.M * self.T * self.gamma + 1))))
            buf = np.zeros(cap, dtype=np.uint32)
        st = self._L.qram_sample_faults(
            self._h, seed, traj0, ntraj, _ptr(n_cand, C.c_uint32), _ptr(dig, C.c_uint64),
            _ptr(n_bad, C.c_uint32), _ptr(bits, C.c_uint64), _ptr(buf, C.c_uint32), cap)
        self._check(st, "qram_sample_faults")
        out = dict(n_cand=n_cand, digest=dig, n_bad=n_bad, bad_bits=bits.reshape(ntraj, w64))
        if dump:
            offs = np.concatenate([[0], np.cumsum(n_cand.astype(np.int64))])
            out["cand_L"] = [buf[offs[t]:offs[t + 1]].copy() for t in range(ntraj)]
        return out

    def _run(self, fn, seed, traj0, ntraj, stats):
        fid = np.zeros(ntraj, dtype=np.float64)
        st_arr = np.zeros(ntraj, dtype=STATS_DTYPE) if stats else None
        st = fn(self._h, seed, traj0, ntraj, _ptr(fid, C.c_double),
                None if st_arr is None else st_arr.ctypes.data_as(C.c_void_p))
        self._check(st, fn.__name__)
        return (fid, st_arr) if stats else fid

    def run_full(self, seed, traj0, ntraj, stats=True):
        return self._run(self._L.qram_run_full, seed, traj0, ntraj, stats)

    def run_pruned(self, seed, traj0, ntraj, stats=True):
        return self._run(self._L.qram_run_pruned, seed, traj0, ntraj, stats)

    def run_plain(self, seed, traj0, ntraj, stats=True):
        return self._run(self._L.qram_run_plain, seed, traj0, ntraj, stats)

    def _run_async(self, fn, seed, traj0, ntraj, d_fid, d_st, stream):
        """d_fid: device tensor of ntraj float64; d_st: device uint8 tensor of
        ntraj*32 bytes or None; stream: torch.cuda.Stream, raw handle or None."""
        if hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        st = fn(self._h, seed, traj0, ntraj, C.c_void_p(d_fid.data_ptr()),
                None if d_st is None else C.c_void_p(d_st.data_ptr()),
                None if stream is None else C.c_void_p(int(stream)))
        self._check(st, fn.__name__)

    def run_full_async(self, seed, traj0, ntraj, d_fid, d_st=None, stream=None):
        self._run_async(self._L.qram_run_full_async, seed, traj0, ntraj, d_fid, d_st, stream)

    def run_pruned_async(self, seed, traj0, ntraj, d_fid, d_st=None, stream=None):
        self._run_async(self._L.qram_run_pruned_async, seed, traj0, ntraj, d_fid, d_st, stream)

    def run_plain_async(self, seed, traj0, ntraj, d_fid, d_st=None, stream=None):
        self._run_async(self._L.qram_run_plain_async, seed, traj0, ntraj, d_fid, d_st, stream)

    def run_pruned_async_noalloc(self, seed, traj0, ntraj, d_fid, d_st=None, stream=None):
        """As run_pruned_async, with the work buffers in the library's static
        per-device scratch array (no device allocation in the call)."""
        self._run_async(self._L.qram_run_pruned_async_noalloc, seed, traj0, ntraj, d_fid, d_st, stream)

    def run_forced(self, mode, cand_L, u_aux, u_fin):
        L = np.ascontiguousarray(cand_L, dtype=np.uint32)
        ua = np.ascontiguousarray(u_aux, dtype=np.float64)
        if len(ua) < self.T:
            raise ValueError("u_aux needs T entries (index = slice)")
        fid = C.c_double()
        st_arr = np.zeros(1, dtype=STATS_DTYPE)
        st = self._L.qram_run_forced(self._h, mode, _ptr(L, C.c_uint32) if len(L) else None, len(L),
                                     _ptr(ua, C.c_double), float(u_fin), C.byref(fid),
                                     st_arr.ctypes.data_as(C.c_void_p))
        self._check(st, "qram_run_forced")
        return fid.value, st_arr[0]

    def export_state(self, mode, seed=0, traj=0, cand_L=None, u_aux=None, u_fin=-1.0, jcap=4096):
        """qram_export_state: the final pre-measurement components of one
        trajectory (sampled, or forced when u_aux is given) and its jump log.
        Returns dict(fid, st, records [ncomp, 3 + lmax] uint32, amp (plain
        mode: complex amplitude of each record), jlog uint32 entries, njl)."""
        K2 = self.K2
        lmax = 2 * self.n + self.k if self.enc == 1 else 4 * self.n + self.k
        ncomp = self.D * K2
        comp = np.zeros(ncomp * (3 + lmax), dtype=np.uint32)
        amp = np.zeros(2 * ncomp)
        jl = np.zeros(max(jcap, 1), dtype=np.uint32)
        njl = C.c_uint32()
        fid = C.c_double()
        st_arr = np.zeros(1, dtype=STATS_DTYPE)
        L = ua = None
        if u_aux is not None:
            ua = np.ascontiguousarray(u_aux, dtype=np.float64)
            if len(ua) < self.T:
                raise ValueError("u_aux needs T entries (index = slice)")
            L = np.ascontiguousarray(cand_L if cand_L is not None else [], dtype=np.uint32)
        st = self._L.qram_export_state(
            self._h, mode, seed, traj, _ptr(L, C.c_uint32) if L is not None and len(L) else None,
            0 if L is None else len(L), _ptr(ua, C.c_double) if ua is not None else None, float(u_fin),
            _ptr(comp, C.c_uint32), ncomp, _ptr(amp, C.c_double), _ptr(jl, C.c_uint32), jcap, C.byref(njl),
            C.byref(fid),
            st_arr.ctypes.data_as(C.c_void_p))
        self._check(st, "qram_export_state")
        return dict(fid=fid.value, st=st_arr[0], records=comp.reshape(ncomp, 3 + lmax),
                    amp=amp[0::2] + 1j * amp[1::2], jlog=jl[:min(njl.value, jcap)].copy(), njl=njl.value)

    def run_jumplog(self, mode, seed, traj0, ntraj, jcap=64):
        """qram_run_jumplog: fidelities, statistics and every trajectory's
        jump log ([ntraj, jcap] uint32 entries, counts [ntraj])."""
        fid = np.zeros(ntraj)
        st_arr = np.zeros(ntraj, dtype=STATS_DTYPE)
        jl = np.zeros(max(ntraj * jcap, 1), dtype=np.uint32)
        njl = np.zeros(ntraj, dtype=np.uint32)
        st = self._L.qram_run_jumplog(self._h, mode, seed, traj0, ntraj, _ptr(fid, C.c_double),
                                      st_arr.ctypes.data_as(C.c_void_p), _ptr(jl, C.c_uint32), jcap,
                                      _ptr(njl, C.c_uint32))
        self._check(st, "qram_run_jumplog")
        return fid, st_arr, jl[:ntraj * jcap].reshape(ntraj, jcap), njl

    def set_launch(self, mode, slots_per_thread, schedule):
        self._check(self._L.qram_set_launch(self._h, mode, slots_per_thread, schedule), "qram_set_launch")

    def set_option(self, option, value):
        self._check(self._L.qram_set_option(self._h, option, int(value)), "qram_set_option")

    def get_launch(self, mode):
        t, s = C.c_int(), C.c_int()
        self._check(self._L.qram_get_launch(self._h, mode, C.byref(t), C.byref(s)), "qram_get_launch")
        return t.value, s.value

    def autotune(self, mode, seed, traj0, ntraj):
        ms = C.c_double()
        self._check(self._L.qram_autotune(self._h, mode, seed, traj0, ntraj, C.byref(ms)), "qram_autotune")
        return ms.value

    def set_timing(self, on=True):
        self._check(self._L.qram_set_timing(self._h, 1 if on else 0), "qram_set_timing")

    def stage_launches(self):
        """Evolution launches inside the batches timed since the last read."""
        n = C.c_uint32()
        self._check(self._L.qram_stage_launches(self._h, C.byref(n)), "qram_stage_launches")
        return n.value

    def stage_times(self):
        """(ms of sampling, classification, evolution summed over batches, batches)."""
        t = np.zeros(3)
        nb = C.c_uint32()
        self._check(self._L.qram_stage_times(self._h, _ptr(t, C.c_double), C.byref(nb)), "qram_stage_times")
        return t, nb.value

    def stage_buckets(self):
        """Per-bucket evolution timing of the current accumulation (read it
        before stage_times): list of dicts ms, launches, ntraj_last, emax."""
        ms = np.zeros(6)
        la, nt, em = (np.zeros(6, dtype=np.uint32) for _ in range(3))
        nb = C.c_int()
        self._check(self._L.qram_stage_buckets(self._h, _ptr(ms, C.c_double), _ptr(la, C.c_uint32),
                                               _ptr(nt, C.c_uint32), _ptr(em, C.c_uint32), C.byref(nb)),
                    "qram_stage_buckets")
        return [dict(ms=float(ms[i]), launches=int(la[i]), ntraj_last=int(nt[i]), emax=int(em[i]))
                for i in range(nb.value)]

    def footprint(self, mode, ntraj):
        """Device bytes held for runs of up to ntraj trajectories per call."""
        b = C.c_uint64()
        self._check(self._L.qram_footprint(self._h, mode, ntraj, C.byref(b)), "qram_footprint")
        return b.value

    def reserve(self, mode, ntraj):
        self._check(self._L.qram_reserve(self._h, mode, ntraj), "qram_reserve")

    def errors(self):
        """Raise if an asynchronous run flagged a capacity overflow."""
        self._check(self._L.qram_errors(self._h), "qram_errors")

    def last_kernel_ms(self):
        t = np.zeros(3)
        self._check(self._L.qram_last_kernel_ms(self._h, _ptr(t, C.c_double)), "qram_last_kernel_ms")
        return t


RESULT_STATE = {0: "waiting", 1: "running", 2: "done", 3: "failed"}


class QramServer:
    """Continuous-batching request server (``qram_server_*``) on the current
    HIP device: admission by device footprint, ``max_active`` overlapping
    execution slots, ``chunk`` trajectories per launch."""

    def __init__(self, hbm_budget_bytes, max_active=8, chunk=8192):
        L = load_library()
        h = C.c_void_p()
        st = L.qram_server_create(int(hbm_budget_bytes), int(max_active), int(chunk), C.byref(h))
        if st:
            raise QramError(st, "qram_server_create")
        self._h, self._L = h, L
        self._keep = {}

    def submit(self, n, k, enc, gamma, memory_bits, seed, shots, mode=QRAM_MODE_PRUNED, traj0=0):
        mem = np.ascontiguousarray(memory_bits, dtype=np.uint32)
        if mem.shape != (1 << n,):
            raise ValueError("memory_bits must hold 2^n words")
        req = QramRequest(n, k, enc, float(gamma), _ptr(mem, C.c_uint32), int(seed), int(traj0), int(shots), int(mode))
        t = C.c_uint64()
        st = self._L.qram_server_submit(self._h, C.byref(req), C.byref(t))
        if st:
            raise QramError(st, "qram_server_submit")
        return t.value

    @staticmethod
    def _as_dict(r):
        return dict(ticket=r.ticket, state=RESULT_STATE.get(r.state, r.state), status=STATUS.get(r.status, r.status),
                    mean=r.mean, sem=r.sem, shots=r.shots, footprint_bytes=r.footprint_bytes,
                    queue_ms=r.queue_ms, latency_ms=r.latency_ms)

    def poll(self, ticket):
        r = QramResult()
        st = self._L.qram_server_poll(self._h, ticket, C.byref(r))
        if st:
            raise QramError(st, "qram_server_poll")
        return self._as_dict(r)

    def wait(self, ticket, timeout_ms=-1.0):
        r = QramResult()
        st = self._L.qram_server_wait(self._h, ticket, float(timeout_ms), C.byref(r))
        if st:
            raise QramError(st, "qram_server_wait")
        return self._as_dict(r)

    def fidelities(self, ticket, shots):
        f = np.zeros(shots, dtype=np.float64)
        st = self._L.qram_server_fidelities(self._h, ticket, _ptr(f, C.c_double), shots)
        if st:
            raise QramError(st, "qram_server_fidelities")
        return f

    def release(self, ticket):
        st = self._L.qram_server_release(self._h, ticket)
        if st:
            raise QramError(st, "qram_server_release")

    def close(self):
        if getattr(self, "_h", None):
            self._L.qram_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
