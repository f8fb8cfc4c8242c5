"""Seeded synthetic inputs shared by the library's users, the tests and the
benchmark.  Holds none of the method's arithmetic: only classical memory
contents and request mixes, drawn with numpy's PCG64 generator."""
from __future__ import annotations

import numpy as np

QUTRIT, QUBIT = 0, 1

# Workloads measured by the benchmark and used as parity cases.  Memory is
# seeded Bernoulli(0.5) with mem_seed = 1000 + id; trajectories use
# seed = 880000 + id.
CONFIGS = {
    1: dict(name="qutrit n=3 k=1 gamma=1e-3", enc=QUTRIT, n=3, k=1, gammas=(1e-3,), ntraj=1000),
    2: dict(name="qubit n=6 k=1 gamma in {1e-4,1e-3,1e-2}", enc=QUBIT, n=6, k=1,
            gammas=(1e-4, 1e-3, 1e-2), ntraj=10000),
    3: dict(name="qubit and qutrit n=10 k=4 gamma=1e-3", encs=(QUBIT, QUTRIT), n=10, k=4,
            gammas=(1e-3,), ntraj=100000),
    5: dict(name="qutrit n=14 k=1 gamma=1e-2", enc=QUTRIT, n=14, k=1, gammas=(1e-2,), ntraj=100000),
}


def memory_words(n: int, k: int, mem_seed: int) -> np.ndarray:
    """2^n memory words of k Bernoulli(0.5) bits (bit b of word i = d_i^(b))."""
    rng = np.random.default_rng(mem_seed)
    bits = rng.integers(0, 2, size=(1 << n, k), dtype=np.uint32)
    return (bits << np.arange(k, dtype=np.uint32)[None, :]).sum(axis=1).astype(np.uint32)


def traj_seed(cfg_id: int) -> int:
    return 880000 + cfg_id


def mem_seed(cfg_id: int) -> int:
    return 1000 + cfg_id


def request_mix(nreq: int, master_seed: int = 4242):
    """Serving mix: n ~ U{4..12}, k ~ U{1,2,4}, encoding ~ U, gamma log-uniform
    in [1e-5, 1e-2], shots log-uniform in [1e3, 1e5]."""
    rng = np.random.default_rng(master_seed)
    out = []
    for r in range(nreq):
        n = int(rng.integers(4, 13))
        k = int(rng.choice([1, 2, 4]))
        enc = int(rng.integers(0, 2))
        gamma = float(10.0 ** rng.uniform(-5, -2))
        shots = int(round(10.0 ** rng.uniform(3, 5)))
        out.append(dict(id=r, n=n, k=k, enc=enc, gamma=gamma, shots=shots,
                        mem_seed=int(rng.integers(0, 2**31)), seed=int(rng.integers(0, 2**62))))
    return out
