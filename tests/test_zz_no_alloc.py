"""The no-allocation entry point (qram_run_pruned_async_noalloc) against
qram_run_pruned_async, through the C ABI: same fidelities (1e-12 relative)
and bit-identical integer statistics, on two calls in a row whose second
input is smaller, and on a second context of the other encoding."""
import ctypes

import numpy as np
import pytest

from paper_2609_34935_amd import STATS_DTYPE, QramContext, load_library
from paper_2609_34935_amd.inputs import memory_words

pytestmark = pytest.mark.gpu

INT_FIELDS = ("n_cand", "n_bad", "ref_addr", "n_explicit", "n_jumps", "first_jump_slice",
              "ref_survived", "q_ground", "flags")


def _run(ctx, fn, seed, traj0, ntraj):
    import torch
    d_fid = torch.full((ntraj,), -1.0, dtype=torch.float64, device="cuda")
    d_st = torch.zeros(ntraj * STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    fn(seed, traj0, ntraj, d_fid, d_st, stream)
    torch.cuda.synchronize()
    ctx.errors()
    return d_fid.cpu().numpy(), np.frombuffer(d_st.cpu().numpy().tobytes(), dtype=STATS_DTYPE)


def _compare(a, b):
    fa, sa = a
    fb, sb = b
    assert np.all(fa >= 0.0) and np.all(fb >= 0.0)
    err = np.abs(fa - fb) / np.maximum(np.abs(fb), 1e-3)
    assert err.max() <= 1e-12, err.max()
    for f in INT_FIELDS:
        assert np.array_equal(sa[f], sb[f]), f
    err = np.abs(sa["fid_pre"] - sb["fid_pre"]) / np.maximum(np.abs(sb["fid_pre"]), 1e-3)
    assert err.max() <= 1e-12


def test_noalloc_matches_pruned_async():
    import torch
    assert torch.cuda.is_available()
    L = load_library()
    assert hasattr(L, "qram_run_pruned_async_noalloc")
    # first call: the bench workload's qubit shape; second call on the same
    # context with a smaller input (fewer trajectories, another range)
    n, k, gamma = 10, 4, 1e-3
    with QramContext(n, k, 1, gamma, memory_words(n, k, 1003)) as ctx:
        print(f"noalloc qubit n={n} k={k} ntraj=3000", flush=True)
        a = _run(ctx, ctx.run_pruned_async_noalloc, 880003, 0, 3000)
        b = _run(ctx, ctx.run_pruned_async, 880003, 0, 3000)
        _compare(a, b)
        print("noalloc second call ntraj=700", flush=True)
        a = _run(ctx, ctx.run_pruned_async_noalloc, 880003, 5000, 700)
        b = _run(ctx, ctx.run_pruned_async, 880003, 5000, 700)
        _compare(a, b)
    # another context and encoding, smaller still: the array keeps the last
    # call's contents, which must not leak into this one
    n, k, gamma = 6, 2, 2e-2
    with QramContext(n, k, 0, gamma, memory_words(n, k, 1002)) as ctx:
        print(f"noalloc qutrit n={n} k={k} ntraj=257", flush=True)
        a = _run(ctx, ctx.run_pruned_async_noalloc, 7, 11, 257)
        b = _run(ctx, ctx.run_pruned_async, 7, 11, 257)
        _compare(a, b)


def test_no_alloc_refuses_plain_engine_contexts():
    """The no-allocation entry serves the trajectory kernel's contexts only;
    a depolarizing context is refused before anything is enqueued."""
    import torch
    assert torch.cuda.is_available()
    from paper_2609_34935_amd import QramError
    n, k = 4, 2
    with QramContext(n, k, 1, 0.01, memory_words(n, k, 3), eps=0.01) as ctx:
        d = torch.zeros(8, dtype=torch.float64, device="cuda")
        with pytest.raises(QramError):
            ctx.run_pruned_async_noalloc(1, 0, 8, d, None, torch.cuda.current_stream())
