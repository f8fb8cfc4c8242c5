"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/qram.h declares, and rejects bad arguments with the
documented status before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qram.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qram_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_2609_34935_amd import qram
    assert declared_functions() == sorted(qram.EXPORTS)


def test_library_exports_every_symbol():
    from paper_2609_34935_amd import load_library
    L = load_library()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_stats_layout():
    from paper_2609_34935_amd import STATS_DTYPE
    assert STATS_DTYPE.itemsize == 32
    assert STATS_DTYPE.fields["fid_pre"][1] == 24


@pytest.mark.parametrize("n,k,enc,gamma,status", [
    (0, 1, 1, 0.1, "QRAM_E_RANGE"), (16, 1, 1, 0.1, "QRAM_E_RANGE"), (15, 1, 0, 0.1, "QRAM_E_RANGE"),
    (3, 4, 1, 0.1, "QRAM_E_RANGE"), (3, 9, 1, 0.1, "QRAM_E_RANGE"), (3, 1, 2, 0.1, "QRAM_E_INVAL"),
    (3, 1, 1, 1.0, "QRAM_E_INVAL"), (3, 1, 1, -0.1, "QRAM_E_INVAL"), (3, 1, 1, float("nan"), "QRAM_E_INVAL"),
    (10, 4, 1, 0.5, "QRAM_E_RANGE")])
def test_create_rejects_bad_arguments(n, k, enc, gamma, status):
    from paper_2609_34935_amd import qram
    L = qram.load_library()
    mem = np.zeros(max(1 << min(n, 15), 1), dtype=np.uint32)
    h = ctypes.c_void_p()
    st = L.qram_create(n, k, enc, gamma, mem.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(h))
    assert qram.STATUS[st] == status
    assert h.value is None
    assert L.qram_last_error(None)


def test_null_arguments():
    from paper_2609_34935_amd import qram
    L = qram.load_library()
    h = ctypes.c_void_p()
    assert qram.STATUS[L.qram_create(3, 1, 1, 0.1, None, ctypes.byref(h))] == "QRAM_E_INVAL"
    L.qram_destroy(None)  # NULL is allowed
    m = ctypes.c_double()
    assert qram.STATUS[L.qram_fidelity(None, 3, ctypes.byref(m), None)] == "QRAM_E_INVAL"


def test_fidelity_helper():
    from paper_2609_34935_amd import qram_fidelity
    f = np.array([1.0, 0.5, 0.0, 0.25])
    m, s = qram_fidelity(f)
    assert abs(m - f.mean()) < 1e-15
    assert abs(s - f.std(ddof=1) / 2) < 1e-15


def test_package_fails_loudly_without_library(tmp_path):
    from paper_2609_34935_amd import qram
    saved = qram._lib
    qram._lib = None
    try:
        with pytest.raises(ImportError):
            qram.load_library(str(tmp_path / "missing.so"))
    finally:
        qram._lib = saved


def test_memory_generator_deterministic():
    from paper_2609_34935_amd.inputs import memory_words
    a = memory_words(10, 4, 1003)
    assert a.shape == (1024,) and a.max() < 16
    assert np.array_equal(a, memory_words(10, 4, 1003))
    assert abs(((a[:, None] >> np.arange(4)) & 1).mean() - 0.5) < 0.03


def test_option_constants_match_header():
    """The binding's option numbers are the header's, and a null context is
    rejected without touching the device."""
    from paper_2609_34935_amd import qram
    text = open(HEADER).read()
    opts = dict((k, int(v)) for k, v in re.findall(r"\b(QRAM_OPT_[A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert opts == {"QRAM_OPT_TIER2_GLOBAL": 1, "QRAM_OPT_GRAPH": 2, "QRAM_OPT_SUBTREE_MARKING": 3}
    for name, value in opts.items():
        assert getattr(qram, name) == value
    L = qram.load_library()
    assert qram.STATUS[L.qram_set_option(None, opts["QRAM_OPT_SUBTREE_MARKING"], 1)] == "QRAM_E_INVAL"
