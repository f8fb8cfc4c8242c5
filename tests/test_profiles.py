"""Host-side checks of the committed counter summaries (no GPU needed): the
source list whose hash a summary records is the one bench.py hashes before it
reports the summary's traffic, so a summary of unchanged kernels is used and
one of changed kernels is not."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_default_sources_match_bench():
    from paper_2609_34935_amd import profile_summary as ps
    bench = load_bench()
    default = [os.path.basename(f) for f in ps.KERNEL_SRCS]
    for key in ("evolve_qubit", "evolve_qutrit"):
        assert list(bench.COUNTERS[key][1]) == default, key


def test_summaries_name_their_sources():
    bench = load_bench()
    for key, (name, srcs) in bench.COUNTERS.items():
        prof = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert len(prof["kernel_sha256"]) == 64, key
        assert prof["hbm_bytes_per_launch"] > 0, key
        listed = prof.get("sources")
        if listed is not None:
            assert [os.path.basename(f) for f in listed] == list(srcs), key


def test_stale_summary_gives_no_traffic(tmp_path, monkeypatch):
    bench = load_bench()
    name, _ = bench.COUNTERS["plain_qubit"]
    prof = json.load(open(os.path.join(ROOT, "profiles", name)))
    prof["kernel_sha256"] = "0" * 64
    (tmp_path / name).write_text(json.dumps(prof))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.traffic_from_profile("plain_qubit") is None
