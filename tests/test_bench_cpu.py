"""CPU: bench.py's host logic -- every global name its functions load is
defined (a mode whose handler was lost fails here, not on the GPU), the
multi-GPU refusal, and the byte accounting of the roofline entry."""
import builtins
import dis
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _global_loads(code):
    for ins in dis.get_instructions(code):
        if ins.opname == "LOAD_GLOBAL":
            yield ins.argval
    for c in code.co_consts:
        if isinstance(c, types.CodeType):
            yield from _global_loads(c)


def test_every_global_name_is_defined():
    missing = set()
    for name, obj in vars(bench).items():
        if isinstance(obj, types.FunctionType) and obj.__module__ == "bench":
            for g in _global_loads(obj.__code__):
                if not hasattr(bench, g) and not hasattr(builtins, g):
                    missing.add((name, g))
    assert not missing, sorted(missing)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_query_kernel_bytes():
    # 12 B per object read once, 8 k + 4 B per query written.
    assert bench.query_kernel_bytes(1_000_000, 1_000_000, 32_000_000) == 12_000_000 + 260_000_000


def _entries(digest):
    return [dict(digest=digest, workload="clustered_1m", leaf_capacity=48, max_level=14,
                 fetch_bytes=10, write_bytes=20, valu_insts=1_000_000),
            dict(digest="stale-digest", workload="clustered_1m", leaf_capacity=64, max_level=12,
                 fetch_bytes=1, write_bytes=2, valu_insts=5)]


def test_traffic_only_for_matching_sources_and_schedule(monkeypatch):
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", _entries(bench.query_source_digest()))
    assert bench.measured_traffic("clustered_1m", 48, 14) == 30
    assert bench.measured_traffic("clustered_1m", 48, 12) is None        # other level
    assert bench.measured_traffic("clustered_1m", 64, 12) is None        # code changed since
    assert bench.measured_traffic("uniform_10k", 48, 14) is None         # other workload
    assert bench.measured_traffic("clustered_1m", 48, 14, "wave") is None  # other flavour


def test_stored_traffic_entries_are_well_formed():
    for m in bench.MEASURED_TRAFFIC:
        assert len(m["digest"]) == 16
        assert m["fetch_bytes"] > 0 and m["write_bytes"] > 0 and m["valu_insts"] > 0
        assert m["leaf_capacity"] >= 1 and 1 <= m["max_level"] <= 16


def test_digest_ignores_comments_not_code():
    here = {f: open(os.path.join(ROOT, "paper_1412_6170_amd", "csrc", f)).read()
            for f in bench.DIGEST_FILES}
    base = bench.query_source_digest(here.get)
    commented = dict(here)
    commented["query.hip"] = "// a new comment\n/* and a block\n comment */\n" + here["query.hip"]
    assert bench.query_source_digest(commented.get) == base
    changed = dict(here)
    changed["query.hpp"] = here["query.hpp"].replace("kQueryClasses = 5", "kQueryClasses = 6")
    assert changed["query.hpp"] != here["query.hpp"]
    assert bench.query_source_digest(changed.get) != base


def test_digest_covers_only_the_flavours_sources():
    files = set(bench.DIGEST_COMMON) | set(bench.DIGEST_FLAVOUR.values())
    here = {f: open(os.path.join(ROOT, "paper_1412_6170_amd", "csrc", f)).read() for f in files}
    lane, group = (bench.query_source_digest(here.get, sweep=s) for s in ("lane", "group"))
    assert lane != group
    edited = dict(here)
    edited["query_group.hip"] = here["query_group.hip"] + "\nint extra_symbol;\n"
    assert bench.query_source_digest(edited.get, sweep="lane") == lane
    assert bench.query_source_digest(edited.get, sweep="group") != group
    edited = dict(here)
    edited["query_device.hpp"] = here["query_device.hpp"] + "\nint extra_symbol;\n"
    assert bench.query_source_digest(edited.get, sweep="lane") != lane
    assert bench.query_source_digest(edited.get, sweep="group") != group


def test_valu_issue_fraction(monkeypatch):
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", _entries(bench.query_source_digest()))
    ms = 0.5
    got = bench.valu_issue("clustered_1m", 48, 14, ms)
    assert got["bound"] == "alu"
    assert abs(got["frac"] - 1_000_000 * 64 / (ms * 1e-3) / (256 * 4 * 16 * 2.4e9)) < 1e-12
    assert bench.valu_issue("clustered_1m", 64, 12, ms) is None
    assert bench.valu_issue("uniform_10k", 48, 14, ms) is None


def test_roofline_names_the_closer_roof(monkeypatch):
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", _entries(bench.query_source_digest()))
    # A large instruction count: the VALU roof is the closer one.
    monkeypatch.setitem(bench.MEASURED_TRAFFIC[0], "valu_insts", 190_000_000)
    r = bench.roofline_entry("clustered_1m", 48, 14, 32, 0.44, 272_000_000)
    assert r["bound"] == "alu" and r["traffic"] == 30
    assert abs(r["hbm_frac"] - 272_000_000 / 0.44e-3 / 8e12) < 1e-9
    # A small one: the HBM roof is.
    monkeypatch.setitem(bench.MEASURED_TRAFFIC[0], "valu_insts", 10)
    r = bench.roofline_entry("clustered_1m", 48, 14, 32, 0.44, 272_000_000)
    assert r["bound"] == "hbm" and abs(r["frac"] - 272_000_000 / 0.44e-3 / 8e12) < 1e-9
    # A configuration without a stored instruction count falls back to HBM.
    r2 = bench.roofline_entry("uniform_10k", 32, 16, 8, 0.06, 1_000_000)
    assert r2["bound"] == "hbm" and r2["unit"] == "GB/s" and r2["traffic"] is None


def test_cpu_model_reads_the_host():
    cpu = bench.cpu_model()
    assert cpu["logical_cpus"] >= 1 and isinstance(cpu["model"], str)
    assert bench.host_threads() >= 1
