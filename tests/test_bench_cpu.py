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


@pytest.mark.parametrize("workload", ["clustered_1m", "uniform_10k"])
def test_traffic_only_for_matching_sources(workload):
    m = bench.MEASURED_TRAFFIC
    got = bench.measured_traffic(workload, m["leaf_capacity"], m.get("max_level", 16))
    if workload != m["workload"] or m["digest"] != bench.query_source_digest():
        assert got is None
    else:
        assert got == m["fetch_bytes"] + m["write_bytes"]


def test_traffic_needs_the_same_maximum_level():
    m = bench.MEASURED_TRAFFIC
    other = 16 if m.get("max_level", 16) != 16 else 12
    assert bench.measured_traffic(m["workload"], m["leaf_capacity"], other) is None


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


def test_valu_issue_fraction():
    m = bench.MEASURED_TRAFFIC
    ms = 0.5
    got = bench.valu_issue(m["workload"], m["leaf_capacity"], m.get("max_level", 16), ms)
    if m["digest"] != bench.query_source_digest():
        assert got is None
        return
    assert got["bound"] == "alu"
    assert abs(got["frac"] - m["valu_insts"] * 64 / (ms * 1e-3) / (256 * 4 * 16 * 2.4e9)) < 1e-12
    assert bench.valu_issue("uniform_10k", m["leaf_capacity"], 16, ms) is None


def test_roofline_names_the_closer_roof():
    m = bench.MEASURED_TRAFFIC
    L = m.get("max_level", 16)
    r = bench.roofline_entry(m["workload"], m["leaf_capacity"], L, 32, 0.44, 272_000_000)
    assert abs(r["hbm_frac" if r["bound"] == "alu" else "frac"]
               - 272_000_000 / 0.44e-3 / 8e12) < 1e-9
    v = bench.valu_issue(m["workload"], m["leaf_capacity"], L, 0.44)
    if v is None:
        assert r["bound"] == "hbm"
    else:
        assert r["bound"] == ("alu" if v["frac"] > r.get("hbm_frac", r["frac"]) else "hbm")
    # A configuration without a stored instruction count falls back to HBM.
    r2 = bench.roofline_entry("uniform_10k", 32, 16, 8, 0.06, 1_000_000)
    assert r2["bound"] == "hbm" and r2["unit"] == "GB/s"


def test_cpu_model_reads_the_host():
    cpu = bench.cpu_model()
    assert cpu["logical_cpus"] >= 1 and isinstance(cpu["model"], str)
    assert bench.host_threads() >= 1
