"""CPU-only checks of the C ABI library: it loads and exports every entry
point include/mknn.h declares, and its pure host helpers behave.  No call
here touches a GPU."""
import ctypes
import os
import re

import pytest

from paper_1412_6170_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "mknn.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"MKNN_API\s+[\w\s\*]+?\b(mknn_\w+)\s*\(", text)))


def test_header_declares_the_four_verbs_and_helpers():
    syms = declared_symbols()
    for verb in ("mknn_load_positions", "mknn_advance_tick", "mknn_query", "mknn_fetch",
                 "mknn_create", "mknn_destroy", "mknn_sync", "mknn_get_stats",
                 "mknn_last_error", "mknn_status_str", "mknn_result_size",
                 "mknn_result_device", "mknn_index_fetch", "mknn_default_leaf_capacity"):
        assert verb in syms


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    raw = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(raw, name), name
    assert lib is not None


def test_status_strings_and_leaf_rule():
    lib = binding.lib()
    for code, name in binding.STATUS.items():
        assert lib.mknn_status_str(code).decode() == name
    assert lib.mknn_status_str(-99).decode() == "MKNN_E_UNKNOWN"
    assert binding.default_leaf_capacity(8) == 192
    assert binding.default_leaf_capacity(32) == 384
    assert binding.default_leaf_capacity(128) == 1536
    assert binding.default_leaf_capacity(200) == 2048


def test_null_arguments_are_rejected_without_a_device():
    lib = binding.lib()
    assert lib.mknn_create(None, None) == -1
    out = ctypes.c_void_p(1)
    assert lib.mknn_create(None, ctypes.byref(out)) == -1 and out.value is None
    assert lib.mknn_destroy(None) == 0
    assert lib.mknn_advance_tick(None) == -1
    assert lib.mknn_sync(None) == -1
    ms = ctypes.c_float()
    assert lib.mknn_query_time(None, 0, 0, ctypes.byref(ms)) == -1
    assert lib.mknn_last_error(None).decode() == "null context"
    cfg = binding.Config()
    cfg.n_max, cfg.q_max, cfg.k_max = 10, 10, 0      # k_max out of range
    assert lib.mknn_create(ctypes.byref(cfg), ctypes.byref(out)) == -1
    cfg.k_max = binding.MKNN_K_LIMIT + 1
    assert lib.mknn_create(ctypes.byref(cfg), ctypes.byref(out)) == -1
    cfg.k_max, cfg.max_level = 8, 17
    assert lib.mknn_create(ctypes.byref(cfg), ctypes.byref(out)) == -1


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libmknn.so")
    with pytest.raises(ImportError):
        binding.lib()


def test_footprint_is_host_only_and_monotone():
    small = binding.footprint(n_max=10_000, k_max=8)
    big = binding.footprint(n_max=1_000_000, k_max=32, leaf_capacity=32)
    more_k = binding.footprint(n_max=1_000_000, k_max=64, leaf_capacity=32)
    assert 0 < small < big < more_k
    # results alone take 8 bytes per slot
    assert big > 1_000_000 * 32 * 8
    with pytest.raises(binding.MknnError):
        binding.footprint(n_max=0)


def test_footprint_at_the_largest_sizes():
    """n_max up to 2^31 - 1 and k_max = 128: sizes are 64-bit and grow
    linearly (no overflow); one past the limits is rejected (n_max, and k_max
    above MKNN_K_LIMIT = 1024)."""
    top = 2 ** 31 - 1
    a = binding.footprint(n_max=top // 2, q_max=top // 2, k_max=128, leaf_capacity=64)
    b = binding.footprint(n_max=top, q_max=top, k_max=128, leaf_capacity=64)
    assert b > 2 ** 40 and 1.9 < b / a < 2.1
    assert b > top * 128 * 8  # the result rows alone
    with pytest.raises(binding.MknnError):
        binding.footprint(n_max=2 ** 31, k_max=8)
    with pytest.raises(binding.MknnError):
        binding.footprint(n_max=1000, k_max=1025)
    assert binding.footprint(n_max=1000, k_max=1024) > binding.footprint(n_max=1000, k_max=128)


def test_readme_c_example_compiles(tmp_path):
    """The C usage example in README.md compiles against include/mknn.h."""
    import re
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "README.md")).read()
    block = re.search(r"```c\n(.*?)```", text, re.S).group(1)
    include = "\n".join(l for l in block.splitlines() if l.startswith("#include"))
    body = "\n".join(l for l in block.splitlines() if not l.startswith("#include"))
    src = tmp_path / "example.c"
    src.write_text(include + "\n#include <stdint.h>\n"
                   "void example(int64_t n, int ticks, float **x, float **y, int32_t *ids,\n"
                   "             float *d2, int32_t *counts)\n{\n" + body + "\n}\n")
    r = subprocess.run(["gcc", "-std=c11", "-fsyntax-only", "-Wall", "-Werror",
                        "-I", os.path.join(root, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_binding_structures_match_the_header(tmp_path):
    """The ctypes mirrors of mknn_config, mknn_stats and mknn_schedule have
    the header's field names, offsets and sizes (a C program compiled
    against include/mknn.h prints them)."""
    import subprocess
    header = open(os.path.join(ROOT, "include", "mknn.h")).read()
    pairs = (("mknn_config", binding.Config), ("mknn_stats", binding.Stats),
             ("mknn_schedule", binding.Schedule))
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mknn.h"', "int main(void) {"]
    for cname, cls in pairs:
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), header, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", " ", body, flags=re.S)
        names = re.findall(r"(\w+)\s*(?:\[\s*\d+\s*\])?\s*;", body)
        assert names == [f for f, _ in cls._fields_], cname
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in names:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in pairs:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)
