"""The C-ABI library loads and exports every symbol include/leiden.h declares,
and the binding's struct layouts match the header (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2410_15451_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "leiden.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(leiden_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == names


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "leiden.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(leiden_opts),'
                   ' sizeof(leiden_stats), offsetof(leiden_opts, stream), offsetof(leiden_stats, nnz),'
                   ' offsetof(leiden_opts, timed_kernel), offsetof(leiden_stats, kt_bytes),'
                   ' sizeof(leiden_tuning), offsetof(leiden_tuning, probe_ms)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    a, b, c, d, e, f, g, h = map(int, subprocess.check_output([str(exe)]).split())
    assert a == ctypes.sizeof(binding.LeidenOpts)
    assert b == ctypes.sizeof(binding.LeidenStats)
    assert c == binding.LeidenOpts.stream.offset
    assert d == binding.LeidenStats.nnz.offset
    assert e == binding.LeidenOpts.timed_kernel.offset
    assert f == binding.LeidenStats.kt_bytes.offset
    assert g == ctypes.sizeof(binding.LeidenTuning)
    assert h == binding.LeidenTuning.probe_ms.offset


def test_default_opts_without_gpu():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    o = binding.default_opts()
    assert (o.tau, o.tau_re_num, o.tau_re_den, o.tol_decline, o.max_iters, o.max_passes) == (1e-2, 3, 5, 10, 20, 10)
    assert (o.move_classes, o.refine_rounds, o.deterministic) == (4, 8, 1)
