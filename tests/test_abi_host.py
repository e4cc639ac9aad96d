"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/odc.h declares; defaults follow the paper."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "odc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(odc_[a-z_]+)\s*\(", src)))


def test_library_exports_declared_symbols():
    from paper_2409_13418_amd import odc
    L = odc.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(odc.EXPORTS) == set(names)


def test_defaults_follow_the_paper():
    from paper_2409_13418_amd import odc
    p = odc.Params()
    odc.load().odc_params_default(C.byref(p), 128)
    assert (p.res, p.iters_1d, p.lin1, p.bin1, p.lin2, p.bin2) == (128, 15, 4, 11, 3, 12)
    assert abs(p.range1 - 0.8) < 1e-7 and abs(p.range2 - math.sqrt(2) / 2) < 1e-7
    assert abs(p.qef_tau - 1e-2) < 1e-9 and p.fp64_cond == 1e6
    assert abs(p.guard_logit - 2 * math.atanh(0.02)) < 1e-7


def test_status_strings():
    from paper_2409_13418_amd import odc
    L = odc.load()
    assert L.odc_status_string(odc.OK) == b"ok"
    assert L.odc_status_string(odc.ERR_CAPACITY) == b"output capacity exceeded"
    assert L.odc_status_string(99) == b"unknown status"


def test_missing_library_fails_loudly(tmp_path):
    from paper_2409_13418_amd import odc
    with pytest.raises(odc.OdcError):
        odc._lib_backup = odc._lib
        try:
            odc._lib = None
            odc.load(str(tmp_path / "nope.so"))
        finally:
            odc._lib = odc._lib_backup


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and member
    offsets (a C program built against include/odc.h prints them)."""
    import shutil
    import subprocess
    from paper_2409_13418_amd import odc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"odc_field": odc.Field, "odc_params": odc.Params,
               "odc_mesh_buffers": odc.MeshBuffers, "odc_mesh_counts": odc.MeshCounts,
               "odc_server_config": odc.ServerConfig, "odc_request_result": odc.RequestResult,
               "odc_server_stats": odc.ServerStats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "odc.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cname, cls in mirrors.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 exits with a message
    (before anything touches a device)."""
    import json
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
