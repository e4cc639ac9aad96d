"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The oracle (gcc, -fsanitize=address,undefined, no recovery) through the
  full pipeline on the three kinds of field, the replay trace (own
  decisions, staged, labels given and topology only), every single-element
  entry point and the building blocks.
* The host side of libodc (hipcc with the sanitizers on the host pass only;
  device code is built as usual but never launched) through what runs
  without a device: argument checks on valid and invalid inputs of every
  kind, scratch planning at every resolution, status strings, NULL handles,
  and context creation.

Each runs in a child process with the sanitizer runtime preloaded; any
report ends it with a non-zero status.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_SCRIPT = r'''
import numpy as np, odc_inputs as I
from oracle import oracle as O
m = O.Oracle(*I.sphere_case(12, 10)).mesh()
assert len(m["tris"]) > 0
for f, g, eps in ((I.csg_random_field(2), I.unit_grid(16, 15), 1e-4),
                  (I.mlp_field(3), I.unit_grid(8, 12), 1e-5)):
    o = O.Oracle(f, g, mlp_tie_eps=eps)
    m = o.mesh()
    words = np.packbits(m["corner_label"], bitorder="little")
    words = np.pad(words, (0, (-len(words)) % 4)).view(np.uint32)
    rec = (m["pair_face"].astype(np.int64) * 2 + (m["pair_info"] & 1)).astype(np.int32)
    for staged in (False, True):
        tr = O.Trace(label_words=words, edge_ids=m["edge_id"], edge_bits=m["edge_bits"],
                     edge_t=m["edge_t"].astype(np.float32), pair_rec=rec,
                     pair_bits=m["pair_bits"], pair_pf=m["pair_pf"], staged=staged)
        m2 = O.Oracle(f, g, mlp_tie_eps=eps, trace=tr).mesh()
        assert tr.mismatched == 0 and np.array_equal(m2["tris"], m["tris"])
        o2 = O.Oracle(f, g, mlp_tie_eps=eps, trace=tr)
        o2.corner_label(1, 2, 3)
        o2.edge_point(int(m["edge_id"][0]))
        o2.pair_point(int(m["pair_face"][0]), 0)
        o2.cell_vertices(int(m["cell_id"][0]))
    tr = O.Trace(label_words=words, labels_given=True)
    O.Oracle(f, g, trace=tr, topology_only=True).mesh()
    o.line_binary(int(m["pair_face"][0]), np.array([0.5, 0.5]), np.array([1.0, 0.0]), 1, 0.8, 4, 11)
    if f.kind == 1:
        o.logit_grad([0.1, 0.2, 0.3], with_margin=True)
        g2 = I.unit_grid(8, 12); g2.ablation = 7
        O.Oracle(f, g2, mlp_tie_eps=eps).mesh()
    O.self_intersections(m["vert"].astype(np.float32), m["tris"][:200])
O.cube_partitions(0x69, 3)
O.qef_solve(np.eye(3), np.zeros((3, 3)))
O.ic_case(np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float), [0.5, 0.5, -1], [0.5, 0.5, 1])
print("oracle clean")
'''

HOST_SCRIPT = r'''
import ctypes as C, sys
import odc_inputs as I
sys.path.insert(0, "paper_2409_13418_amd")
L = C.CDLL(sys.argv[1])
import odc  # the binding's structs only (its loader is not used)
for s in range(-1, 9):
    L.odc_status_string.restype = C.c_char_p
    assert L.odc_status_string(s)
L.odc_last_error.restype = C.c_char_p
assert L.odc_last_error(None)
fake = C.c_void_p(0x1000)   # never dereferenced on the host

def field(kind_, **kw):
    f = odc.Field()
    f.kind = kind_
    if kind_ == 0:
        f.prims, f.n_prims = fake, 3
    else:
        f.weights, f.spheres, f.n_spheres = fake, fake, 32
        f.in_dim, f.width, f.depth, f.n_bands = 39, 256, 4, 6
        f.sdf_gain, f.out_scale = 20.0, 0.3
    for k, v in kw.items():
        setattr(f, k, v)
    return f

def params(res, **kw):
    p = odc.Params()
    L.odc_params_default(C.byref(p), res)
    p.guard_logit = 0.04
    for k, v in kw.items():
        setattr(p, k, v)
    return p

b, fits = C.c_int64(), C.c_int32()
sizes = {}
for res in list(range(1, 70)) + [96, 128, 129, 192, 255, 256, 257, 384, 511, 512]:
    for kind in (0, 1):
        for prec in (0, 1, 2):
            rc = L.odc_plan_scratch(C.byref(field(kind)), C.byref(params(res, precision=prec)),
                                    C.byref(b), C.byref(fits))
            assert rc == 0 and b.value > 0, (res, kind, rc)
            sizes[(res, kind, prec)] = (b.value, fits.value)
assert sizes[(256, 1, 1)][1] == 1 and sizes[(512, 0, 0)][1] == 0
assert sizes[(256, 1, 1)][0] < sizes[(512, 1, 1)][0]
bad_params = [dict(res=0), dict(res=513), dict(iters_1d=0), dict(iters_1d=24), dict(lin1=0),
              dict(bin1=-1), dict(lin2=65), dict(bin2=31), dict(range1=0.0), dict(range2=-1.0),
              dict(qef_tau=1.0), dict(qef_tau=-0.1), dict(precision=3), dict(guard_logit=0.0),
              dict(guard_logit=float("nan")), dict(fp64_cond=0.0), dict(fp64_cond=float("nan")),
              dict(ablation=16), dict(ablation=8), dict(clamp_vertices=2), dict(size=0.0),
              dict(size=float("inf")), dict(coarse_step=3), dict(coarse_step=-1),
              dict(coarse_step=65), dict(res=64, coarse_step=128), dict(coarse_band=-1.0),
              dict(coarse_band=float("nan"))]
for kw in bad_params:
    p = params(kw.get("res", 32), **{k: v for k, v in kw.items() if k != "res"})
    rc = L.odc_plan_scratch(C.byref(field(0)), C.byref(p), C.byref(b), None)
    assert rc == 1, (kw, rc)
for kw, want in ((dict(kind=7), 1), (dict(n_prims=0), 1), (dict(prims=None), 1)):
    assert L.odc_plan_scratch(C.byref(field(0, **kw)), C.byref(params(16)), C.byref(b), None) == want, kw
for kw, want in ((dict(width=128), 5), (dict(depth=9), 5), (dict(depth=0), 5), (dict(in_dim=40), 5),
                 (dict(n_bands=7, in_dim=45), 0), (dict(n_bands=8, in_dim=51), 5),
                 (dict(weights=None), 1), (dict(spheres=None), 1), (dict(n_spheres=0), 1)):
    assert L.odc_plan_scratch(C.byref(field(1, **kw)), C.byref(params(16)), C.byref(b), None) == want, kw
b2 = C.c_int64()
assert L.odc_plan_scratch(C.byref(field(1)), C.byref(params(256, coarse_step=4, coarse_band=1.0)),
                          C.byref(b2), None) == 0
assert L.odc_plan_scratch(C.byref(field(1)), C.byref(params(256)), C.byref(b), None) == 0
assert b2.value > b.value  # the coarse bit sets
p = params(16, ablation=2)
assert L.odc_plan_scratch(C.byref(field(0)), C.byref(p), C.byref(b), None) == 5
assert L.odc_plan_scratch(None, C.byref(params(16)), C.byref(b), None) == 1
assert L.odc_plan_scratch(C.byref(field(0)), C.byref(params(16)), None, None) == 1
for fn, args in (("odc_mesh_extract", (None, None, None, None)), ("odc_mesh_sync", (None, None)),
                 ("odc_mesh_extract_noalloc", (None, None, None, None)),
                 ("odc_get_intermediate", (None, 0, None, 0, None)),
                 ("odc_server_create", (None, None, None)), ("odc_context_set_trace", (None, 1)),
                 ("odc_field_eval", (None, None, 0, None, 0, None))):
    assert getattr(L, fn)(*args) == 1, fn
L.odc_context_destroy(None)
L.odc_server_destroy(None)
h = C.c_void_p()
rc = L.odc_context_create(0, None, C.byref(h))
assert rc in (0, 1, 4), rc    # no device here: INVALID_ARG
if rc == 0:
    L.odc_context_destroy(h)
print("host clean")
'''


def _run(script, env_extra, args=()):
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = os.pathsep.join([ROOT, env.get("PYTHONPATH", "")])
    p = subprocess.run([sys.executable, "-c", script, *args], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path, oracle_mod):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = oracle_mod.build(out=str(tmp_path / "liboracle_san.so"),
                           extra=("-g", "-fsanitize=address,undefined",
                                  "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"))
    out = _run(ORACLE_SCRIPT, {"LD_PRELOAD": asan, "ODC_ORACLE_LIB": lib,
                               "ASAN_OPTIONS": "detect_leaks=0", "OMP_NUM_THREADS": "4"})
    assert "oracle clean" in out


def test_host_library_under_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not shutil.which(hipcc) and not os.path.exists(hipcc) or not rt:
        pytest.skip("no hipcc or clang AddressSanitizer runtime")
    csrc = os.path.join(ROOT, "paper_2409_13418_amd", "csrc")
    lib = str(tmp_path / "libodc_san.so")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-pthread", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-o", lib] + [os.path.join(csrc, f) for f in ("odc_api.hip", "odc_server.hip",
                                                         "odc_kernels.hip", "odc_quality.hip")]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    out = _run(HOST_SCRIPT, {"LD_PRELOAD": rt[-1], "ASAN_OPTIONS": "detect_leaks=0"}, (lib,))
    assert "host clean" in out
