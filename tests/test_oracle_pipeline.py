"""Whole-pipeline properties of the oracle (CPU only)."""
import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M


def _numpy_sphere_labels(res):
    """Brute-force labels of the sphere field, binary32 as specified: corner
    x = lo + g*h, then d2 = (dx^2 + dy^2) + dz^2 < r^2."""
    h = np.float32(1.0 / res)
    g = np.arange(res + 1, dtype=np.float32)
    x = np.float32(-0.5) + g * h
    c = np.array([0.03, -0.02, 0.01], np.float32)
    dx = (x - c[0])[None, None, :]
    dy = (x - c[1])[None, :, None]
    dz = (x - c[2])[:, None, None]
    d2 = (dx * dx + dy * dy) + dz * dz
    return d2 < np.float32(0.35) * np.float32(0.35)


@pytest.mark.parametrize("res,counts", [(8, (142, 284, 144)), (32, (2370, 4740, 2372))])
def test_sphere_counts_and_topology(oracle_mod, res, counts):
    f, g = I.sphere_case(res, 10)
    m = oracle_mod.Oracle(f, g).mesh()
    lab = _numpy_sphere_labels(res)
    assert np.array_equal(m["corner_label"].astype(bool), lab.reshape(-1))
    # independent count of crossing edges / faces with a crossing / cells
    ne = int(np.sum(lab[:, :, 1:] != lab[:, :, :-1]) + np.sum(lab[:, 1:, :] != lab[:, :-1, :]) +
             np.sum(lab[1:, :, :] != lab[:-1, :, :]))
    cube = np.stack([lab[dz:res + dz, dy:res + dy, dx:res + dx]
                     for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
    ncell = int(np.sum(cube.any(0) & ~cube.all(0)))
    assert (len(m["edge_id"]), len(m["pair_face"]), len(m["cell_id"])) == counts
    assert ne == counts[0] and ncell == counts[2]
    ok, why = M.is_closed_oriented_manifold(m["tris"], len(m["vert"]))
    assert ok, why
    assert M.euler_characteristic(m["tris"], len(m["vert"])) == 2
    assert len(m["vert"]) - len(m["tris"]) / 2 == 2
    # outward orientation: triangle normals point away from the centre
    w = -0.5 + m["vert"] * g.h
    P = w[m["tris"]]
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    assert np.all(np.sum(nrm * (P.mean(1) - [0.03, -0.02, 0.01]), 1) > 0)


def test_csg_small_closed_manifold(oracle_mod):
    f = I.csg_random_field(2)
    m = oracle_mod.Oracle(f, I.unit_grid(40)).mesh()
    ok, why = M.is_closed_oriented_manifold(m["tris"], len(m["vert"]))
    assert ok, why
    quads = int(np.sum(m["edge_case"] > 0))
    assert quads == len(m["edge_id"])  # the surface stays inside the domain
    assert len(m["tris"]) == 2 * quads + 2 * m["n_case3"]
    assert len(m["vert"]) == int(m["cell_npart"].sum()) + m["n_case3"]
    assert np.all((m["edge_t"] > 0) & (m["edge_t"] < 1))
    assert m["n_case3"] > 0 and m["n_flipped_faces"] >= 0
    # deterministic
    m2 = oracle_mod.Oracle(f, I.unit_grid(40)).mesh()
    assert np.array_equal(m["tris"], m2["tris"]) and np.array_equal(m["vert"], m2["vert"])


def test_mlp_small_pipeline(oracle_mod):
    f = I.mlp_field(3)
    m = oracle_mod.Oracle(f, I.unit_grid(16, 10), mlp_tie_eps=1e-5).mesh()
    assert len(m["edge_id"]) > 500
    ok, why = M.is_closed_oriented_manifold(m["tris"], len(m["vert"]))
    assert ok, why
    # single-element entry points agree with the full run
    o = oracle_mod.Oracle(f, I.unit_grid(16, 10), mlp_tie_eps=1e-5)
    rng = np.random.default_rng(0)
    for x in rng.choice(len(m["edge_id"]), 5, replace=False):
        t, ts = o.edge_point(m["edge_id"][x])
        assert t == m["edge_t"][x] and ts == m["edge_tie_step"][x]
    for x in rng.choice(len(m["pair_face"]), 5, replace=False):
        slot = m["pair_info"][x] & 15
        n, pf, info, tie = o.pair_point(m["pair_face"][x], slot)
        assert np.array_equal(pf, m["pair_pf"][x]) and info == m["pair_info"][x]
    for x in rng.choice(len(m["cell_id"]), 5, replace=False):
        n, v, pm, tie = o.cell_vertices(m["cell_id"][x])
        vb = m["cell_vbase"][x]
        assert n == m["cell_npart"][x] and pm == m["cell_partmap"][x]
        assert np.array_equal(v, m["vert"][vb:vb + n])


def test_oracle_struct_layouts_match_its_header(tmp_path):
    """The oracle's ctypes mirrors have the C header's sizes and offsets."""
    import ctypes as C
    import os
    import shutil
    import subprocess
    from oracle import oracle as O
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"orc_field": O._Field, "orc_params": O._Params, "orc_mesh": O._Mesh,
               "orc_trace": O._Trace}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "odc_oracle.h"',
             "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.split() for line in out.splitlines())
    for cname, cls in mirrors.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)
