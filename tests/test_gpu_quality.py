"""Self-intersection counts on the GPU (odc_count_self_intersections) against
the oracle's brute force over all pairs: exact integer equality, whatever
the candidate grid's cell size."""
import numpy as np
import pytest

import odc_inputs as I
from gpu_common import gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_13418_amd import odc
    c = odc.Context(0)
    yield c
    c.close()


def _folded_sphere():
    v = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
    t = [[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]
    v = [np.array(p, float) for p in v]
    for _ in range(3):
        mid = {}
        nt = []

        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[k] = len(v) - 1
            return mid[k]
        for a, b, c in t:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nt += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        t = nt
    v = np.array(v)
    v[int(np.argmax(v[:, 2]))] = [0.05, 0.02, -1.4]
    return v, np.array(t)


def test_counts_match_brute_force(ctx, oracle_mod):
    meshes = {"folded sphere": _folded_sphere()}
    A = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]
    for name, B in {"pierce": [[0.2, 0.2, -1], [0.2, 0.2, 1], [0.3, 0.9, 0.5]],
                    "coplanar": [[0.2, 0.2, 0], [1.2, 0.2, 0], [0.2, 1.2, 0]],
                    "apart": [[2, 0, -1], [2, 1, 1], [3, 0, 0]]}.items():
        meshes[name] = (np.array(A + B, float), np.array([[0, 1, 2], [3, 4, 5]]))
    for prec, f, res in ((0, I.mlp_field(3), 24), (0, I.csg_random_field(2), 32)):
        for mode in (0, I.ABL_MDC_SPLIT, I.ABL_LINEAR_1D | I.ABL_MDC_SPLIT):
            g = I.unit_grid(res, 15)
            g.ablation = mode
            r, _ = gpu_run(f, g, precision=prec, ctx=ctx, want_local=False)
            meshes[f"{f.name}{res} ablation {mode}"] = (r["vertices"], r["triangles"])
    nonzero = 0
    for name, (v, t) in meshes.items():
        expect = oracle_mod.self_intersections(v, t)
        vv = np.asarray(v, np.float64)
        tt = np.asarray(t)
        edge = max(float(np.linalg.norm(vv[tt[:, a]] - vv[tt[:, (a + 1) % 3]], axis=1).max())
                   for a in range(3))
        ext = float(np.ptp(vv, axis=0).max())
        # from cubes smaller than the longest edge (a triangle spans several)
        # to one cube holding the whole mesh
        for cell in (edge / 2, edge * 2, ext):
            got = ctx.self_intersections(v, t, cell)
            assert got == expect, (name, cell, got, expect)
        nonzero += expect > 0
        print(f"{name}: {len(t)} triangles, {expect} intersecting pairs")
    assert nonzero >= 3


def test_bad_input_is_rejected(ctx):
    from paper_2409_13418_amd import odc
    v = np.zeros((3, 3), np.float32)
    with pytest.raises(odc.OdcError) as e:
        ctx.self_intersections(v, np.array([[0, 1, 3], [0, 1, 2]], np.int32), 1.0)
    assert e.value.status == odc.ERR_INVALID_ARG
    big = np.array([[0, 0, 0], [100, 0, 0], [0, 100, 0], [1, 1, 1]], np.float32)
    with pytest.raises(odc.OdcError) as e:
        ctx.self_intersections(big, np.array([[0, 1, 2], [0, 1, 3]], np.int32), 0.01)
    assert e.value.status == odc.ERR_INVALID_ARG
    with pytest.raises(odc.OdcError) as e:
        ctx.self_intersections(big, np.array([[0, 1, 2]], np.int32), 0.0)
    assert e.value.status == odc.ERR_INVALID_ARG
