"""Table 3's ablation baselines on the GPU against the oracle: Manifold Dual
Contouring's linear 1D points (Eq. 1), gradient normals (Eq. 2, by
forward-mode differentiation through the network on the matrix cores) and
the plain two-triangle split, alone and as the table's rows (MDC = all three,
+1D = gradient normals and plain split, +2D = plain split), and on an SDF
input (a field whose logit is minus a signed distance): ODC itself, linear
points on psi (mode 9) and the MDC row on psi (mode 15).

Tolerances, derived from the arithmetic:
  linear t      |dt| <= (|dpsi0| + |dpsi1|) / |psi0 - psi1| + 2^-24 with
                |dpsi| <= |dz| / 4 + 2^-24 and |dz| <= 2e-6, the binary32
                logit error the other MLP parity tests observe (|dpsi| <=
                |dz| + 2^-24 for SDF input, where psi is z itself)
  gradients     relative 1e-4 (binary32 forward mode through four 256-wide
                layers; observed ~1e-6), except at a near-switch of the
                gradient's formula: two spheres within 1e-5 of being the
                nearest, or a ReLU input within 1e-5 of 0 (binary32 may take
                the other branch there; both gradients are then valid)
  vertices      1e-5 cell widths, every vertex, whatever the QEF's eigen-gap
                (the kernel redoes small-gap decompositions in binary64)

The oracle replays the GPU's search decisions in staged mode: its 2D
searches start from the GPU's 1D points (linear points differ in the last
bits between binary32 and binary64, which would move the queries) and its
QEF takes the GPU's 1D points, 2D points and gradients, so each stage is
checked on its own: the gradients above against the oracle's, the 3D points
against the oracle's QEF of the same inputs.
"""
import math

import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M
from gpu_common import (check_replayed, compare_discrete, edge_origin, gpu_run, trace_of,
                        vertex_grid_coords, world32)

pytestmark = pytest.mark.gpu

MLP_TIE = 1e-5
DZ = 2e-6


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_13418_amd import odc
    c = odc.Context(0)
    yield c
    c.close()


def _psi(o, g, gp, mode):
    _, _, z = o.label_world(np.array(world32(g, gp), np.float32))
    return z if mode & I.ABL_SDF_INPUT else 0.5 * math.tanh(0.5 * z)


@pytest.mark.parametrize("field,mode", [("occ", 1), ("occ", 2), ("occ", 4), ("occ", 6),
                                        ("occ", 7), ("sdf", 0), ("sdf", 9), ("sdf", 15)])
def test_mlp_ablation_modes(ctx, oracle_mod, field, mode):
    # the SDF input's logit is the occupancy field's over 20: so are its
    # binary32 error and its tie margin
    scale = 1.0 if field == "occ" else 1.0 / 20
    f = I.mlp_field(3) if field == "occ" else I.sdf_mlp_field(3)
    g = I.unit_grid(24, 15)
    g.ablation = mode
    r, _ = gpu_run(f, g, precision=0, ctx=ctx)
    tr = trace_of(oracle_mod, r, staged=True)
    o = oracle_mod.Oracle(f, g, mlp_tie_eps=MLP_TIE * scale, trace=tr)
    m = o.mesh()
    assert tr.mismatched == 0 and tr.unmatched == 0, (tr.mismatched, tr.unmatched)
    assert compare_discrete(r, m) == []
    N = g.res
    et = r["edge_t"].astype(np.float64)
    if mode & I.ABL_LINEAR_1D:
        worst = 0.0
        for x, e in enumerate(m["edge_id"]):
            a, p = edge_origin(e, N)
            q = list(p)
            q[a] += 1
            s0, s1 = _psi(o, g, p, mode), _psi(o, g, q, mode)
            dpsi = DZ * scale if mode & I.ABL_SDF_INPUT else DZ / 4
            bound = 2 * (dpsi + 2.0 ** -24) / abs(s0 - s1) + 2.0 ** -24
            d = abs(et[x] - m["edge_t"][x])
            worst = max(worst, d / bound)
            assert d <= bound, (int(e), et[x], m["edge_t"][x], bound)
        print(f"{field} mode {mode}: linear 1D points within {worst:.2f} of their bound")
    else:
        assert np.array_equal(et, m["edge_t"])
    if mode & I.ABL_GRAD_NORMALS:
        eg = r["edge_grad"].astype(np.float64)
        assert eg.shape == (len(m["edge_id"]), 3)
        rel, near = [], []
        for x, e in enumerate(m["edge_id"]):
            a, p = edge_origin(e, N)
            gp = [np.float32(v) for v in p]
            gp[a] = np.float32(np.float32(p[a]) + np.float32(r["edge_t"][x]))
            _, go, mg = o.logit_grad([float(v) for v in world32(g, gp)], with_margin=True)
            rel.append(np.linalg.norm(eg[x] - go) / np.linalg.norm(go))
            near.append(min(mg) < 1e-5)
        rel, near = np.array(rel), np.array(near)
        print(f"{field} mode {mode}: gradient relative error max {rel[~near].max():.2e} "
              f"({int(near.sum())} near a switch, max there {rel.max():.2e}), "
              f"median {np.median(rel):.2e}")
        assert np.all(rel[~near] <= 1e-4)
        assert near.sum() <= 0.03 * len(near)
    else:
        assert len(r["edge_grad"]) == 0
        # the 2D searches from the GPU's own 1D points: bit-identical
        assert np.array_equal(r["pair_pf"], m["pair_pf"])
    nvp = int(m["cell_npart"].sum())
    vg = vertex_grid_coords(r, N)[:nvp]
    dv = np.max(np.abs(vg - m["vert"][:nvp]), axis=1)
    print(f"{field} mode {mode}: {tr.adopted} near-tie decisions followed; max vertex error "
          f"{dv.max():.2e} cells over {nvp}; {r['n_fp64_cells']} binary64 QEF cells")
    assert np.all(dv <= 1e-5), float(dv.max())
    if mode & I.ABL_MDC_SPLIT:
        assert set(np.unique(r["edge_case"])) <= {0, 1} and r["n_case3"] == 0
        assert np.array_equal(r["edge_case"], m["edge_case"])
        assert np.array_equal(r["triangles"], m["tris"])
    ok, why = M.is_closed_oriented_manifold(r["triangles"], r["n_vertices"])
    assert ok, why


def test_csg_linear_and_split(ctx, oracle_mod):
    f = I.csg_random_field(2)
    g = I.unit_grid(40, 15)
    g.ablation = I.ABL_LINEAR_1D | I.ABL_MDC_SPLIT
    r, _ = gpu_run(f, g, ctx=ctx)
    tr = trace_of(oracle_mod, r)
    m = oracle_mod.Oracle(f, g, trace=tr).mesh()
    assert tr.mismatched == 0 and tr.adopted == 0
    assert compare_discrete(r, m) == []
    assert np.all(r["edge_t"] == 0.5) and np.array_equal(r["edge_t"].astype(np.float64), m["edge_t"])
    assert np.array_equal(r["pair_pf"], m["pair_pf"])
    assert np.array_equal(r["triangles"], m["tris"])
    nvp = int(m["cell_npart"].sum())
    dv = np.max(np.abs(vertex_grid_coords(r, g.res)[:nvp] - m["vert"][:nvp]), axis=1)
    gap = m["vert_gap"][:nvp]
    w = int(np.argmax(dv))
    print(f"csg linear+split: max vertex error {dv.max():.2e} (eigen-gap there {gap[w]:.2e}; "
          f"{int(np.sum(gap < 0.1))} vertices with gap < 0.1); {r['n_fp64_cells']} binary64 "
          f"QEF cells")
    assert np.all(dv <= 1e-5), float(dv.max())


def test_ablation_bits_are_checked(ctx):
    from paper_2409_13418_amd import odc
    g = I.unit_grid(16)
    g.ablation = I.ABL_GRAD_NORMALS
    with pytest.raises(odc.OdcError) as e:
        ctx.extract(odc.DeviceField(I.csg_random_field(2)), odc.default_params(g))
    assert e.value.status == odc.ERR_UNSUPPORTED
    # an unknown bit, and SDF input without the linear points
    for bits in (16, I.ABL_SDF_INPUT, I.ABL_SDF_INPUT | I.ABL_MDC_SPLIT):
        p = odc.default_params(I.unit_grid(16))
        p.ablation = bits
        with pytest.raises(odc.OdcError) as e:
            ctx.extract(odc.DeviceField(I.sdf_mlp_field(3)), p)
        assert e.value.status == odc.ERR_INVALID_ARG, bits


@pytest.mark.parametrize("kind", ["mlp", "csg"])
def test_clamped_vertices(ctx, oracle_mod, kind):
    f = I.mlp_field(3) if kind == "mlp" else I.csg_random_field(2)
    g = I.unit_grid(24 if kind == "mlp" else 32, 15)
    g.clamp = 1
    r, _ = gpu_run(f, g, precision=0, ctx=ctx)
    tr = trace_of(oracle_mod, r)
    m = oracle_mod.Oracle(f, g, mlp_tie_eps=MLP_TIE, trace=tr).mesh()
    nvp = int(m["cell_npart"].sum())
    vl = r["vertices_local"][:nvp]
    assert np.all((vl >= 0.0) & (vl <= 1.0))
    check_replayed(r, m, tr, g.res, f"{kind} clamped")
    ok, why = M.is_closed_oriented_manifold(r["triangles"], r["n_vertices"])
    assert ok, why
