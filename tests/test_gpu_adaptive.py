"""Adaptive corner evaluation (coarse_step > 1): the field is evaluated on a
coarse grid first and on fine corners only inside coarse cells that may hold
the surface.  Where the exactness condition of include/odc.h holds (for MLP
fields a logit band of at least L sqrt(3) S h), the labels, and so the whole
mesh, equal those of the full evaluation bit for bit; the oracle, which
evaluates every corner, checks the result as in the other parity tests.  A
planted feature smaller than a coarse cell shows what the band is for."""
import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M
from gpu_common import MLP_TIE, check_replayed, gpu_run, trace_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_13418_amd import odc
    c = odc.Context(0)
    yield c
    c.close()


def _band(res, step, lip=20.0, margin=1.5):
    """margin x L sqrt(3) S h for the benchmark fields' logit (slope ~sdf_gain)."""
    return float(margin * lip * np.sqrt(3.0) * step / res)


def _same_mesh(a, b, label):
    for k in ("corner_label", "edge_ids", "pairs", "cell_ids", "triangles", "vertices"):
        assert np.array_equal(a[k], b[k]), (label, k)


@pytest.mark.parametrize("res,step,prec", [(64, 4, 1), (64, 8, 0), (96, 4, 2), (256, 4, 1)])
def test_adaptive_mlp_equals_full(ctx, res, step, prec):
    f = I.mlp_field(3)
    g = I.unit_grid(res, 15)
    full, _ = gpu_run(f, g, precision=prec, ctx=ctx, trace=False, want_local=False)
    ad, _ = gpu_run(f, g, precision=prec, ctx=ctx, trace=False, want_local=False,
                    coarse_step=step, coarse_band=_band(res, step))
    _same_mesh(full, ad, f"mlp{res} S={step} prec={prec}")
    nc = (res + 1) ** 3
    assert full["n_corner_queries"] == nc
    frac = ad["n_corner_queries"] / nc
    print(f"mlp{res} S={step} prec={prec}: {ad['n_corner_queries']} corner queries "
          f"({frac:.3f} of {nc}), same mesh")
    coarse = (res // step + 1) ** 3
    assert coarse <= ad["n_corner_queries"] <= nc + coarse
    assert ad["n_queries"] - ad["n_corner_queries"] == full["n_queries"] - nc


@pytest.mark.parametrize("res,step", [(128, 2), (128, 8), (61, 61)])
def test_adaptive_csg_equals_full(ctx, res, step):
    """CSG coarse corners are marked by a signed-distance bound of the solid
    within a coarse cell's diagonal, which is exact by construction: the
    seeded field (thin slivers between its 72 primitives included) meshes as
    with the full evaluation, down to a single coarse cell."""
    f = I.csg_random_field(2)
    g = I.unit_grid(res, 15)
    full, _ = gpu_run(f, g, ctx=ctx, trace=False, want_local=False)
    ad, _ = gpu_run(f, g, ctx=ctx, trace=False, want_local=False, coarse_step=step)
    _same_mesh(full, ad, f"csg{res} S={step}")
    n = (res + 1) ** 3
    print(f"csg{res} S={step}: {ad['n_corner_queries']} corner queries of {n}")
    assert ad["n_corner_queries"] <= n + (res // step + 1) ** 3


def test_adaptive_mlp_replayed_against_oracle(ctx, oracle_mod):
    """The adaptive run against the oracle (which evaluates every corner),
    element by element with its decision traces replayed."""
    f = I.mlp_field(3)
    g = I.unit_grid(40, 15)
    r, _ = gpu_run(f, g, precision=1, ctx=ctx, coarse_step=4, coarse_band=_band(40, 4))
    tr = trace_of(oracle_mod, r)
    m = oracle_mod.Oracle(f, g, mlp_tie_eps=MLP_TIE, trace=tr).mesh()
    dv = check_replayed(r, m, tr, 40, "mlp40 adaptive")
    print(f"mlp40 S=4: {r['n_corner_queries']} corner queries, max vertex error {dv:.1e} cells")


def _small_sphere_field(res, step):
    """The sdf part only (out_scale 0): one sphere of radius 0.4 S h centred in
    a coarse cell (no coarse corner inside it), and one large sphere."""
    f = I.mlp_field(3)
    f.out_scale = 0.0
    S_h = step / res
    c = -0.5 + (res // step // 2 + 0.5) * S_h        # centre of a coarse cell
    f.spheres = np.array([[c, c, c, 0.4 * S_h], [-0.25, -0.25, -0.25, 0.15]], np.float32)
    return f


def test_band_catches_a_feature_inside_a_coarse_cell(ctx):
    """With no band the small sphere, which no coarse corner sees, is lost.
    The band of the exactness condition (20 sqrt(3) S h = 4.33; the sphere's
    logit at its cell's corners is -20 x 0.47 S h = -1.17) marks its cell and
    the mesh equals the full evaluation's."""
    res, step = 64, 8
    f = _small_sphere_field(res, step)
    g = I.unit_grid(res, 15)
    full, _ = gpu_run(f, g, precision=1, ctx=ctx, trace=False, want_local=False)
    lost, _ = gpu_run(f, g, precision=1, ctx=ctx, trace=False, want_local=False,
                      coarse_step=step, coarse_band=0.0)
    kept, _ = gpu_run(f, g, precision=1, ctx=ctx, trace=False, want_local=False,
                      coarse_step=step, coarse_band=4.5)
    assert lost["n_active_cells"] < full["n_active_cells"]
    _same_mesh(full, kept, "small sphere, band 4.5")
    ok, why = M.is_closed_oriented_manifold(lost["triangles"], lost["n_vertices"])
    assert ok, why  # what is left is still a closed manifold


def test_adaptive_job_in_a_batch(ctx):
    from paper_2409_13418_amd import odc
    fm, gm = I.mlp_field(5), I.unit_grid(48, 15)
    fc, gc = I.csg_random_field(4), I.unit_grid(40, 15)
    pm = odc.default_params(gm, odc.PREC_BF16_GUARDED)
    pm.coarse_step, pm.coarse_band = 4, _band(48, 4)
    pc = odc.default_params(gc)
    dfm, dfc = odc.DeviceField(fm), odc.DeviceField(fc)
    alone = [ctx.extract(dfm, pm)["triangles"].cpu().numpy().copy(),
             ctx.extract(dfc, pc)["triangles"].cpu().numpy().copy()]
    full = ctx.extract(dfm, odc.default_params(gm, odc.PREC_BF16_GUARDED))
    assert np.array_equal(full["triangles"].cpu().numpy(), alone[0])
    out = ctx.extract_batch([dfm, dfc], [pm, pc])
    for k in range(2):
        assert np.array_equal(out[k]["triangles"].cpu().numpy(), alone[k]), k
