"""Other network shapes than the benchmark's (depth 4, 6 Fourier bands): the
MLP kernels accept depth 1..8 and 0..7 bands, and the evaluators' layer-1
padding, layer loop and (in the bf16 corner pass) per-layer barriers follow
them.  Per shape: fp32 logits against binary64, the bf16-guarded mesh equal to
the fp32 mesh bit for bit, and corner labels equal to the oracle's away from
its near-ties."""
import numpy as np
import pytest

import odc_inputs as I
from gpu_common import gpu_run

pytestmark = pytest.mark.gpu

FP32_LOGIT_TOL = 4e-6   # half the near-tie band (1e-5) the labels are compared with
SHAPES = [(1, 0), (2, 3), (3, 1), (8, 7)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_13418_amd import odc
    c = odc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("depth,bands", SHAPES)
def test_network_shape(ctx, oracle_mod, depth, bands):
    from paper_2409_13418_amd import odc
    f = I.mlp_field(11 + depth, n_spheres=8, depth=depth, n_bands=bands)
    g = I.unit_grid(20, 12)
    rng = np.random.default_rng(depth)
    pts = rng.uniform(-0.5, 0.5, (2048, 3)).astype(np.float32)
    z = ctx.field_eval(odc.DeviceField(f), pts, odc.PREC_FP32).astype(np.float64)
    o = oracle_mod.Oracle(f, g, mlp_tie_eps=1e-5)
    ref = np.array([o.label_world(p)[2] for p in pts])
    err = np.abs(z - ref)
    print(f"depth {depth}, {bands} bands: fp32 logit error max {err.max():.2e}, "
          f"median |z| {np.median(np.abs(ref)):.2f}")
    assert err.max() < FP32_LOGIT_TOL, float(err.max())
    ra, _ = gpu_run(f, g, precision=0, ctx=ctx, want_local=False)
    rb, _ = gpu_run(f, g, precision=1, ctx=ctx, want_local=False)
    assert np.array_equal(ra["corner_label"], rb["corner_label"])
    assert np.array_equal(ra["triangles"], rb["triangles"])
    assert np.array_equal(ra["vertices"], rb["vertices"])
    m = o.mesh()
    clean = m["corner_tie"] == 0
    assert np.array_equal(rb["corner_label"][clean], m["corner_label"][clean])
    assert rb["n_active_cells"] > 0
