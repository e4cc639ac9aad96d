"""Numerics of the occupancy evaluators (odc_field_eval) against the oracle:
the fp32 matrix-core MLP against binary64, the bf16 one against fp32 and the
guard band, the CSG labels bit for bit."""
import numpy as np
import pytest

import odc_inputs as I

pytestmark = pytest.mark.gpu

FP32_LOGIT_TOL = 4e-6   # < MLP_TIE / 2 of the parity tests (near-tie band 1e-5)
GUARD = 2 * np.arctanh(0.02)


@pytest.fixture(scope="module")
def env():
    from paper_2409_13418_amd import odc
    ctx = odc.Context(0)
    yield odc, ctx
    ctx.close()


def _points(oracle_mod, field, n=4096, seed=0):
    rng = np.random.default_rng(seed)
    uni = rng.uniform(-0.5, 0.5, (n, 3))
    m = oracle_mod.Oracle(field, I.unit_grid(16, 10), mlp_tie_eps=1e-5).mesh()
    near = -0.5 + m["vert"] / 16.0
    near = near + rng.normal(0, 2e-3, near.shape)
    return np.concatenate([uni, near]).astype(np.float32)


def test_mlp_fp32_logits_match_binary64(env, oracle_mod):
    odc, ctx = env
    f = I.mlp_field(3)
    pts = _points(oracle_mod, f)
    z = ctx.field_eval(odc.DeviceField(f), pts, odc.PREC_FP32)
    o = oracle_mod.Oracle(f, I.unit_grid(16))
    ref = np.array([o.label_world(p)[2] for p in pts])
    err = np.abs(z.astype(np.float64) - ref)
    assert err.max() < FP32_LOGIT_TOL, float(err.max())
    # a wrong lane layout or K permutation would give O(1) errors
    assert np.median(np.abs(ref)) > 0.1


@pytest.mark.parametrize("shape", [(3, 6, 4), (5, 0, 1), (7, 7, 8)])
def test_mlp_x3_logits_match_binary64(env, oracle_mod, shape):
    """The split-bf16 evaluation (three bf16 terms per weight and activation,
    six products, binary32 accumulation) carries binary32's error: within the
    same bound as the fp32 matrix-core path, on the benchmark's network and
    on others (depth 1 and 8; no and 7 Fourier bands)."""
    odc, ctx = env
    seed, bands, depth = shape
    f = I.mlp_field(seed, n_bands=bands, depth=depth) if shape != (3, 6, 4) else I.mlp_field(3)
    pts = _points(oracle_mod, f, seed=seed)
    df = odc.DeviceField(f)
    z = ctx.field_eval(df, pts, odc.PREC_BF16_X3).astype(np.float64)
    z32 = ctx.field_eval(df, pts, odc.PREC_FP32).astype(np.float64)
    o = oracle_mod.Oracle(f, I.unit_grid(16))
    ref = np.array([o.label_world(p)[2] for p in pts])
    err, err32 = np.abs(z - ref), np.abs(z32 - ref)
    print(f"x3 logit error {err.max():.2e} (fp32 path {err32.max():.2e}), depth {depth}, "
          f"{bands} bands")
    assert err.max() < FP32_LOGIT_TOL, float(err.max())
    assert np.median(np.abs(ref)) > 0.1


def test_mlp_bf16_error_inside_guard_band(env, oracle_mod):
    """The bf16 logit stays well inside the guard band of the fp32 one, so a
    bf16 sign outside the band equals the fp32 sign."""
    odc, ctx = env
    f = I.mlp_field(3)
    pts = _points(oracle_mod, f, seed=1)
    df = odc.DeviceField(f)
    z32 = ctx.field_eval(df, pts, odc.PREC_FP32)
    z16 = ctx.field_eval(df, pts, odc.PREC_BF16_GUARDED)
    err = np.abs(z16 - z32)
    assert err.max() < GUARD / 2, float(err.max())
    out = np.abs(z16) >= GUARD
    assert np.all(np.sign(z16[out]) == np.sign(z32[out]))


def test_csg_labels_bit_exact(env, oracle_mod):
    odc, ctx = env
    f = I.csg_random_field(2)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-0.5, 0.5, (20000, 3)).astype(np.float32)
    z = ctx.field_eval(odc.DeviceField(f), pts)
    o = oracle_mod.Oracle(f, I.unit_grid(16))
    ref = np.array([o.label_world(p)[0] for p in pts])
    assert np.array_equal(z > 0, ref == 1)
