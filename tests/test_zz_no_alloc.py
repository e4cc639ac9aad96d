"""The allocation-free entry point (odc_mesh_extract_noalloc) against
odc_mesh_extract, through the C ABI.

Both run the same kernels; only where the job's scratch lives differs (one
fixed device array per GPU instead of context-owned buffers), so the meshes
and every intermediate must be identical bit for bit.  Two calls in a row
share the array, the second with a smaller grid, so stale contents of the
first must not leak into the second.  Sizes beyond the array are rejected
before anything runs.
"""
import ctypes as C

import numpy as np
import pytest

import odc_inputs as I

pytestmark = pytest.mark.gpu


def _extract(ctx, entry, field, grid, precision, **kw):
    from paper_2409_13418_amd import odc
    L = odc.load()
    df = odc.DeviceField(field)
    params = odc.default_params(grid, precision)
    for k, v in kw.items():
        setattr(params, k, v)
    n = grid.res
    out = odc.OutputBuffers(8 * n * n + 4096, 16 * n * n + 8192, want_local=True)
    print(f"{entry}: {field.name} res {n} precision {precision}", flush=True)
    ctx._check(getattr(L, entry)(ctx.h, C.byref(df.c), C.byref(params), C.byref(out.c)), entry)
    counts = odc.MeshCounts()
    ctx._check(L.odc_mesh_sync(ctx.h, C.byref(counts)), "odc_mesh_sync")
    c = counts.as_dict()
    v = out.views(c)
    r = {k: t.cpu().numpy() for k, t in v.items()}
    r["counts"] = c
    for name in ("labels", "edge_ids", "edge_t", "pairs", "pair_pf", "cell_ids", "cell_partmap",
                 "vertex_base", "edge_case"):
        r[name] = ctx.intermediate(name)
    return r


def _same(a, b, label):
    ca, cb = dict(a["counts"]), dict(b["counts"])
    assert ca == cb, label
    for k in ("vertices", "triangles", "vertices_local", "vertex_ref", "labels", "edge_ids",
              "edge_t", "pairs", "pair_pf", "cell_ids", "cell_partmap", "vertex_base",
              "edge_case"):
        assert np.array_equal(a[k], b[k]), (label, k)


@pytest.mark.parametrize("kind", ["mlp", "mlp_x3", "mlp_adaptive", "csg"])
def test_noalloc_equals_extract_twice(kind):
    from paper_2409_13418_amd import odc
    ctx = odc.Context(0)
    ctx.set_trace(False)
    try:
        if kind == "mlp":
            field, prec, sizes = I.mlp_field(3), odc.PREC_BF16_GUARDED, (96, 40)
        elif kind == "mlp_x3":  # the split weight terms live in the array too
            field, prec, sizes = I.mlp_field(5), odc.PREC_BF16_X3, (64, 33)
        elif kind == "mlp_adaptive":  # and the coarse bit sets and word list
            field, prec, sizes = I.mlp_field(6), odc.PREC_BF16_GUARDED, (96, 48)
        else:
            field, prec, sizes = I.csg_random_field(2), odc.PREC_FP32, (128, 61)
        for res in sizes:  # the second call is smaller and reuses the array
            g = I.unit_grid(res, 15)
            kw = ({"coarse_step": 4, "coarse_band": 1.5 * 20.0 * 3 ** 0.5 * 4 / res}
                  if kind == "mlp_adaptive" else {})
            ref = _extract(ctx, "odc_mesh_extract", field, g, prec, **kw)
            got = _extract(ctx, "odc_mesh_extract_noalloc", field, g, prec, **kw)
            assert ref["counts"]["n_triangles"] > 0
            _same(ref, got, f"{kind}{res}")
    finally:
        ctx.close()


def test_noalloc_rejects_what_does_not_fit():
    from paper_2409_13418_amd import odc
    L = odc.load()
    ctx = odc.Context(0)
    try:
        df = odc.DeviceField(I.csg_random_field(2))
        params = odc.default_params(I.unit_grid(512, 15))
        out = odc.OutputBuffers(16, 16)
        rc = L.odc_mesh_extract_noalloc(ctx.h, C.byref(df.c), C.byref(params), C.byref(out.c))
        assert rc == odc.ERR_OUT_OF_MEMORY
        assert b"fixed" in L.odc_last_error(ctx.h)
        # the context is still usable afterwards, on the fixed path too
        g = I.unit_grid(32, 15)
        a = _extract(ctx, "odc_mesh_extract", I.csg_random_field(2), g, 0)
        b = _extract(ctx, "odc_mesh_extract_noalloc", I.csg_random_field(2), g, 0)
        _same(a, b, "csg32 after a rejection")
    finally:
        ctx.close()
