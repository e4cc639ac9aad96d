"""C-ABI behaviour on the GPU: argument validation, capacity protocol,
repeatability."""
import ctypes as C

import numpy as np
import pytest

import odc_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_2409_13418_amd import odc
    ctx = odc.Context(0)
    yield odc, ctx
    ctx.close()


def _call(odc, ctx, df, params, vcap, tcap, vbuf=None, tbuf=None):
    b = odc.MeshBuffers()
    b.vertices = vbuf.data_ptr() if vbuf is not None else None
    b.cap_vertices = vcap
    b.triangles = tbuf.data_ptr() if tbuf is not None else None
    b.cap_triangles = tcap
    return odc.load().odc_mesh_extract(ctx.h, C.byref(df.c), C.byref(params), C.byref(b))


def test_invalid_arguments(env):
    odc, ctx = env
    import torch
    f, g = I.sphere_case(16, 10)
    df = odc.DeviceField(f)
    v = torch.zeros(300, device="cuda")
    t = torch.zeros(300, dtype=torch.int32, device="cuda")
    for field, value in (("res", 0), ("res", 513), ("iters_1d", 0), ("iters_1d", 24),
                         ("lin1", 0), ("range1", 0.0), ("precision", 7)):
        p = odc.default_params(g)
        setattr(p, field, value)
        assert _call(odc, ctx, df, p, 100, 100, v, t) == odc.ERR_INVALID_ARG, field
    p = odc.default_params(g)
    assert _call(odc, ctx, df, p, 100, 100, None, t) == odc.ERR_INVALID_ARG
    bad = odc.DeviceField(I.csg_field([I.sphere_record((0, 0, 0), 0.3)]))
    bad.c.n_prims = 0
    assert _call(odc, ctx, bad, p, 100, 100, v, t) == odc.ERR_INVALID_ARG
    mlp = I.mlp_field(3)
    dm = odc.DeviceField(mlp)
    dm.c.width = 128
    assert _call(odc, ctx, dm, p, 100, 100, v, t) == odc.ERR_UNSUPPORTED


def test_capacity_protocol(env):
    """Too-small outputs: CAPACITY with the sizes needed and nothing written
    past the capacities."""
    odc, ctx = env
    import torch
    f, g = I.sphere_case(32, 10)
    df = odc.DeviceField(f)
    p = odc.default_params(g)
    vbuf = torch.full((3 * 200 + 30,), -7.0, device="cuda")
    tbuf = torch.full((3 * 100 + 30,), -7, dtype=torch.int32, device="cuda")
    assert _call(odc, ctx, df, p, 200, 100, vbuf, tbuf) == odc.OK
    c = odc.MeshCounts()
    assert odc.load().odc_mesh_sync(ctx.h, C.byref(c)) == odc.ERR_CAPACITY
    assert c.n_vertices == 2372 and c.n_triangles == 4740
    assert torch.all(vbuf[600:] == -7.0) and torch.all(tbuf[300:] == -7)
    out = ctx.extract(df, p)
    assert out["n_vertices"] == 2372 and out["n_triangles"] == 4740


def test_repeatable_and_reusable(env):
    """Two extractions of one field are bit-identical; a context serves
    fields of different kinds and sizes in turn."""
    odc, ctx = env
    f = I.csg_random_field(2)
    g = I.unit_grid(48)
    df = odc.DeviceField(f)
    a = ctx.extract(df, odc.default_params(g))
    va, ta = a["vertices"].cpu().numpy().copy(), a["triangles"].cpu().numpy().copy()
    ctx.extract(odc.DeviceField(I.mlp_field(3)), odc.default_params(I.unit_grid(12)))
    b = ctx.extract(df, odc.default_params(g))
    assert np.array_equal(va, b["vertices"].cpu().numpy())
    assert np.array_equal(ta, b["triangles"].cpu().numpy())


def test_stage_timing(env):
    odc, ctx = env
    f, g = I.sphere_case(32, 10)
    ctx.set_timing(True)
    ctx.extract(odc.DeviceField(f), odc.default_params(g))
    st = ctx.stage_times()
    ctx.set_timing(False)
    assert set(st) == set(odc.STAGES) and all(v >= 0 for v in st.values())


def test_allocation_failure_is_reported(env):
    """Device allocations refused by the library's failure injection: the
    extraction (first or second scratch buffer) and a server arena report
    OUT_OF_MEMORY with a message, and the context works again afterwards."""
    odc, _ = env
    L = odc.load()
    f, g = I.csg_random_field(2), I.unit_grid(32, 15)
    ctx = odc.Context(0)  # fresh: no job scratch allocated yet
    df = odc.DeviceField(f)
    p = odc.default_params(g)
    try:
        for allowed in (0, 1):
            L.odc_inject_alloc_failures(allowed)
            with pytest.raises(odc.OdcError) as e:
                ctx.extract(df, p)
            assert e.value.status == odc.ERR_OUT_OF_MEMORY, allowed
            assert "failed" in str(e.value) or "refused" in str(e.value)
        L.odc_inject_alloc_failures(0)
        with pytest.raises(odc.OdcError) as e:
            odc.Server(ctx, 1 << 26)
        assert e.value.status == odc.ERR_OUT_OF_MEMORY
    finally:
        L.odc_inject_alloc_failures(-1)
    r = ctx.extract(df, p)
    assert r["n_triangles"] > 0
    ctx.close()
