"""Batched meshing: one launch per stage over many jobs, graph replay, and
the scratch-overflow rerun.  Each job's mesh must be bit-identical to the mesh
of the same field extracted alone."""
import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def odc():
    from paper_2409_13418_amd import odc as m
    return m


def _jobs():
    out = []
    for k, res in enumerate((24, 40, 16, 20, 33, 28)):
        seed = 4000 + k
        f = I.csg_random_field(seed) if k % 2 == 0 else I.mlp_field(seed)
        prec = 1 if k == 3 else 0
        out.append((f, I.unit_grid(res, 15), prec))
    f, g = I.sphere_case(32, 10)
    out.append((f, g, 0))
    return out


def _alone(odc, jobs):
    ctx = odc.Context(0)
    res = []
    for f, g, prec in jobs:
        r = ctx.extract(odc.DeviceField(f), odc.default_params(g, prec))
        res.append((r["vertices"].cpu().numpy().copy(), r["triangles"].cpu().numpy().copy(),
                    (r["n_active_cells"], r["n_search2d_queries"], r["n_guard_corners"])))
    ctx.close()
    return res


def test_batch_equals_alone(odc):
    jobs = _jobs()
    ref = _alone(odc, jobs)
    ctx = odc.Context(0)
    dfs = [odc.DeviceField(f) for f, _, _ in jobs]
    ps = [odc.default_params(g, prec) for _, g, prec in jobs]
    out = ctx.extract_batch(dfs, ps)
    for k, (v, t, nc) in enumerate(ref):
        # the per-job counters (cleared inside the pipeline) match too
        assert (out[k]["n_active_cells"], out[k]["n_search2d_queries"],
                out[k]["n_guard_corners"]) == nc, k
        assert np.array_equal(out[k]["vertices"].cpu().numpy(), v), k
        assert np.array_equal(out[k]["triangles"].cpu().numpy(), t), k
    ctx.close()


def test_graph_replay_matches(odc):
    jobs = _jobs()
    ref = _alone(odc, jobs)
    ctx = odc.Context(0)
    ctx.set_graph(True)
    dfs = [odc.DeviceField(f) for f, _, _ in jobs]
    ps = [odc.default_params(g, prec) for _, g, prec in jobs]
    for rep in range(3):
        out = ctx.extract_batch(dfs, ps)
        for k, (v, t, nc) in enumerate(ref):
            assert (out[k]["n_active_cells"], out[k]["n_search2d_queries"],
                    out[k]["n_guard_corners"]) == nc, (rep, k)
            assert np.array_equal(out[k]["vertices"].cpu().numpy(), v), (rep, k)
            assert np.array_equal(out[k]["triangles"].cpu().numpy(), t), (rep, k)
    # same structure, other fields: the captured graph serves them too
    jobs2 = [(I.csg_random_field(4100 + k) if k % 2 == 0 else I.mlp_field(4100 + k), g, prec)
             for k, (_, g, prec) in enumerate(jobs)]
    ref2 = _alone(odc, jobs2)
    out = ctx.extract_batch([odc.DeviceField(f) for f, _, _ in jobs2], ps)
    for k, (v, t, nc) in enumerate(ref2):
        assert np.array_equal(out[k]["triangles"].cpu().numpy(), t), k
    ctx.close()


def test_scratch_overflow_reruns(odc):
    """A surface far larger than the scratch estimate (a lattice of 512
    spheres at 64^3) overflows the active-set scratch; the sync reruns the
    extraction with room for it and the mesh is complete."""
    recs = []
    for i in range(8):
        for j in range(8):
            for k in range(8):
                c = (-0.4375 + 0.125 * i, -0.4375 + 0.125 * j, -0.4375 + 0.125 * k)
                recs.append(I.sphere_record(c, 0.047))
    f = I.csg_field(recs)
    g = I.unit_grid(64, 12)
    ctx = odc.Context(0)
    r = ctx.extract(odc.DeviceField(f), odc.default_params(g), want_local=True)
    assert r["n_active_edges"] > 12 * 64 * 64 + 4096
    lab = np.unpackbits(ctx.intermediate("labels").view(np.uint8), bitorder="little")
    lab = lab[:65 ** 3].reshape(65, 65, 65).astype(bool)
    ne = int(np.sum(lab[:, :, 1:] != lab[:, :, :-1]) + np.sum(lab[:, 1:] != lab[:, :-1]) +
             np.sum(lab[1:] != lab[:-1]))
    assert r["n_active_edges"] == ne
    ok, why = M.is_closed_oriented_manifold(r["triangles"].cpu().numpy(), r["n_vertices"])
    assert ok, why
    ctx.close()


def test_autotune_keeps_results(odc):
    f = I.csg_random_field(2)
    g = I.unit_grid(48)
    ctx = odc.Context(0)
    df = odc.DeviceField(f)
    p = odc.default_params(g)
    a = ctx.extract(df, p)
    ta = a["triangles"].cpu().numpy().copy()
    chosen = ctx.autotune(df, p)
    assert all(c > 0 for c in chosen)
    b = ctx.extract(df, p)
    assert np.array_equal(ta, b["triangles"].cpu().numpy())
    ctx.close()
