"""Batched meshing: one launch per stage over many jobs, graph replay, and
the scratch-overflow rerun.  Each job's mesh must be bit-identical to the mesh
of the same field extracted alone, and every job of a batch is checked
against the oracle replaying that job's decision traces: CSG jobs and small
MLP jobs element by element over the whole grid, large MLP jobs on seeded
samples (the binary64 network is too slow for every search of a 256^3 grid)."""
import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M
from gpu_common import (MLP_TIE, batch_results, check_replayed, check_sampled_replayed,
                        interior_edge_count, trace_of)

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
        prec = {3: 1, 5: 2}.get(k, 0)   # MLP jobs: fp32, bf16-guarded, split-bf16
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


def _check_job_against_oracle(O, f, g, r, label, sample_rng=None):
    if sample_rng is None:
        tr = trace_of(O, r)
        m = O.Oracle(f, g, mlp_tie_eps=MLP_TIE, trace=tr).mesh()
        dv = check_replayed(r, m, tr, g.res, label)
        return f"{label}: whole grid, {tr.adopted} near-ties followed, max vertex error {dv:.1e}"
    adopted = check_sampled_replayed(r, g, O, f, sample_rng, 600, 40, 20, 15, label)
    ok, why = M.is_closed_oriented_manifold(r["triangles"], r["n_vertices"])
    assert ok, (label, why)
    assert r["n_vertices"] == int(np.sum(r["cell_nf"] & 15)) + r["n_case3"], label
    assert len(r["triangles"]) == 2 * interior_edge_count(r["edge_ids"], g.res) + 2 * r["n_case3"]
    return f"{label}: samples, {adopted} near-ties followed"


def test_batch_jobs_against_oracle(odc, oracle_mod):
    """Every job of a mixed batch (CSG, MLP fp32, bf16-guarded and split-bf16,
    the sphere) against the oracle, whole grids."""
    jobs = _jobs()
    ctx = odc.Context(0)
    ctx.set_trace(True)
    dfs = [odc.DeviceField(f) for f, _, _ in jobs]
    ps = [odc.default_params(g, prec) for _, g, prec in jobs]
    out = ctx.extract_batch(dfs, ps, want_local=True)
    rs = batch_results(ctx, out, [g for _, g, _ in jobs])
    for k, ((f, g, prec), r) in enumerate(zip(jobs, rs)):
        print(_check_job_against_oracle(oracle_mod, f, g, r, f"job {k} {f.name} {g.res}^3"))
    ctx.close()


def test_batched_workload_slice_against_oracle(odc, oracle_mod):
    """Nine shapes of the 64-shape batched workload (seeds 4000.., CSG and MLP
    fields at 64, 96, 128, 192 and 256 cells per axis, MLP bf16-guarded) as
    one autotuned, graph-replayed batch.  CSG jobs against the whole oracle
    mesh; MLP jobs on seeded samples plus whole-mesh identities."""
    cfgs = I.batch_configs(64, 4000)
    pick = [0, 1, 2, 3, 4, 7, 10, 20, 39]
    jobs = [cfgs[i] for i in pick]
    assert {g.res for _, g in jobs} == {64, 96, 128, 192, 256}
    ctx = odc.Context(0)
    ctx.set_trace(True)
    dfs = [odc.DeviceField(f) for f, _ in jobs]
    ps = [odc.default_params(g, odc.PREC_BF16_GUARDED if f.kind == odc.FIELD_MLP else
                             odc.PREC_FP32) for f, g in jobs]
    big = max((k for k in range(len(jobs)) if jobs[k][0].kind == odc.FIELD_MLP),
              key=lambda k: jobs[k][1].res)
    ctx.autotune(dfs[big], ps[big])
    ctx.set_graph(True)
    first = ctx.extract_batch(dfs, ps, want_local=True)       # captured
    tris0 = [o["triangles"].cpu().numpy().copy() for o in first]
    out = ctx.extract_batch(dfs, ps, want_local=True)         # replayed
    rs = batch_results(ctx, out, [g for _, g in jobs])
    rng = np.random.default_rng(40)
    for k, ((f, g), r) in enumerate(zip(jobs, rs)):
        assert np.array_equal(r["triangles"], tris0[k]), k
        label = f"seed {4000 + pick[k]} {f.name} {g.res}^3"
        print(_check_job_against_oracle(oracle_mod, f, g, r, label,
                                        rng if f.kind == odc.FIELD_MLP else None), flush=True)
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


def test_autotune_cache_per_kind_and_resolution(odc):
    """The autotuner's result is cached for the tuned field's kind and
    resolution bucket; other keys fall back to the context default, and an
    explicit launch shape clears the cache.  A batch whose dominant job hits
    the cache meshes exactly as with the default shape."""
    ctx = odc.Context(0)
    f = I.mlp_field(3)
    g = I.unit_grid(48, 15)
    df = odc.DeviceField(f)
    p = odc.default_params(g, odc.PREC_BF16_GUARDED)
    ref = ctx.extract(df, p)["triangles"].cpu().numpy().copy()
    default, hit = ctx.launch_config(odc.FIELD_MLP, 48)
    assert not hit
    ctx.set_launch_config(*default)
    chosen = ctx.autotune(df, p)
    assert ctx.launch_config(odc.FIELD_MLP, 48) == (chosen, True)
    assert ctx.launch_config(odc.FIELD_MLP, 64) == (chosen, True)     # same bucket
    assert ctx.launch_config(odc.FIELD_MLP, 200)[1] is False
    assert ctx.launch_config(odc.FIELD_CSG, 48)[1] is False
    fc, gc = I.csg_random_field(2), I.unit_grid(40, 15)
    out = ctx.extract_batch([df, odc.DeviceField(fc)],
                            [p, odc.default_params(gc)])
    assert np.array_equal(out[0]["triangles"].cpu().numpy(), ref)
    ctx.set_launch_config(*default)
    assert ctx.launch_config(odc.FIELD_MLP, 48) == (default, False)
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
