"""Parity at the workloads' full sizes, in the benchmark's launch shape.

* CSG field at 128^3 (48 boxes + 16 spheres - 8 boxes, seed 2): the oracle
  finishes the whole grid in about a second, so everything is compared
  element by element, exactly as in the small parity tests.
* MLP field at 256^3, bf16-guarded, default context (the configuration the
  benchmark times): the oracle evaluates the network in binary64, which is
  too slow for every search of the grid, so seeded samples of corners,
  crossing edges, face pairs and active cells are recomputed one by one by
  the oracle replaying the GPU's decision traces, at the small tests' bar;
  the properties that hold at any size are checked on the whole mesh.  The
  fp32 path on the same grid must give the same mesh bit for bit, and the
  split-bf16 searches the same topology, their vertices sampled against the
  replaying oracle.
"""
import os

import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M
from gpu_common import (MLP_TIE, check_replayed, check_sampled_replayed, compare_discrete,
                        gpu_run, trace_of)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_13418_amd import odc
    c = odc.Context(0)
    yield c
    c.close()


def test_csg128_full_parity(ctx, oracle_mod):
    f = I.csg_random_field(2)
    g = I.unit_grid(128, 15)
    r, _ = gpu_run(f, g, ctx=ctx)
    tr = trace_of(oracle_mod, r)
    m = oracle_mod.Oracle(f, g, trace=tr).mesh()
    dvmax = check_replayed(r, m, tr, 128, "csg128")
    assert tr.adopted == 0
    ok, why = M.is_closed_oriented_manifold(r["triangles"], r["n_vertices"])
    assert ok, why
    # Chamfer distance to the oracle's mesh: vertices within 1e-5 h bound it by 1e-10 h^2
    vo = np.asarray(g.lo) + m["vert"] * g.h
    ch = M.chamfer_h2(r["vertices"], r["triangles"], vo, m["tris"], g.h, n=20000)
    assert ch <= 1e-10, ch
    print(f"csg128: {len(m['cell_id'])} cells, {len(m['tris'])} triangles, "
          f"max vertex error {dvmax:.2e} cells, Chamfer vs oracle {ch:.2e} h^2")


@pytest.fixture(scope="module")
def mlp256(ctx):
    f = I.mlp_field(3)
    g = I.unit_grid(256, 15)
    r, _ = gpu_run(f, g, precision=1, ctx=ctx)
    return f, g, r


GOLDEN_LABELS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "mlp256_labels.npz")


def test_mlp256_whole_grid_topology(mlp256, oracle_mod):
    """Every one of the 16,974,593 corner labels of the benchmark's grid
    against the oracle's (tests/golden/mlp256_labels.npz, written by
    make_mlp256_labels.py from the binary64 network): equal except at the
    oracle's near-ties, where either label is a correct binary32 evaluation.
    Then the oracle's topology from those labels (crossing edges, face
    pairs, manifold flips, active cells, partitions, vertex numbering)
    against the GPU's whole active sets, bit for bit."""
    f, g, r = mlp256
    gold = np.load(GOLDEN_LABELS)
    assert int(gold["res"]) == g.res and int(gold["seed"]) == 3
    nc = (g.res + 1) ** 3
    lab = np.unpackbits(gold["label_bits"], bitorder="little")[:nc]
    diff = np.nonzero(r["corner_label"] != lab)[0]
    ties = gold["tie_corners"]
    assert np.all(np.isin(diff, ties)), diff[~np.isin(diff, ties)][:10]
    tr = oracle_mod.Trace(label_words=r["labels"], labels_given=True)
    m = oracle_mod.Oracle(f, g, trace=tr, topology_only=True).mesh()
    assert compare_discrete(r, m) == []
    assert len(m["edge_id"]) == r["n_active_edges"] and len(m["cell_id"]) == r["n_active_cells"]
    print(f"mlp256 whole grid: {nc} corners ({len(ties)} oracle near-ties, {len(diff)} taken the "
          f"other way), {len(m['edge_id'])} crossing edges, {len(m['pair_face'])} pairs, "
          f"{len(m['cell_id'])} cells, {m['n_flipped_faces']} flipped faces: all equal")


def test_mlp256_sampled_replayed(mlp256, oracle_mod):
    """Seeded samples in the benchmark's configuration: 3,000 corners (half at
    the ends of crossing edges), 150 crossing edges, 60 pairs and 40 cells,
    each recomputed by the oracle replaying the GPU's traces."""
    f, g, r = mlp256
    rng = np.random.default_rng(11)
    adopted = check_sampled_replayed(r, g, oracle_mod, f, rng, 2000, 150, 60, 40, "mlp256")
    print(f"mlp256: sampled elements at the small tests' bar; {adopted} near-tie "
          f"decisions followed")


def test_mlp256_mesh_properties(mlp256):
    f, g, r = mlp256
    tris = r["triangles"]
    ok, why = M.is_closed_oriented_manifold(tris, r["n_vertices"])
    assert ok, why
    npart = int(np.sum(r["cell_nf"] & 15))
    assert r["n_vertices"] == npart + r["n_case3"]
    # one quad per crossing edge with four in-grid cells, split into two
    # triangles, or four around the edge's 1D point (case 3)
    N, n1 = g.res, g.res + 1
    e = r["edge_ids"].astype(np.int64)
    ea = N * n1 * n1
    a, loc = e // ea, e % ea
    interior = np.ones(len(e), bool)
    for ax in range(3):
        sel = a == ax
        dims = [n1, n1, n1]
        dims[ax] = N
        ijk = [loc[sel] % dims[0], (loc[sel] // dims[0]) % dims[1], loc[sel] // (dims[0] * dims[1])]
        inner = np.ones(int(sel.sum()), bool)
        for o in range(3):
            if o != ax:
                inner &= (ijk[o] > 0) & (ijk[o] < N)
        interior[sel] = inner
    assert len(tris) == 2 * int(interior.sum()) + 2 * r["n_case3"]
    # no clamp to the cell (unclamped QEF points); report how many leave it
    vl = r["vertices_local"][:npart]
    assert np.all(np.isfinite(vl))
    outside = int(np.sum(np.any((vl < 0) | (vl > 1), axis=1)))
    print(f"mlp256: {npart} partition vertices, {outside} outside their cell")


def test_mlp256_bf16_equals_fp32(ctx, mlp256):
    f, g, rb = mlp256
    ra, _ = gpu_run(f, g, precision=0, ctx=ctx, want_local=False)
    assert np.array_equal(ra["corner_label"], rb["corner_label"])
    assert np.array_equal(ra["triangles"], rb["triangles"])
    assert np.array_equal(ra["vertices"], rb["vertices"])
    assert rb["n_guard_corners"] > 0


def test_mlp256_x3_same_topology_and_sampled_replayed(ctx, mlp256, oracle_mod):
    """Split-bf16 searches at 256^3: every corner sign, crossing edge, pair,
    cell, partition map and the vertex numbering equal the guarded path's
    (whose mesh is the fp32 path's); the searches' samples against the
    oracle replaying the split-bf16 decisions, at the small tests' bar; the
    mesh is a closed oriented manifold."""
    f, g, rb = mlp256
    rx, _ = gpu_run(f, g, precision=2, ctx=ctx)
    for k in ("corner_label", "edge_ids", "pairs", "cell_ids", "cell_partmap", "cell_nf"):
        assert np.array_equal(rx[k], rb[k]), k
    npart = int(np.sum(rb["cell_nf"] & 15))
    assert np.array_equal(rx["vertex_ref"][:npart], rb["vertex_ref"][:npart])
    rng = np.random.default_rng(17)
    adopted = check_sampled_replayed(rx, g, oracle_mod, f, rng, 0, 150, 60, 40, "mlp256 x3")
    ok, why = M.is_closed_oriented_manifold(rx["triangles"], rx["n_vertices"])
    assert ok, why
    d = np.max(np.abs(rx["vertices_local"][:npart].astype(np.float64) -
                      rb["vertices_local"][:npart]), axis=1)
    print(f"mlp256 x3: topology equal to the guarded path's; {adopted} near-tie decisions "
          f"followed; vertex difference to the guarded path's: median {np.median(d):.1e}, "
          f"max {d.max():.1e} cells ({int(np.sum(d > 1e-5))} of {npart} above 1e-5)")


def test_sdf256_bf16_equals_fp32_and_sampled_labels(ctx, oracle_mod):
    """The SDF input at 256^3 (the benchmark's zero set, logit 20 times
    flatter): the guard band then holds far more corners, and the guarded
    bf16 path must still give the fp32 path's mesh bit for bit; sampled
    corner labels next to the surface match the oracle (tie band scaled by
    the field's 1/20)."""
    f = I.sdf_mlp_field(3)
    g = I.unit_grid(256, 15)
    rb, _ = gpu_run(f, g, precision=1, ctx=ctx, want_local=False)
    ra, _ = gpu_run(f, g, precision=0, ctx=ctx, want_local=False)
    assert np.array_equal(ra["corner_label"], rb["corner_label"])
    assert np.array_equal(ra["triangles"], rb["triangles"])
    assert np.array_equal(ra["vertices"], rb["vertices"])
    ok, why = M.is_closed_oriented_manifold(rb["triangles"], rb["n_vertices"])
    assert ok, why
    o = oracle_mod.Oracle(f, g, mlp_tie_eps=MLP_TIE / 20)
    n1 = g.res + 1
    rng = np.random.default_rng(13)
    ea = g.res * n1 * n1
    ties = 0
    for e in rb["edge_ids"][rng.integers(0, len(rb["edge_ids"]), 750)]:
        a, loc = int(e) // ea, int(e) % ea
        dims = [n1, n1, n1]
        dims[a] = g.res
        p = [loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])]
        for end in range(2):
            q = list(p)
            q[a] += end
            lab, tie = o.corner_label(*q)
            ties += tie
            c = q[0] + n1 * (q[1] + n1 * q[2])
            assert tie or rb["corner_label"][c] == lab, c
    print(f"sdf256: {rb['n_guard_corners']} guard corners (of {n1 ** 3}), "
          f"1500 sampled corners, {ties} near-ties")
