"""Helpers for GPU parity tests: run the HIP path through the C ABI and compare
with the oracle element by element."""
from __future__ import annotations

import numpy as np

import odc_inputs as I


def gpu_run(field, grid, precision=0, ctx=None, want_local=True):
    from paper_2409_13418_amd import odc
    if ctx is None:
        ctx = odc.Context(0)
    df = odc.DeviceField(field)
    params = odc.default_params(grid, precision)
    out = ctx.extract(df, params, want_local=want_local)
    r = {k: v for k, v in out.items() if not hasattr(v, "cpu")}
    r["vertices"] = out["vertices"].cpu().numpy()
    r["triangles"] = out["triangles"].cpu().numpy()
    if want_local:
        r["vertices_local"] = out["vertices_local"].cpu().numpy()
        r["vertex_ref"] = out["vertex_ref"].cpu().numpy()
    for name in ("labels", "edge_ids", "edge_t", "pairs", "pair_pf", "cell_ids",
                 "cell_partmap", "cell_nf", "vertex_base", "edge_case", "edge_grad"):
        r[name] = ctx.intermediate(name)
    N = grid.res
    nc = (N + 1) ** 3
    bits = np.unpackbits(r["labels"].view(np.uint8), bitorder="little")[:nc]
    r["corner_label"] = bits.astype(np.uint8)
    return r, ctx


def vertex_grid_coords(r, res):
    """GPU vertices in grid units from (reference corner, local offset)."""
    ref = r["vertex_ref"].astype(np.int64)
    n1 = res + 1
    base = np.stack([ref % n1, (ref // n1) % n1, ref // (n1 * n1)], 1).astype(np.float64)
    return base + r["vertices_local"].astype(np.float64)


def compare_discrete(r, m):
    """Bit-exact checks of the integer structure; returns a list of failures."""
    bad = []
    if not np.array_equal(r["corner_label"], m["corner_label"]):
        bad.append(f"labels differ at {int(np.sum(r['corner_label'] != m['corner_label']))} corners")
        return bad
    if not np.array_equal(r["edge_ids"], m["edge_id"]):
        bad.append("crossing edge sets differ")
        return bad
    opairs = (m["pair_face"].astype(np.int64) << 1) | (m["pair_info"] & 1)
    if not np.array_equal(r["pairs"].astype(np.int64), opairs):
        bad.append("face pair sets differ")
    if not np.array_equal(r["cell_ids"], m["cell_id"]):
        bad.append("active cell sets differ")
        return bad
    if not np.array_equal(r["cell_nf"] & 15, m["cell_npart"]):
        bad.append("partition counts differ")
    if not np.array_equal(r["cell_nf"] >> 4, m["cell_flipmask"]):
        bad.append("manifold flips differ")
    # partition maps compared on crossing edges only
    if not np.array_equal(r["cell_partmap"].astype(np.int64), m["cell_partmap"].astype(np.int64)):
        bad.append(f"partition maps differ in {int(np.sum(r['cell_partmap'] != m['cell_partmap']))} cells")
    if not np.array_equal(r["vertex_base"], m["cell_vbase"]):
        bad.append("vertex numbering differs")
    return bad


def mesh_labels_from_oracle(m):
    return m["corner_label"]


def corner_ijk(c, n1):
    return c % n1, (c // n1) % n1, c // (n1 * n1)


def edge_origin(e, N):
    """Axis and lower-corner grid position of edge e (axis-major numbering)."""
    n1 = N + 1
    ea = N * n1 * n1
    a, loc = int(e) // ea, int(e) % ea
    dims = [n1, n1, n1]
    dims[a] = N
    return a, [loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])]


def world32(grid, gp):
    """World point of grid point gp in binary32, x = lo + g h (two rounded
    operations, h = (float)(size / res)), as both sides build query points."""
    h = np.float32(grid.size / grid.res)
    return [np.float32(grid.lo[a]) + np.float32(gp[a]) * h for a in range(3)]


def edge_corners(e, N):
    """The two corner indices of crossing edge e (axis-major edge numbering)."""
    n1 = N + 1
    ea = N * n1 * n1
    a, loc = int(e) // ea, int(e) % ea
    dims = [n1, n1, n1]
    dims[a] = N
    p = [loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])]
    c0 = p[0] + n1 * (p[1] + n1 * p[2])
    p[a] += 1
    return c0, p[0] + n1 * (p[1] + n1 * p[2])


def sampled_labels(r, g, o, rng, n_uniform, n_edges):
    """GPU corner labels against the oracle at uniform corners and at both ends
    of sampled crossing edges; returns the number of near-ties skipped."""
    n1 = g.res + 1
    cs = list(rng.integers(0, n1 ** 3, n_uniform))
    for e in r["edge_ids"][rng.integers(0, len(r["edge_ids"]), n_edges)]:
        cs.extend(edge_corners(e, g.res))
    ties = 0
    for c in cs:
        lab, tie = o.corner_label(*corner_ijk(int(c), n1))
        if tie:
            ties += 1
            continue
        assert r["corner_label"][c] == lab, int(c)
    return len(cs), ties


def interior_edge_count(edge_ids, N):
    """Crossing edges with all four cells inside the grid."""
    n1 = N + 1
    e = edge_ids.astype(np.int64)
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
    return int(interior.sum())
