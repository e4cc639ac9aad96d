"""Helpers for GPU parity tests: run the HIP path through the C ABI and compare
with the oracle element by element."""
from __future__ import annotations

import numpy as np

import odc_inputs as I


VERT_TOL = 1e-5   # cell widths: the stated bar for 3D points
MLP_TIE = 1e-5    # |logit| band the oracle treats as a near-tie (fp32 error < 2.4e-6)

INTERMEDIATE_NAMES = ("labels", "edge_ids", "edge_t", "pairs", "pair_pf", "cell_ids",
                      "cell_partmap", "cell_nf", "vertex_base", "edge_case", "edge_grad")


def gpu_run(field, grid, precision=0, ctx=None, want_local=True, trace=True, **params_kw):
    """Meshes one field through the C ABI and copies every intermediate back;
    with trace, also the searches' decision traces (for a replayed oracle).
    params_kw set further odc_params fields (e.g. coarse_step)."""
    from paper_2409_13418_amd import odc
    if ctx is None:
        ctx = odc.Context(0)
    ctx.set_trace(trace)
    df = odc.DeviceField(field)
    params = odc.default_params(grid, precision)
    for k, v in params_kw.items():
        setattr(params, k, v)
    out = ctx.extract(df, params, want_local=want_local)
    r = {k: v for k, v in out.items() if not hasattr(v, "cpu")}
    r["vertices"] = out["vertices"].cpu().numpy()
    r["triangles"] = out["triangles"].cpu().numpy()
    if want_local:
        r["vertices_local"] = out["vertices_local"].cpu().numpy()
        r["vertex_ref"] = out["vertex_ref"].cpu().numpy()
    for name in INTERMEDIATE_NAMES + (("edge_trace", "pair_trace") if trace else ()):
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
    if "n_flipped_faces" in r and r["n_flipped_faces"] != m["n_flipped_faces"]:
        bad.append(f"flipped-face counts differ: {r['n_flipped_faces']} against "
                   f"{m['n_flipped_faces']}")
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


def batch_results(ctx, outs, grids, trace=True):
    """Per-job results of the last batch on ctx (outputs of extract_batch with
    want_local, plus every intermediate of each job), shaped as gpu_run's."""
    rs = []
    names = INTERMEDIATE_NAMES + (("edge_trace", "pair_trace") if trace else ())
    for k, g in enumerate(grids):
        o = outs[k]
        r = {n: v for n, v in o.items() if not hasattr(v, "cpu")}
        for n in ("vertices", "triangles", "vertices_local", "vertex_ref"):
            r[n] = o[n].cpu().numpy()
        for n in names:
            r[n] = ctx.intermediate(n, job=k)
        nc = (g.res + 1) ** 3
        r["corner_label"] = np.unpackbits(r["labels"].view(np.uint8), bitorder="little")[:nc]
        rs.append(r)
    return rs


def trace_of(O, r, staged=False, labels_given=False):
    """The GPU run's recorded decisions (and, staged, its 1D and 2D points)
    as an oracle replay trace."""
    grad = r.get("edge_grad")
    return O.Trace(label_words=r["labels"], edge_ids=r["edge_ids"], edge_bits=r["edge_trace"],
                   edge_t=r["edge_t"], pair_rec=r["pairs"], pair_bits=r["pair_trace"],
                   pair_pf=r["pair_pf"], staged=staged, labels_given=labels_given,
                   edge_grad=grad if grad is not None and len(grad) else None)


def needed_search_queries(m, g):
    """Sec. 5.2 / App. A.1.3 with early exits, from an oracle mesh's query
    labels: per pair m, each ray's linear samples up to the first label that
    differs from m's (all of them when none does) and its halvings; no
    step-2 rays when step 1 ends at m (pair_info bit 13)."""
    lab = m["pair_bits"][:, 0].astype(np.uint64)
    qm = (m["pair_info"] >> 13) & 1
    total = 0
    for x in range(len(lab)):
        b = int(lab[x])
        sm = b & 1
        n = 1

        def ray(first, n_lin, n_bin):
            for i in range(n_lin):
                if ((b >> (first + i)) & 1) != sm:
                    return i + 1 + n_bin
            return n_lin + n_bin

        n += ray(1, g.lin1, g.bin1)
        if not qm[x]:
            s2 = 1 + g.lin1 + g.bin1
            n += ray(s2, g.lin2, g.bin2) + ray(s2 + g.lin2 + g.bin2, g.lin2, g.bin2)
        total += n
    return total


def check_replayed(r, m, tr, res, label, vert_tol=VERT_TOL):
    """The bar once the oracle has followed the GPU's branches at its own
    near-ties: no other decision differs; integer structure, 1D points and 2D
    points bit-identical; every vertex within vert_tol cell widths; quad
    splits identical except where the binary64 triple product sits within its
    error band.  Returns the largest vertex error."""
    assert tr.mismatched == 0, (label, "decisions away from a near-tie differ", tr.mismatched)
    assert tr.unmatched == 0, (label, tr.unmatched)
    assert compare_discrete(r, m) == [], label
    assert np.array_equal(r["edge_t"].astype(np.float64), m["edge_t"]), label
    dp = np.abs(r["pair_pf"] - m["pair_pf"])
    assert np.array_equal(r["pair_pf"], m["pair_pf"]), (label, float(dp.max()), int(np.argmax(dp) // 2))
    tie = m["edge_case_tie"] != 0
    same = r["edge_case"] == m["edge_case"]
    assert np.all(same | tie), (label, int(np.sum(~same & ~tie)))
    # partition vertices, then (when the quad splits agree, so that the lists
    # align) the case-3 vertices appended after them
    nv = int(m["cell_npart"].sum())
    if np.all(same):
        assert len(r["vertices"]) == len(m["vert"]), label
        assert np.array_equal(r["triangles"], m["tris"]), label
        nv = len(m["vert"])
    dv = np.max(np.abs(vertex_grid_coords(r, res)[:nv] - m["vert"][:nv]), axis=1) if nv else np.zeros(0)
    assert np.all(dv <= vert_tol), (label, float(dv.max()), int(np.argmax(dv)))
    return float(dv.max()) if nv else 0.0


def check_sampled_replayed(r, g, O, f, rng, n_corners, n_edges, n_pairs, n_cells, label):
    """Seeded samples of a large grid, each recomputed one by one by the
    replayed oracle (single-element calls that read the GPU's trace): corner
    labels equal, 1D and 2D points bit-identical, partitions exact and
    vertices within VERT_TOL.  Elements are drawn from the oracle-checked
    label set's crossing lists; returns the adopted near-tie count."""
    tr = trace_of(O, r)
    o = O.Oracle(f, g, mlp_tie_eps=MLP_TIE, trace=tr)
    n1 = g.res + 1
    cs = list(rng.integers(0, n1 ** 3, n_corners))
    for e in r["edge_ids"][rng.integers(0, len(r["edge_ids"]), n_corners // 2)]:
        cs.extend(edge_corners(e, g.res))
    for c in cs:
        lab, tie = o.corner_label(*corner_ijk(int(c), n1))
        assert tie == 0 and r["corner_label"][c] == lab, (label, int(c))
    for x in rng.integers(0, len(r["edge_ids"]), n_edges):
        t, ts = o.edge_point(int(r["edge_ids"][x]))
        assert ts == 0 and float(r["edge_t"][x]) == t, (label, int(x), t)
    for x in rng.integers(0, len(r["pairs"]), n_pairs):
        rec = int(r["pairs"][x])
        n, pf, info, tie = o.pair_point(rec >> 1, rec & 1)
        assert n >= 1 and tie == 0, (label, int(x))
        assert np.array_equal(r["pair_pf"][x], pf), (label, int(x), r["pair_pf"][x], pf)
    vg = vertex_grid_coords(r, g.res)
    for x in rng.integers(0, len(r["cell_ids"]), n_cells):
        cid = int(r["cell_ids"][x])
        n, verts, pm, tie = o.cell_vertices(cid)
        assert n == int(r["cell_nf"][x] & 15) and pm == int(r["cell_partmap"][x]), (label, cid)
        base = int(r["vertex_base"][x])
        dv = np.max(np.abs(vg[base:base + n] - verts))
        assert tie == 0 and dv <= VERT_TOL, (label, cid, dv, tie)
    assert tr.mismatched == 0 and tr.unmatched == 0, (label, tr.mismatched, tr.unmatched)
    return tr.adopted
