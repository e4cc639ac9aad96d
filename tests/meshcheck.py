"""Mesh property checks shared by oracle and GPU tests (pure numpy)."""
from __future__ import annotations

import numpy as np


def edge_incidence(tris: np.ndarray):
    """Directed half-edges -> counts of undirected edges and directed duplicates."""
    t = np.asarray(tris, np.int64)
    he = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    und = np.sort(he, axis=1)
    _, cnt = np.unique(und, axis=0, return_counts=True)
    _, dcnt = np.unique(he, axis=0, return_counts=True)
    return cnt, dcnt


def is_closed_oriented_manifold(tris: np.ndarray, n_vertices: int) -> tuple[bool, str]:
    """Every edge in exactly two triangles with opposite directions, and every
    vertex's triangle fan forms a single cycle."""
    t = np.asarray(tris, np.int64)
    if len(t) == 0:
        return True, "empty"
    if np.any(t[:, 0] == t[:, 1]) or np.any(t[:, 1] == t[:, 2]) or np.any(t[:, 0] == t[:, 2]):
        return False, "degenerate triangle"
    cnt, dcnt = edge_incidence(t)
    if np.any(cnt != 2):
        return False, f"edges with incidence != 2: {int(np.sum(cnt != 2))}"
    if np.any(dcnt != 1):
        return False, f"inconsistently oriented edges: {int(np.sum(dcnt != 1))}"
    # vertex umbrellas: the link of v (edges opposite v) must be a single cycle
    nxt = {}
    for a, b, c in t:
        for v, p, q in ((a, b, c), (b, c, a), (c, a, b)):
            nxt.setdefault(int(v), {})[int(p)] = int(q)
    for v, m in nxt.items():
        start = next(iter(m))
        cur, steps = start, 0
        while True:
            cur = m.get(cur)
            steps += 1
            if cur is None:
                return False, f"open umbrella at vertex {v}"
            if cur == start:
                break
            if steps > len(m):
                return False, f"umbrella loop at vertex {v}"
        if steps != len(m):
            return False, f"vertex {v} umbrella has {len(m)} wedges but cycle of {steps}"
    used = np.unique(t)
    if len(used) != n_vertices:
        return False, f"unused vertices: {n_vertices - len(used)}"
    return True, "ok"


def euler_characteristic(tris: np.ndarray, n_vertices: int) -> int:
    t = np.asarray(tris, np.int64)
    cnt, _ = edge_incidence(t)
    return int(n_vertices - len(cnt) + len(t))


# ------------------------------------------------------------------ Chamfer
def _closest_on_triangles(p, a, b, c):
    """Closest points on triangles (a, b, c) to points p (row-wise), by the
    Voronoi-region method (Ericson, Real-Time Collision Detection, 5.1.5)."""
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = np.einsum("ij,ij->i", ab, ap), np.einsum("ij,ij->i", ac, ap)
    bp = p - b
    d3, d4 = np.einsum("ij,ij->i", ab, bp), np.einsum("ij,ij->i", ac, bp)
    cp = p - c
    d5, d6 = np.einsum("ij,ij->i", ab, cp), np.einsum("ij,ij->i", ac, cp)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    denom = va + vb + vc
    with np.errstate(divide="ignore", invalid="ignore"):
        v = vb / denom
        w = vc / denom
        out = a + ab * v[:, None] + ac * w[:, None]      # interior (NaN if degenerate)
    with np.errstate(divide="ignore", invalid="ignore"):
        # edge regions
        t_ab = d1 / (d1 - d3)
        t_ac = d2 / (d2 - d6)
        t_bc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
    m = (vc <= 0) & (d1 >= 0) & (d3 <= 0)
    out[m] = a[m] + ab[m] * t_ab[m, None]
    m = (vb <= 0) & (d2 >= 0) & (d6 <= 0)
    out[m] = a[m] + ac[m] * t_ac[m, None]
    m = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)
    out[m] = b[m] + (c - b)[m] * t_bc[m, None]
    # vertex regions
    m = (d1 <= 0) & (d2 <= 0)
    out[m] = a[m]
    m = (d3 >= 0) & (d4 <= d3)
    out[m] = b[m]
    m = (d6 >= 0) & (d5 <= d6)
    out[m] = c[m]
    return out


def _sample_surface(v, t, n, rng):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    idx = rng.choice(len(t), n, p=area / area.sum())
    r1 = np.sqrt(rng.random(n))
    r2 = rng.random(n)
    return (1 - r1)[:, None] * a[idx] + (r1 * (1 - r2))[:, None] * b[idx] + (r1 * r2)[:, None] * c[idx]


def sample_surface(v, t, n, seed=0):
    """n area-uniform points on the triangle mesh (v, t)."""
    return _sample_surface(np.asarray(v, np.float64), np.asarray(t), n,
                           np.random.default_rng(seed))


def _to_surface_sq(p, v, t, k=16):
    """Exact squared distance from points p to the triangle mesh (v, t).
    Candidates are the triangles with the k nearest centroids; a point is
    settled once its k-th candidate centroid is farther than its best
    distance plus the largest centroid-to-vertex radius (no other triangle
    can then be closer); the rest are redone with twice as many candidates."""
    from scipy.spatial import cKDTree
    cen = (v[t[:, 0]] + v[t[:, 1]] + v[t[:, 2]]) / 3.0
    rad = np.sqrt(max(float(np.max(np.sum((v[t[:, j]] - cen) ** 2, axis=1))) for j in range(3)))
    tree = cKDTree(cen)
    best = np.full(len(p), np.inf)
    todo = np.arange(len(p))
    while len(todo):
        kk = min(k, len(t))
        dist, cand = tree.query(p[todo], k=kk)
        dist = dist.reshape(len(todo), kk)
        cand = cand.reshape(len(todo), kk)
        b = np.full(len(todo), np.inf)
        for j in range(kk):
            tri = t[cand[:, j]]
            q = _closest_on_triangles(p[todo], v[tri[:, 0]], v[tri[:, 1]], v[tri[:, 2]])
            b = np.fmin(b, np.einsum("ij,ij->i", p[todo] - q, p[todo] - q))
        best[todo] = b
        if kk == len(t):
            break
        settled = dist[:, -1] > np.sqrt(b) + rad
        todo = todo[~settled]
        k *= 2
    return best


def chamfer_h2(va, ta, vb, tb, h, n=100000, seed=0):
    """Symmetric Chamfer distance between two meshes in units of h^2: mean
    squared distance from n area-uniform samples of each mesh to the other
    mesh's surface, averaged over both directions."""
    va, vb = np.asarray(va, np.float64), np.asarray(vb, np.float64)
    ta, tb = np.asarray(ta, np.int64), np.asarray(tb, np.int64)
    if len(ta) == 0 or len(tb) == 0:
        return 0.0 if len(ta) == len(tb) else float("inf")
    rng = np.random.default_rng(seed)
    da = _to_surface_sq(_sample_surface(va, ta, n, rng), vb, tb)
    db = _to_surface_sq(_sample_surface(vb, tb, n, rng), va, ta)
    return float(0.5 * (da.mean() + db.mean()) / (h * h))
