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
