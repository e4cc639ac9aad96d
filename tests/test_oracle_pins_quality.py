"""Pins of the oracle's self-intersection count (CPU only): pairs of
triangles that share no vertex and intersect."""
import numpy as np

import odc_inputs as I
import meshcheck as M


def _count(oracle_mod, v, t):
    return oracle_mod.self_intersections(np.asarray(v, np.float32), np.asarray(t, np.int32))


def test_two_triangles(oracle_mod):
    A = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]
    cases = {
        "piercing": ([[0.2, 0.2, -1], [0.2, 0.2, 1], [0.3, 0.9, 0.5]], 1),
        "above": ([[0.2, 0.2, 0.1], [0.6, 0.2, 0.3], [0.3, 0.5, 0.5]], 0),
        "beside": ([[2, 0, -1], [2, 1, 1], [3, 0, 0]], 0),
        "edge through the interior": ([[0.1, 0.1, -1], [0.1, 0.1, 1], [-1, -1, 0.5]], 1),
        "coplanar overlap": ([[0.2, 0.2, 0], [1.2, 0.2, 0], [0.2, 1.2, 0]], 1),
        "coplanar apart": ([[1.1, 1.1, 0], [2, 1.1, 0], [1.1, 2, 0]], 0),
        "coplanar nested": ([[0.1, 0.1, 0], [0.3, 0.1, 0], [0.1, 0.3, 0]], 1),
    }
    for name, (B, expect) in cases.items():
        v = np.array(A + B, np.float64)
        t = np.array([[0, 1, 2], [3, 4, 5]])
        assert _count(oracle_mod, v, t) == expect, name
        # symmetric in the order of the triangles and of their corners
        assert _count(oracle_mod, v, t[::-1]) == expect, name
        assert _count(oracle_mod, v, np.array([[1, 2, 0], [5, 3, 4]])) == expect, name


def test_shared_vertices_are_not_counted(oracle_mod):
    # two triangles folded through each other but sharing a vertex
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.5, 0.5, -1], [0.3, 0.3, 1]], np.float64)
    t = np.array([[0, 1, 2], [0, 3, 4]])
    assert _count(oracle_mod, v, t) == 0


def test_closed_convex_mesh_has_none(oracle_mod):
    # an octahedron, subdivided twice and pushed onto the unit sphere
    v = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
    t = [[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]
    v = [np.array(p, float) for p in v]
    for _ in range(2):
        mid = {}
        nt = []
        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[k] = len(v) - 1
            return mid[k]
        for a, b, c in t:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nt += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        t = nt
    v = np.array(v)
    t = np.array(t)
    ok, _ = M.is_closed_oriented_manifold(t, len(v))
    assert ok and len(t) == 128
    assert _count(oracle_mod, v, t) == 0
    # push one vertex through the opposite side: its fan now crosses it
    v2 = v.copy()
    top = int(np.argmax(v[:, 2]))
    v2[top] = [0.0, 0.0, -1.5]
    assert _count(oracle_mod, v2, t) > 0


def test_oracle_meshes(oracle_mod):
    """The method's meshes of a smooth field have no self-intersection at this
    size; the plain split does not add any on a convex sphere either."""
    f, g = I.sphere_case(16, 10)
    m = oracle_mod.Oracle(f, g).mesh()
    assert _count(oracle_mod, m["vert"], m["tris"]) == 0
