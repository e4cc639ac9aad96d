"""Pins of the oracle's geometry (CPU only): the QEF (Sec. 4, Eq. 2), the
intersection-free split (App. A.1.5, Eqs. A1-A2), sharp features recovered
from occupancy alone (Sec. 5.2-5.3), and the MLP field definition."""
import math

import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M


def test_qef_three_orthogonal_planes(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(20):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        corner = rng.uniform(0.2, 0.8, 3)
        pts = [corner + rng.uniform(-0.5, 0.5) * Q[(i + 1) % 3] for i in range(3)]
        x, kap = oracle_mod.qef_solve(Q, pts)
        assert np.allclose(x, corner, atol=1e-12)
        assert abs(kap - 1.0) < 1e-9


def test_qef_two_planes_nearest_point_on_line(oracle_mod):
    rng = np.random.default_rng(2)
    for _ in range(20):
        n1 = rng.standard_normal(3); n1 /= np.linalg.norm(n1)
        n2 = rng.standard_normal(3); n2 -= n1 * (n1 @ n2) * 0.3; n2 /= np.linalg.norm(n2)
        d = np.cross(n1, n2); d /= np.linalg.norm(d)
        p_on = rng.uniform(0.3, 0.7, 3)
        pts = [p_on + 0.2 * d, p_on - 0.1 * d + 0.0]
        # both points lie on the line; mass point projects onto it
        x, _ = oracle_mod.qef_solve([n1, n2], pts)
        mass = (pts[0] + pts[1]) / 2
        expect = p_on + ((mass - p_on) @ d) * d
        assert np.allclose(x, expect, atol=1e-10)


def test_qef_one_plane_projects_mass_point(oracle_mod):
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    pts = [np.array([0.1, 0.2, 0.3]), np.array([0.5, 0.1, 0.4]), np.array([0.2, 0.9, 0.1])]
    x, _ = oracle_mod.qef_solve([n, n, n], pts)
    mass = np.mean(pts, axis=0)
    # each point's offset along n is averaged: the solution stays the mass point
    assert np.allclose(x, mass, atol=1e-12)
    # planes through a common plane: solution lies on it
    p0 = np.array([0.5, 0.5, 0.5])
    pts = [p0 + v - n * (n @ v) for v in np.random.default_rng(3).uniform(-0.3, 0.3, (4, 3))]
    x, _ = oracle_mod.qef_solve([n] * 4, pts)
    assert abs((x - p0) @ n) < 1e-12


def test_qef_truncation_treats_shallow_angle_as_flat(oracle_mod):
    """tau = 1e-2 on eigenvalues: planes turning by less than ~11.4 degrees
    act as one plane (the mass point moves only along the mean normal, the
    dominant eigenvector (n1 + n2)/|n1 + n2|)."""
    for deg, flat in ((5.0, True), (30.0, False)):
        a = math.radians(deg)
        n1 = np.array([0.0, 0.0, 1.0])
        n2 = np.array([0.0, math.sin(a), math.cos(a)])
        pts = [np.array([0.3, 0.2, 0.5]), np.array([0.3, 0.8, 0.5])]
        x, _ = oracle_mod.qef_solve([n1, n2], pts)
        mass = (pts[0] + pts[1]) / 2
        if flat:
            v = (n1 + n2) / np.linalg.norm(n1 + n2)
            assert np.linalg.norm(np.cross(x - mass, v)) < 1e-12
        else:
            # the exact intersection line of both planes
            assert abs(n1 @ (x - pts[0])) < 1e-9 and abs(n2 @ (x - pts[1])) < 1e-9


def _square_quad(z_off=0.0):
    # CCW about +x, edge from (0,0,0) (in) to (1,0,0) (out)
    return np.array([[0.5, 0.5, 0.5], [0.5, -0.5, 0.5], [0.5, -0.5, -0.5], [0.5, 0.5, -0.5]])


def test_ic_planar_convex_quad_is_case1(oracle_mod):
    c, tie = oracle_mod.ic_case(_square_quad(), [0, 0, 0], [1, 0, 0])
    assert c == 1 and tie == 0


def _in_tet(x, a, b, c, d, eps):
    T = np.column_stack([b - a, c - a, d - a])
    try:
        lam = np.linalg.solve(T, x - a)
    except np.linalg.LinAlgError:
        return -1.0
    bary = np.array([1 - lam.sum(), *lam])
    return bary.min()


def _diagonal_enclosed(q, pin, pout, i, j):
    """Brute force: sample the open segment q_i q_j and test containment in
    the union of the tetrahedra (v_in, v_out, q_k, q_k+1).  Returns True/False,
    or None when a sample sits on the envelope boundary."""
    worst = np.inf
    for s in np.linspace(0.0, 1.0, 63)[1:-1]:
        x = q[i] + s * (q[j] - q[i])
        best = max(_in_tet(x, pin, pout, q[k], q[(k + 1) % 4], 0) for k in range(4))
        worst = min(worst, best)
    if abs(worst) < 1e-7:
        return None
    return worst > 0


def test_ic_rule_matches_envelope_brute_force(oracle_mod):
    """Case 1 is chosen iff the diagonal q1q3 lies inside the envelope
    v_in v_out - q1q2q3q4; otherwise case 2 iff q2q4 does; otherwise case 3
    (App. A.1.5).  Checked by sampling on random quads wound once about the
    edge (v_in, v_out) = ((0,0,0), (1,0,0)), vertices inside the edge's slab."""
    rng = np.random.default_rng(12)
    pin, pout = np.zeros(3), np.array([1.0, 0.0, 0.0])
    seen = {1: 0, 2: 0, 3: 0}
    checked = 0
    for _ in range(800):
        q = np.zeros((4, 3))
        for k in range(4):
            th = math.pi / 4 + k * math.pi / 2 + rng.uniform(-0.6, 0.6)
            r = rng.uniform(0.15, 1.0)
            q[k] = [rng.uniform(0.02, 0.98), r * math.cos(th), r * math.sin(th)]
        e13 = _diagonal_enclosed(q, pin, pout, 0, 2)
        e24 = _diagonal_enclosed(q, pin, pout, 1, 3)
        if e13 is None or e24 is None:
            continue
        c, tie = oracle_mod.ic_case(q, pin, pout)
        expect = 1 if e13 else (2 if e24 else 3)
        assert c == expect, (q.tolist(), c, expect)
        seen[c] += 1
        checked += 1
    assert checked > 500 and min(seen.values()) >= 5, seen


def _mesh(oracle_mod, f, res, k=15):
    g = I.unit_grid(res, k)
    return oracle_mod.Oracle(f, g).mesh(), g


@pytest.mark.parametrize("rotated", [False, True])
def test_box_corners_are_sharp(oracle_mod, rotated):
    """A box seen only through occupancy: where the cell holding a box corner
    has crossing edges on all three of the corner's planes, its 3D point is
    the corner (2D points of face wedges are exact by Lemma 1, so the QEF
    sees the three true planes).  A rotated corner whose third plane cuts no
    edge of that cell is invisible to it, so the check covers the corners
    the grid samples."""
    rng = np.random.default_rng(4)
    R = None
    if rotated:
        q = rng.standard_normal(4); q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    c = np.array([0.013, -0.021, 0.017])
    half = np.array([0.21, 0.17, 0.19])
    f = I.csg_field([I.box_record(c, half, R)])
    m, g = _mesh(oracle_mod, f, 32)
    ok, why = M.is_closed_oriented_manifold(m["tris"], len(m["vert"]))
    assert ok, why
    Rm = np.eye(3) if R is None else R
    N, h = g.res, g.h
    E = N * (N + 1) * (N + 1)

    def planes_of(grid_pt):
        loc = Rm @ ((-0.5 + grid_pt * h) - c)
        return {(a, int(np.sign(loc[a]))) for a in range(3)
                if abs(abs(loc[a]) - half[a]) < 1e-3 * h}

    edge_pts = {}
    for eid, t in zip(m["edge_id"], m["edge_t"]):
        a = eid // E
        r = eid - a * E
        nx = N if a == 0 else N + 1
        ny = N if a == 1 else N + 1
        pos = np.array([r % nx, (r // nx) % ny, r // (nx * ny)], float)
        pos[a] += t
        edge_pts[eid] = pos
    checked = 0
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                sg = np.array([sx, sy, sz])
                cw = c + Rm.T @ (half * sg)
                gc = (cw + 0.5) / h
                cell = np.floor(gc).astype(int)
                seen = set()
                for p in edge_pts.values():
                    if np.all(p >= cell - 1e-9) and np.all(p <= cell + 1 + 1e-9):
                        seen |= planes_of(p)
                want = {(a, int(sg[a])) for a in range(3)}
                if not want <= seen:
                    continue
                checked += 1
                cid = cell[0] + N * (cell[1] + N * cell[2])
                x = int(np.searchsorted(m["cell_id"], cid))
                vb, npart = m["cell_vbase"][x], m["cell_npart"][x]
                d = np.min(np.linalg.norm(m["vert"][vb:vb + npart] - gc, axis=1))
                assert d < 5e-3, (cw, d)
    assert checked == 8 if not rotated else checked >= 3
    # every vertex lies on the box surface within the search resolution
    world = -0.5 + m["vert"] * h
    loc = (world - c) @ Rm.T
    dist = np.min(np.abs(np.abs(loc) - half), axis=1) / h
    assert np.quantile(dist, 0.9) < 2e-3


def test_plane_vertices_on_plane(oracle_mod):
    n = np.array([0.3, -0.5, 0.81]); n /= np.linalg.norm(n)
    p = np.array([0.02, 0.03, -0.01])
    f = I.csg_field([I.halfspace_record(p, n)])
    m, g = _mesh(oracle_mod, f, 24)
    world = -0.5 + m["vert"] * g.h
    # 1D points sit on the plane within the bisection bound 2^-(k+1); the QEF
    # keeps directions with eigenvalue >= tau * max, which can amplify that
    # error by up to 1/tau where 2D points crowd their 1D points
    d = np.abs((world - p) @ n) / g.h
    assert np.quantile(d, 0.95) < 2.0 ** -14
    assert d.max() < 2.0 ** -16 / 1e-2


def test_mlp_field_definition_by_special_weights(oracle_mod):
    """Weights that make the network compute sin(pi x) - 1/2 exactly (W1
    picks the band-0 sine of x and its negative, biases -1/2 and +1/2,
    identity hidden layers, output relu(a) - relu(b)): with the sdf gain at
    zero, phi' is 1 iff sin(pi x) > 1/2, so on [-0.5,0.5]^3 the surface is
    the plane x = 1/6."""
    W, depth, nb = 8, 3, 2
    in_dim = 3 + 6 * nb
    parts = []
    W1 = np.zeros((W, in_dim)); W1[0, 3] = 1.0; W1[1, 3] = -1.0
    b1 = np.zeros(W); b1[0], b1[1] = -0.5, 0.5
    parts += [W1, b1]
    for _ in range(depth - 1):
        Wh = np.zeros((W, W)); Wh[0, 0] = Wh[1, 1] = 1.0
        parts += [Wh, np.zeros(W)]
    wo = np.zeros(W); wo[0], wo[1] = 1.0, -1.0
    parts += [wo, np.zeros(1)]
    w = np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)
    f = I.Field(kind=I.FIELD_MLP, weights=w, in_dim=in_dim, width=W, depth=depth, n_bands=nb,
                spheres=np.array([[0.0, 0.0, 0.0, 0.1]], np.float32), sdf_gain=0.0,
                out_scale=0.3)
    m, g = _mesh(oracle_mod, f, 8, k=12)
    world = -0.5 + m["vert"] * g.h
    assert len(world) > 0
    assert np.abs(world[:, 0] - 1.0 / 6.0).max() < g.h * 2.0 ** -12
    # and the sdf term alone: a sphere
    f2 = I.Field(kind=I.FIELD_MLP, weights=np.zeros_like(w), in_dim=in_dim, width=W,
                 depth=depth, n_bands=nb,
                 spheres=np.array([[0.03, -0.02, 0.01, 0.3]], np.float32), sdf_gain=20.0,
                 out_scale=0.3)
    m2, g2 = _mesh(oracle_mod, f2, 16, k=12)
    world = -0.5 + m2["vert"] * g2.h
    r = np.linalg.norm(world - np.array([0.03, -0.02, 0.01]), axis=1)
    assert np.abs(r - 0.3).max() < 0.05 * g2.h  # curvature error of the 3D points at r = 4.8 h


def test_mlp_band_indexing(oracle_mod):
    """cos(2 pi y) picked from band 1 (feature 3 + 6*1 + 3 + 1): the surface
    is |y| = 1/4."""
    W, depth, nb = 4, 1, 2
    in_dim = 3 + 6 * nb
    W1 = np.zeros((W, in_dim)); W1[0, 3 + 6 + 3 + 1] = 1.0; W1[1, 3 + 6 + 3 + 1] = -1.0
    wo = np.zeros(W); wo[0], wo[1] = 1.0, -1.0
    w = np.concatenate([W1.reshape(-1), np.zeros(W), wo, np.zeros(1)]).astype(np.float32)
    f = I.Field(kind=I.FIELD_MLP, weights=w, in_dim=in_dim, width=W, depth=depth, n_bands=nb,
                spheres=np.array([[0.0, 0.0, 0.0, 0.1]], np.float32), sdf_gain=0.0,
                out_scale=1.0)
    m, g = _mesh(oracle_mod, f, 10, k=12)
    world = -0.5 + m["vert"] * g.h
    assert len(world) > 0
    # within the 2D-search resolution; a wrong band would put it at 1/8 or 1/16
    assert np.abs(np.abs(world[:, 1]) - 0.25).max() < 2e-3 * g.h
