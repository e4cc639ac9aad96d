"""Pins of the oracle's searches against closed forms (CPU only).

Sec. 5.1 (1D bisection), App. A.1.3 (line-binary search), Sec. 5.2 Lemma 1
with its proof in App. A.1.2 (2D point of a straight line / a wedge).
"""
import math

import numpy as np
import pytest

import odc_inputs as I


def _edge_id(N, a, i, j, k):
    E = N * (N + 1) * (N + 1)
    if a == 0:
        return i + N * (j + (N + 1) * k)
    if a == 1:
        return E + i + (N + 1) * (j + N * k)
    return 2 * E + i + (N + 1) * (j + (N + 1) * k)


def _face_id(N, a, i, j, k):
    F = (N + 1) * N * N
    if a == 0:
        return i + (N + 1) * (j + N * k)
    if a == 1:
        return F + i + N * (j + (N + 1) * k)
    return 2 * F + i + N * (j + N * k)


@pytest.mark.parametrize("seed", range(6))
def test_bisection_plane_closed_form(oracle_mod, seed):
    """Half-space field: the 1D point lies within 2^-(k+1) of the exact
    crossing of the plane with the edge (Sec. 5.1, midpoint of the final
    bracket), plus the binary32 label resolution."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    pt = rng.uniform(-0.2, 0.2, 3)
    f = I.csg_field([I.halfspace_record(pt, n)])
    g = I.unit_grid(16, iters_1d=12)
    o = oracle_mod.Oracle(f, g)
    m = o.mesh()
    assert len(m["edge_id"]) > 20
    h = g.h
    n32 = I.halfspace_record(pt, n)[5:8].astype(np.float64)
    c32 = np.asarray(pt, np.float32).astype(np.float64)
    N = g.res
    E = N * (N + 1) * (N + 1)
    for eid, t in zip(m["edge_id"], m["edge_t"]):
        a = eid // E
        r = eid - a * E
        nx = N if a == 0 else N + 1
        ny = N if a == 1 else N + 1
        pos = np.array([r % nx, (r // nx) % ny, r // (nx * ny)], float)
        p0 = -0.5 + pos * h
        # n.(p0 + s e_a - c) = 0
        s = -np.dot(n32, p0 - c32) / n32[a]
        tstar = s / h
        assert 0.0 < tstar < 1.0
        assert abs(t - tstar) <= 2.0 ** -(g.iters_1d + 1) + 1e-5, (eid, t, tstar)
        # t is the middle of a dyadic bracket: an odd multiple of 2^-(k+1)
        q = t * 2 ** (g.iters_1d + 1)
        assert q == int(q) and int(q) % 2 == 1


def test_bisection_sphere_closed_form(oracle_mod):
    f, g = I.sphere_case(32, 10)
    o = oracle_mod.Oracle(f, g)
    m = o.mesh()
    c = np.array([0.03, -0.02, 0.01], np.float32).astype(np.float64)
    r = float(np.float32(0.35))
    N, h = g.res, g.h
    E = N * (N + 1) * (N + 1)
    worst = 0.0
    for eid, t in zip(m["edge_id"], m["edge_t"]):
        a = eid // E
        rr = eid - a * E
        nx = N if a == 0 else N + 1
        ny = N if a == 1 else N + 1
        pos = np.array([rr % nx, (rr // nx) % ny, rr // (nx * ny)], float)
        p0 = -0.5 + pos * h
        d = p0 - c
        # |d + s e_a|^2 = r^2 -> s^2 + 2 d_a s + |d|^2 - r^2 = 0
        B, Cc = d[a], d @ d - r * r
        disc = B * B - Cc
        roots = [-B - math.sqrt(disc), -B + math.sqrt(disc)]
        ts = [s / h for s in roots if 0.0 <= s / h <= 1.0]
        assert len(ts) == 1
        worst = max(worst, abs(t - ts[0]))
    assert worst <= 2.0 ** -11 + 1e-6


def test_line_binary_halfspace(oracle_mod):
    """Line-binary search (App. A.1.3) along a ray crossing a half-space
    boundary at parameter s*: the near end lies in [s* - R/N 2^-K, s*]; with
    no crossing it ends R/N 2^-K short of R."""
    N = 8
    g = I.unit_grid(N)
    h = g.h
    rng = np.random.default_rng(7)
    fid = _face_id(N, 2, 3, 4, 4)  # normal z at (3,4,4): u = x, v = y
    for trial in range(40):
        sstar = rng.uniform(0.05, 0.75)
        ang = rng.uniform(0, 2 * math.pi)
        d = np.array([math.cos(ang), math.sin(ang)], np.float32)
        p0 = np.array([0.5, 0.5], np.float32)
        # world point where the ray meets the plane; plane normal along d
        wp = np.array([-0.5 + (3 + 0.5 + sstar * d[0]) * h,
                       -0.5 + (4 + 0.5 + sstar * d[1]) * h, -0.5 + 4 * h])
        nrm = np.array([d[0], d[1], 0.0])
        f = I.csg_field([I.halfspace_record(wp, nrm)])  # inside: before the plane
        o = oracle_mod.Oracle(f, g)
        s, q = o.line_binary(fid, p0, d, 1, 0.8, 4, 11)
        step = 0.8 / 4 * 2.0 ** -11
        assert sstar - step - 1e-5 <= s <= sstar + 1e-5, (trial, s, sstar)
    # no crossing within range: everything inside
    f = I.csg_field([I.halfspace_record((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))])
    o = oracle_mod.Oracle(f, I.unit_grid(N))
    fid_low = _face_id(N, 2, 3, 4, 1)
    s, q = o.line_binary(fid_low, np.array([0.5, 0.5], np.float32),
                         np.array([1.0, 0.0], np.float32), 1, 0.8, 4, 11)
    assert abs(s - 0.8 * (1 - 2.0 ** -11 / 4)) < 1e-6


def _wedge_face_case(oracle_mod, apex_uv, n1, n2, convex, N=8, fi=(3, 4, 4)):
    """Face normal z at fi; occupancy inside the face plane is a wedge with
    apex at apex_uv (face-local), boundary lines with in-plane normals n1, n2.
    Returns the oracle's pairs on that face."""
    h = 1.0 / N
    base = np.array([-0.5 + fi[0] * h, -0.5 + fi[1] * h, -0.5 + fi[2] * h])
    apex = base + np.array([apex_uv[0] * h, apex_uv[1] * h, 0.0])
    r1 = I.halfspace_record(apex, (n1[0], n1[1], 0.0))
    r2 = I.halfspace_record(apex, (n2[0], n2[1], 0.0),
                            op=I.OP_INTERSECT if convex else I.OP_UNION)
    f = I.csg_field([r1, r2])
    o = oracle_mod.Oracle(f, I.unit_grid(N, 15))
    return o, _face_id(N, 2, *fi)


def test_lemma1_straight_line_gives_midpoint(oracle_mod):
    """Lemma 1, identical lines: a straight boundary through the face gives
    q = m and p_f = m exactly (App. A.1.2)."""
    rng = np.random.default_rng(11)
    hits = 0
    for trial in range(60):
        ang = rng.uniform(0, 2 * math.pi)
        nrm = (math.cos(ang), math.sin(ang))
        c = rng.uniform(0.3, 0.7, 2)
        o, fid = _wedge_face_case(oracle_mod, c, nrm, nrm, True)
        n, pf, info, tie = o.pair_point(fid, 0)
        if n != 1:
            continue
        hits += 1
        assert (info >> 13) & 1 == 1, trial
        fa, fb = (info >> 4) & 15, (info >> 8) & 15
        ta = o.edge_point(_edge_of(fid, fa))[0]
        tb = o.edge_point(_edge_of(fid, fb))[0]
        P = {0: (ta, 0.0), 1: (ta, 1.0), 2: (0.0, ta), 3: (1.0, ta)}[fa]
        Q = {0: (tb, 0.0), 1: (tb, 1.0), 2: (0.0, tb), 3: (1.0, tb)}[fb]
        m = ((P[0] + Q[0]) / 2, (P[1] + Q[1]) / 2)
        assert pf[0] == m[0] and pf[1] == m[1]
    assert hits > 30


def _edge_of(fid, fe, N=8, fi=(3, 4, 4)):
    i, j, k = fi
    if fe == 0:
        return _edge_id(N, 0, i, j, k)
    if fe == 1:
        return _edge_id(N, 0, i, j + 1, k)
    if fe == 2:
        return _edge_id(N, 1, i, j, k)
    return _edge_id(N, 1, i + 1, j, k)


@pytest.mark.parametrize("convex", [True, False])
def test_lemma1_wedge_gives_apex(oracle_mod, convex):
    """Lemma 1, two lines meeting at u: the 2D point is u within the search
    resolution (step 1: 0.8/4 * 2^-11 cells; step 2: (sqrt2/2)/3 * 2^-12)."""
    rng = np.random.default_rng(5 if convex else 6)
    good = 0
    for trial in range(200):
        apex = rng.uniform(0.25, 0.75, 2)
        a1 = rng.uniform(0, 2 * math.pi)
        a2 = a1 + rng.uniform(0.6, 2.4) * (1 if rng.uniform() < 0.5 else -1)
        n1 = (math.cos(a1), math.sin(a1))
        n2 = (math.cos(a2), math.sin(a2))
        o, fid = _wedge_face_case(oracle_mod, apex, n1, n2, convex)
        n, pf, info, tie = o.pair_point(fid, 0)
        if n != 1:
            continue
        # the lemma needs each boundary line to pass through one of the pair's
        # 1D points: the crossing edges must be cut by different lines
        fa, fb = (info >> 4) & 15, (info >> 8) & 15
        pts = []
        for fe in (fa, fb):
            t = o.edge_point(_edge_of(fid, fe))[0]
            pts.append({0: (t, 0.0), 1: (t, 1.0), 2: (0.0, t), 3: (1.0, t)}[fe])
        on1 = [abs((p[0] - apex[0]) * n1[0] + (p[1] - apex[1]) * n1[1]) < 1e-3 for p in pts]
        on2 = [abs((p[0] - apex[0]) * n2[0] + (p[1] - apex[1]) * n2[1]) < 1e-3 for p in pts]
        if not ((on1[0] and on2[1]) or (on1[1] and on2[0])):
            continue
        # and the apex must be reachable: within step-1 range of m, inside the face
        good += 1
        # the search resolution (~1e-4 cells) spreads along each line by 1/sin
        err = math.hypot(pf[0] - apex[0], pf[1] - apex[1])
        sin = abs(n1[0] * n2[1] - n1[1] * n2[0])
        assert err * sin <= 4e-4, (trial, pf, apex, err)
    assert good > 40
