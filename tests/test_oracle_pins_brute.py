"""Brute-force pins of the oracle's searches and of its manifold fix.

* Sec. 5.1: every 1D point of the sphere at 8^3 equals what dense sampling of
  its edge at all 2^k + 1 dyadic parameters gives (the midpoint of the dyadic
  interval holding the label change).
* App. A.1.3: line-binary searches along random rays agree with dense
  sampling of the same ray (the near end lies within one final bracket of
  the first label change; no change gives R (1 - 2^-k / N)).
* Sec. 5.2 / R9: on a face whose two crossing pairs cut off diagonal inside
  corners, step 1 must search towards the cut-off corner when both sides of
  the chord hold a corner of the other label.  A constructed face with a
  known apex pins the side.
* App. A.1.1 / R8: the oracle's own manifold fix (its face flips, through the
  full pipeline on label-built 2-cell grids) against the brute-force rule on
  all 512 blocks whose shared face is ambiguous.
"""
import numpy as np
import pytest

import odc_inputs as I
from gpu_common import edge_origin, world32


def _label(o, g, gp):
    lab, tie, _ = o.label_world(np.array(world32(g, gp), np.float32))
    assert tie == 0
    return lab


def test_edge_points_match_dense_sampling(oracle_mod):
    f, g = I.sphere_case(8, 10)
    o = oracle_mod.Oracle(f, g)
    m = o.mesh()
    k = g.iters_1d
    # crossing edges counted directly: corners lo + i h are exact in binary64
    # on this grid, inside iff |x - c|^2 < r^2, and no corner lies within
    # 1e-6 of the sphere (so binary32 rounding cannot flip a label)
    c, r = f.prims[0, 2:5].astype(np.float64), float(f.prims[0, 5])
    xs = [g.lo[a] + np.arange(g.res + 1) * (g.size / g.res) for a in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
    assert np.abs(d2 - r * r).min() > 1e-6
    ins = d2 < r * r
    n_cross = sum(int((np.diff(ins, axis=a) != 0).sum()) for a in range(3))
    assert len(m["edge_id"]) == n_cross > 0
    for x, e in enumerate(m["edge_id"]):
        a, p = edge_origin(e, g.res)
        labs = []
        for j in range(2 ** k + 1):
            gp = [np.float32(v) for v in p]
            gp[a] = np.float32(np.float32(p[a]) + np.float32(j / 2 ** k))
            labs.append(_label(o, g, gp))
        labs = np.array(labs)
        change = int(np.argmax(labs != labs[0]))
        assert change > 0 and np.all(labs[change:] != labs[0]), int(e)  # one crossing
        assert m["edge_t"][x] == (change - 0.5) / 2 ** k, (int(e), m["edge_t"][x], change)


def _face_ray_label(o, g, face_pos, a, u, v, P):
    gp = [0.0, 0.0, 0.0]
    gp[a] = np.float32(face_pos[a])
    gp[u] = np.float32(np.float32(face_pos[u]) + np.float32(P[0]))
    gp[v] = np.float32(np.float32(face_pos[v]) + np.float32(P[1]))
    return _label(o, g, gp)


def _decode_face(fid, N):
    n1 = N + 1
    F = n1 * N * N
    a, r = fid // F, fid % F
    dims = [N, N, N]
    dims[a] = n1
    pos = [r % dims[0], (r // dims[0]) % dims[1], r // (dims[0] * dims[1])]
    u, v = [ax for ax in range(3) if ax != a]
    return a, u, v, pos


@pytest.mark.parametrize("seed", [0, 1])
def test_line_binary_matches_dense_sampling(oracle_mod, seed):
    f, g = I.sphere_case(8, 10)
    o = oracle_mod.Oracle(f, g)
    m = o.mesh()
    rng = np.random.default_rng(seed)
    R, n_lin, n_bin = np.float32(0.8), 4, 8
    step = R / n_lin / 2 ** n_bin
    hits = misses = 0
    for fid in rng.choice(np.unique(m["pair_face"]), 40):
        a, u, v, pos = _decode_face(int(fid), g.res)
        p0 = rng.uniform(0, 1, 2).astype(np.float32)
        ang = rng.uniform(0, 2 * np.pi)
        d = np.array([np.cos(ang), np.sin(ang)], np.float32)
        s0 = _face_ray_label(o, g, pos, a, u, v, p0)
        s, q = o.line_binary(int(fid), p0, d, s0, R, n_lin, n_bin)
        # dense samples at a quarter of the final bracket
        dense = np.arange(0, 4 * n_lin * 2 ** n_bin + 1, dtype=np.float64) * (step / 4)
        labs = np.array([_face_ray_label(o, g, pos, a, u, v,
                                         (p0[0] + np.float32(t) * d[0], p0[1] + np.float32(t) * d[1]))
                         for t in dense])
        if np.all(labs == s0):
            misses += 1
            assert s == np.float32(R * (1 - 2.0 ** -n_bin / n_lin)), (int(fid), s)
            continue
        hits += 1
        first = dense[int(np.argmax(labs != s0))]
        assert s <= first <= s + step * (1 + 1e-5) + step / 4, (int(fid), s, first)
    assert hits > 5 and misses > 0


def test_step1_goes_to_the_cut_off_corner(oracle_mod):
    """R9 on a constructed checkerboard face.  Face z = 0 of the 4^3 grid over
    [-0.5, 0.5]^3 at corner (1, 1, 2): face-local (u, v) = (x, y), corners
    c0 = (0,0) and c3 = (1,1) inside, c1 and c2 outside.  Inside near c0 is
    an L of two thin slabs along the face's edges (u < 1/2, v < eps) and
    (u < eps, v < 1/2), so the chord between the crossings (1/2, 0) and
    (0, 1/2) has its midpoint outside.  Both sides of the chord then hold a
    corner whose label differs from m's (c0, and c3 inside a small sphere),
    and the search must go towards c0, the corner the pair cuts off: its
    2D point is then the L's reflex corner (eps, eps), within the searches'
    resolution.  The other side would end near c3's sphere."""
    h, eps = 0.25, 0.05
    x0, y0 = -0.25, -0.25                   # world position of c0
    B1 = I.box_record((x0 + h * 0.0, y0 + h * (eps - 0.5) / 2, 0.0),
                      (h * 0.5, h * (eps + 0.5) / 2, 0.05))
    B2 = I.box_record((x0 + h * (eps - 0.5) / 2, y0 + h * 0.0, 0.0),
                      (h * (eps + 0.5) / 2, h * 0.5, 0.05))
    S3 = I.sphere_record((0.0, 0.0, 0.0), 0.3 * h)
    f = I.csg_field([B1, B2, S3])
    g = I.unit_grid(4, 15)
    o = oracle_mod.Oracle(f, g)
    N = g.res
    fid = 2 * (N + 1) * N * N + 1 + N * (1 + N * 2)   # normal z, min corner (1, 1, 2)
    n, pf, info, tie = o.pair_point(fid, 0)
    assert n == 2 and tie == 0
    assert (info >> 14) & 1                             # ambiguous face
    assert ((info >> 4) & 15, (info >> 8) & 15) == (0, 2)  # the pair around c0
    assert not (info >> 13) & 1                         # q moved off m
    assert np.all(np.abs(pf - eps) < 2e-4), pf
    # the other pair, around c3, ends on c3's sphere
    n, pf3, info3, _ = o.pair_point(fid, 1)
    assert np.linalg.norm(pf3 - 1.0) < 0.31


def test_manifold_fix_through_the_oracle(oracle_mod):
    """Two x-adjacent cells of a 2^3 grid with labels given for their 12
    corners (others outside): the oracle flips their shared ambiguous face
    exactly when both cells' plain partitions merge its two pairs (18 of the
    512 blocks), and afterwards no block has the pairs merged in both."""
    N = 2
    g = I.unit_grid(N, 8)
    dummy = I.csg_field([I.sphere_record((9.0, 9.0, 9.0), 0.1)])

    def merged(pm, side):
        e0 = 4 * 1 + side + 2 * 0   # y-edges of the x-face at x = side
        e1 = 4 * 1 + side + 2 * 1
        return ((pm >> (2 * e0)) & 3) == ((pm >> (2 * e1)) & 3)

    flips = bad_after = blocks = 0
    for code in range(1 << 12):
        lab = np.zeros((N + 1, N + 1, N + 1), np.uint8)   # [z][y][x]
        for n in range(12):
            x, y, z = n % 3, (n // 3) % 2, n // 6
            lab[z, y, x] = (code >> n) & 1
        L = [lab[0, 0, 1], lab[0, 1, 1], lab[1, 0, 1], lab[1, 1, 1]]
        if not (L[0] == L[3] != L[1] == L[2]):
            continue
        blocks += 1
        cfgA = sum(int(lab[c >> 2, (c >> 1) & 1, c & 1]) << c for c in range(8))
        cfgB = sum(int(lab[c >> 2, (c >> 1) & 1, 1 + (c & 1)]) << c for c in range(8))
        bad = merged(oracle_mod.cube_partitions(cfgA, 0)[1], 1) and \
            merged(oracle_mod.cube_partitions(cfgB, 0)[1], 0)
        words = np.packbits(lab.reshape(-1), bitorder="little")
        words = np.pad(words, (0, (-len(words)) % 4)).view(np.uint32)
        tr = oracle_mod.Trace(label_words=words, labels_given=True)
        m = oracle_mod.Oracle(dummy, g, trace=tr, topology_only=True).mesh()
        cells = {int(c): k for k, c in enumerate(m["cell_id"])}
        a, b = cells[0], cells[1]                 # cells (0,0,0) and (1,0,0)
        fa = (int(m["cell_flipmask"][a]) >> 1) & 1  # local face x side 1
        fb = int(m["cell_flipmask"][b]) & 1         # local face x side 0
        assert fa == fb == int(bad), code
        flips += fa
        bad_after += merged(int(m["cell_partmap"][a]), 1) and merged(int(m["cell_partmap"][b]), 0)
    assert blocks == 512 and flips == 18 and bad_after == 0
