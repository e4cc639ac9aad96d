"""Pins of the oracle's ablation baselines (Table 3; CPU only): Manifold Dual
Contouring's linear 1D points (Eq. 1), gradient normals (Eq. 2) and plain
two-triangle split, each replacing one step of the method."""
import math

import numpy as np

import odc_inputs as I
import meshcheck as M


def _biased_mlp(seed=7, width=32, depth=3, n_bands=2):
    """A small MLP field with non-zero biases (so the ReLU masks differ from
    the sign of W h alone)."""
    f = I.mlp_field(seed, n_spheres=4, width=width, depth=depth, n_bands=n_bands)
    w = f.weights.astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    off, fan = 0, f.in_dim
    for _ in range(depth):
        off += width * fan
        w[off:off + width] = rng.normal(0.0, 0.3, width)
        off += width
        fan = width
    f.weights = w.astype(np.float32)
    return f


def _sphere_only(c, r, gain):
    """An MLP field whose network is zero: z = -gain * (|x - c| - r)."""
    f = I.mlp_field(1, n_spheres=1, width=8, depth=2, n_bands=1, sdf_gain=gain)
    f.weights = np.zeros_like(f.weights)
    f.spheres = np.array([[c[0], c[1], c[2], r]], np.float32)
    return f


def test_gradient_matches_central_differences(oracle_mod):
    f = _biased_mlp()
    o = oracle_mod.Oracle(f, I.unit_grid(8))
    rng = np.random.default_rng(3)
    checked = 0
    for x in rng.uniform(-0.45, 0.45, (60, 3)):
        z, g = o.logit_grad(x)
        fd = []
        for h in (1e-5, 5e-6):
            d = np.zeros(3)
            for a in range(3):
                e = np.zeros(3); e[a] = h
                d[a] = (o.logit_grad(x + e)[0] - o.logit_grad(x - e)[0]) / (2 * h)
            fd.append(d)
        if np.abs(fd[0] - fd[1]).max() > 1e-6 * (1 + np.abs(fd[1]).max()):
            continue  # a ReLU kink or the sdf's nearest-sphere switch within h
        assert np.abs(g - fd[1]).max() <= 1e-6 * (1 + np.abs(g).max()), (x, g, fd[1])
        checked += 1
    assert checked >= 50


def test_gradient_of_a_sphere_is_radial(oracle_mod):
    c, r, gain = np.array([0.03, -0.02, 0.01]), 0.3, 20.0
    o = oracle_mod.Oracle(_sphere_only(c, r, gain), I.unit_grid(8))
    rng = np.random.default_rng(4)
    for x in rng.uniform(-0.45, 0.45, (20, 3)):
        z, g = o.logit_grad(x)
        d = x - np.asarray(np.float32(c), np.float64)
        assert abs(z - (-gain * (np.linalg.norm(d) - np.float32(r)))) < 1e-12
        assert np.allclose(g, -gain * d / np.linalg.norm(d), atol=1e-12)


def test_linear_1d_points_on_a_near_plane(oracle_mod):
    """Eq. 1 on a field that is nearly linear across each edge (a sphere of
    radius R = 20 seen through a low gain): the linear 1D point is the true
    crossing up to the curvature of tanh (z/2 - tanh(z/2) < 4e-4 relative for
    |z| <= gain h) and of the distance along the edge (second derivative <=
    1/R, so a deviation <= h^2/(8R), divided by the edge's sdf change)."""
    c = np.array([20.05, 0.3, -0.2])
    f = _sphere_only(c, 20.0, 1.0)
    g = I.unit_grid(16)
    g.ablation = I.ABL_LINEAR_1D
    m = oracle_mod.Oracle(f, g).mesh()
    N, n1 = g.res, g.res + 1
    cf = np.asarray(np.float32(c), np.float64)
    rf = float(np.float32(20.0))
    assert len(m["edge_id"]) > 100
    far_from_mid = 0
    for e, t in zip(m["edge_id"], m["edge_t"]):
        ea = N * n1 * n1
        a, loc = int(e) // ea, int(e) % ea
        dims = [n1, n1, n1]
        dims[a] = N
        p = np.array([loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])], float)
        x0 = -0.5 + p * g.h
        d = np.zeros(3); d[a] = g.h
        # |x0 + s d - c| = r for s in [0, 1]
        A = d @ d; B = 2 * d @ (x0 - cf); Cc = (x0 - cf) @ (x0 - cf) - rf * rf
        roots = [(-B + sg * math.sqrt(B * B - 4 * A * Cc)) / (2 * A) for sg in (-1, 1)]
        s = min(roots, key=lambda q: abs(q - 0.5))
        dsdf = abs(np.linalg.norm(x0 + d - cf) - np.linalg.norm(x0 - cf))
        bound = 1e-3 + g.h ** 2 / (4 * rf) / dsdf
        assert abs(t - s) <= bound, (int(e), t, s, bound)
        far_from_mid += abs(t - 0.5) > 0.1
    assert far_from_mid > 10


def test_linear_1d_points_of_csg_are_midpoints(oracle_mod):
    g = I.unit_grid(12)
    g.ablation = I.ABL_LINEAR_1D
    m = oracle_mod.Oracle(I.csg_random_field(2), g).mesh()
    assert len(m["edge_t"]) > 0 and np.all(m["edge_t"] == 0.5)


def test_mdc_split_keeps_vertices_and_pairs_quads(oracle_mod):
    f = I.csg_random_field(2)
    g0 = I.unit_grid(16)
    g4 = I.unit_grid(16)
    g4.ablation = I.ABL_MDC_SPLIT
    m0 = oracle_mod.Oracle(f, g0).mesh()
    m4 = oracle_mod.Oracle(f, g4).mesh()
    nvp = int(m0["cell_npart"].sum())
    assert np.array_equal(m4["vert"], m0["vert"][:nvp])
    assert m4["n_case3"] == 0 and set(np.unique(m4["edge_case"])) <= {0, 1}
    assert len(m4["tris"]) == 2 * int(np.sum(m4["edge_case"] == 1))
    assert len(m4["tris"]) == 2 * int(np.sum(m0["edge_case"] != 0))
    ok, why = M.is_closed_oriented_manifold(m4["tris"], len(m4["vert"]))
    assert ok, why


def _plane_mlp(n, d, width=8, depth=3, n_bands=1):
    """An MLP field whose logit is exactly n.x - d on the unit cube: neuron 0
    carries n.x + 1 (> 0 there) through every layer, the rest are zero."""
    in_dim = 3 + 6 * n_bands
    parts = []
    W1 = np.zeros((width, in_dim)); W1[0, :3] = n
    b1 = np.zeros(width); b1[0] = 1.0
    parts += [W1, b1]
    for _ in range(depth - 1):
        Wh = np.zeros((width, width)); Wh[0, 0] = 1.0
        parts += [Wh, np.zeros(width)]
    wo = np.zeros(width); wo[0] = 1.0
    parts += [wo, np.array([-1.0 - d])]
    w = np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)
    return I.Field(kind=I.FIELD_MLP, weights=w, in_dim=in_dim, width=width, depth=depth,
                   n_bands=n_bands, spheres=np.array([[0.0, 0.0, 0.0, 0.1]], np.float32),
                   sdf_gain=0.0, out_scale=1.0)


def test_gradient_normals_recover_a_plane(oracle_mod):
    """The gradient of a linear logit is its normal everywhere, so every plane
    of the QEF is the surface and each 3D point is the mass point of its 1D
    points projected onto it: on the plane up to the 1D points' own error
    (2^-16 h after 15 bisection steps)."""
    n = np.array([0.48, 0.6, 0.64])
    nf = n.astype(np.float32).astype(np.float64)
    f = _plane_mlp(n, 0.05)
    o = oracle_mod.Oracle(f, I.unit_grid(8))
    z, gr = o.logit_grad([0.1, -0.2, 0.3])
    assert np.allclose(gr, nf, atol=1e-15)
    g = I.unit_grid(12)
    g.ablation = I.ABL_GRAD_NORMALS
    m = oracle_mod.Oracle(f, g).mesh()
    world = -0.5 + m["vert"] * g.h
    assert len(world) > 50
    dist = np.abs(world @ nf - 0.05) / np.linalg.norm(nf)
    assert dist.max() < 2.0 ** -15 * g.h


def test_gradient_normals_need_an_mlp_field(oracle_mod):
    g = I.unit_grid(8)
    g.ablation = I.ABL_GRAD_NORMALS
    try:
        oracle_mod.Oracle(I.csg_random_field(2), g).mesh()
    except ValueError:
        return
    raise AssertionError("CSG field with gradient normals was accepted")


def test_clamped_vertices_are_the_projection(oracle_mod):
    """The clamp option moves each partition vertex to the nearest point of its
    cell and nothing else: vertices inside stay, the rest are projected."""
    f = I.mlp_field(3)
    g0 = I.unit_grid(16)
    g1 = I.unit_grid(16)
    g1.clamp = 1
    m0 = oracle_mod.Oracle(f, g0, mlp_tie_eps=1e-5).mesh()
    m1 = oracle_mod.Oracle(f, g1, mlp_tie_eps=1e-5).mesh()
    nvp = int(m0["cell_npart"].sum())
    N = g0.res
    owner = np.searchsorted(m0["cell_vbase"], np.arange(nvp), side="right") - 1
    cid = m0["cell_id"][owner]
    c = np.stack([cid % N, (cid // N) % N, cid // (N * N)], 1).astype(float)
    assert np.array_equal(m1["vert"][:nvp], np.clip(m0["vert"][:nvp], c, c + 1))
    outside = np.any((m0["vert"][:nvp] < c) | (m0["vert"][:nvp] > c + 1), axis=1)
    assert outside.sum() > 0


def test_sdf_input_interpolates_the_distance(oracle_mod):
    """SDF input: the logit of a sphere field with gain 1 is minus its signed
    distance, and Eq. 1 on that distance is exact up to the distance's
    curvature along the edge (no tanh term)."""
    c = np.array([20.05, 0.3, -0.2])
    f = _sphere_only(c, 20.0, 1.0)
    g = I.unit_grid(16)
    g.ablation = I.ABL_LINEAR_1D | I.ABL_SDF_INPUT
    m = oracle_mod.Oracle(f, g).mesh()
    N, n1 = g.res, g.res + 1
    cf = np.asarray(np.float32(c), np.float64)
    rf = float(np.float32(20.0))
    for e, t in zip(m["edge_id"], m["edge_t"]):
        ea = N * n1 * n1
        a, loc = int(e) // ea, int(e) % ea
        dims = [n1, n1, n1]
        dims[a] = N
        p = np.array([loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])], float)
        x0 = -0.5 + p * g.h
        d = np.zeros(3); d[a] = g.h
        A = d @ d; B = 2 * d @ (x0 - cf); Cc = (x0 - cf) @ (x0 - cf) - rf * rf
        s = min([(-B + sg * math.sqrt(B * B - 4 * A * Cc)) / (2 * A) for sg in (-1, 1)],
                key=lambda q: abs(q - 0.5))
        dsdf = abs(np.linalg.norm(x0 + d - cf) - np.linalg.norm(x0 - cf))
        assert abs(t - s) <= 1e-9 + g.h ** 2 / (4 * rf) / dsdf, (int(e), t, s)
    # without the linear mode the flag is rejected
    g2 = I.unit_grid(8)
    g2.ablation = I.ABL_SDF_INPUT
    try:
        oracle_mod.Oracle(f, g2).mesh()
    except ValueError:
        return
    raise AssertionError("SDF input without linear 1D points was accepted")


def test_sdf_input_gives_the_occupancy_mesh(oracle_mod):
    """SDF input (s = [psi < 0]): the method reads only the sign of the field,
    so a signed-distance field and an occupancy field with the same zero set
    give the same mesh.  sdf_mlp_field's logit is mlp_field's divided by 20
    (the scale factors round differently, but no decision of this grid falls
    between the two)."""
    g = I.unit_grid(16)
    mo = oracle_mod.Oracle(I.mlp_field(3), g, mlp_tie_eps=1e-6).mesh()
    ms = oracle_mod.Oracle(I.sdf_mlp_field(3), g, mlp_tie_eps=5e-8).mesh()
    # the tie margins scale with the field, so both flag the same decisions
    assert np.array_equal(mo["corner_tie"], ms["corner_tie"])
    assert np.array_equal(mo["corner_label"], ms["corner_label"])
    assert np.array_equal(mo["edge_id"], ms["edge_id"])
    assert np.array_equal(mo["edge_tie_step"], ms["edge_tie_step"])
    assert np.array_equal(mo["edge_t"], ms["edge_t"])
    assert np.array_equal(mo["tris"], ms["tris"])
    assert np.array_equal(mo["pair_pf"], ms["pair_pf"])
    assert np.array_equal(mo["vert_tie"], ms["vert_tie"])
    assert np.array_equal(mo["vert"], ms["vert"])
    # Eq. 1 on the two inputs: psi = z/20 linearly vs tanh(z/2)/2, so the
    # linear points differ, by at most the tanh curvature over an edge
    g1 = I.unit_grid(16)
    g1.ablation = I.ABL_LINEAR_1D
    g2 = I.unit_grid(16)
    g2.ablation = I.ABL_LINEAR_1D | I.ABL_SDF_INPUT
    lo = oracle_mod.Oracle(I.mlp_field(3), g1, mlp_tie_eps=1e-6).mesh()
    ls = oracle_mod.Oracle(I.sdf_mlp_field(3), g2, mlp_tie_eps=5e-8).mesh()
    assert np.array_equal(lo["edge_id"], ls["edge_id"])
    d = np.abs(lo["edge_t"] - ls["edge_t"])
    assert d.max() > 1e-6 and d.max() < 0.5
