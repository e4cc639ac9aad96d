"""Pins of the mesh measurement helpers used by the parity tests and the
benchmark (point-to-surface Chamfer distance)."""
import numpy as np

import meshcheck as M


def _square():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    t = np.array([[0, 1, 2], [1, 3, 2]])
    return v, t


def test_closest_point_never_beaten_by_dense_sampling():
    rng = np.random.default_rng(1)
    a, b, c = rng.random((3, 300, 3))
    p = rng.random((300, 3)) * 2 - 0.5
    q = M._closest_on_triangles(p, a, b, c)
    d = np.linalg.norm(p - q, axis=1)
    u = rng.random((4000, 2))
    flip = u.sum(1) > 1
    u[flip] = 1 - u[flip]
    for i in range(300):
        s = a[i] + (b[i] - a[i]) * u[:, :1] + (c[i] - a[i]) * u[:, 1:]
        assert d[i] <= np.min(np.linalg.norm(s - p[i], axis=1)) + 1e-12


def test_chamfer_identity_and_offset():
    v, t = _square()
    assert M.chamfer_h2(v, t, v, t, 1.0, n=5000) < 1e-28
    # a parallel plane 0.01 away: every sample is exactly 0.01 from the other surface
    assert abs(M.chamfer_h2(v, t, v + [0, 0, 0.01], t, 1.0, n=5000) - 1e-4) < 1e-12
    # units of h^2
    assert abs(M.chamfer_h2(v, t, v + [0, 0, 0.01], t, 0.1, n=5000) - 1e-2) < 1e-10


def test_chamfer_sphere_shift():
    """A closed sphere mesh shifted by s along z: squared distances average
    s^2 <n_z^2> = s^2 / 3 to first order."""
    n = 40
    th, ph = np.meshgrid(np.linspace(0, np.pi, n), np.linspace(0, 2 * np.pi, 2 * n, endpoint=False),
                         indexing="ij")
    v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1).reshape(-1, 3)
    idx = np.arange(n * 2 * n).reshape(n, 2 * n)
    tris = []
    for i in range(n - 1):
        for j in range(2 * n):
            a, b = idx[i, j], idx[i, (j + 1) % (2 * n)]
            c, d = idx[i + 1, j], idx[i + 1, (j + 1) % (2 * n)]
            tris += [[a, c, b], [b, c, d]]
    t = np.array(tris)
    s = 1e-3
    ch = M.chamfer_h2(v, t, v + [0, 0, s], t, 1.0, n=20000)
    assert abs(ch / (s * s) - 1.0 / 3.0) < 0.03, ch / (s * s)
