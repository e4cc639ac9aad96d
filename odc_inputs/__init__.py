"""Seeded synthetic occupancy fields and grids.

The only module shared by the GPU path's callers and the CPU oracle: it draws
field *data* (primitive records, network weights, grid bounds) and holds none
of the meshing arithmetic.  Every array is float32 in the layouts below.

CSG primitive record (20 float32):
    [0] op   0 union, 1 subtract, 2 intersect (left fold; the first op is ignored)
    [1] type 0 sphere, 1 box, 2 half-space
    [2:5]  centre c
    [5:8]  sphere: radius at [5]; box: half extents; half-space: outward normal
    [8:17] box rotation rows R (box-local = R (x - c))
    [17:20] unused

MLP weights (float32, concatenated):
    W1[width][in_dim], b1[width], then for each further hidden layer
    W[width][width], b[width], then w_out[width], b_out[1].
    in_dim = 3 + 6 * n_bands: (x, sin(2^k pi x), cos(2^k pi x)) per band k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PRIM_FLOATS = 20
OP_UNION, OP_SUBTRACT, OP_INTERSECT = 0, 1, 2
PRIM_SPHERE, PRIM_BOX, PRIM_HALFSPACE = 0, 1, 2
FIELD_CSG, FIELD_MLP = 0, 1
# ablation baselines (Table 3): linear 1D points, gradient normals, 2-triangle split
ABL_LINEAR_1D, ABL_GRAD_NORMALS, ABL_MDC_SPLIT, ABL_SDF_INPUT = 1, 2, 4, 8


@dataclasses.dataclass
class Field:
    kind: int
    prims: np.ndarray | None = None          # (n, 20) float32
    weights: np.ndarray | None = None        # flat float32
    in_dim: int = 0
    width: int = 0
    depth: int = 0
    n_bands: int = 0
    spheres: np.ndarray | None = None        # (n, 4) float32
    sdf_gain: float = 0.0
    out_scale: float = 0.0
    name: str = ""


@dataclasses.dataclass
class Grid:
    lo: tuple
    size: float
    res: int
    iters_1d: int = 15
    lin1: int = 4
    bin1: int = 11
    lin2: int = 3
    bin2: int = 12
    range1: float = 0.8
    range2: float = math.sqrt(2.0) / 2.0
    qef_tau: float = 1e-2
    ablation: int = 0   # 0 = the method; bits 1, 2, 4 = the Table 3 baselines
    clamp: int = 0      # 1 = clamp each 3D point into its cell (not the method's reading)

    @property
    def h(self) -> float:
        return self.size / self.res


def unit_grid(res: int, iters_1d: int = 15) -> Grid:
    """[-0.5, 0.5]^3 with `res` cells per axis."""
    return Grid(lo=(-0.5, -0.5, -0.5), size=1.0, res=res, iters_1d=iters_1d)


def _rec(op, typ, c, a=(0.0, 0.0, 0.0), R=None):
    r = np.zeros(PRIM_FLOATS, np.float32)
    r[0], r[1] = op, typ
    r[2:5] = c
    r[5:8] = a
    r[8:17] = (np.eye(3) if R is None else np.asarray(R)).reshape(-1)
    return r


def sphere_record(c, radius, op=OP_UNION):
    return _rec(op, PRIM_SPHERE, c, (radius, 0.0, 0.0))


def box_record(c, half, R=None, op=OP_UNION):
    return _rec(op, PRIM_BOX, c, half, R)


def halfspace_record(point, normal, op=OP_UNION):
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    return _rec(op, PRIM_HALFSPACE, point, n)


def csg_field(records, name="csg") -> Field:
    return Field(kind=FIELD_CSG, prims=np.stack(records).astype(np.float32), name=name)


def _rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def sphere_field() -> Field:
    """Single sphere |x - c| < 0.35, c = (0.03, -0.02, 0.01)."""
    return csg_field([sphere_record((0.03, -0.02, 0.01), 0.35)], name="sphere")


def sphere_case(res: int = 32, iters_1d: int = 10):
    return sphere_field(), unit_grid(res, iters_1d)


def csg_random_field(seed: int = 2, margin: float = 2.0 / 128) -> Field:
    """Union of 48 boxes (24 axis-aligned, 24 rotated; half extents
    U[0.03, 0.15]) and 16 spheres (r U[0.03, 0.12]), minus 8 boxes (half of
    them rotated).  Every added primitive stays `margin` inside [-0.5, 0.5]^3,
    so the surface is closed inside the domain."""
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(48):
        half = rng.uniform(0.03, 0.15, 3)
        if i < 24:
            lim = 0.5 - half - margin
            recs.append(box_record(rng.uniform(-lim, lim), half))
        else:
            R = _rotation(rng)
            lim = 0.5 - float(np.linalg.norm(half)) - margin
            recs.append(box_record(rng.uniform(-lim, lim, 3), half, R))
    for _ in range(16):
        r = rng.uniform(0.03, 0.12)
        lim = 0.5 - r - margin
        recs.append(sphere_record(rng.uniform(-lim, lim, 3), r))
    order = rng.permutation(len(recs))
    recs = [recs[i] for i in order]
    for _ in range(8):
        half = rng.uniform(0.03, 0.15, 3)
        R = _rotation(rng) if rng.uniform() < 0.5 else None
        recs.append(box_record(rng.uniform(-0.4, 0.4, 3), half, R, op=OP_SUBTRACT))
    return csg_field(recs, name=f"csg{seed}")


def mlp_field(seed: int = 3, n_spheres: int = 32, width: int = 256, depth: int = 4,
              n_bands: int = 6, out_scale: float = 0.3, sdf_gain: float = 20.0) -> Field:
    """phi = sigmoid(sdf_gain * (-sdf(x)) + out_scale * MLP(gamma(x))).

    sdf: union of `n_spheres` spheres, centres U[-0.3, 0.3]^3, r U[0.05, 0.15].
    MLP: gamma(x) (3 + 6 n_bands dims) -> depth x width ReLU -> 1, weights
    N(0, 2 / fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    sph = np.zeros((n_spheres, 4), np.float32)
    sph[:, :3] = rng.uniform(-0.3, 0.3, (n_spheres, 3))
    sph[:, 3] = rng.uniform(0.05, 0.15, n_spheres)
    in_dim = 3 + 6 * n_bands
    parts = []
    fan = in_dim
    for _ in range(depth):
        parts.append(rng.standard_normal((width, fan)) * math.sqrt(2.0 / fan))
        parts.append(np.zeros(width))
        fan = width
    parts.append(rng.standard_normal(width) * math.sqrt(2.0 / width))
    parts.append(np.zeros(1))
    w = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    return Field(kind=FIELD_MLP, weights=w, in_dim=in_dim, width=width, depth=depth,
                 n_bands=n_bands, spheres=sph, sdf_gain=sdf_gain, out_scale=out_scale,
                 name=f"mlp{seed}")


def sdf_mlp_field(seed: int = 3) -> Field:
    """A neural signed-distance input (DeepSDF-like): psi = sdf(x) - 0.015
    MLP(gamma(x)), with inside where psi < 0.  Its logit z = -psi is mlp_field's
    logit divided by 20, so the two fields share their zero set (up to the
    rounding of the two scale factors)."""
    f = mlp_field(seed, out_scale=0.015, sdf_gain=1.0)
    f.name = f"sdf{seed}"
    return f


def mlp_weight_count(in_dim: int, width: int, depth: int) -> int:
    return width * in_dim + width + (depth - 1) * (width * width + width) + width + 1


def batch_configs(n: int = 64, seed0: int = 4000):
    """Batched workload: seeds seed0..seed0+n-1, even -> CSG, odd -> MLP,
    resolutions drawn uniformly from {64, 96, 128, 192, 256}."""
    out = []
    for i in range(n):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        res = int(rng.choice([64, 96, 128, 192, 256]))
        field = csg_random_field(seed) if i % 2 == 0 else mlp_field(seed)
        out.append((field, unit_grid(res, 15)))
    return out


def serve_trace(n_requests: int = 1200, rate: float = 20.0, seed: int = 5):
    """Poisson arrivals: (arrival_s, kind, res, field_seed).  Kinds 50/50
    CSG/MLP; res in {64, 128, 256, 512} with weights 0.4/0.3/0.2/0.1."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    kinds = rng.integers(0, 2, n_requests)
    res = rng.choice([64, 128, 256, 512], n_requests, p=[0.4, 0.3, 0.2, 0.1])
    seeds = 100000 + np.arange(n_requests)
    return [(float(t[i]), int(kinds[i]), int(res[i]), int(seeds[i])) for i in range(n_requests)]
