"""ctypes binding of the CPU oracle (odc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "odc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra"]


def build(force: bool = False, out: str = _LIB, extra=()) -> str:
    """Compile liboracle.so with gcc (always when force); `out` and `extra`
    flags build another copy (the sanitizer test's)."""
    if out != _LIB:
        subprocess.check_call(["gcc", *_CFLAGS, *extra, "-o", out, _SRC, "-lm"])
        return out
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "odc_oracle.h"))):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("prims", C.POINTER(C.c_float)), ("n_prims", C.c_int),
                ("weights", C.POINTER(C.c_float)), ("in_dim", C.c_int), ("width", C.c_int),
                ("depth", C.c_int), ("n_bands", C.c_int), ("spheres", C.POINTER(C.c_float)),
                ("n_spheres", C.c_int), ("sdf_gain", C.c_double), ("out_scale", C.c_double),
                ("mlp_tie_eps", C.c_double)]


class _Trace(C.Structure):
    _fields_ = [("label_words", C.POINTER(C.c_uint32)), ("labels_given", C.c_int),
                ("n_edges", C.c_int64), ("edge_id", C.POINTER(C.c_int32)),
                ("edge_bits", C.POINTER(C.c_uint32)), ("edge_t", C.POINTER(C.c_float)),
                ("n_pairs", C.c_int64), ("pair_rec", C.POINTER(C.c_int32)),
                ("pair_bits", C.POINTER(C.c_uint64)), ("pair_pf", C.POINTER(C.c_double)),
                ("edge_grad", C.POINTER(C.c_float)), ("staged", C.c_int), ("adopted", C.c_int64), ("mismatched", C.c_int64),
                ("unmatched", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("size", C.c_double), ("res", C.c_int),
                ("iters_1d", C.c_int), ("lin1", C.c_int), ("bin1", C.c_int), ("lin2", C.c_int),
                ("bin2", C.c_int), ("range1", C.c_float), ("range2", C.c_float),
                ("qef_tau", C.c_double), ("ic_tie_tol", C.c_double), ("n_threads", C.c_int),
                ("ablation", C.c_int), ("clamp", C.c_int), ("topology_only", C.c_int),
                ("trace", C.POINTER(_Trace))]


class Trace:
    """An implementation's recorded occupancy decisions for a replayed oracle
    run (orc_trace in odc_oracle.h): its corner label words, its crossing
    edges with the bisection labels, its pairs with the 2D-search labels and
    evaluated masks, and (staged) its 1D and 2D points.  Where the oracle's
    own decision is a near-tie it follows the recorded branch; elsewhere it
    counts disagreements (`mismatched`, which must stay 0)."""

    def __init__(self, label_words=None, edge_ids=None, edge_bits=None, edge_t=None,
                 pair_rec=None, pair_bits=None, pair_pf=None, staged=False,
                 labels_given=False, edge_grad=None):
        def keep(a, dt):
            return None if a is None else np.ascontiguousarray(a, dt)
        self._a = {"label_words": keep(label_words, np.uint32),
                   "edge_id": keep(edge_ids, np.int32), "edge_bits": keep(edge_bits, np.uint32),
                   "edge_t": keep(edge_t, np.float32), "pair_rec": keep(pair_rec, np.int32),
                   "pair_bits": keep(pair_bits, np.uint64), "pair_pf": keep(pair_pf, np.float64),
                   "edge_grad": keep(edge_grad, np.float32)}
        t = _Trace()
        ctypes_of = {"label_words": C.c_uint32, "edge_id": C.c_int32, "edge_bits": C.c_uint32,
                     "edge_t": C.c_float, "pair_rec": C.c_int32, "pair_bits": C.c_uint64,
                     "pair_pf": C.c_double, "edge_grad": C.c_float}
        for k, a in self._a.items():
            if a is not None:
                setattr(t, k, a.ctypes.data_as(C.POINTER(ctypes_of[k])))
        t.labels_given = int(bool(labels_given))
        t.staged = int(bool(staged))
        t.n_edges = 0 if self._a["edge_id"] is None else len(self._a["edge_id"])
        t.n_pairs = 0 if self._a["pair_rec"] is None else len(self._a["pair_rec"])
        self.t = t

    @property
    def adopted(self):
        return int(self.t.adopted)

    @property
    def mismatched(self):
        return int(self.t.mismatched)

    @property
    def unmatched(self):
        return int(self.t.unmatched)

    def reset(self):
        self.t.adopted = self.t.mismatched = self.t.unmatched = 0


_P = C.POINTER
_MESH_FIELDS = [
    ("res", C.c_int),
    ("n_corners", C.c_int64), ("corner_label", _P(C.c_uint8)), ("corner_tie", _P(C.c_uint8)),
    ("n_edges", C.c_int64), ("edge_id", _P(C.c_int32)), ("edge_t", _P(C.c_double)),
    ("edge_tie_step", _P(C.c_int32)), ("edge_bits", _P(C.c_uint32)),
    ("n_pairs", C.c_int64), ("pair_face", _P(C.c_int32)), ("pair_info", _P(C.c_int32)),
    ("pair_pf", _P(C.c_double)), ("pair_tie", _P(C.c_uint8)), ("pair_sin", _P(C.c_double)),
    ("pair_bits", _P(C.c_uint64)),
    ("n_flipped_faces", C.c_int64),
    ("n_cells", C.c_int64), ("cell_id", _P(C.c_int32)), ("cell_npart", _P(C.c_int32)),
    ("cell_partmap", _P(C.c_int32)), ("cell_flipmask", _P(C.c_int32)),
    ("cell_vbase", _P(C.c_int32)), ("cell_tie", _P(C.c_uint8)),
    ("n_vertices", C.c_int64), ("vert", _P(C.c_double)), ("vert_tie", _P(C.c_uint8)),
    ("vert_kappa", _P(C.c_double)),
    ("vert_gap", _P(C.c_double)),
    ("edge_case", _P(C.c_int32)), ("edge_case_tie", _P(C.c_uint8)),
    ("n_case3", C.c_int64), ("n_tris", C.c_int64), ("tris", _P(C.c_int32)),
]


class _Mesh(C.Structure):
    _fields_ = _MESH_FIELDS


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ODC_ORACLE_LIB: a differently built copy (the sanitizer test's)
        path = os.environ.get("ODC_ORACLE_LIB") or build()
        _lib = C.CDLL(path)
        L = _lib
        L.orc_mesh_extract.argtypes = [_P(_Field), _P(_Params), _P(_Mesh)]
        L.orc_mesh_extract.restype = C.c_int
        L.orc_mesh_free.argtypes = [_P(_Mesh)]
        L.orc_label_world.argtypes = [_P(_Field), _P(C.c_float), _P(C.c_int), _P(C.c_double)]
        L.orc_label_world.restype = C.c_int
        L.orc_corner_label.argtypes = [_P(_Field), _P(_Params), C.c_int, C.c_int, C.c_int,
                                       _P(C.c_int)]
        L.orc_corner_label.restype = C.c_int
        L.orc_edge_point.argtypes = [_P(_Field), _P(_Params), C.c_int64, _P(C.c_int)]
        L.orc_edge_point.restype = C.c_double
        L.orc_pair_point.argtypes = [_P(_Field), _P(_Params), C.c_int64, C.c_int,
                                     _P(C.c_double), _P(C.c_int), _P(C.c_int)]
        L.orc_pair_point.restype = C.c_int
        L.orc_cell_vertices.argtypes = [_P(_Field), _P(_Params), C.c_int64, _P(C.c_double),
                                        _P(C.c_int), _P(C.c_int), _P(C.c_double)]
        L.orc_cell_vertices.restype = C.c_int
        L.orc_line_binary.argtypes = [_P(_Field), _P(_Params), C.c_int64, _P(C.c_float),
                                      _P(C.c_float), C.c_int, C.c_float, C.c_int, C.c_int,
                                      _P(C.c_float), _P(C.c_int)]
        L.orc_line_binary.restype = C.c_float
        L.orc_logit_grad.argtypes = [_P(_Field), _P(C.c_double), _P(C.c_double), _P(C.c_double)]
        L.orc_logit_grad.restype = C.c_double
        L.orc_self_intersections.argtypes = [_P(C.c_float), C.c_int64, _P(C.c_int32), C.c_int64]
        L.orc_self_intersections.restype = C.c_int64
        L.orc_cube_partitions.argtypes = [C.c_int, C.c_int, _P(C.c_int)]
        L.orc_cube_partitions.restype = C.c_int
        L.orc_qef_solve.argtypes = [C.c_int, _P(C.c_double), C.c_double, _P(C.c_double),
                                    _P(C.c_double)]
        L.orc_ic_case.argtypes = [_P(C.c_double), _P(C.c_double), _P(C.c_double), C.c_double,
                                  _P(C.c_int)]
        L.orc_ic_case.restype = C.c_int
    return _lib


def _fptr(a):
    return a.ctypes.data_as(_P(C.c_float)) if a is not None else None


class Oracle:
    """Holds one field and one grid; keeps the numpy buffers alive."""

    def __init__(self, field, grid, mlp_tie_eps: float = 1e-4, ic_tie_tol: float = 1e-5,
                 n_threads: int = 0, trace: "Trace | None" = None, topology_only: bool = False):
        self.field = field
        self.grid = grid
        self._prims = None if field.prims is None else np.ascontiguousarray(field.prims, np.float32)
        self._w = None if field.weights is None else np.ascontiguousarray(field.weights, np.float32)
        self._s = None if field.spheres is None else np.ascontiguousarray(field.spheres, np.float32)
        self.f = _Field(field.kind, _fptr(self._prims),
                        0 if self._prims is None else self._prims.shape[0], _fptr(self._w),
                        field.in_dim, field.width, field.depth, field.n_bands, _fptr(self._s),
                        0 if self._s is None else self._s.shape[0], field.sdf_gain,
                        field.out_scale, mlp_tie_eps)
        self.p = _Params((C.c_double * 3)(*grid.lo), grid.size, grid.res, grid.iters_1d,
                         grid.lin1, grid.bin1, grid.lin2, grid.bin2, grid.range1, grid.range2,
                         grid.qef_tau, ic_tie_tol, n_threads, getattr(grid, "ablation", 0),
                         getattr(grid, "clamp", 0), int(bool(topology_only)),
                         C.pointer(trace.t) if trace is not None else None)
        self.trace = trace

    def mesh(self) -> dict:
        m = _Mesh()
        rc = lib().orc_mesh_extract(C.byref(self.f), C.byref(self.p), C.byref(m))
        if rc != 0:
            raise ValueError(f"oracle rejected the input ({rc})")
        try:
            out = {"res": m.res, "n_flipped_faces": m.n_flipped_faces, "n_case3": m.n_case3}

            def grab(name, n, cols=1):
                ptr = getattr(m, name)
                if n == 0:
                    ctype = ptr._type_
                    return np.zeros((0, cols) if cols > 1 else 0, np.ctypeslib.as_array(
                        (ctype * 1)()).dtype)
                a = np.ctypeslib.as_array(ptr, shape=(n * cols,)).copy()
                return a.reshape(n, cols) if cols > 1 else a

            out["corner_label"] = grab("corner_label", m.n_corners)
            out["corner_tie"] = grab("corner_tie", m.n_corners)
            for k in ("edge_id", "edge_t", "edge_tie_step", "edge_case", "edge_case_tie",
                      "edge_bits"):
                out[k] = grab(k, m.n_edges)
            out["pair_bits"] = grab("pair_bits", m.n_pairs, 2)
            for k in ("pair_face", "pair_info", "pair_tie", "pair_sin"):
                out[k] = grab(k, m.n_pairs)
            out["pair_pf"] = grab("pair_pf", m.n_pairs, 2)
            for k in ("cell_id", "cell_npart", "cell_partmap", "cell_flipmask", "cell_vbase",
                      "cell_tie"):
                out[k] = grab(k, m.n_cells)
            out["vert"] = grab("vert", m.n_vertices, 3)
            out["vert_tie"] = grab("vert_tie", m.n_vertices)
            out["vert_kappa"] = grab("vert_kappa", m.n_vertices)
            out["vert_gap"] = grab("vert_gap", m.n_vertices)
            out["tris"] = grab("tris", m.n_tris, 3)
        finally:
            lib().orc_mesh_free(C.byref(m))
        return out

    # single elements -------------------------------------------------------
    def label_world(self, xyz):
        x = np.asarray(xyz, np.float32)
        tie = C.c_int()
        mg = C.c_double()
        lab = lib().orc_label_world(C.byref(self.f), _fptr(x), C.byref(tie), C.byref(mg))
        return lab, tie.value, mg.value

    def corner_label(self, i, j, k):
        tie = C.c_int()
        return lib().orc_corner_label(C.byref(self.f), C.byref(self.p), i, j, k,
                                      C.byref(tie)), tie.value

    def edge_point(self, eid):
        ts = C.c_int()
        t = lib().orc_edge_point(C.byref(self.f), C.byref(self.p), int(eid), C.byref(ts))
        return t, ts.value

    def pair_point(self, fid, slot):
        pf = (C.c_double * 2)()
        info = C.c_int()
        tie = C.c_int()
        n = lib().orc_pair_point(C.byref(self.f), C.byref(self.p), int(fid), int(slot), pf,
                                 C.byref(info), C.byref(tie))
        return n, np.array(pf[:]), info.value, tie.value

    def cell_vertices(self, cid):
        v = (C.c_double * 12)()
        pm = C.c_int()
        tie = C.c_int()
        kap = (C.c_double * 4)()
        n = lib().orc_cell_vertices(C.byref(self.f), C.byref(self.p), int(cid), v,
                                    C.byref(pm), C.byref(tie), kap)
        return n, np.array(v[:3 * n]).reshape(n, 3), pm.value, tie.value

    def logit_grad(self, x, with_margin=False):
        """Binary64 logit and gradient at a binary64 point (MLP fields); with
        with_margin also (nearest-sphere gap, smallest |ReLU input|)."""
        xd = (C.c_double * 3)(*[float(v) for v in x])
        g = (C.c_double * 3)()
        mg = (C.c_double * 2)()
        z = lib().orc_logit_grad(C.byref(self.f), xd, g, mg)
        if with_margin:
            return z, np.array(g[:]), (mg[0], mg[1])
        return z, np.array(g[:])

    def line_binary(self, fid, p0, d, s0, rng, n_lin, n_bin):
        a = np.asarray(p0, np.float32)
        b = np.asarray(d, np.float32)
        q = (C.c_float * 2)()
        tie = C.c_int()
        s = lib().orc_line_binary(C.byref(self.f), C.byref(self.p), int(fid), _fptr(a), _fptr(b),
                                  int(s0), float(rng), int(n_lin), int(n_bin), q, C.byref(tie))
        return s, np.array(q[:], np.float32)


def cube_partitions(config: int, flipmask: int = 0):
    pm = C.c_int()
    n = lib().orc_cube_partitions(int(config), int(flipmask), C.byref(pm))
    return n, pm.value


def qef_solve(normals, points, tau=1e-2):
    n = len(normals)
    pl = np.zeros((max(n, 1), 6))
    if n:
        pl[:n, :3] = normals
        pl[:n, 3:] = points
    pl = np.ascontiguousarray(pl)
    out = (C.c_double * 3)()
    kap = C.c_double()
    lib().orc_qef_solve(n, pl.ctypes.data_as(_P(C.c_double)), tau, out, C.byref(kap))
    return np.array(out[:]), kap.value


def ic_case(quad, pin, pout, tol=0.0):
    q = np.ascontiguousarray(quad, np.float64)
    a = np.ascontiguousarray(pin, np.float64)
    b = np.ascontiguousarray(pout, np.float64)
    tie = C.c_int()
    c = lib().orc_ic_case(q.ctypes.data_as(_P(C.c_double)), a.ctypes.data_as(_P(C.c_double)),
                          b.ctypes.data_as(_P(C.c_double)), tol, C.byref(tie))
    return c, tie.value


def self_intersections(vertices, tris) -> int:
    """Pairs of vertex-disjoint triangles that intersect (brute force)."""
    v = np.ascontiguousarray(vertices, np.float32)
    t = np.ascontiguousarray(tris, np.int32)
    return int(lib().orc_self_intersections(v.ctypes.data_as(_P(C.c_float)), len(v),
                                            t.ctypes.data_as(_P(C.c_int32)), len(t)))
