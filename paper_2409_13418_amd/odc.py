"""Python binding of libodc.so (include/odc.h): argument marshalling only.

Every step of the meshing path runs in the HIP kernels of libodc.so; this
module moves field arrays to the device with PyTorch, fills the ABI structs
and calls the library.  It refuses to run without the built library.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libodc.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED, ERR_BUSY = range(7)
FIELD_CSG, FIELD_MLP = 0, 1
PREC_FP32, PREC_BF16_GUARDED, PREC_BF16_X3 = 0, 1, 2
INTERMEDIATES = {"labels": (0, np.uint32), "edge_ids": (1, np.int32), "edge_t": (2, np.float32),
                 "pairs": (3, np.int32), "pair_pf": (4, np.float64), "cell_ids": (5, np.int32),
                 "cell_partmap": (6, np.uint32), "cell_nf": (7, np.uint32),
                 "vertex_base": (8, np.int32), "edge_case": (9, np.int32),
                 "edge_grad": (10, np.float32), "edge_trace": (11, np.uint32),
                 "pair_trace": (12, np.uint64)}
_ELEM_BYTES = {"pair_pf": 16, "edge_grad": 12, "pair_trace": 16}
_COLS = {"pair_pf": 2, "edge_grad": 3, "pair_trace": 2}


class OdcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("prims", C.c_void_p), ("n_prims", C.c_int32),
                ("weights", C.c_void_p), ("in_dim", C.c_int32), ("width", C.c_int32),
                ("depth", C.c_int32), ("n_bands", C.c_int32), ("spheres", C.c_void_p),
                ("n_spheres", C.c_int32), ("sdf_gain", C.c_float), ("out_scale", C.c_float)]


class Params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("size", C.c_double), ("res", C.c_int32),
                ("iters_1d", C.c_int32), ("lin1", C.c_int32), ("bin1", C.c_int32),
                ("lin2", C.c_int32), ("bin2", C.c_int32), ("range1", C.c_float),
                ("range2", C.c_float), ("qef_tau", C.c_float), ("fp64_cond", C.c_double),
                ("precision", C.c_int32), ("guard_logit", C.c_float), ("ablation", C.c_int32),
                ("clamp_vertices", C.c_int32), ("coarse_step", C.c_int32),
                ("coarse_band", C.c_float)]


class MeshBuffers(C.Structure):
    _fields_ = [("vertices", C.c_void_p), ("cap_vertices", C.c_int64),
                ("triangles", C.c_void_p), ("cap_triangles", C.c_int64),
                ("vertices_local", C.c_void_p), ("vertex_ref", C.c_void_p)]


class MeshCounts(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_vertices", "n_triangles", "n_active_edges", "n_pairs", "n_active_cells", "n_case3",
        "n_flipped_faces", "n_fp64_cells", "n_guard_corners", "n_queries",
        "n_search2d_queries", "n_search2d_needed", "n_corner_queries")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


SERVE_FIFO, SERVE_SHORTEST, SERVE_BANDED = 0, 1, 2
ABL_LINEAR_1D, ABL_GRAD_NORMALS, ABL_MDC_SPLIT, ABL_SDF_INPUT = 1, 2, 4, 8


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("n_lanes", C.c_int32), ("max_batch", C.c_int32),
                ("max_batch_corners", C.c_int64), ("policy", C.c_int32), ("age_ms", C.c_float),
                ("band", C.c_float)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("attempts", C.c_int32), ("counts", MeshCounts),
                ("submit_ms", C.c_double), ("admit_ms", C.c_double), ("done_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "queued",
                                          "in_flight", "batches", "active_cells")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "window_s",
                                           "cells_per_s")] + \
               [("arena_bytes", C.c_int64), ("arena_peak_bytes", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


EXPORTS = ("odc_status_string", "odc_last_error", "odc_context_create", "odc_context_destroy",
           "odc_params_default", "odc_mesh_extract", "odc_mesh_sync", "odc_get_intermediate",
           "odc_context_set_timing", "odc_get_stage_times", "odc_field_eval",
           "odc_mesh_extract_batch", "odc_mesh_sync_batch", "odc_context_set_graph",
           "odc_autotune", "odc_set_launch_config", "odc_server_create", "odc_server_destroy",
           "odc_server_last_error", "odc_server_footprint", "odc_server_submit",
           "odc_server_poll", "odc_server_wait", "odc_server_get_stats",
           "odc_server_reset_stats", "odc_count_self_intersections",
           "odc_get_job_intermediate", "odc_context_set_trace", "odc_mesh_extract_noalloc",
           "odc_plan_scratch", "odc_inject_alloc_failures", "odc_get_launch_config")
STAGES = ("labels", "classify", "compact", "bisect", "search2d", "cell_count", "cell_qef", "emit")

_lib = None


def load(path: str = LIB_PATH):
    """Loads libodc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OdcError(-1, f"{path} is missing: build it with paper_2409_13418_amd/build.py")
    # PyTorch ships its own HIP runtime; importing it first makes the library
    # bind to that same runtime (one runtime per process, one device view)
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.odc_status_string.argtypes = [C.c_int32]
    L.odc_status_string.restype = C.c_char_p
    L.odc_last_error.argtypes = [C.c_void_p]
    L.odc_last_error.restype = C.c_char_p
    L.odc_context_create.argtypes = [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    L.odc_context_create.restype = C.c_int32
    L.odc_context_destroy.argtypes = [C.c_void_p]
    L.odc_context_destroy.restype = None
    L.odc_params_default.argtypes = [C.POINTER(Params), C.c_int32]
    L.odc_params_default.restype = None
    L.odc_mesh_extract.argtypes = [C.c_void_p, C.POINTER(Field), C.POINTER(Params),
                                   C.POINTER(MeshBuffers)]
    L.odc_mesh_extract.restype = C.c_int32
    L.odc_mesh_sync.argtypes = [C.c_void_p, C.POINTER(MeshCounts)]
    L.odc_mesh_sync.restype = C.c_int32
    L.odc_get_intermediate.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_int64)]
    L.odc_get_intermediate.restype = C.c_int32
    L.odc_get_job_intermediate.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                           C.c_int64, C.POINTER(C.c_int64)]
    L.odc_get_job_intermediate.restype = C.c_int32
    L.odc_context_set_trace.argtypes = [C.c_void_p, C.c_int32]
    L.odc_context_set_trace.restype = C.c_int32
    L.odc_mesh_extract_noalloc.argtypes = [C.c_void_p, C.POINTER(Field), C.POINTER(Params),
                                           C.POINTER(MeshBuffers)]
    L.odc_mesh_extract_noalloc.restype = C.c_int32
    L.odc_plan_scratch.argtypes = [C.POINTER(Field), C.POINTER(Params), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int32)]
    L.odc_plan_scratch.restype = C.c_int32
    L.odc_inject_alloc_failures.argtypes = [C.c_int32]
    L.odc_inject_alloc_failures.restype = C.c_int32
    L.odc_context_set_timing.argtypes = [C.c_void_p, C.c_int32]
    L.odc_context_set_timing.restype = C.c_int32
    L.odc_get_stage_times.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int32,
                                      C.POINTER(C.c_int32)]
    L.odc_get_stage_times.restype = C.c_int32
    L.odc_field_eval.argtypes = [C.c_void_p, C.POINTER(Field), C.c_int32, C.c_void_p, C.c_int64,
                                 C.c_void_p]
    L.odc_field_eval.restype = C.c_int32
    L.odc_mesh_extract_batch.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Field),
                                         C.POINTER(Params), C.POINTER(MeshBuffers)]
    L.odc_mesh_extract_batch.restype = C.c_int32
    L.odc_mesh_sync_batch.argtypes = [C.c_void_p, C.c_int32, C.POINTER(MeshCounts)]
    L.odc_mesh_sync_batch.restype = C.c_int32
    L.odc_context_set_graph.argtypes = [C.c_void_p, C.c_int32]
    L.odc_context_set_graph.restype = C.c_int32
    L.odc_autotune.argtypes = [C.c_void_p, C.POINTER(Field), C.POINTER(Params),
                               C.POINTER(C.c_int32)]
    L.odc_autotune.restype = C.c_int32
    L.odc_set_launch_config.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
    L.odc_set_launch_config.restype = C.c_int32
    L.odc_get_launch_config.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)]
    L.odc_get_launch_config.restype = C.c_int32
    L.odc_server_create.argtypes = [C.c_void_p, C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]
    L.odc_server_create.restype = C.c_int32
    L.odc_server_destroy.argtypes = [C.c_void_p]
    L.odc_server_destroy.restype = None
    L.odc_server_last_error.argtypes = [C.c_void_p]
    L.odc_server_last_error.restype = C.c_char_p
    L.odc_server_footprint.argtypes = [C.c_void_p, C.POINTER(Field), C.POINTER(Params),
                                       C.POINTER(C.c_int64)]
    L.odc_server_footprint.restype = C.c_int32
    L.odc_server_submit.argtypes = [C.c_void_p, C.POINTER(Field), C.POINTER(Params),
                                    C.POINTER(MeshBuffers), C.POINTER(C.c_uint64)]
    L.odc_server_submit.restype = C.c_int32
    L.odc_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]
    L.odc_server_poll.restype = C.c_int32
    L.odc_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(RequestResult)]
    L.odc_server_wait.restype = C.c_int32
    L.odc_server_get_stats.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
    L.odc_server_get_stats.restype = C.c_int32
    L.odc_server_reset_stats.argtypes = [C.c_void_p]
    L.odc_server_reset_stats.restype = C.c_int32
    L.odc_count_self_intersections.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                               C.c_int64, C.c_double, C.POINTER(C.c_int64)]
    L.odc_count_self_intersections.restype = C.c_int32
    _lib = L
    return L


def default_params(grid, precision: int = PREC_FP32) -> Params:
    """odc_params for an odc_inputs.Grid."""
    p = Params()
    load().odc_params_default(C.byref(p), int(grid.res))
    p.lo = (C.c_double * 3)(*grid.lo)
    p.size = float(grid.size)
    p.iters_1d = int(grid.iters_1d)
    p.lin1, p.bin1, p.lin2, p.bin2 = grid.lin1, grid.bin1, grid.lin2, grid.bin2
    p.range1 = float(grid.range1)
    p.range2 = float(grid.range2)
    p.qef_tau = float(grid.qef_tau)
    p.precision = int(precision)
    p.guard_logit = float(2.0 * math.atanh(0.02))
    p.ablation = int(getattr(grid, "ablation", 0))
    p.clamp_vertices = int(getattr(grid, "clamp", 0))
    return p


class DeviceField:
    """An odc_inputs.Field whose arrays live on the GPU (torch tensors)."""

    def __init__(self, field, device="cuda"):
        import torch
        self.kind = field.kind
        self._keep = []

        def dev(a):
            if a is None:
                return None
            t = torch.from_numpy(np.ascontiguousarray(a, np.float32).reshape(-1)).to(device)
            self._keep.append(t)
            return t

        self.prims = dev(field.prims)
        self.weights = dev(field.weights)
        self.spheres = dev(field.spheres)
        f = Field()
        f.kind = field.kind
        f.prims = self.prims.data_ptr() if self.prims is not None else None
        f.n_prims = 0 if field.prims is None else int(field.prims.shape[0])
        f.weights = self.weights.data_ptr() if self.weights is not None else None
        f.in_dim, f.width, f.depth, f.n_bands = field.in_dim, field.width, field.depth, field.n_bands
        f.spheres = self.spheres.data_ptr() if self.spheres is not None else None
        f.n_spheres = 0 if field.spheres is None else int(field.spheres.shape[0])
        f.sdf_gain = float(field.sdf_gain)
        f.out_scale = float(field.out_scale)
        self.c = f


class Context:
    """One libodc context on a torch device; its stream is torch's current one."""

    def __init__(self, device_index: int = 0, stream=None):
        import torch
        L = load()
        self.torch = torch
        self.device = torch.device("cuda", device_index)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        rc = L.odc_context_create(device_index, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise OdcError(rc, f"odc_context_create: {L.odc_status_string(rc).decode()}")
        self.h = h
        self.cap_v = 0
        self.cap_t = 0
        self.vbuf = None
        self.tbuf = None
        self.vloc = None
        self.vref = None

    def close(self):
        if self.h:
            load().odc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            L = load()
            raise OdcError(rc, f"{what}: {L.odc_status_string(rc).decode()}: "
                               f"{L.odc_last_error(self.h).decode()}")

    def _ensure_out(self, nv, nt, want_local):
        torch = self.torch
        if self.vbuf is None or nv > self.cap_v:
            self.cap_v = max(nv, 1024)
            self.vbuf = torch.empty(self.cap_v * 3, dtype=torch.float32, device=self.device)
            self.vloc = torch.empty(self.cap_v * 3, dtype=torch.float32, device=self.device)
            self.vref = torch.empty(self.cap_v, dtype=torch.int32, device=self.device)
        if self.tbuf is None or nt > self.cap_t:
            self.cap_t = max(nt, 2048)
            self.tbuf = torch.empty(self.cap_t * 3, dtype=torch.int32, device=self.device)
        b = MeshBuffers()
        b.vertices = self.vbuf.data_ptr()
        b.cap_vertices = self.cap_v
        b.triangles = self.tbuf.data_ptr()
        b.cap_triangles = self.cap_t
        b.vertices_local = self.vloc.data_ptr() if want_local else None
        b.vertex_ref = self.vref.data_ptr() if want_local else None
        return b

    def extract_async(self, dfield: DeviceField, params: Params, want_local=False,
                      cap_hint=None):
        """Enqueues one mesh extraction into the context's buffers."""
        if cap_hint is None:
            r = params.res
            cap_hint = (max(4096, 8 * r * r), max(8192, 16 * r * r))
        b = self._ensure_out(cap_hint[0], cap_hint[1], want_local)
        rc = load().odc_mesh_extract(self.h, C.byref(dfield.c), C.byref(params), C.byref(b))
        self._check(rc, "odc_mesh_extract")

    def sync(self) -> dict:
        c = MeshCounts()
        rc = load().odc_mesh_sync(self.h, C.byref(c))
        if rc == ERR_CAPACITY:
            return {"capacity": True, **c.as_dict()}
        self._check(rc, "odc_mesh_sync")
        return c.as_dict()

    def extract(self, dfield: DeviceField, params: Params, want_local=False) -> dict:
        """Extracts and waits; grows the outputs and retries once if needed.
        Returns counts plus device tensors 'vertices' (V,3) and 'triangles' (T,3)."""
        self.extract_async(dfield, params, want_local, (self.cap_v, self.cap_t)
                           if self.vbuf is not None else None)
        c = self.sync()
        if c.get("capacity"):
            self.extract_async(dfield, params, want_local,
                               (c["n_vertices"] + 16, c["n_triangles"] + 16))
            c = self.sync()
            if c.get("capacity"):
                raise OdcError(ERR_CAPACITY, "capacity exceeded after growing")
        nv, nt = c["n_vertices"], c["n_triangles"]
        out = dict(c)
        out["vertices"] = self.vbuf[:3 * nv].view(nv, 3)
        out["triangles"] = self.tbuf[:3 * nt].view(nt, 3)
        if want_local:
            out["vertices_local"] = self.vloc[:3 * nv].view(nv, 3)
            out["vertex_ref"] = self.vref[:nv]
        return out

    def field_eval(self, dfield: DeviceField, xyz, precision: int = PREC_FP32) -> np.ndarray:
        """Logits (MLP) or +-1 labels (CSG) at world points xyz (n, 3)."""
        torch = self.torch
        pts = torch.as_tensor(np.ascontiguousarray(xyz, np.float32).reshape(-1, 3),
                              device=self.device)
        z = torch.empty(pts.shape[0], dtype=torch.float32, device=self.device)
        rc = load().odc_field_eval(self.h, C.byref(dfield.c), int(precision),
                                   C.c_void_p(pts.data_ptr()), pts.shape[0],
                                   C.c_void_p(z.data_ptr()))
        self._check(rc, "odc_field_eval")
        return z.cpu().numpy()

    def self_intersections(self, vertices, triangles, cell: float) -> int:
        """Pairs of vertex-disjoint triangles that intersect (device tensors or
        host arrays; counted on this context's GPU)."""
        torch = self.torch
        v = torch.as_tensor(np.asarray(vertices, np.float32) if not torch.is_tensor(vertices)
                            else vertices, device=self.device).float().contiguous()
        t = torch.as_tensor(np.asarray(triangles, np.int32) if not torch.is_tensor(triangles)
                            else triangles, device=self.device).int().contiguous()
        n = C.c_int64()
        rc = load().odc_count_self_intersections(self.h, C.c_void_p(v.data_ptr()), v.numel() // 3,
                                                 C.c_void_p(t.data_ptr()), t.numel() // 3,
                                                 float(cell), C.byref(n))
        self._check(rc, "odc_count_self_intersections")
        return int(n.value)

    def set_graph(self, enable: bool):
        self._check(load().odc_context_set_graph(self.h, 1 if enable else 0), "set_graph")

    def autotune(self, dfield: DeviceField, params: Params):
        """Times candidate launch shapes on this field; returns the chosen
        (grid, element, matrix-core) block counts, cached for the field's
        kind and resolution bucket and kept as this context's default."""
        ch = (C.c_int32 * 3)()
        self._check(load().odc_autotune(self.h, C.byref(dfield.c), C.byref(params), ch),
                    "autotune")
        return tuple(ch)

    def set_launch_config(self, grid_blocks: int, elem_blocks: int, mlp_blocks: int):
        v = (C.c_int32 * 3)(grid_blocks, elem_blocks, mlp_blocks)
        self._check(load().odc_set_launch_config(self.h, v), "set_launch_config")

    def launch_config(self, kind: int, res: int):
        """((grid, element, matrix-core) blocks, from_cache) an extraction
        whose dominant job has this field kind and resolution would use."""
        v = (C.c_int32 * 3)()
        t = C.c_int32()
        self._check(load().odc_get_launch_config(self.h, int(kind), int(res), v, C.byref(t)),
                    "launch_config")
        return tuple(v), bool(t.value)

    def extract_batch(self, dfields, params_list, caps=None, want_local=False):
        """Meshes several fields in one launch per stage.  Returns a list of
        dicts like extract(); outputs live in per-job device tensors."""
        torch = self.torch
        n = len(dfields)
        if caps is None:
            caps = [(max(4096, 8 * p.res * p.res), max(8192, 16 * p.res * p.res))
                    for p in params_list]
        for attempt in range(2):
            fa = (Field * n)(*[d.c for d in dfields])
            pa = (Params * n)(*params_list)
            bufs = (MeshBuffers * n)()
            keep = []
            for k in range(n):
                nv, nt = caps[k]
                v = torch.empty(3 * nv, dtype=torch.float32, device=self.device)
                t = torch.empty(3 * nt, dtype=torch.int32, device=self.device)
                vl = torch.empty(3 * nv, dtype=torch.float32, device=self.device) if want_local else None
                vr = torch.empty(nv, dtype=torch.int32, device=self.device) if want_local else None
                keep.append((v, t, vl, vr))
                bufs[k].vertices = v.data_ptr()
                bufs[k].cap_vertices = nv
                bufs[k].triangles = t.data_ptr()
                bufs[k].cap_triangles = nt
                bufs[k].vertices_local = vl.data_ptr() if vl is not None else None
                bufs[k].vertex_ref = vr.data_ptr() if vr is not None else None
            L = load()
            self._check(L.odc_mesh_extract_batch(self.h, n, fa, pa, bufs), "extract_batch")
            counts = (MeshCounts * n)()
            rc = L.odc_mesh_sync_batch(self.h, n, counts)
            if rc == ERR_CAPACITY and attempt == 0:
                caps = [(max(caps[k][0], counts[k].n_vertices + 16),
                         max(caps[k][1], counts[k].n_triangles + 16)) for k in range(n)]
                continue
            self._check(rc, "sync_batch")
            break
        out = []
        for k in range(n):
            c = counts[k].as_dict()
            v, t, vl, vr = keep[k]
            c["vertices"] = v[:3 * c["n_vertices"]].view(-1, 3)
            c["triangles"] = t[:3 * c["n_triangles"]].view(-1, 3)
            if want_local:
                c["vertices_local"] = vl[:3 * c["n_vertices"]].view(-1, 3)
                c["vertex_ref"] = vr[:c["n_vertices"]]
            out.append(c)
        return out

    def set_timing(self, enable: bool):
        self._check(load().odc_context_set_timing(self.h, 1 if enable else 0), "set_timing")

    def stage_times(self) -> dict:
        """Device milliseconds per stage of the last extraction (timing on)."""
        ms = (C.c_float * 8)()
        n = C.c_int32()
        self._check(load().odc_get_stage_times(self.h, ms, 8, C.byref(n)), "stage_times")
        return {STAGES[i]: float(ms[i]) for i in range(n.value)}

    def intermediate(self, name: str, job: int = 0) -> np.ndarray:
        """A copy of one intermediate array of job `job` of the last extraction
        (host numpy)."""
        which, dt = INTERMEDIATES[name]
        L = load()
        n = C.c_int64()
        rc = L.odc_get_job_intermediate(self.h, job, which, None, 0, C.byref(n))
        if rc not in (OK, ERR_CAPACITY):
            self._check(rc, "odc_get_job_intermediate")
        count = int(n.value)
        elem = _ELEM_BYTES.get(name, 4)
        t = self.torch.empty(max(count * elem, 4), dtype=self.torch.uint8, device=self.device)
        rc = L.odc_get_job_intermediate(self.h, job, which, C.c_void_p(t.data_ptr()),
                                        count * elem, C.byref(n))
        self._check(rc, "odc_get_job_intermediate")
        a = t[:count * elem].cpu().numpy().view(dt)
        return a.reshape(count, _COLS[name]) if name in _COLS else a

    def set_trace(self, enable: bool):
        """Record decision traces of the searches (intermediates edge_trace,
        pair_trace) in later extractions."""
        self._check(load().odc_context_set_trace(self.h, int(bool(enable))), "set_trace")


class OutputBuffers:
    """Device output tensors of one job (vertices, triangles and optionally
    the grid-local vertex form) and the odc_mesh_buffers that point at them."""

    def __init__(self, n_vertices: int, n_triangles: int, device="cuda", want_local=False):
        import torch
        self.v = torch.empty(3 * n_vertices, dtype=torch.float32, device=device)
        self.t = torch.empty(3 * n_triangles, dtype=torch.int32, device=device)
        self.vl = torch.empty(3 * n_vertices, dtype=torch.float32, device=device) \
            if want_local else None
        self.vr = torch.empty(n_vertices, dtype=torch.int32, device=device) if want_local else None
        b = MeshBuffers()
        b.vertices = self.v.data_ptr()
        b.cap_vertices = n_vertices
        b.triangles = self.t.data_ptr()
        b.cap_triangles = n_triangles
        b.vertices_local = self.vl.data_ptr() if want_local else None
        b.vertex_ref = self.vr.data_ptr() if want_local else None
        self.c = b

    def views(self, counts: dict) -> dict:
        nv, nt = counts["n_vertices"], counts["n_triangles"]
        out = {"vertices": self.v[:3 * nv].view(-1, 3), "triangles": self.t[:3 * nt].view(-1, 3)}
        if self.vl is not None:
            out["vertices_local"] = self.vl[:3 * nv].view(-1, 3)
            out["vertex_ref"] = self.vr[:nv]
        return out


class Server:
    """Continuous-batching request loop of libodc (odc_server_*) on the
    context's GPU.  Field tensors and output buffers of a submitted job must
    stay alive until wait() returns for its ticket; submit() keeps references
    to the objects it is given until then."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, lanes: int = 2, max_batch: int = 16,
                 max_batch_corners: int = 0, policy: int = SERVE_FIFO, age_ms: float = 0.0,
                 band: float = 0.0):
        L = load()
        self.ctx = ctx
        cfg = ServerConfig(int(hbm_budget_bytes), int(lanes), int(max_batch),
                           int(max_batch_corners), int(policy), float(age_ms), float(band))
        h = C.c_void_p()
        rc = L.odc_server_create(ctx.h, C.byref(cfg), C.byref(h))
        if rc != OK:
            raise OdcError(rc, f"odc_server_create: {L.odc_status_string(rc).decode()}: "
                               f"{L.odc_last_error(ctx.h).decode()}")
        self.h = h
        self._held = {}

    def close(self):
        if self.h:
            load().odc_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            L = load()
            raise OdcError(rc, f"{what}: {L.odc_status_string(rc).decode()}: "
                               f"{L.odc_server_last_error(self.h).decode()}")

    def footprint(self, dfield: DeviceField, params: Params) -> int:
        b = C.c_int64()
        self._check(load().odc_server_footprint(self.h, C.byref(dfield.c), C.byref(params),
                                                C.byref(b)), "footprint")
        return int(b.value)

    def submit(self, dfield: DeviceField, params: Params, out: OutputBuffers) -> int:
        """Queues one job; returns its ticket at once."""
        t = C.c_uint64()
        self._check(load().odc_server_submit(self.h, C.byref(dfield.c), C.byref(params),
                                             C.byref(out.c), C.byref(t)), "submit")
        self._held[t.value] = (dfield, params, out)
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        self._check(load().odc_server_poll(self.h, ticket, C.byref(d)), "poll")
        return bool(d.value)

    def wait(self, ticket: int) -> dict:
        """Blocks until the job is done; returns its status, counts and
        host timestamps (ms since the server started) and releases it."""
        r = RequestResult()
        self._check(load().odc_server_wait(self.h, ticket, C.byref(r)), "wait")
        self._held.pop(ticket, None)
        out = r.counts.as_dict()
        out.update(status=int(r.status), attempts=int(r.attempts), submit_ms=r.submit_ms,
                   admit_ms=r.admit_ms, done_ms=r.done_ms,
                   latency_ms=r.done_ms - r.submit_ms)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        self._check(load().odc_server_get_stats(self.h, C.byref(st)), "stats")
        return st.as_dict()

    def reset_stats(self):
        self._check(load().odc_server_reset_stats(self.h), "reset_stats")
