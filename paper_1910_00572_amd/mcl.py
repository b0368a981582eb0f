"""Python binding of the C ABI in include/mcl.h (argument marshalling only).

Every computation runs in libmcl.so's HIP kernels.  PyTorch supplies device
memory (the workspaces are torch uint8 tensors) and the current HIP stream.
Importing this module fails loudly when libmcl.so has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmcl.so")

F32, BF16, F16 = 0, 1, 2
DTYPES = {"f32": F32, "bf16": BF16, "f16": F16}
MASK_BEFORE_BLUR, WALL_NORMALIZE, SUBCELL_GATE, SCAN_F32, INTEGER_SHIFT, ANISOTROPIC = 1, 2, 4, 8, 16, 32
DEFAULT_FLAGS = MASK_BEFORE_BLUR | WALL_NORMALIZE
OK, EINVAL, ENOMEM, EDEGENERATE, EDEVICE, ESTATE = range(6)
STATUS_NAMES = {0: "MCL_OK", 1: "MCL_EINVAL", 2: "MCL_ENOMEM", 3: "MCL_EDEGENERATE",
                4: "MCL_EDEVICE", 5: "MCL_ESTATE"}

# Every symbol include/mcl.h declares.
ABI_SYMBOLS = [
    "mcl_last_error", "mcl_map_workspace_bytes", "mcl_map_create", "mcl_map_destroy",
    "mcl_filter_workspace_bytes", "mcl_init_belief", "mcl_filter_destroy", "mcl_step_odometry",
    "mcl_apply_scan", "mcl_normalize", "mcl_read_belief", "mcl_export_belief", "mcl_scan_sqdist",
    "mcl_get_info", "mcl_step_batch", "mcl_batch_workspace_bytes", "mcl_sample_cells",
    "mcl_apply_scan_sampled", "mcl_dither", "mcl_match_workspace_bytes", "mcl_best_match",
    "mcl_difficulty", "mcl_batch_create", "mcl_batch_step", "mcl_batch_counts", "mcl_batch_destroy",
    "mcl_export_scalars", "mcl_apply_scan_batch", "mcl_step_batch_noalloc",
]


class MapDesc(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("cell_m", c_double),
                ("occupancy", c_void_p), ("range_table", c_void_p), ("n_dirs", c_int32),
                ("max_range_m", c_double)]


class Params(ctypes.Structure):
    _fields_ = [("n_theta", c_int32), ("sigma_xy_cells", c_double), ("sigma_theta_bins", c_double),
                ("radius_xy", c_int32), ("radius_theta", c_int32), ("storage", c_int32),
                ("flags", c_uint32), ("sigma_lateral_cells", c_double), ("launch_shape", c_int32 * 7)]


class Pose(ctypes.Structure):
    _fields_ = [("i", c_int32), ("j", c_int32), ("k", c_int32), ("x_m", c_double), ("y_m", c_double),
                ("theta_rad", c_double), ("prob", c_double)]

    def as_tuple(self):
        return (self.k, self.j, self.i)


class Info(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("n_theta", c_int32), ("pitch", c_int32),
                ("storage", c_int32), ("radius", c_int32), ("tile_x", c_int32), ("tile_y", c_int32),
                ("theta_chunks", c_int32), ("workgroups", c_int32), ("steps", c_int64),
                ("theta_offset_rad", c_double), ("log_norm", c_double), ("status", c_int32),
                ("belief_device", c_void_p), ("state_bytes", c_uint64)]


class MclError(RuntimeError):
    def __init__(self, status, message, readout=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        # read_belief on a degenerate filter still fills its outputs (the last
        # belief that had mass): (belief, Pose, theta_offset, log_norm)
        self.readout = readout


_lib = None


def load_library(path: str = _LIB_PATH):
    """Load libmcl.so (raises if it is missing) and declare the ABI signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1910_00572_amd.build`")
    lib = ctypes.CDLL(path)
    lib.mcl_last_error.restype = ctypes.c_char_p
    lib.mcl_last_error.argtypes = []
    lib.mcl_map_workspace_bytes.restype = c_size_t
    lib.mcl_map_workspace_bytes.argtypes = [POINTER(MapDesc), POINTER(Params)]
    lib.mcl_map_create.restype = c_int
    lib.mcl_map_create.argtypes = [POINTER(MapDesc), POINTER(Params), c_void_p, c_size_t, c_void_p,
                                   POINTER(c_void_p)]
    lib.mcl_map_destroy.restype = None
    lib.mcl_map_destroy.argtypes = [c_void_p]
    lib.mcl_filter_workspace_bytes.restype = c_size_t
    lib.mcl_filter_workspace_bytes.argtypes = [c_void_p, POINTER(Params)]
    lib.mcl_init_belief.restype = c_int
    lib.mcl_init_belief.argtypes = [c_void_p, POINTER(Params), c_void_p, c_size_t, c_void_p, c_void_p,
                                    c_double, POINTER(c_void_p)]
    lib.mcl_filter_destroy.restype = None
    lib.mcl_filter_destroy.argtypes = [c_void_p]
    lib.mcl_step_odometry.restype = c_int
    lib.mcl_step_odometry.argtypes = [c_void_p, c_double, c_double, c_double]
    lib.mcl_apply_scan.restype = c_int
    lib.mcl_apply_scan.argtypes = [c_void_p, c_void_p, c_int32, c_double]
    lib.mcl_normalize.restype = c_int
    lib.mcl_normalize.argtypes = [c_void_p, POINTER(c_double)]
    lib.mcl_read_belief.restype = c_int
    lib.mcl_read_belief.argtypes = [c_void_p, c_void_p, POINTER(Pose), POINTER(c_double), POINTER(c_double)]
    lib.mcl_export_belief.restype = c_int
    lib.mcl_export_belief.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.mcl_scan_sqdist.restype = c_int
    lib.mcl_scan_sqdist.argtypes = [c_void_p, c_void_p, c_int32, c_void_p]
    lib.mcl_get_info.restype = c_int
    lib.mcl_get_info.argtypes = [c_void_p, c_int, POINTER(Info)]
    lib.mcl_step_batch.restype = c_int
    lib.mcl_step_batch.argtypes = [POINTER(c_void_p), c_void_p, c_int32, c_void_p, c_size_t, c_void_p]
    lib.mcl_batch_workspace_bytes.restype = c_size_t
    lib.mcl_batch_workspace_bytes.argtypes = [c_int32]
    lib.mcl_sample_cells.restype = c_int
    lib.mcl_sample_cells.argtypes = [c_void_p, c_int32, c_void_p]
    lib.mcl_apply_scan_sampled.restype = c_int
    lib.mcl_apply_scan_sampled.argtypes = [c_void_p, c_void_p, c_int32, c_double, c_void_p]
    lib.mcl_dither.restype = c_int
    lib.mcl_dither.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p]
    lib.mcl_match_workspace_bytes.restype = c_size_t
    lib.mcl_match_workspace_bytes.argtypes = [c_void_p, c_int32, c_int32]
    lib.mcl_best_match.restype = c_int
    lib.mcl_best_match.argtypes = [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]
    lib.mcl_difficulty.restype = c_int
    lib.mcl_difficulty.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_double, c_void_p]
    lib.mcl_batch_create.restype = c_int
    lib.mcl_batch_create.argtypes = [c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.mcl_batch_step.restype = c_int
    lib.mcl_batch_step.argtypes = [c_void_p, POINTER(c_void_p), c_void_p, c_int32]
    lib.mcl_batch_counts.restype = c_int
    lib.mcl_batch_counts.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
    lib.mcl_step_batch_noalloc.restype = c_int
    lib.mcl_step_batch_noalloc.argtypes = [POINTER(c_void_p), c_void_p, c_int32, c_void_p]
    lib.mcl_apply_scan_batch.restype = c_int
    lib.mcl_apply_scan_batch.argtypes = [POINTER(c_void_p), c_void_p, c_int32, c_void_p, c_int32]
    lib.mcl_export_scalars.restype = c_int
    lib.mcl_export_scalars.argtypes = [c_void_p, c_void_p]
    lib.mcl_batch_destroy.restype = None
    lib.mcl_batch_destroy.argtypes = [c_void_p]
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().mcl_last_error().decode(errors="replace")


def _check(status):
    if status != OK:
        raise MclError(status, last_error())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _params(n_theta=1, sigma_xy=0.0, sigma_theta=0.0, radius_xy=-1, radius_theta=-1, storage="f32",
            flags=DEFAULT_FLAGS, sigma_lateral=0.0, launch_shape=None) -> Params:
    shape = (c_int32 * 7)(*(list(launch_shape or []) + [0] * 7)[:7])
    return Params(int(n_theta), float(sigma_xy), float(sigma_theta), int(radius_xy), int(radius_theta),
                  DTYPES[storage] if isinstance(storage, str) else int(storage), int(flags), float(sigma_lateral),
                  shape)


class Map:
    """Traversability, wall weights and (optional) quantised range table on the GPU."""

    def __init__(self, occupancy, cell_m, sigma_xy, *, radius_xy=-1, flags=DEFAULT_FLAGS,
                 range_table=None, max_range_m=0.0, stream=None):
        import torch
        lib = load_library()
        occ = np.ascontiguousarray(occupancy, dtype=np.uint8)
        self.height, self.width = occ.shape
        self.cell_m = float(cell_m)
        self.sigma_xy = float(sigma_xy)
        self.radius_xy = int(radius_xy)
        self.flags = int(flags)
        rt = None
        n_dirs = 0
        if range_table is not None:
            rt = np.ascontiguousarray(range_table, dtype=np.float32)
            n_dirs = rt.shape[-1]
        self.n_dirs = n_dirs
        self.max_range_m = float(max_range_m)
        desc = MapDesc(self.width, self.height, self.cell_m, occ.ctypes.data,
                       rt.ctypes.data if rt is not None else None, n_dirs, self.max_range_m)
        prm = _params(sigma_xy=sigma_xy, radius_xy=radius_xy, flags=flags)
        nbytes = lib.mcl_map_workspace_bytes(byref(desc), byref(prm))
        if nbytes == 0:
            _check(lib.mcl_map_create(byref(desc), byref(prm), None, 0, None, byref(c_void_p())))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = c_void_p()
        _check(lib.mcl_map_create(byref(desc), byref(prm), c_void_p(self.workspace.data_ptr()), nbytes,
                                  _stream_handle(stream), byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcl_map_destroy(self.handle)
            self.handle = None


class Filter:
    """One belief tensor on the GPU (init_belief)."""

    def __init__(self, map: Map, n_theta, sigma_theta, *, radius_theta=-1, storage="f32", init=None,
                 theta0=0.0, stream=None, sigma_lateral=0.0, launch_shape=None):
        """launch_shape (testing and tuning only): the step kernel's launch shape, as
        mcl_params.launch_shape; None lets the library choose."""
        import torch
        lib = load_library()
        self.map = map
        self.n_theta = int(n_theta)
        self.storage = storage
        self.params = _params(n_theta, map.sigma_xy, sigma_theta, map.radius_xy, radius_theta, storage,
                              map.flags, sigma_lateral, launch_shape)
        nbytes = lib.mcl_filter_workspace_bytes(map.handle, byref(self.params))
        if nbytes == 0:
            _check(lib.mcl_init_belief(map.handle, byref(self.params), None, 0, None, None, 0.0,
                                       byref(c_void_p())))
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        init_ptr = None
        if init is not None:
            self._init = np.ascontiguousarray(init, dtype=np.float32)
            assert self._init.shape == (self.n_theta, map.height, map.width)
            init_ptr = self._init.ctypes.data
        self.stream = stream
        # the torch stream the filter's work runs on; outputs handed back as
        # tensors are ordered after it on the caller's current stream
        self._tstream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        _check(lib.mcl_init_belief(map.handle, byref(self.params), c_void_p(self.workspace.data_ptr()), nbytes,
                                   _stream_handle(stream), init_ptr, float(theta0), byref(h)))
        self.handle = h
        self._init = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcl_filter_destroy(self.handle)
            self.handle = None

    # the five calls of the boundary, as methods
    def step_odometry(self, u, v, w):
        _check(_lib.mcl_step_odometry(self.handle, float(u), float(v), float(w)))

    def apply_scan(self, ranges_m, sigma_m):
        z = np.ascontiguousarray(ranges_m, dtype=np.float32)
        _check(_lib.mcl_apply_scan(self.handle, z.ctypes.data, len(z), float(sigma_m)))

    def normalize(self) -> float:
        ln = c_double()
        _check(_lib.mcl_normalize(self.handle, byref(ln)))
        return ln.value

    def read_belief(self, want_belief=True):
        """Returns (belief float32 (T, H, W) or None, Pose, theta_offset, log_norm)."""
        out = np.empty((self.n_theta, self.map.height, self.map.width), np.float32) if want_belief else None
        pose = Pose()
        th = c_double()
        ln = c_double()
        st = _lib.mcl_read_belief(self.handle, out.ctypes.data if out is not None else None, byref(pose),
                                  byref(th), byref(ln))
        if st == EDEGENERATE:
            raise MclError(st, last_error(), readout=(out, pose, th.value, ln.value))
        _check(st)
        return out, pose, th.value, ln.value

    def export_belief(self, with_map=False):
        """Normalised FP32 belief (and belief map) as CUDA tensors."""
        import torch
        out = torch.empty((self.n_theta, self.map.height, self.map.width), dtype=torch.float32, device="cuda")
        bm = torch.empty((self.map.height, self.map.width), dtype=torch.float32, device="cuda") if with_map else None
        _check(_lib.mcl_export_belief(self.handle, c_void_p(out.data_ptr()),
                                      c_void_p(bm.data_ptr()) if bm is not None else None))
        self._order_after()
        return (out, bm) if with_map else out

    def _order_after(self):
        """Order the caller's current stream after the work enqueued on the filter's stream."""
        import torch
        cur = torch.cuda.current_stream()
        if cur != self._tstream:
            cur.wait_stream(self._tstream)

    def export_scalars(self, out=None):
        """Device float64 tensor [log_norm, status] as of the work enqueued so far (async)."""
        import torch
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device="cuda")
        _check(_lib.mcl_export_scalars(self.handle, c_void_p(out.data_ptr())))
        self._order_after()
        return out

    def scan_sqdist(self, ranges_m):
        import torch
        z = np.ascontiguousarray(ranges_m, dtype=np.float32)
        out = torch.empty((self.n_theta, self.map.height, self.map.width), dtype=torch.int32, device="cuda")
        _check(_lib.mcl_scan_sqdist(self.handle, z.ctypes.data, len(z), c_void_p(out.data_ptr())))
        self._order_after()
        return out

    def sample_cells(self, n_samples, out=None):
        """Floyd-Steinberg sample mask of the belief map: uint8 CUDA tensor (H, W)."""
        import torch
        if out is None:
            out = torch.empty((self.map.height, self.map.width), dtype=torch.uint8, device="cuda")
        _check(_lib.mcl_sample_cells(self.handle, int(n_samples), c_void_p(out.data_ptr())))
        self._order_after()
        return out

    def apply_scan_sampled(self, ranges_m, sigma_m, mask):
        """Observation update on the states of the cells of `mask` (uint8 CUDA tensor (H, W))."""
        assert mask.dtype.itemsize == 1 and mask.is_contiguous() and mask.is_cuda
        assert tuple(mask.shape) == (self.map.height, self.map.width)
        z = np.ascontiguousarray(ranges_m, dtype=np.float32)
        _check(_lib.mcl_apply_scan_sampled(self.handle, z.ctypes.data, len(z), float(sigma_m),
                                           c_void_p(mask.data_ptr())))

    def info(self, sync=True) -> Info:
        inf = Info()
        _check(_lib.mcl_get_info(self.handle, int(sync), byref(inf)))
        return inf


# ---- module-level names of the boundary --------------------------------------------

def init_belief(map: Map, n_theta, sigma_theta, **kw) -> Filter:
    return Filter(map, n_theta, sigma_theta, **kw)


def step_odometry(f: Filter, u, v, w):
    f.step_odometry(u, v, w)


def apply_scan(f: Filter, ranges_m, sigma_m):
    f.apply_scan(ranges_m, sigma_m)


def apply_scan_batch(filters, ranges_m, sigma_m):
    """Scan updates of several filters of one map (n scans, one std-dev each) in shared launches."""
    if not filters:
        return
    arr = (c_void_p * len(filters))(*[f.handle.value for f in filters])
    z = np.ascontiguousarray(ranges_m, dtype=np.float32)
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma_m, np.float64), (len(filters),)))
    assert z.ndim == 2 and z.shape[0] == len(filters)
    _check(load_library().mcl_apply_scan_batch(arr, z.ctypes.data, z.shape[1], sig.ctypes.data, len(filters)))


def normalize(f: Filter) -> float:
    return f.normalize()


def read_belief(f: Filter, want_belief=True):
    return f.read_belief(want_belief)


def sample_cells(f: Filter, n_samples, out=None):
    return f.sample_cells(n_samples, out)


def apply_scan_sampled(f: Filter, ranges_m, sigma_m, mask):
    f.apply_scan_sampled(ranges_m, sigma_m, mask)


def dither(intensity, out=None, stream=None):
    """Floyd-Steinberg mask (uint8 CUDA tensor) of a float32 CUDA image (H, W)."""
    import torch
    assert intensity.dtype == torch.float32 and intensity.is_contiguous() and intensity.is_cuda
    H, W = intensity.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=intensity.device)
    _check(load_library().mcl_dither(c_void_p(intensity.data_ptr()), int(W), int(H), c_void_p(out.data_ptr()),
                                     _stream_handle(stream)))
    return out


def best_match(map: Map, n_theta, ranges_m, batch=64, stream=None):
    """Best matching free state of each query scan (map difficulty): (cell j*W+i, heading, D) arrays."""
    import torch
    lib = load_library()
    z = np.ascontiguousarray(ranges_m, dtype=np.float32)
    if map.n_dirs == 0:
        raise MclError(ESTATE, "the map has no range table")
    if z.ndim != 2 or z.shape[1] != map.n_dirs:
        raise MclError(EINVAL, f"ranges must be (n_queries, {map.n_dirs}), got {z.shape}")
    n = z.shape[0]
    nbytes = lib.mcl_match_workspace_bytes(map.handle, int(n_theta), int(batch))
    if nbytes == 0:
        raise MclError(ESTATE if map.n_dirs == 0 else EINVAL, "no workspace for these arguments")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    cell = np.empty(n, np.int32)
    head = np.empty(n, np.int32)
    dist = np.empty(n, np.int32)
    _check(lib.mcl_best_match(map.handle, int(n_theta), z.ctypes.data, n, int(batch), cell.ctypes.data,
                              head.ctypes.data, dist.ctypes.data, c_void_p(ws.data_ptr()), nbytes,
                              _stream_handle(stream)))
    return cell, head, dist


def difficulty(map: Map, query_cells, best_cells, threshold_m=1.0):
    """D_M: fraction of query cells whose best match lies more than threshold_m away."""
    lib = load_library()
    q = np.ascontiguousarray(query_cells, dtype=np.int32)
    b = np.ascontiguousarray(best_cells, dtype=np.int32)
    if q.shape != b.shape:
        raise MclError(EINVAL, "query and best cell lists differ in length")
    out = c_double()
    _check(lib.mcl_difficulty(map.handle, q.ctypes.data, b.ctypes.data, len(q), float(threshold_m), byref(out)))
    return out.value


class BatchWorkspace:
    """Device job table of step_batch for up to `max_filters` filters."""

    def __init__(self, max_filters):
        import torch
        lib = load_library()
        self.max_filters = int(max_filters)
        n = lib.mcl_batch_workspace_bytes(self.max_filters)
        if n == 0:
            raise MclError(EINVAL, "batch size out of range")
        self.nbytes = n
        self.tensor = torch.empty(n, dtype=torch.uint8, device="cuda")


def step_batch(filters, uvw, workspace: BatchWorkspace, stream=None):
    """One odometry step for each filter in as few launches as possible (serving).

    uvw: (n, 3) float64 robot-frame increments.  Results are bitwise identical
    to stepping each filter alone.
    """
    assert len(filters) <= workspace.max_filters
    arr = (c_void_p * len(filters))(*[f.handle.value for f in filters])
    u = np.ascontiguousarray(uvw, dtype=np.float64)
    _check(load_library().mcl_step_batch(arr, u.ctypes.data, len(filters), c_void_p(workspace.tensor.data_ptr()),
                                         workspace.nbytes, _stream_handle(stream)))


def step_batch_noalloc(filters, uvw, stream=None):
    """step_batch without a workspace: the job table is the library's own static device array."""
    arr = (c_void_p * len(filters))(*[f.handle.value for f in filters])
    u = np.ascontiguousarray(uvw, dtype=np.float64)
    _check(load_library().mcl_step_batch_noalloc(arr, u.ctypes.data, len(filters), _stream_handle(stream)))


class BatchRunner:
    """Graph-replayed batched steps (mcl_batch_*): one HIP graph per launch
    structure, replayed while the set of filters keeps its shape.  Runs on
    `stream` (default: the current stream), which must not be the default
    NULL stream; the filters must be driven on the same stream."""

    def __init__(self, max_filters, stream=None):
        import torch
        lib = load_library()
        self.max_filters = int(max_filters)
        n = lib.mcl_batch_workspace_bytes(self.max_filters)
        if n == 0:
            raise MclError(EINVAL, "batch size out of range")
        self.workspace = torch.empty(n, dtype=torch.uint8, device="cuda")
        h = c_void_p()
        _check(lib.mcl_batch_create(self.max_filters, c_void_p(self.workspace.data_ptr()), n,
                                    _stream_handle(stream), byref(h)))
        self.handle = h

    def step(self, filters, uvw):
        """One odometry step for each filter; uvw: (n, 3) robot-frame increments."""
        arr = (c_void_p * len(filters))(*[f.handle.value for f in filters])
        u = np.ascontiguousarray(uvw, dtype=np.float64)
        _check(_lib.mcl_batch_step(self.handle, arr, u.ctypes.data, len(filters)))

    def counts(self):
        """(graph captures, graph replays) so far."""
        c, r = c_int64(), c_int64()
        _check(_lib.mcl_batch_counts(self.handle, byref(c), byref(r)))
        return c.value, r.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcl_batch_destroy(self.handle)
            self.handle = None
