"""Thin ctypes binding of libkatsevich.so (include/katsevich.h).

Argument marshalling only: every step of the reconstruction runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream; no torch type crosses
the C ABI.  If the library has not been built this module raises on first use: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p, c_char_p

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkatsevich.so")


class KatsevichError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"katsevich status {status}: {msg}")
        self.status = status


class _Geometry(ctypes.Structure):
    _fields_ = [("R", c_double), ("D", c_double), ("feed_per_turn", c_double),
                ("lambda0", c_double), ("z0", c_double), ("lambda_first", c_double),
                ("dalpha", c_double), ("col_offset", c_double), ("dw", c_double),
                ("row_offset", c_double), ("n_views", c_int64), ("views_per_turn", c_int32),
                ("det_cols", c_int32), ("det_rows", c_int32), ("reserved", c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("dx", c_double), ("dy", c_double), ("dz", c_double), ("x_first", c_double),
                ("y_first", c_double), ("z_first", c_double), ("nx", c_int32), ("ny", c_int32),
                ("nz", c_int32), ("reserved", c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("n_psi", c_int32), ("n_threads", c_int32), ("flags", c_int32),
                ("bp_slices", c_int32), ("hilbert_mode", c_int32)]


class _DevSizes(ctypes.Structure):
    _fields_ = [("scratch_bytes", c_uint64), ("table_bytes", c_uint64),
                ("pi_li_offset", c_uint64), ("pi_lo_offset", c_uint64),
                ("pi_nfirst_offset", c_uint64), ("pi_nlast_offset", c_uint64),
                ("fov_offset", c_uint64), ("n_table_slices", c_int32), ("reserved", c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("table_bytes", c_uint64), ("workspace_bytes", c_uint64),
                ("filtered_bytes", c_uint64), ("workspace_bytes_filter", c_uint64),
                ("first_view", c_int64), ("last_view", c_int64), ("n_vv", c_int64),
                ("n_valid_voxels", c_int64), ("n_pitches", c_int32),
                ("slices_per_pitch", c_int32), ("n_table_slices", c_int32), ("n_psi", c_int32),
                ("window_views", c_int32), ("window_lo", c_int32), ("fft_len", c_int32),
                ("commensurate", c_int32), ("gf_rows", c_int32), ("gf_cols", c_int32),
                ("atan_degree", c_int32), ("bp_slices", c_int32), ("bp_box_rows", c_int32),
                ("bp_box_cols", c_int32), ("half_sample", c_int32), ("hilbert_mode", c_int32)]


FLAG_HALF_SAMPLE_DERIVATIVE = 1   # KATS_FLAG_HALF_SAMPLE_DERIVATIVE (include/katsevich.h)
FLAG_DETERMINISTIC_ADJOINT = 2    # KATS_FLAG_DETERMINISTIC_ADJOINT
HILBERT_AUTO, HILBERT_FFT, HILBERT_MFMA = 0, 1, 2   # KATS_HILBERT_* (include/katsevich.h)

# table id -> (C enum, numpy dtype, shape key)
TABLES = {
    "fr_row": (1, np.int32, "psi_cols"), "fr_weight": (2, np.float64, "psi_cols"),
    "br_kappa": (3, np.int32, "rows_cols"), "br_weight": (4, np.float64, "rows_cols"),
    "psi_hat": (5, np.float64, "rows_cols"), "pi_li": (6, np.float64, "tab"),
    "pi_lo": (7, np.float64, "tab"), "pi_nfirst": (8, np.int32, "tab"),
    "pi_nlast": (9, np.int32, "tab"), "fov": (10, np.uint8, "tab"), "valid": (11, np.uint8, "vol"),
}

EXPORTED = ["katsevich_plan", "katsevich_plan_query", "katsevich_plan_bind",
            "katsevich_plan_export", "katsevich_recon", "katsevich_filter",
            "katsevich_backproject", "katsevich_recon_backward", "katsevich_backproject_batch",
            "katsevich_plan_destroy", "katsevich_status_string", "katsevich_last_error",
            "katsevich_plan_device", "katsevich_plan_device_sizes",
            "katsevich_sparse_upsample", "katsevich_data_scratch_bytes", "katsevich_max",
            "katsevich_add_noise", "katsevich_rmse_ssim", "katsevich_rmse_ssim_noscratch"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkatsevich.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise KatsevichError(-1, f"{path} not found: build it with "
                                 "`python -m paper_2201_02309_amd.build`")
    lib = ctypes.CDLL(path)
    lib.katsevich_plan.argtypes = [POINTER(_Geometry), POINTER(_Grid), POINTER(_Options),
                                   POINTER(c_void_p)]
    lib.katsevich_plan_query.argtypes = [c_void_p, POINTER(_Info)]
    lib.katsevich_plan_bind.argtypes = [c_void_p, c_void_p, c_uint64, c_void_p]
    lib.katsevich_plan_export.argtypes = [c_void_p, c_int, c_void_p, c_uint64]
    lib.katsevich_recon.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p]
    lib.katsevich_filter.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p]
    lib.katsevich_backproject.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.katsevich_recon_backward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_uint64,
                                             c_void_p]
    lib.katsevich_backproject_batch.argtypes = [POINTER(c_void_p), POINTER(c_void_p),
                                                POINTER(c_void_p), c_int, c_void_p]
    lib.katsevich_plan_device.argtypes = [POINTER(_Geometry), POINTER(_Grid), POINTER(_Options),
                                          c_void_p, c_uint64, c_void_p, c_uint64, c_void_p,
                                          POINTER(c_void_p)]
    lib.katsevich_plan_device.restype = c_int
    lib.katsevich_plan_device_sizes.argtypes = [POINTER(_Geometry), POINTER(_Grid), POINTER(_Options),
                                                POINTER(_DevSizes)]
    lib.katsevich_plan_device_sizes.restype = c_int
    lib.katsevich_sparse_upsample.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p]
    lib.katsevich_sparse_upsample.restype = c_int
    lib.katsevich_data_scratch_bytes.argtypes = []
    lib.katsevich_data_scratch_bytes.restype = c_uint64
    lib.katsevich_max.argtypes = [c_void_p, c_uint64, c_void_p, c_void_p, c_uint64, c_void_p]
    lib.katsevich_max.restype = c_int
    lib.katsevich_add_noise.argtypes = [c_void_p, c_void_p, c_uint64, c_void_p, c_double, c_double,
                                        c_uint64, c_void_p]
    lib.katsevich_add_noise.restype = c_int
    lib.katsevich_rmse_ssim.argtypes = [c_void_p, c_void_p, c_uint64, c_void_p, c_void_p, c_uint64,
                                        c_void_p]
    lib.katsevich_rmse_ssim.restype = c_int
    lib.katsevich_rmse_ssim_noscratch.argtypes = [c_void_p, c_void_p, c_uint64, c_void_p, c_void_p]
    lib.katsevich_rmse_ssim_noscratch.restype = c_int
    lib.katsevich_plan_destroy.argtypes = [c_void_p]
    lib.katsevich_plan_destroy.restype = None
    lib.katsevich_status_string.argtypes = [c_int]
    lib.katsevich_status_string.restype = c_char_p
    lib.katsevich_last_error.argtypes = []
    lib.katsevich_last_error.restype = c_char_p
    for name in EXPORTED[:9]:
        getattr(lib, name).restype = c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def _check(lib, status):
    if status != 0:
        raise KatsevichError(status, lib.katsevich_last_error().decode() or
                             lib.katsevich_status_string(status).decode())


def _geom_struct(g: dict) -> _Geometry:
    return _Geometry(R=g["R"], D=g["D"], feed_per_turn=g["feed_per_turn"],
                     lambda0=g.get("lambda0", 0.0), z0=g.get("z0", 0.0),
                     lambda_first=g.get("lambda_first", 0.0), dalpha=g["dalpha"],
                     col_offset=g.get("col_offset", 0.0), dw=g["dw"],
                     row_offset=g.get("row_offset", 0.0), n_views=int(g["n_views"]),
                     views_per_turn=int(g["views_per_turn"]), det_cols=int(g["det_cols"]),
                     det_rows=int(g["det_rows"]), reserved=0)


def _grid_struct(g: dict) -> _Grid:
    return _Grid(dx=g["dx"], dy=g["dy"], dz=g["dz"], x_first=g["x_first"], y_first=g["y_first"],
                 z_first=g["z_first"], nx=int(g["nx"]), ny=int(g["ny"]), nz=int(g["nz"]),
                 reserved=0)


def _stream_handle(device=None):
    import torch
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A float64 host plan (katsevich_plan) plus its device tables (katsevich_plan_bind).

    geom / grid: dicts with the fields of katsevich_geometry / katsevich_grid."""

    def __init__(self, geom: dict, grid: dict, n_psi: int = 0, n_threads: int = 0,
                 bind: bool = True, device=None, bp_slices: int = 0, gpu_plan: bool = False,
                 half_sample: bool = False, keep_pi_scratch: bool = False,
                 deterministic_adjoint: bool = False, hilbert_mode: int = 0):
        """gpu_plan: build the whole plan on the GPU (katsevich_plan_device) on `device` and
        its current stream, straight into the plan's table tensor (the plan is then bound
        whatever `bind` says); otherwise on the host (katsevich_plan).  keep_pi_scratch
        (gpu_plan only): keep the build's scratch, whose float64 PI tables pi_tables() reads.
        half_sample: KATS_FLAG_HALF_SAMPLE_DERIVATIVE (derivative at the centres of the
        sinogram's 2 x 2 (lambda, alpha) cells).  deterministic_adjoint:
        KATS_FLAG_DETERMINISTIC_ADJOINT (bit-reproducible recon_backward).  hilbert_mode:
        HILBERT_AUTO, HILBERT_FFT or HILBERT_MFMA (the Hilbert filter as register FFTs or as
        a Toeplitz product on the matrix cores)."""
        self._lib = load_library()
        self.geom = dict(geom)
        self.grid = dict(grid)
        self._h = c_void_p()
        self.tables = None
        self._ws = None
        self.device = None
        self._pi_scratch = None
        opts = _Options(n_psi=int(n_psi), n_threads=int(n_threads),
                        flags=(FLAG_HALF_SAMPLE_DERIVATIVE if half_sample else 0) |
                        (FLAG_DETERMINISTIC_ADJOINT if deterministic_adjoint else 0),
                        bp_slices=int(bp_slices), hilbert_mode=int(hilbert_mode))
        g, gr = _geom_struct(geom), _grid_struct(grid)
        if gpu_plan:
            import torch
            dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
            sz = _DevSizes()
            _check(self._lib, self._lib.katsevich_plan_device_sizes(byref(g), byref(gr), byref(opts),
                                                                    byref(sz)))
            with torch.cuda.device(dev):
                scratch = torch.empty(max(int(sz.scratch_bytes), 256), dtype=torch.uint8, device=dev)
                tables = torch.empty(max(int(sz.table_bytes), 256), dtype=torch.uint8, device=dev)
                _check(self._lib, self._lib.katsevich_plan_device(
                    byref(g), byref(gr), byref(opts), c_void_p(scratch.data_ptr()),
                    c_uint64(scratch.numel()), c_void_p(tables.data_ptr()), c_uint64(tables.numel()),
                    _stream_handle(dev), byref(self._h)))
            self.tables, self.device = tables, dev
            if keep_pi_scratch:
                self._pi_scratch = (scratch, {k: getattr(sz, k) for k, _ in _DevSizes._fields_})
            del scratch
        else:
            _check(self._lib, self._lib.katsevich_plan(byref(g), byref(gr), byref(opts),
                                                       byref(self._h)))
        info = _Info()
        _check(self._lib, self._lib.katsevich_plan_query(self._h, byref(info)))
        self.info = {k: getattr(info, k) for k, _ in _Info._fields_}
        if bind and self.tables is None:
            self.bind(device)

    def pi_tables(self) -> dict:
        """Float64 PI tables of a plan built with gpu_plan=True, keep_pi_scratch=True, read
        from the build's scratch: li, lo (view units), nf, nl (first / last covered view),
        fov, each [n_table_slices, ny, nx]."""
        if self._pi_scratch is None:
            raise KatsevichError(-1, "pi_tables needs a plan built with gpu_plan=True, keep_pi_scratch=True")
        scratch, sz = self._pi_scratch
        n = int(sz["n_table_slices"]) * int(self.grid["ny"]) * int(self.grid["nx"])
        shape = (int(sz["n_table_slices"]), int(self.grid["ny"]), int(self.grid["nx"]))
        host = scratch.cpu().numpy()
        out = {}
        for key, off, dt in (("li", "pi_li_offset", np.float64), ("lo", "pi_lo_offset", np.float64),
                             ("nf", "pi_nfirst_offset", np.int32), ("nl", "pi_nlast_offset", np.int32),
                             ("fov", "fov_offset", np.uint8)):
            o = int(sz[off])
            out[key] = host[o:o + n * np.dtype(dt).itemsize].view(dt).reshape(shape).copy()
        return out

    # ------------------------------------------------------------------ device side
    def bind(self, device=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nbytes = max(int(self.info["table_bytes"]), 256)
        with torch.cuda.device(dev):
            self.tables = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _check(self._lib, self._lib.katsevich_plan_bind(
                self._h, c_void_p(self.tables.data_ptr()), c_uint64(nbytes), _stream_handle(dev)))
        self.device = dev
        return self

    def workspace(self, ws=None):
        import torch
        need = int(self.info["workspace_bytes"])
        if ws is not None:
            return ws
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def release_workspace(self):
        self._ws = None

    # ------------------------------------------------------------------ host side
    def export(self, name: str) -> np.ndarray:
        which, dtype, shape_key = TABLES[name]
        i, g, gr = self.info, self.geom, self.grid
        cols = int(g["det_cols"]) - int(i["half_sample"])     # columns of the filtered grid
        shape = {"psi_cols": (i["n_psi"], cols),
                 "rows_cols": (g["det_rows"], cols),
                 "tab": (i["n_table_slices"], gr["ny"], gr["nx"]),
                 "vol": (gr["nz"], gr["ny"], gr["nx"])}[shape_key]
        out = np.empty(shape, dtype=dtype)
        _check(self._lib, self._lib.katsevich_plan_export(self._h, which,
                                                          out.ctypes.data_as(c_void_p),
                                                          c_uint64(out.nbytes)))
        return out

    @property
    def n_filtered(self) -> int:
        return max(0, int(self.info["last_view"]) - int(self.info["first_view"]) + 1)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.katsevich_plan_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _require(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise KatsevichError(-3, f"{name} must be a contiguous float32 CUDA tensor of shape "
                                 f"{tuple(shape)}, got {getattr(t, 'shape', None)} "
                                 f"{getattr(t, 'dtype', None)}")


def _sino_shape(plan):
    g = plan.geom
    return (int(g["n_views"]), int(g["det_rows"]), int(g["det_cols"]))


def _vol_shape(plan):
    gr = plan.grid
    return (int(gr["nz"]), int(gr["ny"]), int(gr["nx"]))


def recon(plan: Plan, sino, out=None, ws=None):
    """katsevich_recon on the current stream: sino [n_views, rows, cols] -> vol [nz, ny, nx]."""
    import torch
    _require(sino, _sino_shape(plan), "sino")
    if out is None:
        out = torch.empty(_vol_shape(plan), dtype=torch.float32, device=sino.device)
    _require(out, _vol_shape(plan), "out")
    ws = plan.workspace(ws)
    _check(plan._lib, plan._lib.katsevich_recon(plan.handle, c_void_p(sino.data_ptr()),
                                                c_void_p(out.data_ptr()), c_void_p(ws.data_ptr()),
                                                c_uint64(ws.numel() * ws.element_size()),
                                                _stream_handle(sino.device)))
    return out


PAD = 2   # zero border (cells) around every filtered view, see include/katsevich.h


def filtered_shape(plan: Plan):
    """Shape of the g^F buffer: [n_filtered, gf_rows, gf_cols] (zero border of PAD cells;
    gf_cols is cols + 2 PAD rounded up to a multiple of 4)."""
    return (plan.n_filtered, int(plan.info["gf_rows"]), int(plan.info["gf_cols"]))


def filter_views(plan: Plan, sino, out=None, ws=None):
    """katsevich_filter: sino -> zero-padded g^F of views first_view..last_view."""
    import torch
    _require(sino, _sino_shape(plan), "sino")
    shape = filtered_shape(plan)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=sino.device)
    _require(out, shape, "out")
    ws = plan.workspace(ws)
    _check(plan._lib, plan._lib.katsevich_filter(plan.handle, c_void_p(sino.data_ptr()),
                                                 c_void_p(out.data_ptr()), c_void_p(ws.data_ptr()),
                                                 c_uint64(ws.numel() * ws.element_size()),
                                                 _stream_handle(sino.device)))
    return out


def backproject(plan: Plan, gF, out=None):
    """katsevich_backproject: zero-padded g^F (views first_view..last_view) -> vol."""
    import torch
    shape = filtered_shape(plan)
    _require(gF, shape, "gF")
    if out is None:
        out = torch.empty(_vol_shape(plan), dtype=torch.float32, device=gF.device)
    _require(out, _vol_shape(plan), "out")
    _check(plan._lib, plan._lib.katsevich_backproject(plan.handle, c_void_p(gF.data_ptr()),
                                                      c_void_p(out.data_ptr()),
                                                      _stream_handle(gF.device)))
    return out


def backproject_batch(plans, gFs, vols=None):
    """katsevich_backproject_batch: grouped launches backprojecting every (plans[i], gFs[i])
    into vols[i] (allocated if None).  Returns the volumes."""
    import torch
    n = len(plans)
    if n == 0:
        return []
    lib = plans[0]._lib
    if vols is None:
        vols = [torch.empty(_vol_shape(p), dtype=torch.float32, device=g.device)
                for p, g in zip(plans, gFs)]
    for p, g, v in zip(plans, gFs, vols):
        _require(g, filtered_shape(p), "gF")
        _require(v, _vol_shape(p), "vol")
    arr = c_void_p * n
    hp = arr(*[p.handle.value for p in plans])
    hg = arr(*[g.data_ptr() for g in gFs])
    hv = arr(*[v.data_ptr() for v in vols])
    _check(lib, lib.katsevich_backproject_batch(hp, hg, hv, n, _stream_handle(gFs[0].device)))
    return vols


# ---------------------------------------------------------------- data path and metrics
def _f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise KatsevichError(-1, f"{name}: expected a contiguous float32 CUDA tensor")
    return t


def _data_scratch(device):
    import torch
    lib = load_library()
    return torch.empty(max(int(lib.katsevich_data_scratch_bytes()), 256), dtype=torch.uint8,
                       device=device)


def sparse_upsample(sparse, cols: int, step: int = 4, out=None):
    """katsevich_sparse_upsample: [..., ceil(cols/step)] sparse columns -> [..., cols]."""
    import torch
    _f32(sparse, "sparse")
    if int(cols) < 1 or int(step) < 1:
        raise KatsevichError(-1, f"need cols >= 1 and step >= 1 (got {cols}, {step})")
    ns = (int(cols) + int(step) - 1) // int(step)
    if sparse.shape[-1] != ns:
        raise KatsevichError(-3, f"sparse: last dimension {sparse.shape[-1]} != ceil(cols/step) = {ns}")
    shape = tuple(sparse.shape[:-1]) + (int(cols),)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=sparse.device)
    _f32(out, "out")
    if tuple(out.shape) != shape:
        raise KatsevichError(-3, f"out: shape {tuple(out.shape)} != {shape}")
    lib = load_library()
    _check(lib, lib.katsevich_sparse_upsample(c_void_p(sparse.data_ptr()), c_void_p(out.data_ptr()),
                                              c_int64(sparse.numel() // ns), c_int32(int(cols)),
                                              c_int32(int(step)), _stream_handle(sparse.device)))
    return out


def max_value(x, scratch=None, out=None):
    """katsevich_max: device float32 tensor [1] holding max(x)."""
    import torch
    _f32(x, "x")
    scratch = _data_scratch(x.device) if scratch is None else scratch
    out = torch.empty(1, dtype=torch.float32, device=x.device) if out is None else out
    lib = load_library()
    _check(lib, lib.katsevich_max(c_void_p(x.data_ptr()), c_uint64(x.numel()), c_void_p(out.data_ptr()),
                                  c_void_p(scratch.data_ptr()), c_uint64(scratch.numel()),
                                  _stream_handle(x.device)))
    return out


def add_noise(g, I0: float = 1e5, var: float = 0.5, seed: int = 0, d_max=None, out=None):
    """katsevich_add_noise (Sec. III-C noise model); d_max defaults to max_value(g)."""
    import torch
    _f32(g, "g")
    d_max = max_value(g) if d_max is None else d_max
    if out is None:
        out = torch.empty_like(g)
    _f32(out, "out")
    if out.shape != g.shape:
        raise KatsevichError(-3, "out: shape differs from g")
    lib = load_library()
    _check(lib, lib.katsevich_add_noise(c_void_p(g.data_ptr()), c_void_p(out.data_ptr()),
                                        c_uint64(g.numel()), c_void_p(d_max.data_ptr()),
                                        c_double(I0), c_double(var), c_uint64(int(seed)),
                                        _stream_handle(g.device)))
    return out


def rmse_ssim(f, ref, scratch=None, result=None):
    """katsevich_rmse_ssim: device float64 tensor [2] = (RMSE, SSIM) of f against ref."""
    import torch
    _f32(f, "f")
    _f32(ref, "ref")
    if f.shape != ref.shape:
        raise KatsevichError(-3, "f and ref differ in shape")
    scratch = _data_scratch(f.device) if scratch is None else scratch
    result = torch.empty(2, dtype=torch.float64, device=f.device) if result is None else result
    lib = load_library()
    _check(lib, lib.katsevich_rmse_ssim(c_void_p(f.data_ptr()), c_void_p(ref.data_ptr()),
                                        c_uint64(f.numel()), c_void_p(result.data_ptr()),
                                        c_void_p(scratch.data_ptr()), c_uint64(scratch.numel()),
                                        _stream_handle(f.device)))
    return result


def rmse_ssim_noscratch(f, ref, result=None):
    """katsevich_rmse_ssim_noscratch: as rmse_ssim, with the library's static device scratch
    (no scratch buffer; calls overlapping on one GPU race)."""
    import torch
    _f32(f, "f")
    _f32(ref, "ref")
    if f.shape != ref.shape:
        raise KatsevichError(-3, "f and ref differ in shape")
    result = torch.empty(2, dtype=torch.float64, device=f.device) if result is None else result
    lib = load_library()
    _check(lib, lib.katsevich_rmse_ssim_noscratch(c_void_p(f.data_ptr()), c_void_p(ref.data_ptr()),
                                                  c_uint64(f.numel()), c_void_p(result.data_ptr()),
                                                  _stream_handle(f.device)))
    return result


def recon_backward(plan: Plan, grad_vol, out=None, ws=None):
    """katsevich_recon_backward: exact adjoint, grad_vol [nz, ny, nx] -> grad_sino."""
    import torch
    _require(grad_vol, _vol_shape(plan), "grad_vol")
    if out is None:
        out = torch.empty(_sino_shape(plan), dtype=torch.float32, device=grad_vol.device)
    _require(out, _sino_shape(plan), "out")
    ws = plan.workspace(ws)
    _check(plan._lib, plan._lib.katsevich_recon_backward(
        plan.handle, c_void_p(grad_vol.data_ptr()), c_void_p(out.data_ptr()),
        c_void_p(ws.data_ptr()), c_uint64(ws.numel() * ws.element_size()),
        _stream_handle(grad_vol.device)))
    return out


def _autograd_function():
    import torch

    class KatsevichFn(torch.autograd.Function):
        """Differentiable reconstruction: forward = katsevich_recon, backward = its exact
        adjoint katsevich_recon_backward (the operator is linear, nothing is saved but the
        plan).  Accepts [n_views, rows, cols] or a batch [B, n_views, rows, cols]."""

        @staticmethod
        def forward(ctx, sino, plan):
            ctx.plan = plan
            s = sino.contiguous()
            if s.dim() == 4:
                return torch.stack([recon(plan, s[b]) for b in range(s.shape[0])])
            return recon(plan, s)

        @staticmethod
        def backward(ctx, grad):
            plan = ctx.plan
            g = grad.contiguous()
            if g.dim() == 4:
                out = torch.stack([recon_backward(plan, g[b]) for b in range(g.shape[0])])
            else:
                out = recon_backward(plan, g)
            return out, None

    return KatsevichFn


class _LazyFn:
    _fn = None

    def __getattr__(self, name):
        if _LazyFn._fn is None:
            _LazyFn._fn = _autograd_function()
        return getattr(_LazyFn._fn, name)


KatsevichFn = _LazyFn()
