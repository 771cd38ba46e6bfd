"""ctypes wrapper of synth/libsynth_project.so: the FP64 closed-form ellipsoid projector on
the GPU, used to make large synthetic sinograms resident in HBM (harness only)."""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_DIR, "libsynth_project.so")
SRC = os.path.join(_DIR, "projector.hip")
_lib = None


def build():
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("synth projector build failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} missing: run __graft_entry__.build()")
        _lib = ctypes.CDLL(LIB)
        _lib.synth_project_ellipsoids.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_longlong, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_void_p]
        _lib.synth_project_ellipsoids.restype = ctypes.c_int
    return _lib


def ellipsoid_records(ph: dict) -> np.ndarray:
    n = len(ph["density"])
    rec = np.zeros((n, 16))
    for i in range(n):
        rec[i, 0:3] = ph["centre"][i]
        rec[i, 3:12] = (ph["rot"][i] / ph["axes"][i][None, :]).reshape(-1)
        rec[i, 12] = ph["density"][i]
    return rec


def project(ph: dict, geom: dict, views=None, device="cuda", out=None):
    """float32 sinogram [n_views(or len(views)), rows, cols] on the GPU (FP64 arithmetic)."""
    import torch
    assert ph["kind"] == "ellipsoids"
    lib = _load()
    if views is None:
        view0, nv = 0, int(geom["n_views"])
    else:
        view0, nv = int(views[0]), int(views[-1]) - int(views[0]) + 1
    rows, cols = int(geom["det_rows"]), int(geom["det_cols"])
    if out is None:
        out = torch.empty((nv, rows, cols), dtype=torch.float32, device=device)
    rec = torch.tensor(ellipsoid_records(ph), dtype=torch.float64, device=device)
    scan = np.array([geom["R"], geom["D"], geom["feed_per_turn"] / (2 * math.pi),
                     geom.get("lambda0", 0.0), geom.get("z0", 0.0), geom.get("lambda_first", 0.0),
                     2 * math.pi / geom["views_per_turn"], geom["dalpha"],
                     geom.get("col_offset", 0.0), geom["dw"], geom.get("row_offset", 0.0)],
                    dtype=np.float64)
    stream = ctypes.c_void_p(torch.cuda.current_stream(out.device).cuda_stream)
    st = lib.synth_project_ellipsoids(scan.ctypes.data_as(ctypes.c_void_p), rows, cols,
                                      ctypes.c_void_p(rec.data_ptr()), rec.shape[0], view0, nv,
                                      ctypes.c_void_p(out.data_ptr()), stream)
    if st != 0:
        raise RuntimeError("synth projector launch failed")
    torch.cuda.current_stream(out.device).synchronize()
    del rec
    return out
