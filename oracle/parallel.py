"""Process-parallel drivers of the float64 oracle, for full-size checks and CPU timing.

TEST INFRASTRUCTURE ONLY: used by tests/ and the cpu_baseline leg of bench.py.  Nothing here
adds arithmetic: every worker calls the oracle's own functions (katsevich_oracle) on a part
of the work -- a slice of the table pitch for the PI lines (Sec. II pre-calculating step 2),
a block of views for the filtering chain (Sec. II steps 1-6), one slice for the
backprojection (step 7), one view for the transpose of the backprojection -- and the parent
puts the parts together in the order of katsevich_oracle.recon(mode="pitch").

Workers are spawned (fresh interpreters: no state of the parent, e.g. a GPU runtime, is
inherited), each limited to one BLAS thread; large arrays travel through POSIX shared memory.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import get_context, shared_memory

import numpy as np

from . import katsevich_oracle as O

TWO_PI = 2.0 * math.pi
_LIMIT = None


def default_workers() -> int:
    """Processes to use: the CPUs this process may run on, at most 16 (the host share of one
    GPU on the machines this runs on)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:                      # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _init_worker():
    global _LIMIT
    from threadpoolctl import threadpool_limits
    _LIMIT = threadpool_limits(limits=1)


def pool(workers: int):
    return ProcessPoolExecutor(max_workers=workers, mp_context=get_context("spawn"),
                               initializer=_init_worker)


class Shared:
    """A numpy array in POSIX shared memory; `spec` names it for attach() in a worker."""

    def __init__(self, shape, dtype, src=None):
        dtype = np.dtype(dtype)
        size = max(1, int(np.prod(shape)) * dtype.itemsize)
        self.shm = shared_memory.SharedMemory(create=True, size=size)
        self.arr = np.ndarray(shape, dtype, buffer=self.shm.buf)
        if src is not None:
            self.arr[...] = src
        self.spec = (self.shm.name, tuple(shape), dtype.str)

    def close(self):
        self.arr = None
        self.shm.close()
        self.shm.unlink()


def attach(spec):
    name, shape, dtype = spec
    shm = shared_memory.SharedMemory(name=name)
    return shm, np.ndarray(shape, np.dtype(dtype), buffer=shm.buf)


# ----------------------------------------------------------------------------- PI tables
def _pi_slice(geom, grid, j):
    scan = O.Scan(geom)
    x, y = O.grid_xy(grid)
    Y, X = np.meshgrid(y, x, indexing="ij")
    Z = np.full(X.shape, grid["z_first"] + j * grid["dz"])
    lam_i, lam_o = O.pi_line(scan, X, Y, Z)
    li, lo, nf, nl = O.pi_view_bounds(scan, lam_i, lam_o)
    return j, lam_i, lam_o, li, lo, nf, nl, O.in_fov(scan, X, Y)


def pitch_tables(geom: dict, grid: dict, workers: int | None = None, ex=None):
    """katsevich_oracle.pitch_tables, one slice of the table pitch per task."""
    scan = O.Scan(geom)
    pit = O.Pitches(scan, grid)
    shape = (pit.n_tab, int(grid["ny"]), int(grid["nx"]))
    out = {k: np.empty(shape) for k in ("lam_i", "lam_o", "li", "lo")}
    out.update(nf=np.empty(shape, np.int64), nl=np.empty(shape, np.int64),
               fov=np.empty(shape, bool))
    own = ex is None
    ex = ex or pool(workers or default_workers())
    try:
        futs = [ex.submit(_pi_slice, geom, grid, j) for j in range(pit.n_tab)]
        for f in futs:
            j, *vals = f.result()
            for key, v in zip(("lam_i", "lam_o", "li", "lo", "nf", "nl", "fov"), vals):
                out[key][j] = v
    finally:
        if own:
            ex.shutdown()
    fov = out["fov"]
    out["n_lo"] = int(out["nf"][fov].min()) - 1
    out["n_hi"] = int(out["nl"][fov].max()) + 1
    out["pitches"] = pit
    return out


# ----------------------------------------------------------------------------- filtering
def _filter_block(geom, n_psi, gspec, a, b, ospec, a0):
    """g^F of views a .. b-1 (indices into the shared input block) -> output rows a-a0 .."""
    shm_g, g = attach(gspec)
    shm_o, out = attach(ospec)
    try:
        scan = O.Scan(geom, n_psi)
        lo, hi = max(a - 1, 0), min(b + 1, g.shape[0])
        res = O.filter_views(scan, g[lo:hi])
        # filter_views leaves the first / last view of its block at 0: only views with both
        # neighbours inside the block are taken from it
        for n in range(a, b):
            if lo < n < hi - 1:
                out[n - a0] = res[n - lo]
            else:
                out[n - a0] = 0.0
    finally:
        del g, out
        shm_g.close()
        shm_o.close()


def filter_views(geom: dict, g, n_psi: int = 0, workers: int | None = None, ex=None,
                 block: int = 64):
    """katsevich_oracle.filter_views of a block of consecutive views (first / last view 0),
    split into blocks of views that each worker filters with their neighbours."""
    g = np.asarray(g)
    V = g.shape[0]
    gs = Shared(g.shape, np.float64, g)
    os_ = Shared(g.shape, np.float64)
    own = ex is None
    ex = ex or pool(workers or default_workers())
    try:
        futs = [ex.submit(_filter_block, geom, n_psi, gs.spec, a, min(a + block, V), os_.spec, 0)
                for a in range(0, V, block)]
        for f in futs:
            f.result()
        out = os_.arr.copy()
    finally:
        if own:
            ex.shutdown()
        gs.close()
        os_.close()
    out[0] = 0.0
    out[-1] = 0.0
    return out


# ----------------------------------------------------------------------------- backprojection
def _bp_slice(geom, grid, fspec, a, k, iz, j, li, lo, nf, nl, m):
    shm, gF = attach(fspec)
    try:
        scan = O.Scan(geom)
        x, y = O.grid_xy(grid)
        Y2, X2 = np.meshgrid(y, x, indexing="ij")
        zj = grid["z_first"] + j * grid["dz"]
        vals = O.backproject(scan, gF, a, X2[m], Y2[m], np.full(int(m.sum()), zj), li, lo, nf, nl,
                             lam_shift=TWO_PI * k)
    finally:
        del gF
        shm.close()
    return iz, vals


def warm(_=None) -> int:
    """A no-op task: submitting one per worker starts every worker process (interpreter and
    imports) before a timed region."""
    return os.getpid()


def recon(geom: dict, grid: dict, g, workers: int | None = None, tables=None, ex=None):
    """katsevich_oracle.recon(mode="pitch") with the PI lines, the filtering of each pitch
    window and the backprojection of each slice spread over worker processes (those of the
    executor ex when given)."""
    scan = O.Scan(geom)
    g = np.asarray(g)
    nx, ny, nz = int(grid["nx"]), int(grid["ny"]), int(grid["nz"])
    f = np.zeros((nz, ny, nx))
    valid = np.zeros((nz, ny, nx), dtype=bool)
    own = ex is None
    ex = ex or pool(workers or default_workers())
    try:
        tab = tables or pitch_tables(geom, grid, ex=ex)
        pit = tab["pitches"]
        for k in range(pit.n_pitches):
            sl, js = pit.slices(k)
            shift = k * scan.Nv
            a = max(tab["n_lo"] + shift, 0)
            b = min(tab["n_hi"] + shift, scan.N - 1)
            if b - a < 2:
                continue
            nf = tab["nf"][js] + shift
            nl = tab["nl"][js] + shift
            vk = O.valid_mask(scan, nf, nl, tab["fov"][js])
            valid[sl] = vk
            if not vk.any():
                continue
            gF = filter_views(geom, g[a:b + 1], ex=ex)
            fs = Shared(gF.shape, np.float64, gF)
            try:
                futs = []
                for jj, (iz, j) in enumerate(zip(sl, js)):
                    m = vk[jj]
                    if not m.any():
                        continue
                    futs.append(ex.submit(_bp_slice, geom, grid, fs.spec, a, k, int(iz), int(j),
                                          tab["li"][j][m] + shift, tab["lo"][j][m] + shift,
                                          nf[jj][m], nl[jj][m], m))
                for fu in futs:
                    iz, vals = fu.result()
                    f[iz][valid[iz]] = vals
            finally:
                fs.close()
    finally:
        if own:
            ex.shutdown()
    return f, valid


# ----------------------------------------------------------------------------- adjoint views
def _bpT_view(geom, grid, tspec, fspec, n):
    """Transpose of the backprojection into view n alone, summed over every pitch whose
    voxels' PI windows contain it."""
    shms, arrs = zip(*(attach(s) for s in tspec))
    shm_f, fbar = attach(fspec)
    li, lo, nf, nl, fov = arrs
    try:
        scan = O.Scan(geom)
        pit = O.Pitches(scan, grid)
        x, y = O.grid_xy(grid)
        Y2, X2 = np.meshgrid(y, x, indexing="ij")
        out = np.zeros((scan.rows, scan.cols))
        for k in range(pit.n_pitches):
            sl, js = pit.slices(k)
            shift = k * scan.Nv
            for iz, j in zip(sl, js):
                nfk, nlk = nf[j] + shift, nl[j] + shift
                m = O.valid_mask(scan, nfk, nlk, fov[j]) & (nfk <= n) & (n <= nlk)
                if not m.any():
                    continue
                cnt = int(m.sum())
                zj = grid["z_first"] + j * grid["dz"]
                out += O.backproject_T(scan, fbar[iz][m], n, 1, X2[m], Y2[m], np.full(cnt, zj),
                                       li[j][m] + shift, lo[j][m] + shift, np.full(cnt, n),
                                       np.full(cnt, n), lam_shift=TWO_PI * k)[0]
    finally:
        del arrs, fbar, li, lo, nf, nl, fov, m
        for s in shms:
            s.close()
        shm_f.close()
    return n, out


def adjoint_views(geom: dict, grid: dict, fbar, views, workers: int | None = None, tables=None):
    """Rows of katsevich_oracle.recon_T(fbar) at the given sinogram views, without the rest:
    the transpose of the backprojection into views n-1, n, n+1 (every voxel whose PI window
    contains them, over all pitches), then the transpose of the filter chain on that
    three-view block, whose middle view is the cotangent of view n (the derivative in lambda
    couples each view to its two neighbours only).  Returns {n: [rows, cols]}."""
    scan = O.Scan(geom)
    need = sorted({int(m) for n in views for m in (n - 1, n, n + 1) if 0 <= m < scan.N})
    with pool(workers or default_workers()) as ex:
        tab = tables or pitch_tables(geom, grid, ex=ex)
        ts = [Shared(tab[k].shape, tab[k].dtype, tab[k]) for k in ("li", "lo", "nf", "nl", "fov")]
        fs = Shared(np.shape(fbar), np.float64, fbar)
        try:
            futs = [ex.submit(_bpT_view, geom, grid, [t.spec for t in ts], fs.spec, m)
                    for m in need]
            gFbar = dict(f.result() for f in futs)
        finally:
            for t in ts:
                t.close()
            fs.close()
    out = {}
    zero = np.zeros((scan.rows, scan.cols))
    for n in views:
        blk = np.stack([zero] + [gFbar.get(m, zero) for m in (n - 1, n, n + 1)] + [zero])
        out[int(n)] = O.filter_views_T(scan, blk)[2]
    return out
