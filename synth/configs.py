"""Workload recipes: helical scan geometry + voxel grid for each benchmark configuration.

Conventions (shared vocabulary of the C-ABI structs ``katsevich_geometry`` and
``katsevich_grid``):

* helix  a(lambda) = (R cos(lambda+lambda0), R sin(lambda+lambda0), z0 + P lambda / 2pi)
  (paper Sec. II, helix equation), P = table feed per turn;
* view n sits at lambda_n = lambda_first + n * 2pi / views_per_turn;
* curved detector (radius D about the source): column c at fan angle
  alpha_c = (c - (cols-1)/2 + col_offset) * dalpha, row r at height
  w_r = (r - (rows-1)/2 + row_offset) * dw  (paper Sec. III-C, detector coordinates);
* voxel (ix, iy, iz) at (x_first + ix dx, y_first + iy dy, z_first + iz dz),
  stored [nz, ny, nx] with x fastest.

Detector sizing (a recipe, not part of the method): the half fan angle covers the
radius r_cov of everything that must be reconstructed, alpha_m = asin(r_cov / R),
dalpha = 2 alpha_m / (cols - 1); the rows cover the Tam-Danielsson window with a
10 % margin, i.e. the outermost row centres sit at +-1.1 * w_TD where
w_TD = (D P / 2pi R) (pi/2 + alpha_m) / cos(alpha_m) is the TD boundary height at
the fan edge.  The z spacing divides the feed so that slices repeat every pitch.
"""
from __future__ import annotations

import math

import numpy as np
from dataclasses import dataclass, field, asdict


@dataclass
class Geometry:
    R: float
    D: float
    feed_per_turn: float
    views_per_turn: int
    n_views: int
    det_cols: int
    det_rows: int
    dalpha: float
    dw: float
    lambda0: float = 0.0
    z0: float = 0.0
    lambda_first: float = 0.0
    col_offset: float = 0.0
    row_offset: float = 0.0

    def as_dict(self):
        return asdict(self)


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x_first: float
    y_first: float
    z_first: float

    def as_dict(self):
        return asdict(self)


@dataclass
class Workload:
    name: str
    geom: Geometry
    grid: Grid
    phantom: dict = field(default_factory=dict)   # recipe for synth.phantom.make_phantom
    seed: int = 0
    n_psi: int = 0                                 # 0 -> 2*rows+1
    batch: int = 1

    def as_dict(self):
        return {"name": self.name, "geom": self.geom.as_dict(), "grid": self.grid.as_dict(),
                "phantom": dict(self.phantom), "seed": self.seed, "n_psi": self.n_psi,
                "batch": self.batch}


def detector_for(R, D, feed, cols, rows, r_cov, td_margin=1.1):
    """(dalpha, dw) of the sizing recipe in the module docstring."""
    h = feed / (2.0 * math.pi)
    alpha_m = math.asin(r_cov / R)
    dalpha = 2.0 * alpha_m / (cols - 1)
    w_td = D * h / R * (0.5 * math.pi + alpha_m) / math.cos(alpha_m)
    dw = 2.0 * td_margin * w_td / (rows - 1)
    return dalpha, dw


def centred_grid(geom: Geometry, nx, ny, nz, dxy, dz) -> Grid:
    """Grid centred on the z axis and on the mid-height of the acquired helix."""
    h = geom.feed_per_turn / (2.0 * math.pi)
    dlam = 2.0 * math.pi / geom.views_per_turn
    lam_last = geom.lambda_first + (geom.n_views - 1) * dlam
    zmid = geom.z0 + 0.5 * h * (geom.lambda_first + lam_last)
    return Grid(nx=nx, ny=ny, nz=nz, dx=dxy, dy=dxy, dz=dz,
                x_first=-0.5 * (nx - 1) * dxy, y_first=-0.5 * (ny - 1) * dxy,
                z_first=zmid - 0.5 * (nz - 1) * dz)


def corner_radius(nx, ny, dxy):
    return math.hypot(0.5 * (nx - 1) * dxy, 0.5 * (ny - 1) * dxy)


R_DEFAULT = 570.0
D_DEFAULT = 1040.0
# keep every voxel centre a little inside the field-of-view cylinder so that no
# voxel sits on its boundary (an inclusion decision taken by rounding)
FOV_MARGIN_MM = 0.05


def make_workload(name, *, feed, cols, rows, views_per_turn, turns, nxy, nz, dxy,
                  slices_per_pitch=None, dz=None, r_cov=None, phantom=None, seed=0,
                  n_psi=0, batch=1, R=R_DEFAULT, D=D_DEFAULT) -> Workload:
    if dz is None:
        dz = feed / slices_per_pitch
    rc = corner_radius(nxy, nxy, dxy) + FOV_MARGIN_MM
    if r_cov is not None:
        rc = max(rc, r_cov)
    dalpha, dw = detector_for(R, D, feed, cols, rows, rc)
    geom = Geometry(R=R, D=D, feed_per_turn=feed, views_per_turn=views_per_turn,
                    n_views=views_per_turn * turns, det_cols=cols, det_rows=rows,
                    dalpha=dalpha, dw=dw)
    grid = centred_grid(geom, nxy, nxy, nz, dxy, dz)
    return Workload(name=name, geom=geom, grid=grid, phantom=phantom or {}, seed=seed,
                    n_psi=n_psi, batch=batch)


def config1() -> Workload:
    """Parity case: 128x16 curved detector, feed 24 mm/turn, 360 views/turn x 3 turns,
    64^3 grid at 1 mm (24 slices per pitch), 8 ellipsoids in a 28 mm cylinder."""
    return make_workload(
        "parity-64^3", feed=24.0, cols=128, rows=16, views_per_turn=360, turns=3,
        nxy=64, nz=64, dxy=1.0, slices_per_pitch=24, r_cov=28.0 + 25.0,
        phantom={"kind": "ellipsoids", "n": 8, "centre_radius": 28.0,
                 "semi_axes": (5.0, 25.0), "density": (0.1, 1.0), "inserts": 0},
        seed=1001)


def _clinical_phantom(nxy, dxy, n_ell, n_ins):
    half = 0.5 * nxy * dxy
    return {"kind": "ellipsoids", "n": n_ell, "centre_radius": 0.45 * half,
            "semi_axes": (0.06 * half, 0.35 * half), "density": (0.1, 1.0),
            "bound_radius": 0.95 * half, "inserts": n_ins, "insert_radius": (2.0, 6.0),
            "insert_density": 0.02}


def config2() -> Workload:
    """Clinical high pitch: 736x64 detector, feed 76.8 mm/turn, 1160 views/turn x 6 turns,
    512^2 x 128 grid at 0.7 mm in-plane; z spacing 76.8/77 mm (nominal 1.0 mm, made
    commensurate with the feed so per-pitch tables repeat exactly)."""
    return make_workload(
        "clinical-512^2x128", feed=76.8, cols=736, rows=64, views_per_turn=1160, turns=6,
        nxy=512, nz=128, dxy=0.7, slices_per_pitch=77,
        phantom=_clinical_phantom(512, 0.7, 12, 20), seed=1002)


def config3(b=0) -> Workload:
    """Sparse detector + differentiation: 184 columns, feed 96 mm/turn, 6 turns,
    256^2 x 64 grid at 1.4 mm in-plane, 2.0 mm in z (48 slices per pitch)."""
    return make_workload(
        "sparse-256^2x64", feed=96.0, cols=184, rows=64, views_per_turn=1160, turns=6,
        nxy=256, nz=64, dxy=1.4, slices_per_pitch=48,
        phantom=_clinical_phantom(256, 1.4, 12, 20), seed=1003 + b, batch=4)


def config5() -> Workload:
    """Large volume: 736x64 detector, 2304 views/turn x 24 turns, feed 64 mm/turn,
    512^3 grid at 0.7 mm in-plane, 64/107 mm in z (nominal 0.6 mm)."""
    return make_workload(
        "large-512^3", feed=64.0, cols=736, rows=64, views_per_turn=2304, turns=24,
        nxy=512, nz=512, dxy=0.7, slices_per_pitch=107,
        phantom=_clinical_phantom(512, 0.7, 24, 50), seed=1005)


def tiny(nxy=24, nz=16, cols=48, rows=8, views_per_turn=72, turns=3, feed=24.0,
         slices_per_pitch=None, dxy=2.0, seed=7, n_ell=4) -> Workload:
    """Small CPU-test geometry in the same family (R=570, D=1040, curved detector)."""
    if slices_per_pitch is None:
        slices_per_pitch = max(1, int(round(feed / dxy)))
    half = 0.5 * nxy * dxy
    return make_workload(
        f"tiny-{nxy}^2x{nz}", feed=feed, cols=cols, rows=rows,
        views_per_turn=views_per_turn, turns=turns, nxy=nxy, nz=nz, dxy=dxy,
        slices_per_pitch=slices_per_pitch,
        phantom={"kind": "ellipsoids", "n": n_ell, "centre_radius": 0.4 * half,
                 "semi_axes": (0.1 * half, 0.4 * half), "density": (0.1, 1.0),
                 "bound_radius": 0.95 * half, "inserts": 0},
        seed=seed)


def network_pitch(nxy=512, dxy=1.0, cols=627, rows=16, views_per_turn=360, turns=4, h=3.5,
                  slices=10, seed=3001) -> Workload:
    """One pitch of the network workload of Sec. III-C at p = 7 pi (h = 3.5 mm/rad): R = 595,
    D = 1085.6, a curved detector of 627 columns at 0.0625 deg with the quarter-column offset,
    16 rows covering the Tam-Danielsson window + 10 %, 360 views per turn; a 512 x 512 grid
    at 1 mm in-plane and the pitch's 10 slices at 2 pi h / 10 (the paper's 11 z positions
    from 0 to 2 pi h include both ends; 10 of them repeat every pitch).  The field of view
    (radius R sin(alpha_m) ~ 199 mm) leaves the grid's corners out.  Seeded ellipsoids
    inside the field of view."""
    R, D = 595.0, 1085.6
    feed = 2.0 * math.pi * h
    dalpha = math.pi / 2880.0                          # 0.0625 degree
    alpha_m = (0.5 * (cols - 1) + 0.25) * dalpha
    w_td = D * h / R * (0.5 * math.pi + alpha_m) / math.cos(alpha_m)
    dw = 2.0 * 1.1 * w_td / (rows - 1)
    geom = Geometry(R=R, D=D, feed_per_turn=feed, views_per_turn=views_per_turn,
                    n_views=views_per_turn * turns, det_cols=cols, det_rows=rows,
                    dalpha=dalpha, dw=dw, col_offset=0.25)
    grid = centred_grid(geom, nxy, nxy, slices, dxy, feed / slices)
    r_fov = R * math.sin(alpha_m - 0.25 * dalpha) * 0.9
    ph = {"kind": "ellipsoids", "n": 10, "centre_radius": 0.45 * r_fov,
          "semi_axes": (0.06 * r_fov, 0.35 * r_fov), "density": (0.1, 1.0),
          "bound_radius": 0.95 * r_fov, "inserts": 20, "insert_radius": (2.0, 6.0),
          "insert_density": 0.02}
    return Workload(name=f"network-pitch-{nxy}^2x{slices}", geom=geom, grid=grid, phantom=ph,
                    seed=seed)


def with_helix_offsets(wl: Workload, lambda0=0.7, z0=-13.2, lambda_first=0.31) -> Workload:
    """The same workload on a helix with the source at angle lambda0 and height z0 at
    lambda = 0 and the first view at lambda_first (not on the view grid), the grid moved
    with the helix (centred on its new mid-height)."""
    geom = Geometry(**dict(wl.geom.as_dict(), lambda0=lambda0, z0=z0, lambda_first=lambda_first))
    g = wl.grid
    grid = centred_grid(geom, g.nx, g.ny, g.nz, g.dx, g.dz)
    grid.x_first, grid.y_first = g.x_first, g.y_first
    return Workload(name=wl.name + "-offsets", geom=geom, grid=grid, phantom=dict(wl.phantom),
                    seed=wl.seed, n_psi=wl.n_psi, batch=wl.batch)


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}


SERVING_GRIDS = ((256, 32, 1.4), (256, 96, 1.4), (512, 64, 0.7), (512, 160, 0.7))


def serving_request(i: int) -> Workload:
    """Request i of the serving workload, drawn with numpy default_rng(2000 + i): grid from
    {256^2x32, 256^2x96 at 1.4 mm, 512^2x64, 512^2x160 at 0.7 mm}, feed U[40, 96] mm/turn,
    2..10 turns, 736 or 184 (4x sparse) columns, 64 rows, 1160 views/turn; z spacing the
    feed divided by round(feed / 1 mm) so that slices repeat every pitch."""
    rng = np.random.default_rng(2000 + i)
    nxy, nz, dxy = SERVING_GRIDS[int(rng.integers(0, len(SERVING_GRIDS)))]
    feed = float(rng.uniform(40.0, 96.0))
    turns = int(rng.integers(2, 11))
    cols = 736 if rng.uniform() < 0.5 else 184
    ns = max(1, int(round(feed / 1.0)))
    return make_workload(f"serve-{i}", feed=feed, cols=cols, rows=64, views_per_turn=1160,
                         turns=turns, nxy=nxy, nz=nz, dxy=dxy, slices_per_pitch=ns,
                         phantom=_clinical_phantom(nxy, dxy, 12, 20), seed=2000 + i)


def serving_arrivals(n: int, rate: float = 20.0, seed: int = 1004, saturated: bool = False):
    """Poisson arrival times (seconds) of n requests at `rate` per second, or all at 0."""
    if saturated:
        return np.zeros(n)
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
