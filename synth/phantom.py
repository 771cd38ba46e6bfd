"""Seeded phantoms with closed-form line integrals (FP64, NumPy).

Two phantom kinds:

* ``ellipsoids``: additive constant-density ellipsoids.  The line integral of one
  ellipsoid along p(t) = s + t d is density * |d| * 2 sqrt(disc) / A, where the ray is
  mapped into the ellipsoid's unit-sphere frame q = diag(1/a) Q^T (p - c):
  A = |d'|^2, B = s'.d', C = |s'|^2 - 1, disc = B^2 - A C (0 when negative).
* ``gaussians``: additive isotropic Gaussian blobs amp * exp(-|p-c|^2 / (2 sigma^2)),
  whose line integral is amp * sigma * sqrt(2 pi) * exp(-dist^2 / (2 sigma^2)) with dist
  the distance from c to the line.  Smooth everywhere (used by quadrature checks).

Rays of a helical scan start at the source a(lambda_n) and point at the curved
detector cell (alpha_c, w_r): direction D sin(alpha) e_u + D cos(alpha) e_v + w e_z
with e_u = (-sin b, cos b, 0), e_v = (-cos b, -sin b, 0), b = lambda + lambda0.
These are the scan conventions of the helix and detector (paper Sec. II and III-C).
"""
from __future__ import annotations

import math
import numpy as np


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _inside_any(centres, axes, rots, p):
    for c, a, Q in zip(centres, axes, rots):
        q = (Q.T @ (p - c)) / a
        if float(q @ q) <= 1.0:
            return True
    return False


def make_phantom(recipe: dict, grid: dict, seed: int) -> dict:
    """Draw a phantom from ``recipe`` (see synth.configs) with numpy default_rng(seed).

    Ellipsoid centres are uniform (by area) in a cylinder of radius
    recipe['centre_radius'] about the z axis and uniform in z over the grid's z extent.
    """
    rng = np.random.default_rng(seed)
    kind = recipe.get("kind", "ellipsoids")
    z_lo = grid["z_first"]
    z_hi = grid["z_first"] + (grid["nz"] - 1) * grid["dz"]
    if kind == "gaussians":
        n = recipe["n"]
        centres = []
        for _ in range(n):
            r = recipe["centre_radius"] * math.sqrt(rng.uniform())
            ph = rng.uniform(0, 2 * math.pi)
            centres.append([r * math.cos(ph), r * math.sin(ph), rng.uniform(z_lo, z_hi)])
        lo, hi = recipe["sigma"]
        return {"kind": "gaussians", "centre": np.array(centres, dtype=np.float64),
                "sigma": rng.uniform(lo, hi, size=n),
                "amp": rng.uniform(*recipe.get("amp", (0.5, 1.0)), size=n)}
    centres, axes, rots, dens = [], [], [], []
    bound = recipe.get("bound_radius", None)
    while len(centres) < recipe["n"]:
        r = recipe["centre_radius"] * math.sqrt(rng.uniform())
        ph = rng.uniform(0, 2 * math.pi)
        c = np.array([r * math.cos(ph), r * math.sin(ph), rng.uniform(z_lo, z_hi)])
        a = rng.uniform(*recipe["semi_axes"], size=3)
        Q = _random_rotation(rng)
        d = rng.uniform(*recipe["density"])
        if bound is not None and r + a.max() > bound:
            continue
        centres.append(c); axes.append(a); rots.append(Q); dens.append(d)
    n_ins = recipe.get("inserts", 0)
    tries = 0
    while n_ins > 0 and tries < 100000:
        tries += 1
        r = recipe["centre_radius"] * math.sqrt(rng.uniform())
        ph = rng.uniform(0, 2 * math.pi)
        c = np.array([r * math.cos(ph), r * math.sin(ph), rng.uniform(z_lo, z_hi)])
        if not _inside_any(centres[:recipe["n"]], axes[:recipe["n"]], rots[:recipe["n"]], c):
            continue
        rad = rng.uniform(*recipe["insert_radius"])
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        centres.append(c); axes.append(np.full(3, rad)); rots.append(np.eye(3))
        dens.append(sign * recipe["insert_density"])
        n_ins -= 1
    return {"kind": "ellipsoids", "centre": np.array(centres), "axes": np.array(axes),
            "rot": np.array(rots), "density": np.array(dens)}


def line_integrals(ph: dict, src: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Line integrals along the full lines p(t) = src + t d (src, d: [..., 3], FP64)."""
    src = np.asarray(src, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros(np.broadcast_shapes(src.shape, d.shape)[:-1])
    dn = np.sqrt(np.sum(d * d, axis=-1))
    if ph["kind"] == "gaussians":
        u = d / dn[..., None]
        for c, s, amp in zip(ph["centre"], ph["sigma"], ph["amp"]):
            p = c - src
            proj = np.sum(p * u, axis=-1)
            dist2 = np.maximum(np.sum(p * p, axis=-1) - proj * proj, 0.0)
            out += amp * s * math.sqrt(2 * math.pi) * np.exp(-dist2 / (2 * s * s))
        return out
    for c, a, Q, rho in zip(ph["centre"], ph["axes"], ph["rot"], ph["density"]):
        M = Q / a[None, :]          # columns scaled: q = M^T (p - c)
        sp = (src - c) @ M
        dp = d @ M
        A = np.sum(dp * dp, axis=-1)
        B = np.sum(sp * dp, axis=-1)
        C = np.sum(sp * sp, axis=-1) - 1.0
        disc = np.maximum(B * B - A * C, 0.0)
        out += rho * dn * 2.0 * np.sqrt(disc) / A
    return out


def density(ph: dict, pts: np.ndarray) -> np.ndarray:
    """Phantom value at points pts [..., 3]."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros(pts.shape[:-1])
    if ph["kind"] == "gaussians":
        for c, s, amp in zip(ph["centre"], ph["sigma"], ph["amp"]):
            r2 = np.sum((pts - c) ** 2, axis=-1)
            out += amp * np.exp(-r2 / (2 * s * s))
        return out
    for c, a, Q, rho in zip(ph["centre"], ph["axes"], ph["rot"], ph["density"]):
        q = ((pts - c) @ Q) / a
        out += np.where(np.sum(q * q, axis=-1) <= 1.0, rho, 0.0)
    return out


def surface_distance_ok(ph: dict, pts: np.ndarray, margin: float) -> np.ndarray:
    """True where pts are (to first order) farther than ``margin`` from every ellipsoid
    surface: |s - 1| / |grad s| > margin with s = |diag(1/a) Q^T (p - c)|."""
    pts = np.asarray(pts, dtype=np.float64)
    ok = np.ones(pts.shape[:-1], dtype=bool)
    if ph["kind"] != "ellipsoids":
        return ok
    for c, a, Q in zip(ph["centre"], ph["axes"], ph["rot"]):
        q = ((pts - c) @ Q) / a
        s = np.sqrt(np.sum(q * q, axis=-1))
        g = (q / a) @ Q.T / np.maximum(s, 1e-30)[..., None]
        gn = np.sqrt(np.sum(g * g, axis=-1))
        ok &= np.abs(s - 1.0) > margin * gn
    return ok


def scan_rays(geom: dict, views):
    """Source points and directions of every detector cell of the given views.

    Returns (src [V,1,1,3], dir [V,rows,cols,3])."""
    views = np.asarray(views)
    dlam = 2 * math.pi / geom["views_per_turn"]
    h = geom["feed_per_turn"] / (2 * math.pi)
    lam = geom["lambda_first"] + views * dlam
    b = lam + geom["lambda0"]
    cols, rows = geom["det_cols"], geom["det_rows"]
    alpha = (np.arange(cols) - 0.5 * (cols - 1) + geom["col_offset"]) * geom["dalpha"]
    w = (np.arange(rows) - 0.5 * (rows - 1) + geom["row_offset"]) * geom["dw"]
    R, D = geom["R"], geom["D"]
    cb, sb = np.cos(b), np.sin(b)
    src = np.stack([R * cb, R * sb, geom["z0"] + h * lam], axis=-1)[:, None, None, :]
    eu = np.stack([-sb, cb, np.zeros_like(b)], axis=-1)[:, None, None, :]
    ev = np.stack([-cb, -sb, np.zeros_like(b)], axis=-1)[:, None, None, :]
    ez = np.array([0.0, 0.0, 1.0])
    sa = np.sin(alpha)[None, None, :, None]
    ca = np.cos(alpha)[None, None, :, None]
    ww = w[None, :, None, None]
    d = D * sa * eu + D * ca * ev + ww * ez
    return src, d


def project(ph: dict, geom: dict, views=None, chunk=64) -> np.ndarray:
    """Closed-form sinogram g[n, r, c] (FP64) of the phantom for the given views."""
    if views is None:
        views = np.arange(geom["n_views"])
    views = np.asarray(views)
    out = np.empty((len(views), geom["det_rows"], geom["det_cols"]))
    for i in range(0, len(views), chunk):
        v = views[i:i + chunk]
        src, d = scan_rays(geom, v)
        out[i:i + len(v)] = line_integrals(ph, src, d)
    return out
