"""Plain FP64 NumPy oracle of pitch-by-pitch Katsevich FBP on a curved detector.

TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py.  It shares no code with the HIP library.

Every step follows the implementation of the Katsevich inversion formula in
Sec. II of the paper (derivative at constant direction, length-correction weighting,
forward height rebinning onto kappa-lines, 1-D Hilbert transform in alpha, backward
height rebinning, post-cosine weighting, PI-window backprojection), in the paper's
order and notation.  Points the paper leaves open are fixed as follows (one reading
each):

* derivative: central differences in lambda and alpha on the native grid, detector
  data taken as 0 outside the columns; the first and last acquired views get no
  derivative (set to 0) -- no valid voxel ever uses them;
* kappa-lines: n_psi (default 2*rows+1, odd) uniform psi samples on
  [-pi/2-alpha_m, pi/2+alpha_m], psi_k = (k-(n_psi-1)/2) dpsi, alpha_m = max |alpha_c|;
* forward rebinning: linear in w, rows outside the detector contribute 0;
* Hilbert: kernel h_H(sin(alpha-alpha')) sampled as the band-limited discrete Hilbert
  kernel times gamma/sin(gamma): K[m] = (1 - cos(pi m)) dalpha / (pi sin(m dalpha)),
  summed over all detector columns (zero data outside the fan);
* backward rebinning: psi_hat = root of w = w_kappa(alpha, psi) on the monotone branch
  of w_kappa through psi = 0 (the root of smallest |psi|), found by bisection and
  clamped to that branch; linear interpolation between neighbouring kappa-lines;
* PI lines: lambda_i found by bisection on the chord-height equation;
* backprojection: bilinear interpolation in (alpha, w) with 0 outside the detector;
  the PI interval enters through the coverage weight
  c_n = clamp(min(n + 1/2 - l_i, l_o - n + 1/2), 0, 1) in view units, i.e. the overlap of
  view cell [n-1/2, n+1/2] with [l_i, l_o]; constant factor dlambda / (2 pi);
* validity: a voxel is reconstructed iff it lies inside the field-of-view cylinder
  (radius R sin(min(-alpha_first, alpha_last))) and every view with c_n > 0, together
  with both derivative neighbours, was acquired; otherwise its value is 0.

Option (half=True): the derivative of eq. Deriv at the centre of each 2 x 2 cell of
(lambda, alpha) samples, every partial derivative the mean of the two forward differences
across the cell.  The filtered data then live on the grid lambda_{n+1/2}, alpha_{c+1/2}
(half_sample_geometry), on which every later step runs unchanged; the validity rule keeps
its one-view margin in that grid.

All arithmetic is float64 and round-to-nearest.  Integer tables are floor() of float64
values.
"""
from __future__ import annotations

import math
import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------------
# geometry (Sec. II helix equation; Sec. III-C detector coordinates)
# ----------------------------------------------------------------------------------
class Scan:
    """Quantities derived from a geometry dict (see synth.configs for the fields)."""

    def __init__(self, geom: dict, n_psi: int = 0):
        self.geom = dict(geom)
        self.R = float(geom["R"])
        self.D = float(geom["D"])
        self.P = float(geom["feed_per_turn"])
        self.h = self.P / TWO_PI                      # P / 2pi, helix rise per radian
        self.lambda0 = float(geom.get("lambda0", 0.0))
        self.z0 = float(geom.get("z0", 0.0))
        self.lambda_first = float(geom.get("lambda_first", 0.0))
        self.Nv = int(geom["views_per_turn"])
        self.N = int(geom["n_views"])
        self.dlam = TWO_PI / self.Nv
        self.cols = int(geom["det_cols"])
        self.rows = int(geom["det_rows"])
        self.dalpha = float(geom["dalpha"])
        self.dw = float(geom["dw"])
        self.col_offset = float(geom.get("col_offset", 0.0))
        self.row_offset = float(geom.get("row_offset", 0.0))
        self.alpha = (np.arange(self.cols) - 0.5 * (self.cols - 1) + self.col_offset) * self.dalpha
        self.w = (np.arange(self.rows) - 0.5 * (self.rows - 1) + self.row_offset) * self.dw
        self.alpha_m = max(abs(self.alpha[0]), abs(self.alpha[-1]))
        self.r_fov = self.R * math.sin(min(-self.alpha[0], self.alpha[-1]))
        self.psi_max = 0.5 * math.pi + self.alpha_m
        self.n_psi = int(n_psi) if n_psi else 2 * self.rows + 1
        self.dpsi = 2.0 * self.psi_max / (self.n_psi - 1)
        self.psi = (np.arange(self.n_psi) - 0.5 * (self.n_psi - 1)) * self.dpsi

    def lam(self, n):
        """lambda of view index n."""
        return self.lambda_first + np.asarray(n, dtype=np.float64) * self.dlam


# ----------------------------------------------------------------------------------
# Sec. II steps 1-2: derivative at constant direction + length-correction weighting
# ----------------------------------------------------------------------------------
def derivative_lw(scan: Scan, g) -> np.ndarray:
    """g2 = D / sqrt(D^2 + w^2) * (dg/dq + dg/dalpha) at q = lambda  (eqs. Deriv, LW).

    g holds consecutive views [V, rows, cols]; the first and last view of the block get 0.
    """
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros_like(g)
    if g.shape[0] < 3:
        return out
    d_lam = (g[2:] - g[:-2]) / (2.0 * scan.dlam)
    gp = np.pad(g[1:-1], ((0, 0), (0, 0), (1, 1)))          # zero outside the columns
    d_alpha = (gp[:, :, 2:] - gp[:, :, :-2]) / (2.0 * scan.dalpha)
    lw = scan.D / np.sqrt(scan.D ** 2 + scan.w ** 2)
    out[1:-1] = lw[None, :, None] * (d_lam + d_alpha)
    return out


def half_sample_geometry(geom: dict) -> dict:
    """Grid of the filtered data under the half-sample derivative: views at lambda_{n+1/2}
    (n = 0 .. N-2) and columns at alpha_{c+1/2} (c = 0 .. cols-2).  Columns are centred on
    the detector, so one column fewer at the same offset puts them half a column on."""
    h = dict(geom)
    h["lambda_first"] = float(geom.get("lambda_first", 0.0)) + math.pi / int(geom["views_per_turn"])
    h["det_cols"] = int(geom["det_cols"]) - 1
    h["n_views"] = int(geom["n_views"]) - 1
    return h


def derivative_lw_half(scan_h: Scan, g) -> np.ndarray:
    """Eqs. Deriv and LW at the cell centres (lambda_{n+1/2}, alpha_{c+1/2}): each partial
    derivative is the mean of the two forward differences across the 2 x 2 cell of native
    samples (n, n+1) x (c, c+1).  g: native views [V, rows, cols] -> [V-1, rows, cols-1];
    scan_h is the Scan of half_sample_geometry."""
    g = np.asarray(g, dtype=np.float64)
    d_lam = (g[1:, :, :-1] - g[:-1, :, :-1] + g[1:, :, 1:] - g[:-1, :, 1:]) / (2.0 * scan_h.dlam)
    d_alpha = (g[:-1, :, 1:] - g[:-1, :, :-1] + g[1:, :, 1:] - g[1:, :, :-1]) / (2.0 * scan_h.dalpha)
    lw = scan_h.D / np.sqrt(scan_h.D ** 2 + scan_h.w ** 2)
    return lw[None, :, None] * (d_lam + d_alpha)


# ----------------------------------------------------------------------------------
# Sec. II step 3: forward height rebinning onto kappa-lines (eqs. FR, w_k)
# ----------------------------------------------------------------------------------
def w_kappa(scan: Scan, alpha, psi):
    """w_kappa(alpha, psi) = D P / (2 pi R) (psi cos(alpha) + psi / tan(psi) sin(alpha)),
    with psi / tan(psi) := 1 at psi = 0 (R_o read as R, P as the feed per turn)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        pcot = np.where(psi == 0.0, 1.0, psi / np.tan(psi))
    return scan.D * scan.h / scan.R * (psi * np.cos(alpha) + pcot * np.sin(alpha))


def forward_rebin_table(scan: Scan):
    """Row coordinate of w_kappa(alpha_c, psi_k): r0 = floor(s), t = s - r0 with
    s = w_kappa / dw + (rows-1)/2 - row_offset.  Shapes [n_psi, cols]."""
    wk = w_kappa(scan, scan.alpha[None, :], scan.psi[:, None])
    s = wk / scan.dw + 0.5 * (scan.rows - 1) - scan.row_offset
    r0 = np.floor(s)
    return r0.astype(np.int64), s - r0


def _rows_or_zero(g2, r, c_idx, rows):
    ok = (r >= 0) & (r < rows)
    return g2[:, np.clip(r, 0, rows - 1), c_idx] * ok


def forward_rebin(scan: Scan, g2, table=None) -> np.ndarray:
    """g3[n, k, c] = g2(lambda_n, alpha_c, w_kappa(alpha_c, psi_k)), linear in w."""
    r0, t = forward_rebin_table(scan) if table is None else table
    c_idx = np.arange(scan.cols)[None, :]
    return (1.0 - t) * _rows_or_zero(g2, r0, c_idx, scan.rows) + \
        t * _rows_or_zero(g2, r0 + 1, c_idx, scan.rows)


# ----------------------------------------------------------------------------------
# Sec. II step 4: Hilbert transform in alpha at constant psi (eq. HF with h_H of e4)
# ----------------------------------------------------------------------------------
def hilbert_taps(scan: Scan) -> np.ndarray:
    """K[m], m = -(cols-1) .. cols-1 (index m + cols - 1):
    (1 - cos(pi m)) dalpha / (pi sin(m dalpha)); 0 for even m."""
    m = np.arange(-(scan.cols - 1), scan.cols)
    K = np.zeros(m.shape)
    odd = (m % 2) != 0
    K[odd] = 2.0 * scan.dalpha / (math.pi * np.sin(m[odd] * scan.dalpha))
    return K


def hilbert_matrix(scan: Scan) -> np.ndarray:
    """T[c, c'] = K[c - c']."""
    K = hilbert_taps(scan)
    c = np.arange(scan.cols)
    return K[(c[:, None] - c[None, :]) + scan.cols - 1]


def hilbert(scan: Scan, g3, T=None) -> np.ndarray:
    """g4[..., c] = sum_c' K[c - c'] g3[..., c']."""
    T = hilbert_matrix(scan) if T is None else T
    g3 = np.asarray(g3)
    return (g3.reshape(-1, g3.shape[-1]) @ T.T).reshape(g3.shape)


# ----------------------------------------------------------------------------------
# Sec. II steps 5-6: backward height rebinning + post-cosine weighting (eqs. BR, PW)
# ----------------------------------------------------------------------------------
def _bisect(f, lo, hi, iters=200):
    """Root of an increasing function on [lo, hi] (f(lo) <= 0 <= f(hi)); vectorised;
    iterates until the bracket stops shrinking and returns its midpoint."""
    lo = np.array(lo, dtype=np.float64)
    hi = np.array(hi, dtype=np.float64)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        live = (mid > lo) & (mid < hi)
        if not live.any():
            break
        fm = f(mid)
        go_up = live & (fm < 0.0)
        go_dn = live & (fm > 0.0)
        hit = live & (fm == 0.0)
        lo = np.where(go_up | hit, mid, lo)
        hi = np.where(go_dn | hit, mid, hi)
    return 0.5 * (lo + hi)


def dw_kappa_dpsi(scan: Scan, alpha, psi):
    """d w_kappa / d psi = D P/(2 pi R) (cos(alpha) + sin(alpha)(cot(psi) - psi/sin^2(psi)))."""
    return scan.D * scan.h / scan.R * (
        np.cos(alpha) + np.sin(alpha) * (1.0 / np.tan(psi) - psi / np.sin(psi) ** 2))


def monotone_branch(scan: Scan):
    """Per column, the interval [psi_lo, psi_hi] of the branch of w_kappa(alpha_c, .)
    through psi = 0 on which it increases (turning points or +-psi_max)."""
    lo = np.full(scan.cols, -scan.psi_max)
    hi = np.full(scan.cols, scan.psi_max)
    for c, a in enumerate(scan.alpha):
        if a > 0 and dw_kappa_dpsi(scan, a, scan.psi_max) < 0:
            # derivative falls from cos(alpha) > 0 at 0+ to < 0 at psi_max: one crossing
            hi[c] = _bisect(lambda p: -dw_kappa_dpsi(scan, a, p), 1e-3, scan.psi_max)
        if a < 0 and dw_kappa_dpsi(scan, a, -scan.psi_max) < 0:
            lo[c] = _bisect(lambda p: dw_kappa_dpsi(scan, a, p), -scan.psi_max, -1e-3)
    return lo, hi


def psi_hat(scan: Scan) -> np.ndarray:
    """psi_hat(alpha_c, w_r) [rows, cols]: smallest-|psi| solution of w = w_kappa, i.e. the
    root on the monotone branch through 0, clamped to that branch's end points."""
    lo, hi = monotone_branch(scan)
    out = np.empty((scan.rows, scan.cols))
    for c, a in enumerate(scan.alpha):
        w_lo = w_kappa(scan, a, lo[c])
        w_hi = w_kappa(scan, a, hi[c])
        w = scan.w
        root = _bisect(lambda p: w_kappa(scan, a, p) - w,
                       np.full(scan.rows, lo[c]), np.full(scan.rows, hi[c]))
        out[:, c] = np.where(w <= w_lo, lo[c], np.where(w >= w_hi, hi[c], root))
    return out


def backward_rebin_table(scan: Scan):
    """kappa index k0 (<= n_psi-2) and weight t of psi_hat: q = psi_hat/dpsi + (n_psi-1)/2
    clamped to [0, n_psi-1].  Shapes [rows, cols]."""
    q = psi_hat(scan) / scan.dpsi + 0.5 * (scan.n_psi - 1)
    q = np.clip(q, 0.0, scan.n_psi - 1.0)
    k0 = np.minimum(np.floor(q), scan.n_psi - 2)
    return k0.astype(np.int64), q - k0


def backward_rebin_cos(scan: Scan, g4, table=None) -> np.ndarray:
    """gF[n, r, c] = cos(alpha_c) g4(lambda_n, alpha_c, psi_hat(alpha_c, w_r))."""
    k0, t = backward_rebin_table(scan) if table is None else table
    c_idx = np.arange(scan.cols)[None, :]
    g4 = np.asarray(g4)
    return np.cos(scan.alpha)[None, None, :] * (
        (1.0 - t) * g4[:, k0, c_idx] + t * g4[:, k0 + 1, c_idx])


class FilterTables:
    def __init__(self, scan: Scan):
        self.fr = forward_rebin_table(scan)
        self.br = backward_rebin_table(scan)
        self.T = hilbert_matrix(scan)


def filter_views(scan: Scan, g, tables: FilterTables | None = None, chunk=256,
                 progress=None, half=False) -> np.ndarray:
    """Steps 1-6 of Sec. II on a block of consecutive views -> g^F (first/last view 0).
    half: scan is the half-sample grid and g the V+1 native views around its V views."""
    tables = tables or FilterTables(scan)
    g = np.asarray(g, dtype=np.float64)
    if half:
        V = g.shape[0] - 1
        out = np.zeros((max(V, 0), scan.rows, scan.cols))
        for a in range(0, V, chunk):
            if progress is not None:
                progress(a, V)
            b = min(V, a + chunk)
            g2 = derivative_lw_half(scan, g[a:b + 1])
            g3 = forward_rebin(scan, g2, tables.fr)
            g4 = hilbert(scan, g3, tables.T)
            out[a:b] = backward_rebin_cos(scan, g4, tables.br)
        return out
    V = g.shape[0]
    out = np.zeros((V, scan.rows, scan.cols))
    for a in range(1, V - 1, chunk):
        if progress is not None:
            progress(a, V)
        b = min(V - 1, a + chunk)
        g2 = derivative_lw(scan, g[a - 1:b + 1])[1:-1]
        g3 = forward_rebin(scan, g2, tables.fr)
        g4 = hilbert(scan, g3, tables.T)
        out[a:b] = backward_rebin_cos(scan, g4, tables.br)
    return out


# ----------------------------------------------------------------------------------
# PI lines (Sec. II pre-calculating step 2), by bisection on the chord height
# ----------------------------------------------------------------------------------
def _chord(scan: Scan, s, x, y):
    """For the in-plane chord from source angle s + lambda0 through (x, y): the angle
    it spans (counter-clockwise, in (0, 2pi)) and the fraction t of (x, y) along it."""
    b = s + scan.lambda0
    Sx, Sy = scan.R * np.cos(b), scan.R * np.sin(b)
    dx, dy = x - Sx, y - Sy
    tau = -2.0 * (Sx * dx + Sy * dy) / (dx * dx + dy * dy)   # second circle crossing
    Ex, Ey = Sx + tau * dx, Sy + tau * dy
    span = np.mod(np.arctan2(Sx * Ey - Sy * Ex, Sx * Ex + Sy * Ey), TWO_PI)
    return span, 1.0 / tau


def pi_line(scan: Scan, x, y, z):
    """(lambda_i, lambda_o) of the PI line through (x, y, z): the chord of the helix with
    lambda_o - lambda_i < 2pi containing the point.  lambda_i solves
    z0 + h (s + t(s) span(s)) = z on s in ((z-z0)/h - 2pi, (z-z0)/h)."""
    x, y, z = np.broadcast_arrays(np.asarray(x, np.float64), np.asarray(y, np.float64),
                                  np.asarray(z, np.float64))
    zr = (z - scan.z0) / scan.h

    def F(s):
        span, t = _chord(scan, s, x, y)
        return scan.z0 + scan.h * (s + t * span) - z

    s = _bisect(F, zr - TWO_PI, zr)
    span, _ = _chord(scan, s, x, y)
    return s, s + span


def pi_view_bounds(scan: Scan, lam_i, lam_o):
    """PI interval in global view units l = (lambda - lambda_first)/dlambda and the first /
    last view with non-zero coverage: n_first = floor(l_i - 1/2) + 1,
    n_last = ceil(l_o + 1/2) - 1."""
    li = (np.asarray(lam_i) - scan.lambda_first) / scan.dlam
    lo = (np.asarray(lam_o) - scan.lambda_first) / scan.dlam
    nf = (np.floor(li - 0.5) + 1).astype(np.int64)
    nl = (np.ceil(lo + 0.5) - 1).astype(np.int64)
    return li, lo, nf, nl


def in_fov(scan: Scan, x, y):
    return np.asarray(x) ** 2 + np.asarray(y) ** 2 <= scan.r_fov ** 2


# ----------------------------------------------------------------------------------
# Sec. II step 7: PI-window backprojection with v*, alpha*, w*
# ----------------------------------------------------------------------------------
def project_point(scan: Scan, lam, x, y, z):
    """(v*, alpha*, w*) of points (x, y, z) seen from a(lam) (Sec. II step 7):
    v* = R - x cos(lam+lambda0) - y sin(lam+lambda0),
    alpha* = arctan((-x sin(lam+lambda0) + y cos(lam+lambda0)) / v*),
    w* = D cos(alpha*) / v* (z - z0 - P lam / 2pi)."""
    b = lam + scan.lambda0
    v = scan.R - x * np.cos(b) - y * np.sin(b)
    a_s = np.arctan((-x * np.sin(b) + y * np.cos(b)) / v)
    w_s = scan.D * np.cos(a_s) / v * (z - scan.z0 - scan.h * lam)
    return v, a_s, w_s


def detector_coords(scan: Scan, alpha_s, w_s):
    """Fractional (row, col) of detector position (alpha, w)."""
    cc = alpha_s / scan.dalpha + 0.5 * (scan.cols - 1) - scan.col_offset
    rr = w_s / scan.dw + 0.5 * (scan.rows - 1) - scan.row_offset
    return rr, cc


def bilinear(scan: Scan, img, rr, cc):
    """img[rows, cols] at fractional (row, col); 0 outside the detector."""
    r0 = np.floor(rr).astype(np.int64)
    c0 = np.floor(cc).astype(np.int64)
    tr = rr - r0
    tc = cc - c0

    def at(r, c):
        ok = (r >= 0) & (r < scan.rows) & (c >= 0) & (c < scan.cols)
        return img[np.clip(r, 0, scan.rows - 1), np.clip(c, 0, scan.cols - 1)] * ok

    return (1 - tr) * ((1 - tc) * at(r0, c0) + tc * at(r0, c0 + 1)) + \
        tr * ((1 - tc) * at(r0 + 1, c0) + tc * at(r0 + 1, c0 + 1))


def backproject(scan: Scan, gF, n0, x, y, z, li, lo, nf, nl, lam_shift=0.0):
    """f = dlambda/(2 pi) sum_n c_n / v*_n g^F(lambda_n, alpha*_n, w*_n) at points (x, y, z).

    gF holds filtered views n0 .. n0 + len - 1 (global indices).  The geometry of view
    n is evaluated at lambda_n - lam_shift (lam_shift = 2 pi k with pitch-0 coordinates
    for pitch k).  li, lo, nf, nl are in global view units."""
    x, y, z = (np.asarray(a, np.float64).ravel() for a in (x, y, z))
    li, lo = np.asarray(li, np.float64).ravel(), np.asarray(lo, np.float64).ravel()
    nf, nl = np.asarray(nf).ravel(), np.asarray(nl).ravel()
    acc = np.zeros(x.shape)
    if x.size == 0:
        return acc
    for n in range(int(nf.min()), int(nl.max()) + 1):
        idx = np.nonzero((n >= nf) & (n <= nl))[0]
        if idx.size == 0:
            continue
        lam = scan.lambda_first + n * scan.dlam - lam_shift
        v, a_s, w_s = project_point(scan, lam, x[idx], y[idx], z[idx])
        rr, cc = detector_coords(scan, a_s, w_s)
        val = bilinear(scan, gF[n - n0], rr, cc)
        c = np.clip(np.minimum(n + 0.5 - li[idx], lo[idx] - n + 0.5), 0.0, 1.0)
        acc[idx] += c * val / v
    return acc * scan.dlam / TWO_PI


# ----------------------------------------------------------------------------------
# grid, pitches, validity (Sec. II periodicity + reconstruction step)
# ----------------------------------------------------------------------------------
class Pitches:
    """Pitch structure of a grid: slices_per_pitch = P / dz when that is an integer
    (then slice iz = k * Ns + j of pitch k sits at z_j + k P), otherwise a single
    'pitch' holding every slice (no reuse)."""

    def __init__(self, scan: Scan, grid: dict):
        self.grid = dict(grid)
        nz, dz = int(grid["nz"]), float(grid["dz"])
        ns = int(round(scan.P / dz))
        if ns >= 1 and abs(ns * dz - scan.P) <= 1e-9 * scan.P:
            self.commensurate = True
            self.ns = ns
        else:
            self.commensurate = False
            self.ns = nz
        self.n_tab = min(self.ns, nz)
        self.n_pitches = -(-nz // self.ns)

    def slices(self, k):
        """Global slice indices of pitch k and their in-pitch index j."""
        a = k * self.ns
        b = min(a + self.ns, int(self.grid["nz"]))
        return np.arange(a, b), np.arange(b - a)


def grid_xy(grid: dict):
    x = grid["x_first"] + np.arange(grid["nx"]) * grid["dx"]
    y = grid["y_first"] + np.arange(grid["ny"]) * grid["dy"]
    return x, y


def pitch_tables(scan: Scan, grid: dict, pit: Pitches | None = None):
    """Sec. II pre-calculating step 2 on the slices of the first pitch: PI lines of
    every (j, y, x), their view bounds, the FOV flag and the pitch view window
    [n_lo, n_hi] (global units for pitch 0, one extra view each side for the
    derivative).  Arrays are [n_tab, ny, nx]."""
    pit = pit or Pitches(scan, grid)
    x, y = grid_xy(grid)
    zj = grid["z_first"] + np.arange(pit.n_tab) * grid["dz"]
    Z, Y, X = np.meshgrid(zj, y, x, indexing="ij")
    lam_i, lam_o = pi_line(scan, X, Y, Z)
    li, lo, nf, nl = pi_view_bounds(scan, lam_i, lam_o)
    fov = in_fov(scan, X, Y)
    n_lo = int(nf[fov].min()) - 1
    n_hi = int(nl[fov].max()) + 1
    return {"lam_i": lam_i, "lam_o": lam_o, "li": li, "lo": lo, "nf": nf, "nl": nl,
            "fov": fov, "n_lo": n_lo, "n_hi": n_hi, "pitches": pit}


def valid_mask(scan: Scan, nf, nl, fov):
    return fov & (nf - 1 >= 0) & (nl + 1 <= scan.N - 1)


def recon(scan: Scan, grid: dict, g, mode="pitch", tables=None, ftables=None, half=False):
    """Full reconstruction f[nz, ny, nx] and validity mask.

    half: half-sample derivative; scan is the Scan of half_sample_geometry(native geometry)
    and g the native sinogram [N + 1, rows, cols + 1].

    mode="pitch": the paper's scheme -- PI tables of the first pitch reused for every
    pitch k (lambda shifted by 2 pi k), each pitch filtering its own lambda-sliced
    sinogram window [n_lo + k Nv, n_hi + k Nv] (clipped to the scan).
    mode="whole": filter the whole scan once and solve the PI lines of every voxel at
    its own z (no periodicity used)."""
    g = np.asarray(g)
    nx, ny, nz = int(grid["nx"]), int(grid["ny"]), int(grid["nz"])
    f = np.zeros((nz, ny, nx))
    valid = np.zeros((nz, ny, nx), dtype=bool)
    x, y = grid_xy(grid)
    ftables = ftables or FilterTables(scan)
    ext = 1 if half else 0                  # native views beyond the last filtered one
    if mode == "whole":
        gF = filter_views(scan, g, ftables, half=half)
        z = grid["z_first"] + np.arange(nz) * grid["dz"]
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        lam_i, lam_o = pi_line(scan, X, Y, Z)
        li, lo, nf, nl = pi_view_bounds(scan, lam_i, lam_o)
        valid = valid_mask(scan, nf, nl, in_fov(scan, X, Y))
        for iz in range(nz):
            m = valid[iz]
            if m.any():
                f[iz][m] = backproject(scan, gF, 0, X[iz][m], Y[iz][m], Z[iz][m],
                                       li[iz][m], lo[iz][m], nf[iz][m], nl[iz][m])
        return f, valid
    tab = tables or pitch_tables(scan, grid)
    pit = tab["pitches"]
    Y2, X2 = np.meshgrid(y, x, indexing="ij")
    for k in range(pit.n_pitches):
        sl, js = pit.slices(k)
        shift = k * scan.Nv
        a = max(tab["n_lo"] + shift, 0)
        b = min(tab["n_hi"] + shift, scan.N - 1)
        if b - a < 2:
            continue
        nf = tab["nf"][js] + shift
        nl = tab["nl"][js] + shift
        vk = valid_mask(scan, nf, nl, tab["fov"][js])
        valid[sl] = vk
        if not vk.any():
            continue
        gF = filter_views(scan, g[a:b + 1 + ext], ftables, half=half)
        for jj, (iz, j) in enumerate(zip(sl, js)):
            m = vk[jj]
            if not m.any():
                continue
            zj = grid["z_first"] + j * grid["dz"]
            f[iz][m] = backproject(scan, gF, a, X2[m], Y2[m], np.full(m.sum(), zj),
                                   tab["li"][j][m] + shift, tab["lo"][j][m] + shift,
                                   nf[jj][m], nl[jj][m], lam_shift=TWO_PI * k)
    return f, valid


# ----------------------------------------------------------------------------------
# exact transpose of the discrete operator (adjoint), FP64
# ----------------------------------------------------------------------------------
def backproject_T(scan: Scan, fbar, n0, nviews, x, y, z, li, lo, nf, nl, lam_shift=0.0):
    """Transpose of backproject(): scatter dlambda/(2 pi) c_n / v*_n * fbar(x) into the four
    bilinear taps of view n.  Returns gFbar for views n0 .. n0 + nviews - 1."""
    x, y, z = (np.asarray(a, np.float64).ravel() for a in (x, y, z))
    fbar = np.asarray(fbar, np.float64).ravel()
    li, lo = np.asarray(li, np.float64).ravel(), np.asarray(lo, np.float64).ravel()
    nf, nl = np.asarray(nf).ravel(), np.asarray(nl).ravel()
    out = np.zeros((nviews, scan.rows, scan.cols))
    if x.size == 0:
        return out
    s = scan.dlam / TWO_PI
    for n in range(int(nf.min()), int(nl.max()) + 1):
        idx = np.nonzero((n >= nf) & (n <= nl))[0]
        if idx.size == 0:
            continue
        lam = scan.lambda_first + n * scan.dlam - lam_shift
        v, a_s, w_s = project_point(scan, lam, x[idx], y[idx], z[idx])
        rr, cc = detector_coords(scan, a_s, w_s)
        c = np.clip(np.minimum(n + 0.5 - li[idx], lo[idx] - n + 0.5), 0.0, 1.0)
        amp = s * c / v * fbar[idx]
        r0 = np.floor(rr).astype(np.int64)
        c0 = np.floor(cc).astype(np.int64)
        tr, tc = rr - r0, cc - c0
        img = out[n - n0]
        for dr, wr in ((0, 1 - tr), (1, tr)):
            for dc, wc in ((0, 1 - tc), (1, tc)):
                r, cidx = r0 + dr, c0 + dc
                ok = (r >= 0) & (r < scan.rows) & (cidx >= 0) & (cidx < scan.cols)
                np.add.at(img, (r[ok], cidx[ok]), (amp * wr * wc)[ok])
    return out


def filter_views_T(scan: Scan, gFbar, tables: FilterTables | None = None,
                   half=False) -> np.ndarray:
    """Transpose of filter_views() on a block of consecutive views (half: returns the
    V+1 native views [V+1, rows, cols+1])."""
    tables = tables or FilterTables(scan)
    gFbar = np.asarray(gFbar, np.float64)
    V = gFbar.shape[0]
    if half:
        gbar = np.zeros((V + 1, scan.rows, scan.cols + 1))
        views = range(0, V)
    else:
        gbar = np.zeros_like(gFbar)
        if V < 3:
            return gbar
        views = range(1, V - 1)
    k0, tb = tables.br
    r0, tf = tables.fr
    c_idx = np.arange(scan.cols)
    cosa = np.cos(scan.alpha)
    lw = scan.D / np.sqrt(scan.D ** 2 + scan.w ** 2)
    for n in views:
        gf = gFbar[n] * cosa[None, :]
        g4 = np.zeros((scan.n_psi, scan.cols))                 # BR^T (scatter)
        np.add.at(g4, (k0, np.broadcast_to(c_idx, k0.shape)), (1 - tb) * gf)
        np.add.at(g4, (k0 + 1, np.broadcast_to(c_idx, k0.shape)), tb * gf)
        g3 = g4 @ tables.T                                      # H^T
        g2 = np.zeros((scan.rows, scan.cols))                   # FR^T (scatter)
        for dr, wt in ((0, 1 - tf), (1, tf)):
            r = r0 + dr
            ok = (r >= 0) & (r < scan.rows)
            np.add.at(g2, (r[ok], np.broadcast_to(c_idx, r.shape)[ok]), (wt * g3)[ok])
        g1 = lw[:, None] * g2                                   # LW^T
        if half:                                                # half-sample Deriv^T
            a, b = 1.0 / (2 * scan.dlam), 1.0 / (2 * scan.dalpha)
            gbar[n, :, :-1] -= (a + b) * g1
            gbar[n, :, 1:] += (b - a) * g1
            gbar[n + 1, :, :-1] += (a - b) * g1
            gbar[n + 1, :, 1:] += (a + b) * g1
            continue
        gbar[n + 1] += g1 / (2 * scan.dlam)                     # Deriv^T (lambda)
        gbar[n - 1] -= g1 / (2 * scan.dlam)
        gbar[n, :, 1:] += g1[:, :-1] / (2 * scan.dalpha)        # Deriv^T (alpha)
        gbar[n, :, :-1] -= g1[:, 1:] / (2 * scan.dalpha)
    return gbar


def recon_T(scan: Scan, grid: dict, fbar, tables=None, ftables=None, half=False) -> np.ndarray:
    """Exact transpose of recon(mode="pitch"): volume cotangent -> sinogram cotangent.
    Views shared by adjacent pitches accumulate.  half: as in recon (native-shaped result)."""
    nx, ny = int(grid["nx"]), int(grid["ny"])
    fbar = np.asarray(fbar, np.float64)
    ext = 1 if half else 0
    gbar = np.zeros((scan.N + ext, scan.rows, scan.cols + ext))
    x, y = grid_xy(grid)
    ftables = ftables or FilterTables(scan)
    tab = tables or pitch_tables(scan, grid)
    pit = tab["pitches"]
    Y2, X2 = np.meshgrid(y, x, indexing="ij")
    for k in range(pit.n_pitches):
        sl, js = pit.slices(k)
        shift = k * scan.Nv
        a = max(tab["n_lo"] + shift, 0)
        b = min(tab["n_hi"] + shift, scan.N - 1)
        if b - a < 2:
            continue
        nf = tab["nf"][js] + shift
        nl = tab["nl"][js] + shift
        vk = valid_mask(scan, nf, nl, tab["fov"][js])
        if not vk.any():
            continue
        gFbar = np.zeros((b - a + 1, scan.rows, scan.cols))
        for jj, (iz, j) in enumerate(zip(sl, js)):
            m = vk[jj]
            if not m.any():
                continue
            zj = grid["z_first"] + j * grid["dz"]
            gFbar += backproject_T(scan, fbar[iz][m], a, b - a + 1, X2[m], Y2[m],
                                   np.full(m.sum(), zj), tab["li"][j][m] + shift,
                                   tab["lo"][j][m] + shift, nf[jj][m], nl[jj][m],
                                   lam_shift=TWO_PI * k)
        gbar[a:b + 1 + ext] += filter_views_T(scan, gFbar, ftables, half=half)
    return gbar


# ----------------------------------------------------------------------------------
# counts used by the measurement (N_vv = number of (voxel, view) pairs with c_n > 0)
# ----------------------------------------------------------------------------------
def n_voxel_views(scan: Scan, grid: dict, tables=None) -> int:
    tab = tables or pitch_tables(scan, grid)
    pit = tab["pitches"]
    total = 0
    for k in range(pit.n_pitches):
        sl, js = pit.slices(k)
        shift = k * scan.Nv
        nf = tab["nf"][js] + shift
        nl = tab["nl"][js] + shift
        vk = valid_mask(scan, nf, nl, tab["fov"][js])
        total += int((nl - nf + 1)[vk].sum())
    return total
