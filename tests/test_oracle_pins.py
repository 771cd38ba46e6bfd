"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than itself: a closed
form, an explicit geometric construction, an invariant, a brute-force or library
computation of the continuous quantity, or convergence under refinement.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from synth import configs, phantom


# Helix offsets of Sec. II (lambda0: angle of the source at lambda = 0, z0: its height) and a
# first view that is not a multiple of the view step; the geometric pins run with and
# without them, so that a dropped or mis-signed offset anywhere fails one of them.
OFFSETS = {"lambda0": 0.7, "z0": -13.2, "lambda_first": 0.31}


def _scan(offsets=False, **kw):
    wl = configs.tiny(**kw)
    geom = wl.geom.as_dict()
    if offsets:
        geom.update(OFFSETS)
    return O.Scan(geom), wl


with_offsets = pytest.mark.parametrize("offsets", [False, True], ids=["no-offsets", "offsets"])


# ---------------------------------------------------------------- phantom / projector
def test_ellipsoid_line_integral_vs_marching():
    """Closed-form chord length vs boundary crossings located by bisection of the
    inside test along the ray (a different computation of the same length)."""
    rng = np.random.default_rng(0)
    ph = phantom.make_phantom({"kind": "ellipsoids", "n": 1, "centre_radius": 5.0,
                               "semi_axes": (5.0, 20.0), "density": (1.0, 1.0)},
                              {"z_first": -5.0, "nz": 2, "dz": 10.0}, 3)
    c, a, Q = ph["centre"][0], ph["axes"][0], ph["rot"][0]

    def inside(p):
        q = (Q.T @ (p - c)) / a
        return q @ q <= 1.0

    for _ in range(20):
        src = rng.normal(size=3) * 5 + np.array([200.0, 0, 0])
        tgt = c + rng.normal(size=3) * 6
        d = tgt - src
        ts = np.linspace(0.0, 2.0, 4001)
        ins = np.array([inside(src + t * d) for t in ts])
        length = 0.0
        edges = np.nonzero(ins[1:] != ins[:-1])[0]
        cross = []
        for e in edges:
            lo, hi = ts[e], ts[e + 1]
            state_lo = ins[e]
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                if inside(src + mid * d) == state_lo:
                    lo = mid
                else:
                    hi = mid
            cross.append(0.5 * (lo + hi))
        for i in range(0, len(cross), 2):
            length += (cross[i + 1] - cross[i]) * np.linalg.norm(d)
        got = phantom.line_integrals(ph, src, d)
        assert abs(got - length) <= 1e-9 * max(1.0, length)


def test_gaussian_line_integral_vs_quadrature():
    ph = {"kind": "gaussians", "centre": np.array([[3.0, -2.0, 5.0]]),
          "sigma": np.array([4.0]), "amp": np.array([0.7])}
    rng = np.random.default_rng(1)
    for _ in range(10):
        src = np.array([300.0, 10.0, 0.0]) + rng.normal(size=3)
        d = np.array([-1.0, 0.0, 0.0]) + 0.02 * rng.normal(size=3)
        u = d / np.linalg.norm(d)
        val, _ = integrate.quad(lambda t: phantom.density(ph, src + t * u), 200, 400,
                                epsabs=1e-13, epsrel=1e-12, limit=200)
        assert abs(phantom.line_integrals(ph, src, d) - val) < 1e-9


# ---------------------------------------------------------------- geometry (v*, alpha*, w*)
@with_offsets
def test_backprojection_coordinates_vs_ray_cylinder_intersection(offsets):
    """alpha*, v*, w* of the backprojection step equal the detector cell hit by the ray
    source -> x, found by intersecting that ray with the curved detector (a cylinder of
    radius D about the source, axis parallel to z)."""
    scan, _ = _scan(offsets)
    rng = np.random.default_rng(2)
    for _ in range(50):
        x, y, z = rng.uniform(-30, 30), rng.uniform(-30, 30), rng.uniform(-20, 60)
        lam = rng.uniform(-3, 20)
        b = lam + scan.lambda0
        a = np.array([scan.R * math.cos(b), scan.R * math.sin(b), scan.z0 + scan.h * lam])
        d = np.array([x, y, z]) - a
        p = a + d * scan.D / math.hypot(d[0], d[1])          # on the detector cylinder
        eu = np.array([-math.sin(b), math.cos(b), 0.0])
        ev = np.array([-math.cos(b), -math.sin(b), 0.0])
        alpha_ref = math.atan2((p - a) @ eu, (p - a) @ ev)
        w_ref = p[2] - a[2]
        v, al, w = O.project_point(scan, lam, x, y, z)
        assert abs(v - d @ ev) < 1e-10
        assert abs(al - alpha_ref) < 1e-13
        assert abs(w - w_ref) < 1e-10


@with_offsets
def test_w_kappa_is_the_kappa_plane_on_the_detector(offsets):
    """Points of the kappa-plane through a(l), a(l+psi), a(l+2psi), seen from a(l), land
    on the detector curve w = w_kappa(alpha, psi) (R_o = R, P = feed per turn)."""
    scan, _ = _scan(offsets, feed=40.0)
    rng = np.random.default_rng(3)
    lam = 0.7
    b = lam + scan.lambda0
    a = lambda l: np.array([scan.R * math.cos(l + scan.lambda0),
                            scan.R * math.sin(l + scan.lambda0), scan.z0 + scan.h * l])
    eu = np.array([-math.sin(b), math.cos(b), 0.0])
    ev = np.array([-math.cos(b), -math.sin(b), 0.0])
    for psi in (-2.0, -1.1, -0.3, 0.2, 0.9, 1.9):
        p0, p1, p2 = a(lam), a(lam + psi), a(lam + 2 * psi)
        for _ in range(6):
            s1, s2 = rng.uniform(0.1, 1.0, size=2)
            q = p0 + s1 * (p1 - p0) + s2 * (p2 - p0) - p0
            alpha = math.atan2(q @ eu, q @ ev)
            if q @ ev <= 0:
                continue
            w = scan.D * q[2] / math.hypot(q @ eu, q @ ev)
            assert abs(O.w_kappa(scan, alpha, psi) - w) < 1e-9 * max(1, abs(w))


# ---------------------------------------------------------------- PI lines
@with_offsets
def test_pi_line_axis_closed_form(offsets):
    scan, _ = _scan(offsets)
    z = np.array([-10.0, 0.0, 7.3, 55.0])
    li, lo = O.pi_line(scan, np.zeros(4), np.zeros(4), z)
    ref = (z - scan.z0) / scan.h - math.pi / 2
    assert np.allclose(li, ref, atol=1e-12, rtol=0)
    assert np.allclose(lo, ref + math.pi, atol=1e-12, rtol=0)


@with_offsets
def test_pi_line_chord_contains_point_and_spans(offsets):
    scan, _ = _scan(offsets, feed=60.0)
    rng = np.random.default_rng(4)
    x = rng.uniform(-150, 150, 400)
    y = rng.uniform(-150, 150, 400)
    z = rng.uniform(-40, 90, 400)
    keep = x * x + y * y < 150 ** 2
    x, y, z = x[keep], y[keep], z[keep]
    li, lo = O.pi_line(scan, x, y, z)
    a = lambda l: np.stack([scan.R * np.cos(l + scan.lambda0), scan.R * np.sin(l + scan.lambda0),
                            scan.z0 + scan.h * l], -1)
    A, B = a(li), a(lo)
    P = np.stack([x, y, z], -1)
    t = np.sum((P - A) * (B - A), -1) / np.sum((B - A) ** 2, -1)
    dist = np.linalg.norm(A + t[:, None] * (B - A) - P, axis=-1)
    assert dist.max() < 1e-9
    assert (t > 0).all() and (t < 1).all()
    rho = np.hypot(x, y)
    span = lo - li
    assert (span >= math.pi - 2 * np.arcsin(rho / scan.R) - 1e-12).all()
    assert (span <= math.pi + 2 * np.arcsin(rho / scan.R) + 1e-12).all()


@with_offsets
def test_pi_line_periodicity(offsets):
    """lambda_{i,o}(x, y, z + kP) = lambda_{i,o}(x, y, z) + 2 k pi  (Sec. II periodicity)."""
    scan, _ = _scan(offsets, feed=50.0)
    rng = np.random.default_rng(5)
    x, y, z = rng.uniform(-100, 100, (3, 200))
    li0, lo0 = O.pi_line(scan, x, y, z)
    for k in (1, 3, -2):
        li, lo = O.pi_line(scan, x, y, z + k * scan.P)
        assert np.abs(li - li0 - 2 * math.pi * k).max() < 1e-11
        assert np.abs(lo - lo0 - 2 * math.pi * k).max() < 1e-11


@with_offsets
def test_pi_endpoints_project_on_tam_danielsson_boundaries(offsets):
    """Seen from a(lambda_i), x projects on the upper TD boundary
    w_top(alpha) = (D P / 2pi R)(pi/2 - alpha)/cos(alpha); from a(lambda_o) on the lower one
    w_bot(alpha) = -(D P / 2pi R)(pi/2 + alpha)/cos(alpha) (closed form for the curved
    detector, derived from the projection of the adjacent helix turns)."""
    scan, _ = _scan(offsets, feed=70.0)
    rng = np.random.default_rng(6)
    x, y, z = rng.uniform(-120, 120, 100), rng.uniform(-120, 120, 100), rng.uniform(0, 80, 100)
    li, lo = O.pi_line(scan, x, y, z)
    k = scan.D * scan.h / scan.R
    _, al, w = O.project_point(scan, li, x, y, z)
    assert np.abs(w - k * (math.pi / 2 - al) / np.cos(al)).max() < 1e-8
    _, al, w = O.project_point(scan, lo, x, y, z)
    assert np.abs(w + k * (math.pi / 2 + al) / np.cos(al)).max() < 1e-8


# ---------------------------------------------------------------- derivative (eq. Deriv)
def test_derivative_at_constant_direction_converges():
    """Central differences in (lambda, alpha) converge at second order to the exact
    derivative at constant ray direction, obtained from the closed-form line integral
    by moving the source along the helix with the direction held fixed."""
    ph = {"kind": "gaussians", "centre": np.array([[10.0, -5.0, 30.0], [-20.0, 15.0, 25.0]]),
          "sigma": np.array([12.0, 8.0]), "amp": np.array([1.0, 0.6])}
    errs = []
    for level in range(3):
        nv = 360 * 2 ** level
        cols = 64 * 2 ** level
        wl = configs.make_workload("d", feed=40.0, cols=cols, rows=8, views_per_turn=nv,
                                   turns=1, nxy=16, nz=4, dxy=4.0, slices_per_pitch=10,
                                   r_cov=60.0)
        geom = wl.geom.as_dict()
        scan = O.Scan(geom)
        n = nv // 4
        g = phantom.project(ph, geom, views=[n - 1, n, n + 1])
        g1 = O.derivative_lw(scan, g)[1] / (scan.D / np.sqrt(scan.D ** 2 + scan.w ** 2))[:, None]
        src, d = phantom.scan_rays(geom, [n])
        lam = scan.lam(n)
        eps = 1e-5

        def src_at(l):
            return np.array([scan.R * math.cos(l + scan.lambda0),
                             scan.R * math.sin(l + scan.lambda0), scan.z0 + scan.h * l])
        exact = (phantom.line_integrals(ph, src_at(lam + eps), d[0]) -
                 phantom.line_integrals(ph, src_at(lam - eps), d[0])) / (2 * eps)
        sl = slice(cols // 4, 3 * cols // 4)        # away from the zero-padded edges
        errs.append(np.abs(g1[:, sl] - exact[:, sl]).max() / np.abs(exact[:, sl]).max())
    print(errs)
    assert errs[0] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


# ---------------------------------------------------------------- Hilbert (eqs. HF, e4)
def test_hilbert_kernel_odd_and_transpose_is_negative():
    scan, _ = _scan(cols=33)
    K = O.hilbert_taps(scan)
    assert np.array_equal(K, -K[::-1])
    T = O.hilbert_matrix(scan)
    assert np.array_equal(T.T, -T)


def test_hilbert_direct_equals_fft_convolution():
    scan, _ = _scan(cols=75)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(5, scan.cols))
    K = O.hilbert_taps(scan)
    nfft = 256
    spec = np.fft.rfft(np.concatenate([K[scan.cols - 1:], np.zeros(nfft - 2 * scan.cols + 1),
                                       K[:scan.cols - 1]]), nfft)
    y_fft = np.fft.irfft(np.fft.rfft(x, nfft) * spec, nfft)[:, :scan.cols]
    assert np.abs(O.hilbert(scan, x) - y_fft).max() < 1e-12 * np.abs(y_fft).max()


def test_hilbert_converges_to_principal_value_integral():
    """The discrete kernel converges (second order) to the continuous
    PV int dalpha' g(alpha') / (pi sin(alpha - alpha')) of a smooth compact g, evaluated
    with QUADPACK's Cauchy-weight rule."""
    half = 0.3
    g = lambda a: np.where(np.abs(a) < half, (1 - (a / half) ** 2) ** 4, 0.0)
    probes = np.array([-0.21, -0.05, 0.1, 0.27])
    ref = []
    for a0 in probes:
        f = lambda ap: float(g(ap)) * ((a0 - ap) / math.sin(a0 - ap) if ap != a0 else 1.0) / math.pi
        val, _ = integrate.quad(f, -half, half, weight="cauchy", wvar=a0, epsabs=1e-14)
        ref.append(-val)
    ref = np.array(ref)
    errs = []
    for level in range(3):
        cols = 120 * 2 ** level + 1
        dalpha = 0.8 / (cols - 1)
        wl = configs.tiny(cols=cols)
        geom = dict(wl.geom.as_dict(), dalpha=dalpha)
        scan = O.Scan(geom)
        out = O.hilbert(scan, g(scan.alpha)[None, :])[0]
        got = np.interp(probes, scan.alpha, out)
        errs.append(np.abs(got - ref).max())
    assert errs[-1] < 2e-4 * np.abs(ref).max()
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ---------------------------------------------------------------- backward rebinning
@pytest.mark.parametrize("cfg", ["tiny", "wide"])
def test_psi_hat_is_smallest_root_on_monotone_branch(cfg):
    if cfg == "tiny":
        scan, _ = _scan()
    else:  # a wide fan where w_kappa turns over inside [-psi_max, psi_max]
        wl = configs.make_workload("w", feed=76.8, cols=184, rows=64, views_per_turn=1160,
                                   turns=1, nxy=256, nz=4, dxy=1.4, slices_per_pitch=77)
        scan = O.Scan(wl.geom.as_dict())
    ph = O.psi_hat(scan)
    lo, hi = O.monotone_branch(scan)
    if cfg == "wide":
        assert (hi < scan.psi_max).any()          # turning points really occur
    grid = np.linspace(-scan.psi_max, scan.psi_max, 20001)
    for c in range(0, scan.cols, max(1, scan.cols // 23)):
        a = scan.alpha[c]
        # branch ends are turning points (derivative 0) or the psi range ends
        for e in (lo[c], hi[c]):
            if abs(abs(e) - scan.psi_max) > 1e-12:
                assert abs(O.dw_kappa_dpsi(scan, a, e)) < 1e-7
        wk = O.w_kappa(scan, a, grid)
        for r in range(scan.rows):
            p = ph[r, c]
            assert lo[c] - 1e-15 <= p <= hi[c] + 1e-15
            if lo[c] < p < hi[c]:
                assert abs(O.w_kappa(scan, a, p) - scan.w[r]) < 1e-9
                # no root with a smaller |psi| (dense scan for sign changes)
                s = np.sign(wk - scan.w[r])
                roots = grid[np.nonzero(s[1:] != s[:-1])[0]]
                assert np.abs(roots).min() >= abs(p) - 2 * (grid[1] - grid[0])


# ---------------------------------------------------------------- backprojection
def test_backprojection_of_constant_matches_closed_form():
    """g^F = 1 gives f = (1/2pi) int_{lambda_i}^{lambda_o} dl / v*(l), with
    int db / (R - rho cos(b - phi)) = 2/sqrt(R^2-rho^2) atan(sqrt((R+rho)/(R-rho)) tan((b-phi)/2));
    the coverage-weighted sum converges at second order in dlambda."""
    rng = np.random.default_rng(8)
    x, y = rng.uniform(-20, 20, (2, 30))
    errs = []
    for level in range(3):
        scan, wl = _scan(views_per_turn=90 * 2 ** level, cols=96, rows=16, turns=4)
        z = np.full(30, 45.0)
        li, lo = O.pi_line(scan, x, y, z)
        li_v, lo_v, nf, nl = O.pi_view_bounds(scan, li, lo)
        gF = np.ones((scan.N, scan.rows, scan.cols))
        f = O.backproject(scan, gF, 0, x, y, z, li_v, lo_v, nf, nl)
        rho, phi = np.hypot(x, y), np.arctan2(y, x)
        R = scan.R
        F = lambda b: 2 / np.sqrt(R * R - rho * rho) * np.arctan(
            np.sqrt((R + rho) / (R - rho)) * np.tan((b - phi) / 2))
        bi, bo = li + scan.lambda0, lo + scan.lambda0
        # split at b - phi = pi (tan branch) where needed
        k = np.ceil((bi - phi - math.pi) / (2 * math.pi))
        cut = phi + math.pi + 2 * math.pi * k
        whole = np.where(cut < bo, (F(cut - 1e-12) - F(bi)) + (F(bo) - F(cut + 1e-12)),
                         F(bo) - F(bi))
        ref = whole / (2 * math.pi)
        errs.append(np.abs(f - ref).max() / np.abs(ref).max())
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ---------------------------------------------------------------- end to end
def test_uniform_ball_reconstructs_positive_density():
    """Sign reading: the +1/(2 pi) backprojection with this detector frame recovers +1
    inside a uniform ball."""
    scan, wl = _scan(nxy=24, nz=12, cols=64, rows=8, views_per_turn=90)
    gr = wl.grid.as_dict()
    zc = gr["z_first"] + 0.5 * (gr["nz"] - 1) * gr["dz"]
    ph = {"kind": "ellipsoids", "centre": np.array([[0, 0, zc]]), "axes": np.array([[15.0] * 3]),
          "rot": np.array([np.eye(3)]), "density": np.array([1.0])}
    g = phantom.project(ph, scan.geom)
    f, valid = O.recon(scan, gr, g)
    c = gr["nz"] // 2
    core = f[c, 9:15, 9:15]
    assert valid[c].all()
    assert np.abs(core - 1.0).max() < 0.02


def test_recon_converges_to_phantom_under_refinement():
    """Relative L2 error inside the phantom (farther than 6 mm = 1.5 coarsest voxels from
    every surface) decreases monotonically as every sampling step is halved."""
    ph = {"kind": "ellipsoids",
          "centre": np.array([[0.0, 0.0, 36.0], [6.0, -4.0, 34.0]]),
          "axes": np.array([[30.0, 22.0, 26.0], [8.0, 10.0, 9.0]]),
          "rot": np.array([O_rot(0.3), O_rot(1.1)]), "density": np.array([1.0, 0.5])}
    errs = []
    for level in range(3):
        s = 2 ** level
        wl = configs.make_workload("c", feed=24.0, cols=32 * s, rows=4 * s, views_per_turn=60 * s,
                                   turns=3, nxy=16 * s, nz=8 * s, dxy=4.0 / s,
                                   slices_per_pitch=6 * s, r_cov=45.0)
        scan = O.Scan(wl.geom.as_dict())
        gr = wl.grid.as_dict()
        g = phantom.project(ph, scan.geom)
        f, valid = O.recon(scan, gr, g)
        xs = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
        zs = gr["z_first"] + np.arange(gr["nz"]) * gr["dz"]
        Z, Y, X = np.meshgrid(zs, xs, xs, indexing="ij")
        P = np.stack([X, Y, Z], -1)
        truth = phantom.density(ph, P)
        m = valid & phantom.surface_distance_ok(ph, P, 6.0) & (truth > 0)
        assert m.sum() > 20
        errs.append(np.linalg.norm((f - truth)[m]) / np.linalg.norm(truth[m]))
    print(errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.01


def O_rot(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def test_pitch_by_pitch_equals_whole_scan():
    """Reusing the first pitch's PI tables for every pitch (lambda + 2 k pi) and filtering
    each pitch's own lambda-window gives the whole-scan result (Sec. II periodicity)."""
    wl = configs.tiny(nxy=16, nz=30, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    scan = O.Scan(wl.geom.as_dict())
    gr = wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    g = phantom.project(ph, scan.geom).astype(np.float32)
    tab = O.pitch_tables(scan, gr)
    assert tab["pitches"].n_pitches == 3
    fp, vp = O.recon(scan, gr, g, mode="pitch", tables=tab)
    fw, vw = O.recon(scan, gr, g, mode="whole")
    assert np.array_equal(vp, vw) and vp.any()
    assert np.abs(fp - fw).max() <= 1e-10 * np.abs(fw).max()


def test_sinogram_shift_by_one_turn_shifts_volume_by_one_pitch():
    wl = configs.tiny(nxy=16, nz=24, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    scan = O.Scan(wl.geom.as_dict())
    gr = wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    g = phantom.project(ph, scan.geom).astype(np.float32)
    f, v = O.recon(scan, gr, g)
    g_shift = np.zeros_like(g)
    g_shift[scan.Nv:] = g[:-scan.Nv]             # data of the object moved up by P
    fs, vs = O.recon(scan, gr, g_shift)
    ns = 12
    both = v[:-ns] & vs[ns:]
    assert both.any()
    assert np.abs(fs[ns:][both] - f[:-ns][both]).max() <= 1e-10 * np.abs(f).max()


# ---------------------------------------------------------------- helix offsets (Sec. II)
def _offset_case(**over):
    wl = configs.tiny(nxy=14, nz=16, cols=48, rows=8, views_per_turn=72, turns=4, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    geom = dict(wl.geom.as_dict(), **OFFSETS)
    geom.update(over)
    gr = configs.centred_grid(configs.Geometry(**geom), 14, 14, 16, 2.0, 2.0).as_dict()
    rng = np.random.default_rng(21)
    g = rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
    return geom, gr, g


def test_rotating_the_helix_rotates_the_volume():
    """lambda0 -> lambda0 + pi/2 turns every source position by pi/2 about the axis, so the
    same data describe the object turned by pi/2: the reconstruction at (x, y) equals the
    first one at (y, -x).  On a square grid centred on the axis that is an index map, and
    the discrete operator (v*, alpha*, w*, PI lines, coverage, validity) must follow it
    exactly; a lambda0 dropped or mis-signed in any of them breaks it."""
    geom, gr, g = _offset_case()
    f0, v0 = O.recon(O.Scan(geom), gr, g)
    f1, v1 = O.recon(O.Scan(dict(geom, lambda0=geom["lambda0"] + 0.5 * math.pi)), gr, g)
    n = gr["nx"]
    # f1[iz, iy, ix] is f0 at (x, y) = (y_iy, -x_ix): column iy, row n - 1 - ix
    rot0 = np.transpose(f0[:, ::-1, :], (0, 2, 1))
    rotv = np.transpose(v0[:, ::-1, :], (0, 2, 1))
    assert np.array_equal(v1, rotv) and v1.sum() > 500
    assert np.abs(f1 - rot0).max() <= 1e-9 * np.abs(f0).max()
    # and the volume itself is not symmetric under that turn (the check has teeth)
    assert np.abs(f0 - rot0)[v0 & rotv].max() > 0.1 * np.abs(f0).max()


def test_raising_the_helix_raises_the_volume():
    """z0 -> z0 + 3 dz lifts every source position by three slices, so the same data describe
    the object lifted by 3 dz: slice iz of the new reconstruction equals slice iz - 3 of the
    first wherever both are valid."""
    geom, gr, g = _offset_case()
    k = 3
    f0, v0 = O.recon(O.Scan(geom), gr, g)
    f1, v1 = O.recon(O.Scan(dict(geom, z0=geom["z0"] + k * gr["dz"])), gr, g)
    both = v1[k:] & v0[:-k]
    assert both.sum() > 500
    assert np.array_equal(v1[k:][both], v0[:-k][both])
    assert np.abs(f1[k:] - f0[:-k])[both].max() <= 1e-9 * np.abs(f0).max()
    assert np.abs(f1 - f0)[v0 & v1].max() > 0.1 * np.abs(f0).max()


def test_pitch_by_pitch_equals_whole_scan_with_offsets():
    """The periodicity of Sec. II (tables of the first pitch reused with lambda + 2 k pi) holds
    for any lambda0, z0 and first view angle."""
    geom, gr, g = _offset_case()
    scan = O.Scan(geom)
    tab = O.pitch_tables(scan, gr)
    assert tab["pitches"].n_pitches >= 2
    fp, vp = O.recon(scan, gr, g, mode="pitch", tables=tab)
    fw, vw = O.recon(scan, gr, g, mode="whole")
    assert np.array_equal(vp, vw) and vp.any()
    assert np.abs(fp - fw).max() <= 1e-10 * np.abs(fw).max()


def test_ball_reconstructs_with_helix_offsets():
    """A uniform ball seen by a helix with lambda0, z0 and a first view off the view grid
    (data from the closed-form projector, which places the source independently)
    reconstructs to +1 inside."""
    wl = configs.tiny(nxy=24, nz=12, cols=64, rows=8, views_per_turn=90)
    geom = dict(wl.geom.as_dict(), **OFFSETS)
    gr = configs.centred_grid(configs.Geometry(**geom), 24, 24, 12, 2.0, 2.0).as_dict()
    zc = gr["z_first"] + 0.5 * (gr["nz"] - 1) * gr["dz"]
    ph = {"kind": "ellipsoids", "centre": np.array([[0, 0, zc]]), "axes": np.array([[15.0] * 3]),
          "rot": np.array([np.eye(3)]), "density": np.array([1.0])}
    f, valid = O.recon(O.Scan(geom), gr, phantom.project(ph, geom))
    c = gr["nz"] // 2
    assert valid[c, 9:15, 9:15].all()
    assert np.abs(f[c, 9:15, 9:15] - 1.0).max() < 0.02


# ---------------------------------------------------------------- adjoint
def test_oracle_adjoint_dot_product():
    wl = configs.tiny(nxy=12, nz=12, cols=32, rows=6, views_per_turn=48, turns=3, feed=24.0,
                      dxy=3.0, slices_per_pitch=8)
    scan = O.Scan(wl.geom.as_dict())
    gr = wl.grid.as_dict()
    rng = np.random.default_rng(9)
    g = rng.normal(size=(scan.N, scan.rows, scan.cols))
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"]))
    tab = O.pitch_tables(scan, gr)
    f, valid = O.recon(scan, gr, g, tables=tab)
    gbar = O.recon_T(scan, gr, fbar, tables=tab)
    lhs = float(np.sum(f * fbar))
    rhs = float(np.sum(g * gbar))
    assert valid.any()
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(f) * np.linalg.norm(fbar) * 10


# ---------------------------------------------------------------- half-sample derivative option
def test_half_sample_derivative_converges():
    """The 2 x 2 cell stencil converges at second order to the exact derivative at constant
    ray direction at the cell centre (lambda_{n+1/2}, alpha_{c+1/2}), obtained from the
    closed-form line integral with the source moved along the helix."""
    ph = {"kind": "gaussians", "centre": np.array([[10.0, -5.0, 30.0], [-20.0, 15.0, 25.0]]),
          "sigma": np.array([12.0, 8.0]), "amp": np.array([1.0, 0.6])}
    errs = []
    for level in range(3):
        nv = 360 * 2 ** level
        cols = 64 * 2 ** level
        wl = configs.make_workload("d", feed=40.0, cols=cols, rows=8, views_per_turn=nv,
                                   turns=1, nxy=16, nz=4, dxy=4.0, slices_per_pitch=10,
                                   r_cov=60.0)
        geom = wl.geom.as_dict()
        gh = O.half_sample_geometry(geom)
        sh = O.Scan(gh)
        n = nv // 4
        g = phantom.project(ph, geom, views=[n, n + 1])
        g1 = O.derivative_lw_half(sh, g)[0] / (sh.D / np.sqrt(sh.D ** 2 + sh.w ** 2))[:, None]
        src, d = phantom.scan_rays(gh, [n])           # rays of the half-sample cell centres
        lam = sh.lam(n)
        eps = 1e-5

        def src_at(l):
            return np.array([sh.R * math.cos(l + sh.lambda0),
                             sh.R * math.sin(l + sh.lambda0), sh.z0 + sh.h * l])
        exact = (phantom.line_integrals(ph, src_at(lam + eps), d[0]) -
                 phantom.line_integrals(ph, src_at(lam - eps), d[0])) / (2 * eps)
        sl = slice(cols // 4, 3 * cols // 4)
        errs.append(np.abs(g1[:, sl] - exact[:, sl]).max() / np.abs(exact[:, sl]).max())
    print(errs)
    assert errs[0] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_half_sample_geometry_is_the_cell_centres():
    geom = configs.tiny(cols=32, rows=6, views_per_turn=48, turns=3).geom.as_dict()
    geom["col_offset"] = 0.25
    s, sh = O.Scan(geom), O.Scan(O.half_sample_geometry(geom))
    assert sh.cols == s.cols - 1 and sh.N == s.N - 1 and sh.rows == s.rows
    assert np.allclose(sh.alpha, 0.5 * (s.alpha[:-1] + s.alpha[1:]), rtol=0, atol=1e-15)
    assert np.allclose(sh.lam(np.arange(sh.N)), 0.5 * (s.lam(np.arange(s.N - 1)) +
                                                       s.lam(np.arange(1, s.N))), atol=1e-13)
    assert np.array_equal(sh.w, s.w)


def test_half_sample_uniform_ball_reconstructs_positive_density():
    """As the central-difference ball test; the averaged stencil smooths across columns, so
    its error in alpha is larger at equal sampling (64 columns: 5 %, 128: 1.2 %, i.e. second
    order), and the test uses 128 columns."""
    wl = configs.tiny(nxy=24, nz=12, cols=128, rows=8, views_per_turn=90)
    geom = wl.geom.as_dict()
    sh = O.Scan(O.half_sample_geometry(geom))
    gr = wl.grid.as_dict()
    zc = gr["z_first"] + 0.5 * (gr["nz"] - 1) * gr["dz"]
    ph = {"kind": "ellipsoids", "centre": np.array([[0, 0, zc]]), "axes": np.array([[15.0] * 3]),
          "rot": np.array([np.eye(3)]), "density": np.array([1.0])}
    g = phantom.project(ph, geom)
    f, valid = O.recon(sh, gr, g, half=True)
    c = gr["nz"] // 2
    # (the half-sample grid has one column less, so the FOV loses the grid corners)
    assert valid[c, 9:15, 9:15].all()
    assert np.abs(f[c, 9:15, 9:15] - 1.0).max() < 0.02


def test_half_sample_recon_converges_with_central():
    """Both derivative stencils discretise the same formula: on a smooth phantom inside the
    fan, each reconstruction converges to the phantom at second order (error / 4 when the
    view, column and row steps halve) and their difference shrinks with it."""
    errs = []
    for cols, rows, vpt in ((64, 8, 120), (128, 16, 240)):
        ph = {"kind": "gaussians", "centre": np.array([[4.0, -3.0, 0.0], [-6.0, 5.0, 0.0]]),
              "sigma": np.array([6.0, 4.0]), "amp": np.array([1.0, 0.5])}
        wl = configs.make_workload("h", feed=24.0, cols=cols, rows=rows, views_per_turn=vpt,
                                   turns=3, nxy=16, nz=6, dxy=2.0, slices_per_pitch=12,
                                   r_cov=50.0)
        geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
        ph["centre"][:, 2] = gr["z_first"] + 0.5 * (gr["nz"] - 1) * gr["dz"]
        g = phantom.project(ph, geom)
        f0, v0 = O.recon(O.Scan(geom), gr, g)
        f1, v1 = O.recon(O.Scan(O.half_sample_geometry(geom)), gr, g, half=True)
        m = v0 & v1
        assert m.sum() > 1000
        P = np.stack(np.meshgrid(gr["z_first"] + np.arange(gr["nz"]) * gr["dz"],
                                 gr["y_first"] + np.arange(gr["ny"]) * gr["dy"],
                                 gr["x_first"] + np.arange(gr["nx"]) * gr["dx"],
                                 indexing="ij")[::-1], -1)
        truth = phantom.density(ph, P)
        nrm = np.linalg.norm(truth[m])
        errs.append((np.linalg.norm((f0 - truth)[m]) / nrm, np.linalg.norm((f1 - truth)[m]) / nrm,
                     np.linalg.norm((f1 - f0)[m]) / nrm))
    print(errs)
    (c0, h0, d0), (c1, h1, d1) = errs
    assert c0 < 0.05 and h0 < 0.05 and d0 < 0.03
    assert c0 / c1 > 3.0 and h0 / h1 > 3.0 and d0 / d1 > 3.0


def test_oracle_adjoint_dot_product_half_sample():
    wl = configs.tiny(nxy=12, nz=12, cols=32, rows=6, views_per_turn=48, turns=3, feed=24.0,
                      dxy=3.0, slices_per_pitch=8)
    geom = wl.geom.as_dict()
    sh = O.Scan(O.half_sample_geometry(geom))
    gr = wl.grid.as_dict()
    rng = np.random.default_rng(11)
    g = rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"]))
    tab = O.pitch_tables(sh, gr)
    f, valid = O.recon(sh, gr, g, tables=tab, half=True)
    gbar = O.recon_T(sh, gr, fbar, tables=tab, half=True)
    assert gbar.shape == g.shape and valid.any()
    lhs, rhs = float(np.sum(f * fbar)), float(np.sum(g * gbar))
    assert abs(lhs - rhs) <= 1e-11 * np.linalg.norm(f) * np.linalg.norm(fbar)


# ---------------------------------------------------------------- detector offsets
def test_shifted_detector_reconstructs_the_same_object():
    """A detector whose centre is moved by (2.5 columns, 1.5 rows) and widened to cover the
    same fan and Tam-Danielsson window sees the same rays at other indices; its
    reconstruction stays that of the phantom.  Read with the offsets' signs flipped, the
    same data give an error near 100 %."""
    ph = {"kind": "gaussians", "centre": np.array([[4.0, -3.0, 0.0], [-6.0, 5.0, 0.0]]),
          "sigma": np.array([6.0, 4.0]), "amp": np.array([1.0, 0.5])}
    wl = configs.make_workload("h", feed=24.0, cols=64, rows=8, views_per_turn=120, turns=3,
                               nxy=16, nz=6, dxy=2.0, slices_per_pitch=12, r_cov=50.0)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph["centre"][:, 2] = gr["z_first"] + 0.5 * (gr["nz"] - 1) * gr["dz"]
    shifted = dict(geom, det_cols=geom["det_cols"] + 6, col_offset=2.5,
                   det_rows=geom["det_rows"] + 4, row_offset=1.5)
    g1 = phantom.project(ph, shifted)
    f0, v0 = O.recon(O.Scan(geom), gr, phantom.project(ph, geom))
    f1, v1 = O.recon(O.Scan(shifted), gr, g1)
    f2, v2 = O.recon(O.Scan(dict(shifted, col_offset=-2.5, row_offset=-1.5)), gr, g1)
    m = v0 & v1 & v2
    P = np.stack(np.meshgrid(gr["z_first"] + np.arange(gr["nz"]) * gr["dz"],
                             gr["y_first"] + np.arange(gr["ny"]) * gr["dy"],
                             gr["x_first"] + np.arange(gr["nx"]) * gr["dx"], indexing="ij")[::-1], -1)
    truth = phantom.density(ph, P)
    nrm = np.linalg.norm(truth[m])
    e1 = np.linalg.norm((f1 - truth)[m]) / nrm
    d = np.linalg.norm((f1 - f0)[m]) / nrm
    e2 = np.linalg.norm((f2 - truth)[m]) / nrm
    print(e1, d, e2)
    assert m.sum() > 1000 and e1 < 0.05 and d < 0.01 and e2 > 0.5
