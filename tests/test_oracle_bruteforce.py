"""Brute-force quadrature of the continuous Katsevich inversion formula (paper Sec. II,
eqs. e1-e4) at single voxels, written independently of the oracle:

  f(x) = -1/(2 pi) int_{lambda_i}^{lambda_o} dl |x - a(l)|^-1 g^F(l, theta),
  g^F(l, theta) = PV int_0^{2 pi} dgamma h_H(sin gamma) g'(l, cos gamma theta + sin gamma theta x m),
  h_H(s) = 1/(pi s),  g' = derivative in the source position at fixed direction,

with m the unit normal of the kappa-plane through a(l), a(l+psi), a(l+2psi) of smallest |psi|
containing the ray, oriented as sgn(psi) (a(l+psi)-a(l)) x (a(l+2psi)-a(l)).

The phantom is a sum of Gaussian blobs (smooth, so every integrand is smooth): g' is the
analytic gradient of the closed-form blob line integral dotted with da/dl; the gamma
principal value is taken after subtracting F(0)(1+cos g)/2 + F(pi)(1-cos g)/2 (whose PV
integrals over a period vanish) with the midpoint rule; lambda uses Gauss-Legendre nodes.
The PI interval comes from the closed-form chord condition solved by bisection here.

Pins: (1) the brute force reproduces the phantom density (the formula is exact);
(2) the discretised oracle converges to it under refinement.
"""
import math

import numpy as np
import pytest

import oracle as O
from synth import configs, phantom

R, P = 570.0, 40.0
H = P / (2 * math.pi)
BLOBS = {"kind": "gaussians",
         "centre": np.array([[5.0, -3.0, 30.0], [-25.0, 10.0, 24.0], [18.0, 22.0, 36.0]]),
         "sigma": np.array([16.0, 9.0, 11.0]), "amp": np.array([1.0, 0.6, 0.8])}


def a_of(l):
    return np.array([R * math.cos(l), R * math.sin(l), H * l])


def da_of(l):
    return np.array([-R * math.sin(l), R * math.cos(l), H])


def blob_gprime(src, dirs, dsrc):
    """d/dq of the divergent-beam transform g(q, u) = int_0^inf f(src(q) + t u) dt of the
    blobs at fixed direction u.  For one blob, with p = c - src, t0 = p.u,
    d^2 = |p|^2 - t0^2: g = amp sigma sqrt(pi/2) (1 + erf(t0 / (sigma sqrt 2))) exp(-d^2/2sigma^2)
    and grad_src g = -amp exp(-|p|^2 / 2 sigma^2) u + (g / sigma^2) (p - t0 u)."""
    from scipy.special import erf
    u = dirs / np.linalg.norm(dirs, axis=-1, keepdims=True)
    out = np.zeros(dirs.shape[:-1])
    for c, s, amp in zip(BLOBS["centre"], BLOBS["sigma"], BLOBS["amp"]):
        p = c - src
        pu = u @ p
        d2 = p @ p - pu * pu
        L = amp * s * math.sqrt(math.pi / 2) * (1 + erf(pu / (s * math.sqrt(2)))) * \
            np.exp(-d2 / (2 * s * s))
        grad = (L / (s * s))[..., None] * (p[None, :] - pu[..., None] * u) - \
            amp * math.exp(-(p @ p) / (2 * s * s)) * u
        out += grad @ dsrc
    return out


def kappa_normal(l, theta):
    """Unit normal m of the smallest-|psi| kappa-plane containing the ray (l, theta)."""
    a0 = a_of(l)

    def a_vec(ls):
        return np.stack([R * np.cos(ls), R * np.sin(ls), H * ls], -1)

    def n_of(psi):
        psi = np.asarray(psi, float)
        return np.cross(a_vec(l + psi) - a0, a_vec(l + 2 * psi) - a0)

    # n(psi).theta ~ psi^3 near 0: scan psi^-3 n(psi).theta for sign changes
    grid = np.concatenate([-np.geomspace(math.pi - 1e-6, 1e-4, 3000), np.geomspace(1e-4, math.pi - 1e-6, 3000)])
    vals = (n_of(grid) @ theta) / grid ** 3
    idx = np.nonzero(np.sign(vals[1:]) != np.sign(vals[:-1]))[0]
    idx = [i for i in idx if grid[i] * grid[i + 1] > 0]            # not across psi = 0
    best = None
    for i in idx:
        lo, hi = grid[i], grid[i + 1]
        flo = vals[i]
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            fm = n_of(mid) @ theta / mid ** 3
            if np.sign(fm) == np.sign(flo):
                lo, flo = mid, fm
            else:
                hi = mid
        r = 0.5 * (lo + hi)
        if best is None or abs(r) < abs(best):
            best = r
    if best is None:      # theta along the psi -> 0 limit plane
        best = 1e-4
    n = n_of(best) * math.copysign(1.0, best)
    return n / np.linalg.norm(n)


def gF_continuous(l, theta, n_gamma=512):
    m = kappa_normal(l, theta)
    e2 = np.cross(theta, m)
    g = (np.arange(n_gamma) + 0.5) * 2 * math.pi / n_gamma
    src = a_of(l)
    dsrc = da_of(l)
    dirs = np.cos(g)[:, None] * theta[None, :] + np.sin(g)[:, None] * e2[None, :]
    F = blob_gprime(src, dirs, dsrc)
    F0 = blob_gprime(src, theta[None, :], dsrc)[0]
    Fpi = blob_gprime(src, -theta[None, :], dsrc)[0]
    reg = (F - F0 * (1 + np.cos(g)) / 2 - Fpi * (1 - np.cos(g)) / 2) / (math.pi * np.sin(g))
    return reg.sum() * 2 * math.pi / n_gamma


def pi_interval(x):
    """lambda_i < lambda_o with x on the chord a(lambda_i) a(lambda_o), span < 2 pi
    (bisection on the chord height; in-plane chord by line-circle intersection)."""
    X = np.asarray(x, float)

    def chord(s):
        S = a_of(s)[:2]
        d = X[:2] - S
        tau = -2 * (S @ d) / (d @ d)
        E = S + tau * d
        span = math.atan2(S[0] * E[1] - S[1] * E[0], S @ E) % (2 * math.pi)
        return span, 1.0 / tau

    def f(s):
        span, t = chord(s)
        return H * (s + t * span) - X[2]

    lo, hi = X[2] / H - 2 * math.pi, X[2] / H
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    s = 0.5 * (lo + hi)
    return s, s + chord(s)[0]


def f_bruteforce(x, n_lambda=96):
    li, lo = pi_interval(x)
    nodes, weights = np.polynomial.legendre.leggauss(n_lambda)
    ls = 0.5 * (lo - li) * nodes + 0.5 * (lo + li)
    acc = 0.0
    for l, w in zip(ls, weights):
        d = np.asarray(x) - a_of(l)
        r = np.linalg.norm(d)
        acc += w * gF_continuous(l, d / r) / r
    return -acc * 0.5 * (lo - li) / (2 * math.pi)


POINTS = [(0.0, 0.0, 30.0), (8.0, -6.0, 28.0), (-20.0, 9.0, 25.0), (15.0, 20.0, 34.0)]


@pytest.fixture(scope="module")
def brute():
    return np.array([f_bruteforce(p) for p in POINTS])


def test_continuous_formula_reproduces_phantom(brute):
    truth = phantom.density(BLOBS, np.array(POINTS))
    print("bruteforce", brute, "truth", truth)
    assert np.abs(brute - truth).max() < 2e-6 * truth.max()


def test_discretised_oracle_converges_to_continuous_formula(brute):
    ref = brute
    errs = []
    for level in range(2):
        s = 2 ** level
        wl = configs.make_workload("bf", feed=P, cols=96 * s, rows=12 * s, views_per_turn=240 * s,
                                   turns=3, nxy=4, nz=4, dxy=1.0, slices_per_pitch=40, r_cov=110.0)
        geom = wl.geom.as_dict()
        scan = O.Scan(geom)
        pts = np.array(POINTS)
        li, lo = O.pi_line(scan, pts[:, 0], pts[:, 1], pts[:, 2])
        li_v, lo_v, nf, nl = O.pi_view_bounds(scan, li, lo)
        a, b = int(nf.min()) - 1, int(nl.max()) + 1
        assert a >= 0 and b <= scan.N - 1
        g = phantom.project(BLOBS, geom, views=np.arange(a, b + 1))
        gF = O.filter_views(scan, g)
        f = O.backproject(scan, gF, a, pts[:, 0], pts[:, 1], pts[:, 2], li_v, lo_v, nf, nl)
        errs.append(np.abs(f - ref).max() / np.abs(ref).max())
    print("oracle vs continuous formula", errs)
    assert errs[1] < 2e-2
    assert errs[1] < 0.5 * errs[0]
