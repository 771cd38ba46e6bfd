"""Plain float64 NumPy oracle of the sparse-detector data path and the image metrics.

TEST INFRASTRUCTURE ONLY: used by tests/ and bench.py's cpu_baseline leg.  It shares no code
with the HIP library.

* Sec. III-C data preparation: keep every 4th detector column (alpha_sp = alpha[0:4:end]),
  interpolate back to the full column grid, add 'Gaussian+Poisson' noise:
  counts from lambda = I0 exp(-g / M) (M the maximum of the upsampled sinogram), then
  g_in = M log(I0 / counts).  Readings where the paper leaves a choice:
  - interpolation: linear in alpha between neighbouring kept columns, the last kept
    column's value held beyond it (numpy.interp's end rule);
  - the printed 'g = g + poisson(g) + Gaussian' is taken as counts = Poisson(lambda) +
    N(0, var): adding a Poisson draw to its own mean would double the photon count.  The
    Poisson draw is its normal limit lambda + sqrt(lambda) z1 (lambda >= I0 / e = 3.7e4 here,
    where the two laws differ by O(lambda^-1/2) in distribution); counts below one photon
    are raised to 1;
  - the normal variates come from the counter-based generator Philox4x64-10 (Salmon et
    al., SC'11): elements 2b and 2b+1 share the block of counter (b, 0, 0, 0) and key
    (seed, 0); the even one takes its words (x0, x1), the odd one (x2, x3), as the 24-bit
    uniforms u1 = ((first >> 40) + 1) 2^-24, u2 = (second >> 40) 2^-24, and
    z1, z2 = sqrt(-2 ln u1) (cos, sin)(2 pi u2) (Box-Muller).
* Sec. IV metrics: RMSE = sqrt(||f - f_GT||^2 / n); SSIM of the whole image as one window
  with population means, variances and covariance and c1 = (0.01 range(f_GT))^2,
  c2 = (0.03 range(f_GT))^2 (the paper calls sigma a variance but squares it in the
  formula; sigma^2 is read as the variance).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 128-bit product of uint64 arrays as (hi, lo), from 32-bit halves."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds.  counter: uint64 [..., 4]; key: (k0, k1).  Each round maps
    (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)) and
    then advances the key by the Weyl constants."""
    with np.errstate(over="ignore"):
        c = [np.array(counter[..., i], dtype=np.uint64) for i in range(4)]
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        for _ in range(10):
            hi0, lo0 = _mulhilo64(_M0, c[0])
            hi1, lo1 = _mulhilo64(_M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = k0 + _W0
            k1 = k1 + _W1
    return np.stack(c, axis=-1)


def sparse_sample(g, step=4):
    """Columns 0, step, 2 step, ... of the sinogram (alpha_sp = alpha_cor[0:step:end])."""
    return np.asarray(g)[..., ::step]


def sparse_upsample(gs, cols, step=4):
    """Linear interpolation in alpha from the kept columns back to cols columns."""
    gs = np.asarray(gs, np.float64)
    xk = np.arange(gs.shape[-1]) * step
    xc = np.arange(cols)
    flat = gs.reshape(-1, gs.shape[-1])
    out = np.empty((flat.shape[0], cols))
    for i in range(flat.shape[0]):
        out[i] = np.interp(xc, xk, flat[i])
    return out.reshape(gs.shape[:-1] + (cols,))


def normals_at(idx, seed):
    """(z1, z2) of the given element indices (any order, any size of the full array)."""
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = np.zeros((idx.size, 4), np.uint64)
    ctr[:, 0] = idx >> np.uint64(1)
    x = philox4x64_10(ctr, (seed, 0))
    odd = (idx & np.uint64(1)).astype(bool)
    first = np.where(odd, x[:, 2], x[:, 0])
    second = np.where(odd, x[:, 3], x[:, 1])
    u1 = ((first >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (second >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    rho = np.sqrt(-2.0 * np.log(u1))
    return rho * np.cos(2.0 * np.pi * u2), rho * np.sin(2.0 * np.pi * u2)


def add_noise_at(g_values, idx, M, I0=1e5, var=0.5, seed=0):
    """The noisy values of the elements idx whose data are g_values (same rule as add_noise)."""
    g = np.asarray(g_values, np.float64)
    z1, z2 = normals_at(idx, seed)
    lam = I0 * np.exp(-g / M)
    counts = np.maximum(lam + np.sqrt(lam) * z1 + np.sqrt(var) * z2, 1.0)
    return M * np.log(I0 / counts)


def normals(n, seed):
    """(z1, z2) of elements 0 .. n-1."""
    nb = (n + 1) // 2
    ctr = np.zeros((nb, 4), np.uint64)
    ctr[:, 0] = np.arange(nb, dtype=np.uint64)
    x = philox4x64_10(ctr, (seed, 0))
    first = np.stack([x[:, 0], x[:, 2]], axis=1).ravel()[:n]       # even, odd elements
    second = np.stack([x[:, 1], x[:, 3]], axis=1).ravel()[:n]
    u1 = ((first >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (second >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    rho = np.sqrt(-2.0 * np.log(u1))
    return rho * np.cos(2.0 * np.pi * u2), rho * np.sin(2.0 * np.pi * u2)


def add_noise(g, M=None, I0=1e5, var=0.5, seed=0):
    """Noisy sinogram of Sec. III-C (readings in the module docstring)."""
    g = np.asarray(g, np.float64)
    M = float(g.max()) if M is None else float(M)
    z1, z2 = normals(g.size, seed)
    lam = I0 * np.exp(-g.ravel() / M)
    counts = np.maximum(lam + np.sqrt(lam) * z1 + np.sqrt(var) * z2, 1.0)
    return (M * np.log(I0 / counts)).reshape(g.shape)


def rmse(f, ref):
    f, ref = np.asarray(f, np.float64), np.asarray(ref, np.float64)
    return float(np.sqrt(np.sum((f - ref) ** 2) / f.size))


def ssim(f, ref):
    f, ref = np.asarray(f, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    mf, mr = f.mean(), ref.mean()
    vf, vr = np.mean((f - mf) ** 2), np.mean((ref - mr) ** 2)
    cov = np.mean((f - mf) * (ref - mr))
    rng = ref.max() - ref.min()
    c1, c2 = (0.01 * rng) ** 2, (0.03 * rng) ** 2
    return float((2 * mf * mr + c1) * (2 * cov + c2) / ((mf ** 2 + mr ** 2 + c1) * (vf + vr + c2)))
