"""The Hilbert filter as a Toeplitz product on the matrix cores (hilbert_mode 2) against the
register-FFT path and the FP64 oracle: the filtered views of both paths agree to a few 1e-7
relative (float16 pairs with float32 accumulation), also for inputs scaled by 1e+-6 (the
power-of-two range scaling), odd detector widths and the half-sample derivative; the
reconstruction meets the oracle bar."""
import numpy as np
import pytest

import oracle as O
from synth import configs, phantom

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")
KK = pytest.importorskip("paper_2201_02309_amd.katsevich")

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


CASES = {
    "parity-64^3": (configs.config1, {}),
    "clinical-512^2x128": (configs.config2, {}),
    "sparse-184-columns": (configs.config3, {}),
    "odd-47-columns": (lambda: configs.tiny(nxy=16, nz=8, cols=47, rows=8, views_per_turn=72,
                                            turns=4, feed=24.0, dxy=2.0), {}),
    "parity-64^3 half-sample": (configs.config1, {"half_sample": True}),
    # the other product widths: 2 fragments per wave (257-512 columns), 4 (769-1024), the
    # largest detector a plan accepts and a ragged width beside it
    "wide-300-columns": (lambda: configs.tiny(nxy=16, nz=8, cols=300, rows=8, views_per_turn=72,
                                              turns=4, feed=24.0, dxy=2.0), {}),
    "wide-1023-columns": (lambda: configs.tiny(nxy=16, nz=8, cols=1023, rows=8, views_per_turn=72,
                                               turns=4, feed=24.0, dxy=2.0), {}),
    "max-1024-columns": (lambda: configs.tiny(nxy=16, nz=8, cols=1024, rows=8, views_per_turn=72,
                                              turns=4, feed=24.0, dxy=2.0), {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_matrix_core_hilbert_matches_fft(name):
    dev = _dev()
    make, kw = CASES[name]
    wl = make()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print(f"[case] hilbert mode 2 vs 1: {name}", flush=True)
    pf = K.Plan(g, gr, device=0, hilbert_mode=1, **kw)
    pm = K.Plan(g, gr, device=0, hilbert_mode=2, **kw)
    gen = torch.Generator(device=dev).manual_seed(11)
    base = torch.rand((g["n_views"], g["det_rows"], g["det_cols"]), device=dev, generator=gen)
    for scale in (1.0, 1e6, 1e-6):
        sino = base * scale
        a = KK.filter_views(pf, sino)
        b = KK.filter_views(pm, sino)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(b).all())
        rel = float((a - b).double().norm() / a.double().norm())
        mx = float((a - b).abs().max() / a.abs().max())
        print(f"[parity] {name} x{scale:g}: matrix cores vs FFT rel-L2 {rel:.3e}, "
              f"max-abs/peak {mx:.3e}", flush=True)
        assert rel <= 1e-6 and mx <= 5e-6


def test_matrix_core_hilbert_filter_and_recon_vs_oracle():
    dev = _dev()
    wl = configs.config1()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino_np = phantom.project(ph, g).astype(np.float32)
    scan = O.Scan(g)
    plan = K.Plan(g, gr, device=0, hilbert_mode=2)
    a, b = plan.info["first_view"], plan.info["last_view"]
    sino = torch.from_numpy(sino_np).to(dev)
    P = KK.PAD
    gF = KK.filter_views(plan, sino).cpu().numpy()[:, P:-P, P:-P]
    ref = O.filter_views(scan, sino_np[a - 1:b + 2])[1:-1]
    rel = np.linalg.norm(gF - ref) / np.linalg.norm(ref)
    print(f"[parity] matrix-core filter stage vs oracle: rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-5
    vol = K.recon(plan, sino).cpu().numpy()
    rvol, valid = O.recon(scan, gr, sino_np)
    d = (vol - rvol)[valid]
    relv = float(np.linalg.norm(d) / np.linalg.norm(rvol[valid]))
    peak = float(np.abs(rvol[valid]).max())
    print(f"[parity] matrix-core recon vs oracle: rel-L2 {relv:.3e}, max-abs "
          f"{np.abs(d).max():.3e} (peak {peak:.3f})", flush=True)
    assert relv <= 1e-5 and np.abs(d).max() <= 1e-4 * peak and np.all(vol[~valid] == 0)
