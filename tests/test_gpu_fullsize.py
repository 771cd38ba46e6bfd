"""Full-size parity of the adjoint (the differentiation use of Sec. III-B) and of the forward
on the sparse-detector workload, in the launch configuration the benchmark times.

The FP64 oracle runs in worker processes (oracle.parallel: the oracle's own functions on
slices and views).  For the adjoint the oracle does not need the whole transpose: the
sinogram cotangent of view n depends only on the filtered-data cotangents of views n-1, n,
n+1 (the derivative in lambda couples neighbours), and each of those is the transpose of
the backprojection over every voxel whose PI window contains that view.  Those rows are
compared element by element with the GPU's katsevich_recon_backward over the whole scan.
Bars: relative L2 <= 1e-5, max |error| <= 1e-4 of the largest reference value."""
import numpy as np
import pytest

import oracle as O
from oracle import parallel as OP
from synth import configs, phantom

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
MAX_ABS_OF_PEAK = 1e-4


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _views_to_check(plan):
    """Views near both ends of the filtered range, inside the part of the first and of the
    last pitch window that no other pitch uses, and in the overlap of two pitch windows."""
    info = plan.info
    a, b = info["first_view"], info["last_view"]
    lo, W, Nv = info["window_lo"], info["window_views"], plan.geom["views_per_turn"]
    k_last = info["n_pitches"] - 1
    cand = [a + 1, lo + Nv // 2, lo + Nv + (W - Nv) // 2, lo + k_last * Nv + W - Nv // 2, b - 1]
    return sorted({int(min(max(n, a), b)) for n in cand})


def _compare_rows(name, gs, ref_rows, plan):
    """The sampled rows against the oracle's, to the bar of the gradient: relative L2 over
    the sampled part of the gradient (all checked views together) <= 1e-5, and every
    element within 1e-4 of the largest reference value.  Per-view relative errors are
    printed: at views near the ends of the filtered range, where few voxels contribute and
    the derivative's difference of neighbouring views cancels, a view's own norm is orders
    of magnitude below the bulk and its relative error shows the float32 rounding of the
    terms that cancel, which the max-abs bar bounds."""
    info = plan.info
    a, b = info["first_view"], info["last_view"]
    peak = max(float(np.abs(r).max()) for r in ref_rows.values())
    num = den = 0.0
    worst_abs = 0.0
    for n, ref in ref_rows.items():
        got = gs[n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(ref) > 0
        d = got - ref
        num += float(np.sum(d * d))
        den += float(np.sum(ref * ref))
        mx = float(np.abs(d).max())
        worst_abs = max(worst_abs, mx)
        print(f"[parity] {name} adjoint view {n}: rel-L2 {np.linalg.norm(d) / np.linalg.norm(ref):.3e} "
              f"max-abs {mx:.3e} (row norm {np.linalg.norm(ref):.3e}, peak {peak:.3e})", flush=True)
    rel = (num / den) ** 0.5
    print(f"[parity] {name} adjoint, {len(ref_rows)} views together: rel-L2 {rel:.3e}, "
          f"max-abs {worst_abs:.3e} = {worst_abs / peak:.2e} of peak", flush=True)
    assert rel <= REL_L2 and worst_abs <= MAX_ABS_OF_PEAK * peak
    # nothing outside the filtered views and their derivative neighbours
    assert int(torch.count_nonzero(gs[:max(a - 1, 0)])) == 0
    assert int(torch.count_nonzero(gs[b + 2:])) == 0
    return rel


def _adjoint_rows(wl, name, seed):
    dev = _dev()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print(f"[case] {name} adjoint at full size", flush=True)
    plan = K.Plan(geom, gr, device=0)
    rng = np.random.default_rng(seed)
    fbar = rng.standard_normal((gr["nz"], gr["ny"], gr["nx"]), dtype=np.float32)
    gs = K.recon_backward(plan, torch.from_numpy(fbar).to(dev))
    torch.cuda.synchronize()
    views = _views_to_check(plan)
    print(f"[oracle] {name}: PI tables and adjoint rows of views {views} "
          f"on {OP.default_workers()} processes", flush=True)
    ref = OP.adjoint_views(geom, gr, fbar.astype(np.float64), views)
    _compare_rows(name, gs, ref, plan)


def test_adjoint_rows_clinical_full_size():
    """512^2 x 128 clinical workload (two pitches)."""
    _adjoint_rows(configs.config2(), "clinical 512^2x128", 41)


def test_adjoint_rows_large_volume_full_size():
    """512^3 / 55296-view workload (five pitches, 3999-view windows)."""
    _adjoint_rows(configs.config5(), "large 512^3", 43)


def test_sparse_workload_forward_and_gradient_full_size():
    """Sparse-detector workload (184 columns, 256^2 x 64) at full size: the whole GPU volume
    against the oracle's, voxel by voxel; then the gradient of 0.5 ||(A g - f) valid||^2
    through KatsevichFn against the oracle's A^T of its own residual, at sampled views."""
    dev = _dev()
    from synth import gpu_projector
    wl = configs.config3(0)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print("[case] sparse workload forward + gradient at full size", flush=True)
    plan = K.Plan(geom, gr, device=0)
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = gpu_projector.project(ph, geom, device=dev)
    x = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
    y = gr["y_first"] + np.arange(gr["ny"]) * gr["dy"]
    z = gr["z_first"] + np.arange(gr["nz"]) * gr["dz"]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    f = phantom.density(ph, np.stack([X, Y, Z], -1)).astype(np.float32)
    valid = plan.export("valid").astype(bool)
    s = sino.clone().requires_grad_(True)
    out = K.KatsevichFn.apply(s, plan)
    vmask = torch.from_numpy(valid).to(dev)
    loss = 0.5 * (((out - torch.from_numpy(f).to(dev)) * vmask) ** 2).sum()
    loss.backward()
    vol = out.detach().cpu().numpy()
    g_host = sino.cpu().numpy()
    print(f"[oracle] sparse workload: full reconstruction on {OP.default_workers()} processes",
          flush=True)
    tab = OP.pitch_tables(geom, gr)
    ref, vref = OP.recon(geom, gr, g_host, tables=tab)
    assert np.array_equal(vref, valid)
    peak = float(f.max())
    d = (vol - ref)[valid]
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref[valid]))
    print(f"[parity] sparse workload full volume: rel-L2 {rel:.3e} max-abs {np.abs(d).max():.3e} "
          f"({int(valid.sum())} valid voxels)", flush=True)
    assert np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and np.abs(d).max() <= MAX_ABS_OF_PEAK * peak
    resid = (ref - f) * valid
    views = _views_to_check(plan)
    print(f"[oracle] sparse workload: gradient rows of views {views}", flush=True)
    rows = OP.adjoint_views(geom, gr, resid, views, tables=tab)
    _compare_rows("sparse workload gradient", s.grad, rows, plan)
