"""The deterministic adjoint (KATS_FLAG_DETERMINISTIC_ADJOINT): 64-bit fixed-point
accumulation of the transposed backprojection.  Two calls give the same bits; the result
meets the same parity bars as the default adjoint against the FP64 oracle's transpose and
in the dot-product test, on both kernel paths (boxes in LDS, boxes beyond the LDS tile
scattered to HBM), and agrees with the default float adjoint to rounding; at full size
(clinical 512^2 x 128) it is bit-reproducible too."""
import time

import numpy as np
import pytest

import oracle as O
from synth import configs

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("case", ["fits", "hbm"])
def test_deterministic_adjoint_parity_and_reproducibility(case):
    dev = _dev()
    if case == "fits":
        wl = configs.tiny(nxy=12, nz=20, cols=40, rows=8, views_per_turn=60, turns=4, feed=24.0,
                          dxy=2.5, slices_per_pitch=8)
    else:
        wl = configs.tiny(nxy=16, nz=16, cols=48, rows=32, views_per_turn=72, turns=4, feed=24.0,
                          dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print(f"[case] deterministic adjoint, {case}", flush=True)
    plan = K.Plan(geom, gr, device=0, deterministic_adjoint=True)
    fits = plan.info["bp_box_rows"] <= 32 and plan.info["bp_box_cols"] <= 64
    assert fits == (case == "fits")
    rng = np.random.default_rng(23)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    fb = torch.from_numpy(fbar).to(dev)
    a = K.recon_backward(plan, fb)
    b = K.recon_backward(plan, fb)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    got = a.cpu().numpy()
    ref = O.recon_T(O.Scan(geom), gr, fbar.astype(np.float64))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    default = K.recon_backward(K.Plan(geom, gr, device=0), fb).cpu().numpy()
    rel_d = np.linalg.norm(got - default) / np.linalg.norm(default)
    x = torch.from_numpy(rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
                         .astype(np.float32)).to(dev)
    Ax = K.recon(plan, x).double()
    lhs = float((Ax * fb.double()).sum())
    rhs = float((x.double() * a.double()).sum())
    dot = abs(lhs - rhs) / (float(Ax.norm()) * float(np.linalg.norm(fbar)))
    print(f"[parity] deterministic adjoint {case}: vs oracle rel-L2 {rel:.3e}, vs default adjoint "
          f"{rel_d:.3e}, dot product {dot:.3e}", flush=True)
    assert rel <= REL_L2 and rel_d <= 1e-6 and dot <= 1e-5
    # a zero cotangent gives exact zeros (scale 1, nothing accumulated)
    z = K.recon_backward(plan, torch.zeros_like(fb))
    assert int(torch.count_nonzero(z)) == 0


def test_deterministic_adjoint_full_size_reproducible():
    dev = _dev()
    wl = configs.config2()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print("[case] deterministic adjoint, clinical 512^2 x 128", flush=True)
    plan = K.Plan(geom, gr, device=0, gpu_plan=True, deterministic_adjoint=True)
    g = torch.Generator(device=dev).manual_seed(9)
    fb = torch.randn((gr["nz"], gr["ny"], gr["nx"]), device=dev, generator=g)
    a = K.recon_backward(plan, fb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = K.recon_backward(plan, fb)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    assert torch.equal(a, b)
    ref = K.recon_backward(K.Plan(geom, gr, device=0, gpu_plan=True), fb)
    rel = float((a - ref).norm() / ref.norm())
    print(f"[parity] deterministic adjoint at full size: bit-identical twice, {ms:.1f} ms, vs "
          f"default adjoint rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-6
