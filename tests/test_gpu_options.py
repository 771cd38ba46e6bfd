"""GPU parity of the plan options against the oracle: the half-sample derivative
(KATS_FLAG_HALF_SAMPLE_DERIVATIVE; the oracle's half=True on its cell-centre grid) in the
forward reconstruction and its adjoint, and detector column / row offsets (the paper's
quarter-column offset and a shifted, widened detector)."""
import numpy as np
import pytest

import oracle as O
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


def _points(gr):
    z = gr["z_first"] + np.arange(gr["nz"]) * gr["dz"]
    y = gr["y_first"] + np.arange(gr["ny"]) * gr["dy"]
    x = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], -1)


def _parity(name, geom, gr, ph, half=False, **plan_kw):
    dev = _dev()
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(O.half_sample_geometry(geom) if half else geom)
    ref, valid = O.recon(scan, gr, sino, half=half)
    plan = K.Plan(geom, gr, device=0, half_sample=half, **plan_kw)
    assert plan.info["half_sample"] == int(half)
    assert np.array_equal(valid, plan.export("valid").astype(bool))
    vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
    peak = max(float(phantom.density(ph, _points(gr)).max()), 0.1)
    d = (vol - ref)[valid]
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref[valid]))
    mx = float(np.abs(d).max())
    print(f"[parity] {name}: rel-L2 {rel:.3e}  max-abs {mx:.3e}  peak {peak:.3f}  "
          f"valid {int(valid.sum())}", flush=True)
    assert valid.any() and np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak


def test_half_sample_recon_parity_config1():
    wl = configs.config1()
    gr = wl.grid.as_dict()
    print("[case] parity-64^3, half-sample derivative", flush=True)
    _parity("half-sample config1", wl.geom.as_dict(), gr,
            phantom.make_phantom(wl.phantom, gr, wl.seed), half=True)


@pytest.mark.parametrize("bp_slices", [8, 32])
def test_half_sample_recon_ragged_grid(bp_slices):
    wl = configs.tiny(nxy=16, nz=29, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gr.update(nx=13, ny=11, x_first=-12.0 + 0.3, y_first=-10.0 - 0.7)
    print(f"[case] ragged 13x11x29 half-sample, bp_slices {bp_slices}", flush=True)
    _parity(f"half-sample ragged bp_slices={bp_slices}", geom, gr,
            phantom.make_phantom(wl.phantom, gr, wl.seed), half=True, bp_slices=bp_slices)


@pytest.fixture(scope="module")
def half_adj():
    wl = configs.tiny(nxy=12, nz=20, cols=40, rows=8, views_per_turn=60, turns=4, feed=24.0,
                      dxy=2.5, slices_per_pitch=8)
    return wl.geom.as_dict(), wl.grid.as_dict()


def test_half_sample_adjoint_dot_product_and_oracle(half_adj):
    dev = _dev()
    geom, gr = half_adj
    plan = K.Plan(geom, gr, device=0, half_sample=True)
    rng = np.random.default_rng(15)
    x = torch.from_numpy(rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
                         .astype(np.float32)).to(dev)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    y = torch.from_numpy(fbar).to(dev)
    Ax = K.recon(plan, x).double()
    ATy = K.recon_backward(plan, y)
    assert ATy.shape == x.shape
    lhs = float((Ax * y.double()).sum())
    rhs = float((x.double() * ATy.double()).sum())
    rel = abs(lhs - rhs) / (float(Ax.norm()) * float(y.double().norm()))
    print(f"[parity] half-sample adjoint dot product: {rel:.3e}", flush=True)
    assert rel <= 1e-5
    ref = O.recon_T(O.Scan(O.half_sample_geometry(geom)), gr, fbar.astype(np.float64), half=True)
    got = ATy.cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"[parity] half-sample adjoint vs oracle: rel-L2 {rel:.3e}", flush=True)
    assert rel <= REL_L2


@pytest.mark.parametrize("offsets", [(0.25, 0.0), (0.25, -0.2), (2.5, 1.5)])
def test_detector_offsets_parity(offsets):
    """Quarter-column offset (the paper's detector), a row offset, and a detector shifted
    by (2.5, 1.5) cells and widened by (6, 4) cells to keep covering the fan and the
    Tam-Danielsson window."""
    co, ro = offsets
    wl = configs.config1()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    geom.update(col_offset=co, row_offset=ro)
    if co > 1:
        geom.update(det_cols=geom["det_cols"] + 6, det_rows=geom["det_rows"] + 4)
    print(f"[case] parity-64^3 with detector offsets {offsets}", flush=True)
    _parity(f"offsets {offsets}", geom, gr, phantom.make_phantom(wl.phantom, gr, wl.seed))
