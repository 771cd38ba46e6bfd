"""GPU tests of the device PI-line solve (katsevich_plan_device): the plan it builds equals
the host plan (integer tables identical, float64 PI limits to rounding), and reconstructs
the same volume."""
import time

import numpy as np
import pytest

from synth import configs, phantom

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


CASES = {
    "parity-64^3": configs.config1,
    "serving-12 (512^2x160, 44 slices/pitch)": lambda: configs.serving_request(12),
    "sparse-256^2x64": configs.config3,
    "non-commensurate": lambda: configs.tiny(nxy=20, nz=9, slices_per_pitch=None, feed=23.0,
                                             dxy=2.1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_plan_equals_host_plan(name):
    _dev()
    wl = CASES[name]()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    t0 = time.perf_counter()
    host = K.Plan(g, gr, bind=False)
    t1 = time.perf_counter()
    gpu = K.Plan(g, gr, bind=False, gpu_plan=True, device=0)
    t2 = time.perf_counter()
    print(f"[plan] {name}: host {t1 - t0:.3f} s, with GPU PI lines {t2 - t1:.3f} s", flush=True)
    for key in ("first_view", "last_view", "n_vv", "n_valid_voxels", "window_views", "window_lo",
                "n_pitches", "n_table_slices", "bp_box_rows", "bp_box_cols", "table_bytes"):
        assert host.info[key] == gpu.info[key], key
    for t in ("pi_nfirst", "pi_nlast", "fov", "valid", "fr_row", "br_kappa"):
        assert np.array_equal(host.export(t), gpu.export(t)), t
    for t in ("pi_li", "pi_lo"):
        d = np.abs(host.export(t) - gpu.export(t)).max()
        print(f"[plan] {name}: max |{t} host - gpu| = {d:.3e} views", flush=True)
        assert d <= 1e-9


def test_reconstruction_with_device_plan():
    dev = _dev()
    wl = configs.config1()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = torch.from_numpy(phantom.project(ph, g).astype(np.float32)).to(dev)
    host = K.Plan(g, gr, device=0)
    gpu = K.Plan(g, gr, device=0, gpu_plan=True)
    a = K.recon(host, sino)
    b = K.recon(gpu, sino)
    torch.cuda.synchronize()
    rel = float((a - b).norm() / a.norm())
    print(f"[plan] recon with host vs device plan: rel-L2 {rel:.3e}", flush=True)
    assert rel <= 1e-6
