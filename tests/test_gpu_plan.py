"""GPU tests of the device plan builder (katsevich_plan_device): every table computed on the
GPU in float64 equals the host plan's (integer tables bit for bit, float64 tables to the
last bits of the libm functions), its PI limits agree with the oracle's bisection directly,
and it reconstructs the same volume."""
import time

import numpy as np
import pytest

import oracle as O
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
    "parity-64^3 offsets": lambda: configs.with_helix_offsets(configs.config1()),
    "serving-12 (512^2x160, 44 slices/pitch)": lambda: configs.serving_request(12),
    "sparse-256^2x64": configs.config3,
    "clinical-512^2x128": configs.config2,
    "non-commensurate": lambda: configs.tiny(nxy=20, nz=9, slices_per_pitch=None, feed=23.0,
                                             dxy=2.1),
}

INFO_KEYS = ("first_view", "last_view", "n_vv", "n_valid_voxels", "window_views", "window_lo",
             "n_pitches", "n_table_slices", "slices_per_pitch", "n_psi", "fft_len", "atan_degree",
             "bp_box_rows", "bp_box_cols", "workspace_bytes", "filtered_bytes")


def _device_plan(g, gr):
    t0 = time.perf_counter()
    p = K.Plan(g, gr, gpu_plan=True, device=0, keep_pi_scratch=True)
    return p, time.perf_counter() - t0


@pytest.mark.parametrize("name", list(CASES))
def test_device_plan_equals_host_plan(name):
    _dev()
    wl = CASES[name]()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print(f"[case] device plan {name}", flush=True)
    t0 = time.perf_counter()
    host = K.Plan(g, gr, bind=False)
    t_host = time.perf_counter() - t0
    _device_plan(g, gr)                                   # first use loads the kernels
    gpu, t_gpu = _device_plan(g, gr)
    print(f"[plan] {name}: host {t_host:.3f} s, device {t_gpu * 1e3:.1f} ms", flush=True)
    for key in INFO_KEYS:
        assert host.info[key] == gpu.info[key], key
    for t in ("fr_row", "br_kappa", "valid"):
        assert np.array_equal(host.export(t), gpu.export(t)), t
    for t in ("fr_weight", "br_weight", "psi_hat"):
        d = np.abs(host.export(t) - gpu.export(t)).max()
        assert d <= 1e-12, (t, d)
    pt = gpu.pi_tables()
    for key, t in (("nf", "pi_nfirst"), ("nl", "pi_nlast"), ("fov", "fov")):
        assert np.array_equal(host.export(t).astype(np.int64), pt[key].astype(np.int64)), t
    for key, t in (("li", "pi_li"), ("lo", "pi_lo")):
        d = np.abs(host.export(t) - pt[key]).max()
        print(f"[plan] {name}: max |{t} host - device| = {d:.3e} views", flush=True)
        assert d <= 1e-9


@pytest.mark.parametrize("name", ["parity-64^3", "parity-64^3 offsets", "clinical-512^2x128"])
def test_device_pi_lines_match_oracle_bisection(name):
    """The device PI limits (Newton on the chord angle with the projection step) against the
    oracle's bisection on the chord-height equation, in view units, and the integer first /
    last covered views bit for bit; every voxel of the parity cases, 20000 sampled voxels
    of the clinical table pitch."""
    _dev()
    wl = CASES[name]()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gpu, _ = _device_plan(g, gr)
    pt = gpu.pi_tables()
    scan = O.Scan(g)
    shape = pt["li"].shape
    idx = np.arange(pt["li"].size)
    if idx.size > 20000:
        idx = np.random.default_rng(7).choice(idx, 20000, replace=False)
    j, iy, ix = np.unravel_index(idx, shape)
    X = gr["x_first"] + ix * gr["dx"]
    Y = gr["y_first"] + iy * gr["dy"]
    Z = gr["z_first"] + j * gr["dz"]
    lam_i, lam_o = O.pi_line(scan, X, Y, Z)
    li, lo, nf, nl = O.pi_view_bounds(scan, lam_i, lam_o)
    di = np.abs(pt["li"].reshape(-1)[idx] - li).max()
    do = np.abs(pt["lo"].reshape(-1)[idx] - lo).max()
    print(f"[parity] {name}: device PI limits vs oracle bisection, {idx.size} voxels: "
          f"max |li| diff {di:.3e}, |lo| diff {do:.3e} views", flush=True)
    assert di <= 1e-9 and do <= 1e-9
    assert np.array_equal(pt["nf"].reshape(-1)[idx], nf)
    assert np.array_equal(pt["nl"].reshape(-1)[idx], nl)
    assert np.array_equal(pt["fov"].reshape(-1)[idx].astype(bool), O.in_fov(scan, X, Y))


def test_reconstruction_with_device_plan():
    dev = _dev()
    wl = configs.config1()
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino_np = phantom.project(ph, g).astype(np.float32)
    sino = torch.from_numpy(sino_np).to(dev)
    host = K.Plan(g, gr, device=0)
    gpu = K.Plan(g, gr, device=0, gpu_plan=True)
    a = K.recon(host, sino)
    b = K.recon(gpu, sino)
    torch.cuda.synchronize()
    rel = float((a - b).norm() / a.norm())
    print(f"[plan] recon with host vs device plan: rel-L2 {rel:.3e}, bit-identical "
          f"{bool(torch.equal(a, b))}", flush=True)
    assert rel <= 1e-6
    ref, valid = O.recon(O.Scan(g), gr, sino_np)
    got = b.cpu().numpy()
    d = (got - ref)[valid]
    rel_o = float(np.linalg.norm(d) / np.linalg.norm(ref[valid]))
    print(f"[parity] recon with the device plan vs oracle: rel-L2 {rel_o:.3e}", flush=True)
    assert rel_o <= 1e-5 and np.all(got[~valid] == 0)
    # a rebind moves the device-built tables to another buffer
    gpu.bind(0)
    c = K.recon(gpu, sino)
    assert torch.equal(b, c)
