"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
float32 inputs.  Bar (floating point): relative L2 <= 1e-5 and max |error| <= 1e-4 of the
phantom peak over valid voxels; invalid voxels exactly 0.  Integer tables are compared bit
for bit in test_plan_host.py."""
import math

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


def _grid_points(gr):
    x = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
    y = gr["y_first"] + np.arange(gr["ny"]) * gr["dy"]
    z = gr["z_first"] + np.arange(gr["nz"]) * gr["dz"]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], -1)


def _report(name, got, ref, valid, peak):
    d = (got - ref)[valid]
    rel = float(np.linalg.norm(d) / max(np.linalg.norm(ref[valid]), 1e-30))
    mx = float(np.abs(d).max()) if d.size else 0.0
    print(f"[parity] {name}: rel-L2 {rel:.3e}  max-abs {mx:.3e}  peak {peak:.3f}  "
          f"valid {int(valid.sum())}", flush=True)
    return rel, mx


class _Case:
    def __init__(self, wl, n_psi=0):
        self.wl = wl
        self.geom, self.grid = wl.geom.as_dict(), wl.grid.as_dict()
        self.scan = O.Scan(self.geom, n_psi)
        self.ph = phantom.make_phantom(wl.phantom, self.grid, wl.seed)
        self.sino = phantom.project(self.ph, self.geom).astype(np.float32)
        self.tab = O.pitch_tables(self.scan, self.grid)
        self.ftab = O.FilterTables(self.scan)
        self._ref = None
        self.peak = float(phantom.density(self.ph, _grid_points(self.grid)).max())

    @property
    def ref(self):
        if self._ref is None:
            self._ref = O.recon(self.scan, self.grid, self.sino, tables=self.tab, ftables=self.ftab)
        return self._ref


@pytest.fixture(scope="module")
def case1():
    return _Case(configs.config1())


@pytest.fixture(scope="module")
def plan1(case1):
    _dev()
    return K.Plan(case1.geom, case1.grid, device=0)


def test_filter_stage_parity(case1, plan1):
    dev = _dev()
    a, b = plan1.info["first_view"], plan1.info["last_view"]
    print(f"[case] config1 filter views {a}..{b}", flush=True)
    gFp = K.filter_views(plan1, torch.from_numpy(case1.sino).to(dev)).cpu().numpy()
    P = K.katsevich.PAD
    assert np.all(gFp[:, :P] == 0) and np.all(gFp[:, -P:] == 0)
    assert np.all(gFp[:, :, :P] == 0) and np.all(gFp[:, :, -P:] == 0)
    gF = gFp[:, P:-P, P:-P]
    ref = O.filter_views(case1.scan, case1.sino[a - 1:b + 2], case1.ftab)[1:-1]
    rel = np.linalg.norm(gF - ref) / np.linalg.norm(ref)
    mx = np.abs(gF - ref).max() / np.abs(ref).max()
    print(f"[parity] filter stage: rel-L2 {rel:.3e} max-abs/max {mx:.3e}", flush=True)
    assert rel <= REL_L2 and mx <= 1e-5


def test_backprojection_stage_parity(case1, plan1):
    """The GPU backprojector fed the oracle's g^F (rounded to float32) against the oracle
    backprojection of the same float32 g^F."""
    dev = _dev()
    a, b = plan1.info["first_view"], plan1.info["last_view"]
    gF64 = O.filter_views(case1.scan, case1.sino[a - 1:b + 2], case1.ftab)[1:-1]
    gF32 = gF64.astype(np.float32)
    P = K.katsevich.PAD
    gF32p = np.pad(gF32, ((0, 0), (P, P), (P, P)))
    vol = K.backproject(plan1, torch.from_numpy(gF32p).to(dev)).cpu().numpy()
    full = np.zeros((case1.scan.N, case1.scan.rows, case1.scan.cols), np.float32)
    full[a:b + 1] = gF32
    ref = np.zeros_like(vol, dtype=np.float64)
    tab, gr, scan = case1.tab, case1.grid, case1.scan
    x = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
    y = gr["y_first"] + np.arange(gr["ny"]) * gr["dy"]
    Y2, X2 = np.meshgrid(y, x, indexing="ij")
    valid = np.zeros(vol.shape, bool)
    pit = tab["pitches"]
    for k in range(pit.n_pitches):
        sl, js = pit.slices(k)
        s = k * scan.Nv
        for iz, j in zip(sl, js):
            nf, nl = tab["nf"][j] + s, tab["nl"][j] + s
            m = O.valid_mask(scan, nf, nl, tab["fov"][j])
            valid[iz] = m
            zj = gr["z_first"] + j * gr["dz"]
            ref[iz][m] = O.backproject(scan, full, 0, X2[m], Y2[m], np.full(m.sum(), zj),
                                       tab["li"][j][m] + s, tab["lo"][j][m] + s, nf[m], nl[m],
                                       lam_shift=2 * math.pi * k)
    rel, mx = _report("backprojection stage", vol, ref, valid, case1.peak)
    assert np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * case1.peak


def test_recon_parity_config1(case1, plan1):
    dev = _dev()
    vol = K.recon(plan1, torch.from_numpy(case1.sino).to(dev)).cpu().numpy()
    ref, valid = case1.ref
    assert np.array_equal(valid, plan1.export("valid").astype(bool))
    rel, mx = _report("recon config1", vol, ref, valid, case1.peak)
    assert np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * case1.peak


@pytest.mark.parametrize("bp_slices", [8, 32])
def test_recon_parity_slice_run_variants(case1, bp_slices):
    """The 8- and 32-slice backprojection kernels meet the same bar as the default."""
    dev = _dev()
    plan = K.Plan(case1.geom, case1.grid, device=0, bp_slices=bp_slices)
    vol = K.recon(plan, torch.from_numpy(case1.sino).to(dev)).cpu().numpy()
    ref, valid = case1.ref
    rel, mx = _report(f"recon config1 bp_slices={bp_slices}", vol, ref, valid, case1.peak)
    assert np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * case1.peak


@pytest.mark.parametrize("shape", [(13, 11, 29), (9, 17, 5), (1, 1, 3)])
def test_recon_ragged_grids(shape):
    """Grids that are not multiples of the 8 x 8 tile or of the slice run, spanning pitch
    boundaries (12 slices per pitch), down to a single voxel column."""
    dev = _dev()
    nx, ny, nz = shape
    wl = configs.tiny(nxy=16, nz=nz, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gr.update(nx=nx, ny=ny, x_first=-0.5 * (nx - 1) * 2.0 + 0.3, y_first=-0.5 * (ny - 1) * 2.0 - 0.7)
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(geom)
    ref, valid = O.recon(scan, gr, sino)
    plan = K.Plan(geom, gr, device=0)
    vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
    peak = max(float(phantom.density(ph, _grid_points(gr)).max()), 0.1)
    print(f"[case] ragged {shape}", flush=True)
    rel, mx = _report(f"ragged {shape}", vol, ref, valid, peak)
    assert np.all(vol[~valid] == 0)
    if valid.any():
        assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak


@pytest.mark.parametrize("R,degree", [(30.0, 7), (26.0, -1)])
def test_wide_fan_geometries(R, degree):
    """Short helix radii: a fan of +-0.79 rad takes the backprojector's general column
    coordinate (degree-7 polynomial in tan^2, the instance a degree-4 fit cannot serve) and
    +-0.96 rad the library atan2f (no polynomial of degree <= 8 meets the fit bound);
    recon against the oracle at the bar, the adjoint against the oracle's transpose."""
    dev = _dev()
    wl = configs.make_workload(f"wide-fan-R{R:g}", feed=24.0, cols=96, rows=16, views_per_turn=144,
                               turns=3, nxy=16, nz=12, dxy=2.0, slices_per_pitch=12, R=R, D=2.0 * R,
                               phantom=configs.tiny(nxy=16).phantom, seed=7)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(geom)
    ref, valid = O.recon(scan, gr, sino)
    peak = float(phantom.density(ph, _grid_points(gr)).max())
    rng = np.random.default_rng(8)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    refT = O.recon_T(scan, gr, fbar.astype(np.float64))
    for kw in ({}, {"gpu_plan": True}):
        print(f"[case] wide fan R = {R:g} mm, plan {kw}", flush=True)
        plan = K.Plan(geom, gr, device=0, **kw)
        assert plan.info["atan_degree"] == degree
        vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
        rel, mx = _report(f"wide fan R={R:g} {kw}", vol, ref, valid, peak)
        assert valid.sum() > 0 and np.all(vol[~valid] == 0)
        assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak
        got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev)).cpu().numpy()
        relT = np.linalg.norm(got - refT) / np.linalg.norm(refT)
        print(f"[parity] wide fan R={R:g} {kw} adjoint vs oracle: rel-L2 {relT:.3e}", flush=True)
        assert relT <= REL_L2


@pytest.mark.parametrize("variant", ["thin-slices", "thick-slices", "anisotropic-voxels",
                                     "partial-field-of-view", "tall-detector", "tight-detector"])
def test_slice_and_voxel_shape_variants(variant):
    """Slice spacing far below the detector row spacing (rows per slice ~0.1: many slices
    share a row in the adjoint's row merging), far above it (~3 rows per slice: the walk
    skips rows), non-square voxels (dx != dy), and a fan narrower than the grid (field of
    view radius 14.9 mm against 21.2 mm grid corners: a third of the voxels invalid, their
    lanes idle inside the tiles, the projections truncated), detector rows covering 1.5
    times the Tam-Danielsson window and only 1 % more than it (projections reaching the edge
    rows, footprint boxes clipped at the padded detector): recon against the oracle at the
    bar, the adjoint against the oracle's transpose."""
    dev = _dev()
    spp = {"thin-slices": 96, "thick-slices": 3}.get(variant, 12)
    nz = {"thin-slices": 40, "thick-slices": 6}.get(variant, 16)
    wl = configs.tiny(nxy=16, nz=nz, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=spp)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    if variant == "anisotropic-voxels":
        gr.update(nx=12, ny=20, dx=2.6, dy=1.5, x_first=-0.5 * 11 * 2.6, y_first=-0.5 * 19 * 1.5)
    if variant == "partial-field-of-view":
        geom["dalpha"] *= 0.7
    if variant == "tall-detector":
        geom["dw"] *= 1.5 / 1.1                   # the recipe's rows cover 1.1 x the window
    if variant == "tight-detector":
        geom["dw"] *= 1.01 / 1.1
    print(f"[case] {variant}: dz {gr['dz']:.3f} mm, dw {geom['dw']:.3f} mm", flush=True)
    plan = K.Plan(geom, gr, device=0)
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(geom)
    ref, valid = O.recon(scan, gr, sino)
    vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
    peak = float(phantom.density(ph, _grid_points(gr)).max())
    rel, mx = _report(variant, vol, ref, valid, peak)
    assert valid.sum() > 0 and np.all(vol[~valid] == 0)
    if variant == "partial-field-of-view":
        assert 0 < int((~valid).sum()) < valid.size
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak
    rng = np.random.default_rng(9)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev)).cpu().numpy()
    refT = O.recon_T(scan, gr, fbar.astype(np.float64))
    relT = np.linalg.norm(got - refT) / np.linalg.norm(refT)
    print(f"[parity] {variant} adjoint vs oracle: rel-L2 {relT:.3e}", flush=True)
    assert relT <= REL_L2


@pytest.mark.parametrize("n_psi", [5, 64, 200])
def test_kappa_line_counts(n_psi):
    """Other numbers of kappa-lines than the default 2 rows + 1: few (5), even (64: the FFT
    pairs kappa rows two per transform, the matrix-core tiles group 16 lines), many (200);
    both Hilbert paths against the oracle with the same count, and the adjoint against the
    oracle's transpose."""
    dev = _dev()
    wl = configs.tiny(nxy=16, nz=12, cols=48, rows=8, views_per_turn=72, turns=5, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print(f"[case] n_psi = {n_psi}", flush=True)
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(geom, n_psi)
    ref, valid = O.recon(scan, gr, sino)
    peak = float(phantom.density(ph, _grid_points(gr)).max())
    for mode in (1, 2):
        plan = K.Plan(geom, gr, device=0, n_psi=n_psi, hilbert_mode=mode)
        assert plan.info["n_psi"] == n_psi
        vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
        rel, mx = _report(f"n_psi {n_psi} hilbert_mode {mode}", vol, ref, valid, peak)
        assert np.all(vol[~valid] == 0)
        assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak
    rng = np.random.default_rng(10)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev)).cpu().numpy()
    refT = O.recon_T(scan, gr, fbar.astype(np.float64))
    relT = np.linalg.norm(got - refT) / np.linalg.norm(refT)
    print(f"[parity] n_psi {n_psi} adjoint vs oracle: rel-L2 {relT:.3e}", flush=True)
    assert relT <= REL_L2


def test_long_hulls_take_the_exact_fallback():
    """3000 views per turn: a workgroup's hull (the union of its voxels' PI windows over a
    pitch) spans ~4200 views, beyond the per-view group-word tables of both backprojectors,
    which then evaluate every slice group's coverage at every view.  Forward against the
    oracle, adjoint against the oracle transpose and by the dot product."""
    dev = _dev()
    wl = configs.tiny(nxy=16, nz=8, cols=48, rows=8, views_per_turn=3000, turns=3, feed=24.0,
                      dxy=2.0, slices_per_pitch=8)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    print("[case] long hulls, 3000 views per turn", flush=True)
    plan = K.Plan(geom, gr, device=0)
    nf, nl = plan.export("pi_nfirst").astype(np.int64), plan.export("pi_nlast").astype(np.int64)
    ok = nf <= nl
    assert ok.any() and int(nl[ok].max() - nf[ok].min() + 1) > 2048
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    scan = O.Scan(geom)
    ref, valid = O.recon(scan, gr, sino)
    vol = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
    peak = max(float(phantom.density(ph, _grid_points(gr)).max()), 0.1)
    rel, mx = _report("long hulls", vol, ref, valid, peak)
    assert valid.any() and np.all(vol[~valid] == 0)
    assert rel <= REL_L2 and mx <= MAX_ABS_OF_PEAK * peak
    rng = np.random.default_rng(8)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev))
    ref_T = O.recon_T(scan, gr, fbar.astype(np.float64))
    rel_T = np.linalg.norm(got.cpu().numpy() - ref_T) / np.linalg.norm(ref_T)
    x = torch.from_numpy(sino).to(dev)
    Ax = K.recon(plan, x).double()
    y = torch.from_numpy(fbar).to(dev).double()
    dot = abs(float((Ax * y).sum()) - float((x.double() * got.double()).sum()))
    dot /= float(Ax.norm()) * float(y.norm())
    print(f"[parity] long hulls adjoint: vs oracle rel-L2 {rel_T:.3e}, dot product {dot:.3e}",
          flush=True)
    assert rel_T <= REL_L2 and dot <= 1e-5


@pytest.mark.parametrize("dz_mm", [200.0, -200.0])
def test_grid_beyond_the_scan_reconstructs_to_zero(dz_mm):
    """Degenerate plan: the grid lies above (or below) every slice the helix covers, so no
    voxel is valid and no view is filtered; recon writes zeros over a volume that held other
    values, and the adjoint (float and deterministic) writes zeros over the whole sinogram;
    the plan built on the GPU says the same."""
    dev = _dev()
    wl = configs.config1()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gr["z_first"] += dz_mm
    print(f"[case] grid beyond the scan, z shifted {dz_mm} mm", flush=True)
    for kw in ({}, {"gpu_plan": True}, {"deterministic_adjoint": True}):
        plan = K.Plan(geom, gr, device=0, **kw)
        assert plan.info["n_vv"] == 0 and plan.n_filtered == 0
        assert not plan.export("valid").any()
        g = torch.rand((geom["n_views"], geom["det_rows"], geom["det_cols"]), device=dev,
                       generator=torch.Generator(dev).manual_seed(5))
        vol = torch.full((gr["nz"], gr["ny"], gr["nx"]), 7.0, device=dev)
        K.recon(plan, g, out=vol)
        gs = torch.full_like(g, 7.0)
        K.recon_backward(plan, torch.rand_like(vol), out=gs)
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(vol)) == 0 and int(torch.count_nonzero(gs)) == 0


def test_device_plan_rejects_a_grid_outside_the_field_of_view():
    """No voxel inside the field of view: the device builder refuses the plan, like the host
    builder."""
    _dev()
    wl = configs.config1()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gr = dict(gr, nx=4, ny=4, x_first=200.0, y_first=200.0)        # r > r_fov = 53 mm
    for kw in ({}, {"gpu_plan": True}):
        with pytest.raises(K.KatsevichError, match="field of view"):
            K.Plan(geom, gr, device=0, **kw)


def test_turn_shift_gives_pitch_shift_bit_exact():
    """Sinogram shifted by one turn (views_per_turn views) -> volume shifted by one pitch,
    bit for bit: every pitch uses identical pitch-relative geometry and no atomics."""
    dev = _dev()
    wl = configs.tiny(nxy=24, nz=36, cols=48, rows=8, views_per_turn=72, turns=6, feed=24.0,
                      dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = phantom.project(ph, geom).astype(np.float32)
    sh = np.zeros_like(sino)
    sh[72:] = sino[:-72]
    plan = K.Plan(geom, gr, device=0)
    v0 = K.recon(plan, torch.from_numpy(sino).to(dev)).cpu().numpy()
    v1 = K.recon(plan, torch.from_numpy(sh).to(dev)).cpu().numpy()
    valid = plan.export("valid").astype(bool)
    both = valid[:-12] & valid[12:]
    assert both.any()
    assert np.array_equal(v1[12:][both], v0[:-12][both])


def test_recon_is_deterministic(case1, plan1):
    dev = _dev()
    s = torch.from_numpy(case1.sino).to(dev)
    a = K.recon(plan1, s).cpu().numpy()
    b = K.recon(plan1, s).cpu().numpy()
    assert np.array_equal(a, b)


def test_wrong_shapes_are_rejected(case1, plan1):
    dev = _dev()
    with pytest.raises(K.KatsevichError):
        K.recon(plan1, torch.zeros((3, 4, 5), device=dev))
    with pytest.raises(K.KatsevichError):
        K.recon(plan1, torch.zeros((case1.scan.N, case1.scan.rows, case1.scan.cols),
                                   dtype=torch.float64, device=dev))


# ------------------------------------------------------------------ clinical config (sampled)
def _sampled_parity(wl, name, n, z_ends, x_edges, half=False, seed=11):
    """GPU volume of the whole workload at n random voxels plus voxels near the z ends and
    the FOV edge, against the oracle computed voxel by voxel from the same float32
    sinogram (filtering only the views the plan uses)."""
    dev = _dev()
    from synth import gpu_projector
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    print(f"[case] {name} sampled parity", flush=True)
    plan = K.Plan(geom, gr, device=0, half_sample=half)
    a, b = plan.info["first_view"], plan.info["last_view"]
    hi = b + 2 + (1 if half else 0)             # sinogram views a-1 .. hi-1 feed the filter
    sino_d = torch.zeros((geom["n_views"], geom["det_rows"], geom["det_cols"]),
                         dtype=torch.float32, device=dev)
    gpu_projector.project(ph, geom, views=np.arange(a - 1, hi), out=sino_d[a - 1:hi])
    # the GPU projector against the closed form on the host, on a few views
    chk = np.array([a - 1, (a + b) // 2, hi - 1])
    host = phantom.project(ph, geom, views=chk)
    got = sino_d[torch.from_numpy(chk).to(dev)].cpu().numpy()
    assert np.abs(got - host).max() <= 1e-5 * np.abs(host).max()
    vol = K.recon(plan, sino_d).cpu().numpy()
    torch.cuda.synchronize()
    sino = sino_d[a - 1:hi].cpu().numpy()
    del sino_d
    scan = O.Scan(O.half_sample_geometry(geom) if half else geom)
    rng = np.random.default_rng(seed)
    ze = np.asarray(z_ends)
    iz = np.concatenate([rng.integers(0, gr["nz"], n), np.tile(ze, 24 // len(ze))])
    iy = np.concatenate([rng.integers(0, gr["ny"], n), rng.integers(0, gr["ny"], 24)])
    ix = np.concatenate([rng.integers(0, gr["nx"], n), np.tile(x_edges, 24 // len(x_edges))])
    valid = plan.export("valid").astype(bool)[iz, iy, ix]
    pit = O.Pitches(scan, gr)
    k, j = iz // pit.ns, iz % pit.ns
    x = gr["x_first"] + ix * gr["dx"]
    y = gr["y_first"] + iy * gr["dy"]
    zj = gr["z_first"] + j * gr["dz"]
    Li, Lo = O.pi_line(scan, x, y, zj)
    li, lo, nf, nl = O.pi_view_bounds(scan, Li, Lo)
    ref = np.zeros(len(iz))
    prog = lambda i, n: print(f"[oracle] filtering view {i} of {n}", flush=True)
    gF = O.filter_views(scan, sino, O.FilterTables(scan), progress=prog, half=half)
    print("[oracle] backprojecting sampled voxels", flush=True)
    for kk in np.unique(k):
        m = (k == kk) & valid
        sh = kk * scan.Nv
        ref[m] = O.backproject(scan, gF, a - 1, x[m], y[m], zj[m], li[m] + sh, lo[m] + sh,
                               nf[m] + sh, nl[m] + sh, lam_shift=2 * math.pi * kk)
    got = vol[iz, iy, ix]
    coarse = dict(gr, nx=gr["nx"] // 4, ny=gr["ny"] // 4, nz=max(gr["nz"] // 4, 1),
                  dx=4 * gr["dx"], dy=4 * gr["dy"], dz=4 * gr["dz"])
    peak = float(phantom.density(ph, _grid_points(coarse)).max())
    d = (got - ref)[valid]
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref[valid]))
    print(f"[parity] {name} sampled: rel-L2 {rel:.3e} max-abs {np.abs(d).max():.3e} "
          f"({int(valid.sum())} valid of {len(iz)})", flush=True)
    assert valid.sum() > n // 2
    assert np.all(got[~valid] == 0)
    assert rel <= REL_L2 and np.abs(d).max() <= MAX_ABS_OF_PEAK * peak


def test_clinical_config_sampled_parity():
    """512^2 x 128 clinical workload at full size, in the launch configuration the
    benchmark times."""
    _sampled_parity(configs.config2(), "config2", 300, [0, 1, 76, 77, 126, 127], [0, 511, 3, 508])


def test_clinical_config_half_sample_sampled_parity():
    """The same workload with the half-sample derivative."""
    _sampled_parity(configs.config2(), "config2 half-sample", 200, [0, 1, 76, 77, 126, 127],
                    [0, 511, 3, 508], half=True, seed=13)


def test_sparse_detector_config_sampled_parity():
    """Sparse-detector geometry (184 columns at 96 mm/turn, 256^2 x 64 grid): w_kappa turns
    over inside the psi range and the footprint boxes exceed the LDS tile (the kernels'
    HBM path)."""
    _sampled_parity(configs.config3(), "config3", 300, [0, 1, 47, 48, 62, 63], [0, 255, 2, 253],
                    seed=17)


# ------------------------------------------------------------------ adjoint
@pytest.fixture(scope="module")
def small_adj():
    wl = configs.tiny(nxy=12, nz=20, cols=40, rows=8, views_per_turn=60, turns=4, feed=24.0,
                      dxy=2.5, slices_per_pitch=8)
    return wl.geom.as_dict(), wl.grid.as_dict()


def test_adjoint_dot_product(small_adj):
    dev = _dev()
    geom, gr = small_adj
    plan = K.Plan(geom, gr, device=0)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
                         .astype(np.float32)).to(dev)
    y = torch.from_numpy(rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)).to(dev)
    Ax = K.recon(plan, x).double()
    ATy = K.recon_backward(plan, y).double()
    lhs = float((Ax * y.double()).sum())
    rhs = float((x.double() * ATy).sum())
    rel = abs(lhs - rhs) / (float(Ax.norm()) * float(y.double().norm()))
    print(f"[parity] adjoint dot product: {rel:.3e}", flush=True)
    assert rel <= 1e-5


def test_adjoint_matches_oracle_transpose(small_adj):
    dev = _dev()
    geom, gr = small_adj
    plan = K.Plan(geom, gr, device=0)
    rng = np.random.default_rng(6)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev)).cpu().numpy()
    ref = O.recon_T(O.Scan(geom), gr, fbar.astype(np.float64))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"[parity] adjoint vs oracle: rel-L2 {rel:.3e}", flush=True)
    assert rel <= REL_L2


@pytest.mark.parametrize("case,bp_slices", [("fits", 8), ("fits", 32), ("hbm", 16), ("hbm", 8)])
def test_adjoint_kernel_instances(case, bp_slices):
    """The adjoint's kernel instances against the oracle's transpose: 8- and 32-slice runs,
    and a 32-row detector whose footprint boxes (36 rows) exceed the LDS tile, so its views
    scatter through the HBM path."""
    dev = _dev()
    if case == "fits":
        wl = configs.tiny(nxy=12, nz=20, cols=40, rows=8, views_per_turn=60, turns=4, feed=24.0,
                          dxy=2.5, slices_per_pitch=8)
    else:
        wl = configs.tiny(nxy=16, nz=16, cols=48, rows=32, views_per_turn=72, turns=4, feed=24.0,
                          dxy=2.0, slices_per_pitch=12)
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    plan = K.Plan(geom, gr, device=0, bp_slices=bp_slices)
    lr = 64 if bp_slices >= 32 else 32
    fits = plan.info["bp_box_rows"] <= lr and plan.info["bp_box_cols"] <= 64
    assert fits == (case == "fits")
    rng = np.random.default_rng(21)
    fbar = rng.normal(size=(gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)
    got = K.recon_backward(plan, torch.from_numpy(fbar).to(dev)).cpu().numpy()
    ref = O.recon_T(O.Scan(geom), gr, fbar.astype(np.float64))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    x = torch.from_numpy(rng.normal(size=(geom["n_views"], geom["det_rows"], geom["det_cols"]))
                         .astype(np.float32)).to(dev)
    Ax = K.recon(plan, x).double()
    lhs = float((Ax * torch.from_numpy(fbar).to(dev).double()).sum())
    rhs = float((x.double() * torch.from_numpy(got).to(dev).double()).sum())
    dot = abs(lhs - rhs) / (float(Ax.norm()) * float(np.linalg.norm(fbar)))
    print(f"[parity] adjoint {case} bp_slices={bp_slices} (boxes {plan.info['bp_box_rows']}x"
          f"{plan.info['bp_box_cols']}): vs oracle rel-L2 {rel:.3e}, dot product {dot:.3e}", flush=True)
    assert rel <= REL_L2 and dot <= 1e-5


def test_autograd_function_gradient(small_adj):
    dev = _dev()
    geom, gr = small_adj
    plan = K.Plan(geom, gr, device=0)
    rng = np.random.default_rng(7)
    s = torch.from_numpy(rng.normal(size=(2, geom["n_views"], geom["det_rows"], geom["det_cols"]))
                         .astype(np.float32)).to(dev).requires_grad_(True)
    target = torch.from_numpy(rng.normal(size=(2, gr["nz"], gr["ny"], gr["nx"])).astype(np.float32)).to(dev)
    out = K.KatsevichFn.apply(s, plan)
    loss = 0.5 * ((out - target) ** 2).sum()
    loss.backward()
    for bidx in range(2):
        expect = K.recon_backward(plan, (out[bidx] - target[bidx]).detach().contiguous())
        assert torch.allclose(s.grad[bidx], expect, rtol=0, atol=1e-6 * float(expect.abs().max()))
