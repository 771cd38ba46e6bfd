"""GPU tests of the grouped multi-request backprojection and the serving loop: every
request's volume is bit-identical alone (plain katsevich_recon) and in the mix, and equal to
the FP64 oracle's reconstruction to the parity bar (relative L2 <= 1e-5, max |error| <=
1e-4 of the phantom peak over valid voxels, invalid voxels 0)."""
import numpy as np
import pytest

import oracle as O
from synth import configs, phantom

torch = pytest.importorskip("torch")
K = pytest.importorskip("paper_2201_02309_amd")
from paper_2201_02309_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _small_requests():
    """Five small scans of different lengths, pitches and grids (two share a geometry)."""
    specs = [dict(nxy=24, nz=16, cols=48, rows=8, views_per_turn=72, turns=3, feed=24.0, dxy=2.0),
             dict(nxy=20, nz=30, cols=40, rows=8, views_per_turn=60, turns=5, feed=30.0, dxy=2.0,
                  slices_per_pitch=15),
             dict(nxy=33, nz=9, cols=64, rows=10, views_per_turn=90, turns=4, feed=20.0, dxy=1.5,
                  slices_per_pitch=10),
             dict(nxy=24, nz=16, cols=48, rows=8, views_per_turn=72, turns=3, feed=24.0, dxy=2.0),
             dict(nxy=17, nz=40, cols=36, rows=8, views_per_turn=64, turns=6, feed=36.0, dxy=2.5,
                  slices_per_pitch=18)]
    out = []
    for i, sp in enumerate(specs):
        wl = configs.tiny(seed=50 + i, **sp)
        g, gr = wl.geom.as_dict(), wl.grid.as_dict()
        ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
        out.append((g, gr, phantom.project(ph, g).astype(np.float32)))
    return out


def _wide_box_request():
    """A scan whose backprojection footprint boxes exceed the LDS tile (wide fan of fine
    columns over coarse voxels), so its tiles take the kernel path with HBM taps."""
    wl = configs.tiny(nxy=24, nz=12, cols=160, rows=8, views_per_turn=72, turns=3, feed=24.0,
                      dxy=8.0, seed=61)
    g, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    return g, gr, phantom.project(ph, g).astype(np.float32)


def test_packed_backprojection_equals_single_launches():
    dev = _dev()
    # 19 items: more than one group of 16, both kernel paths
    reqs = (_small_requests() * 4)[:18] + [_wide_box_request()]
    plans = [K.Plan(g, gr, device=0) for g, gr, _ in reqs]
    fits = [p.info["bp_box_rows"] <= 32 and p.info["bp_box_cols"] <= 64 for p in plans]
    assert any(fits) and not all(fits)
    gFs = [K.filter_views(p, torch.from_numpy(s).to(dev)) for p, (_, _, s) in zip(plans, reqs)]
    alone = [K.backproject(p, gF) for p, gF in zip(plans, gFs)]
    mixed = K.backproject_batch(plans, gFs)
    torch.cuda.synchronize()
    for i, (a, m) in enumerate(zip(alone, mixed)):
        print(f"[serve] packed item {i}: shape {tuple(a.shape)}", flush=True)
        assert torch.equal(a, m)


def _oracle_parity(r):
    ref, valid = O.recon(O.Scan(r.geom), r.grid, r.sino.cpu().numpy())
    got = r.volume.cpu().numpy()
    x = r.grid["x_first"] + np.arange(r.grid["nx"]) * r.grid["dx"]
    y = r.grid["y_first"] + np.arange(r.grid["ny"]) * r.grid["dy"]
    z = r.grid["z_first"] + np.arange(r.grid["nz"]) * r.grid["dz"]
    d = (got - ref)[valid]
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref[valid]))
    print(f"[parity] served request {r.rid} vs oracle: rel-L2 {rel:.3e}, max-abs "
          f"{np.abs(d).max():.3e}, {int(valid.sum())} valid voxels", flush=True)
    assert valid.sum() > 0 and np.all(got[~valid] == 0)
    peak = float(np.abs(ref[valid]).max())
    assert rel <= 1e-5 and np.abs(d).max() <= 1e-4 * peak
    del x, y, z


@pytest.mark.parametrize("saturated", [True, False])
def test_served_results_equal_alone(saturated):
    dev = _dev()
    reqs = _small_requests()
    cache = serve.PlanCache(dev, workers=2)
    arrivals = configs.serving_arrivals(len(reqs), rate=200.0, seed=3, saturated=saturated)
    rs = [serve.Request(rid=i, arrival=float(t), geom=g, grid=gr,
                        sino=torch.from_numpy(s).to(dev))
          for i, ((g, gr, s), t) in enumerate(zip(reqs, arrivals))]
    srv = serve.Server(cache, budget_bytes=64 << 20, max_batch=3, keep_volumes=True)
    done = srv.run(rs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert srv.arena.used == 0
    for r in done:
        plan = cache.get_blocking(r.geom, r.grid)
        alone = K.recon(plan, r.sino)
        torch.cuda.synchronize()
        print(f"[serve] request {r.rid}: latency {r.latency * 1e3:.1f} ms hit={r.cache_hit}",
              flush=True)
        assert torch.equal(alone, r.volume)
        if saturated:
            _oracle_parity(r)
    assert cache.misses >= 4 and len(cache.plans) == 4      # two requests share a geometry
    cache.close()


def test_served_results_with_plans_evicted():
    """A table budget that holds no plan: every plan is dropped once its requests complete
    (a request holds its plan from arrival to completion), and the served volumes are still
    those of plain katsevich_recon and of the oracle."""
    dev = _dev()
    reqs = _small_requests()
    cache = serve.PlanCache(dev, workers=2, table_budget=1)
    rs = [serve.Request(rid=i, arrival=0.002 * i, geom=g, grid=gr, sino=torch.from_numpy(s).to(dev))
          for i, (g, gr, s) in enumerate(reqs)]
    srv = serve.Server(cache, budget_bytes=64 << 20, max_batch=2, keep_volumes=True)
    done = srv.run(rs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs) and not any(r.error for r in done)
    assert cache.evicted >= 3 and not cache.inuse
    for r in sorted(done, key=lambda r: r.rid)[:3]:
        plan = K.Plan(r.geom, r.grid, device=0)
        alone = K.recon(plan, r.sino)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.volume)
        _oracle_parity(r)
    cache.close()


def test_admission_budget_smaller_than_two_requests_queues_them():
    dev = _dev()
    reqs = _small_requests()[:3]
    cache = serve.PlanCache(dev, workers=1)
    rs = [serve.Request(rid=i, arrival=0.0, geom=g, grid=gr, sino=torch.from_numpy(s).to(dev))
          for i, (g, gr, s) in enumerate(reqs)]
    biggest = max(serve.footprint(cache.get_blocking(r.geom, r.grid)) for r in rs)
    srv = serve.Server(cache, budget_bytes=biggest, max_batch=8)
    done = srv.run(rs)
    assert len(done) == 3 and srv.arena.used == 0
    # one request in flight at a time: admissions strictly after earlier completions
    order = sorted(done, key=lambda r: r.t_admit)
    for a, b in zip(order, order[1:]):
        assert b.t_admit >= a.t_done
    cache.close()
