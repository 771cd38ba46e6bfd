#!/usr/bin/env python3
"""Benchmark: pitch-by-pitch Katsevich reconstruction of the clinical high-pitch workload
(512^2 x 128 grid, 736 x 64 curved detector, 1160 views/turn x 6 turns, feed 76.8 mm/turn)
on one MI355X.

One step = one pass of the whole hot path over one synthetic sinogram resident in HBM:
katsevich_filter (derivative + length weighting, forward rebinning, Hilbert, backward
rebinning + cosine) followed by katsevich_backproject (PI-window backprojection of every
pitch with the shared per-pitch tables).  Throughput = (voxel, view) updates with non-zero
PI coverage per second; volumes/s = 1 / step time.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 work of one (voxel, view) update of the backprojection (FMA = 2 flops):
# detector row 2, floor/fraction 2, bilinear interpolation 9, PI coverage weight 4,
# weighted accumulation 3.
BP_FLOP_PER_UPDATE = 20
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, sino_dev, nz_sample=16, iz0=24):
    """Time the FP64 oracle (oracle.parallel: the oracle's own functions spread over one
    worker process per host core, BLAS limited to one thread each) on a slab of the
    workload: nz_sample consecutive 512 x 512 slices from z index iz0, reconstructed
    pitch-style from the same device-resident sinogram (copied to the host untimed).  The
    PI tables of the slab are built first and timed apart, like the GPU's plan; the rate is
    the slab's (voxel, view) updates over the filtering + backprojection time."""
    import numpy as np

    from oracle import parallel as OP

    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    sub = dict(gr)
    sub["nz"] = nz_sample
    sub["z_first"] = gr["z_first"] + iz0 * gr["dz"]
    g_host = sino_dev.cpu().numpy()
    workers = OP.default_workers()
    with OP.pool(workers) as ex:
        list(ex.map(OP.warm, range(4 * workers)))           # start every worker, untimed
        t0 = time.perf_counter()
        tab = OP.pitch_tables(geom, sub, ex=ex)
        t_tab = time.perf_counter() - t0
        t0 = time.perf_counter()
        f, valid = OP.recon(geom, sub, g_host, tables=tab, ex=ex)
        t = time.perf_counter() - t0
    updates = int(((tab["nl"] - tab["nf"] + 1) * valid).sum())
    views = int(tab["n_hi"] - tab["n_lo"] + 1)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": updates / t / 1e9, "unit": "Gvoxel-view/s", "cores": workers,
            "kind": "oracle",
            "sample": f"slices {iz0}..{iz0 + nz_sample - 1} (512 x 512 each) of the clinical "
                      f"workload: filtering of the {views} views of their pitch window and "
                      f"backprojection of {int(valid.sum())} voxels ({updates:.3e} updates) in "
                      f"{t:.1f} s on {workers} worker processes (float64 NumPy, 1 BLAS thread "
                      f"each); their PI tables took {t_tab:.1f} s more, not counted",
            "seconds": round(t, 3), "pi_tables_seconds": round(t_tab, 3),
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "host_cpus_affinity": affinity,
            "finite": bool(np.isfinite(f).all())}


def serving_bench(duration=60.0, rate=20.0, budget=200e9, n_saturated=300):
    """Serving workload as specified: Poisson arrivals at `rate` per second for `duration`
    seconds, request i drawn by synth.configs.serving_request(i) (grids 256^2x32 .. 512^2x160,
    feed U[40,96] mm/turn, 2-10 turns, dense or 4x-sparse columns, 64 rows, 1160 views/turn),
    so that nearly every request brings a new geometry.  Both sides start from a cold plan
    cache and build every plan on the GPU inside the request's latency: the
    continuous-batching server against one-at-a-time katsevich_recon (FIFO) on the same
    trace, then both on the first n_saturated requests all arriving at once.  Sinograms are
    views of one pre-generated random scan resident in HBM outside the budget (their values
    do not change the work), copied device to device on admission inside the budget."""
    import numpy as np
    import torch

    from paper_2201_02309_amd import serve
    from synth import configs

    dev = torch.device("cuda", 0)
    arrivals = configs.serving_arrivals(int(rate * duration * 2) + 50, rate=rate)
    arrivals = arrivals[arrivals < duration]
    n = len(arrivals)
    wls = [configs.serving_request(i) for i in range(n)]
    geoms = [(wl.geom.as_dict(), wl.grid.as_dict()) for wl in wls]
    shapes = [(g["n_views"], g["det_rows"], g["det_cols"]) for g, _ in geoms]
    pool = torch.rand(max(int(np.prod(sh)) for sh in shapes), device=dev)
    sinos = [pool[:int(np.prod(sh))].view(sh) for sh in shapes]

    def reqs(idx, saturated):
        return [serve.Request(rid=i, arrival=0.0 if saturated else float(arrivals[i]),
                              geom=geoms[i][0], grid=geoms[i][1], sino=sinos[i]) for i in idx]

    # warm-up on other geometries (kernel loading), untimed, then cold caches per run
    warm = [configs.serving_request(100000 + i) for i in range(4)]
    wc = serve.PlanCache(dev, workers=2)
    ws = serve.Server(wc, budget_bytes=budget)
    ws.run([serve.Request(rid=i, arrival=0.0, geom=w.geom.as_dict(), grid=w.grid.as_dict(),
                          sino=pool[:w.geom.n_views * 64 * w.geom.det_cols].view(
                              w.geom.n_views, 64, w.geom.det_cols)) for i, w in enumerate(warm)])
    serve.summarize(serve.serve_sequential(wc, [serve.Request(
        rid=0, arrival=0.0, geom=warm[0].geom.as_dict(), grid=warm[0].grid.as_dict(),
        sino=pool[:warm[0].geom.n_views * 64 * warm[0].geom.det_cols].view(
            warm[0].geom.n_views, 64, warm[0].geom.det_cols))]))
    torch.cuda.synchronize()
    ws.close()
    wc.close()
    del ws, wc
    print(f"[bench] serving: {n} requests over {duration:.0f} s, {len({serve.plan_key(g, gr) for g, gr in geoms})} "
          f"distinct geometries", file=sys.stderr, flush=True)
    out = {"workload": f"serving: Poisson {rate:g} req/s for {duration:g} s ({n} requests), "
                       f"cold plan caches, plans built on the GPU inside latency; saturated: "
                       f"the first {min(n, n_saturated)} requests at t = 0",
           "hbm_budget_bytes": budget, "group_work_updates": serve.GROUP_WORK}
    for name, idx, sat in (("poisson", range(n), False),
                           ("saturated", range(min(n, n_saturated)), True)):
        cache = serve.PlanCache(dev, workers=2)
        srv = serve.Server(cache, budget_bytes=budget)
        served_r = srv.run(reqs(idx, sat))
        torch.cuda.synchronize()
        served = serve.summarize(served_r)
        served["plans_evicted"] = cache.evicted
        srv.close()
        cache.close()
        del srv, cache
        torch.cuda.empty_cache()
        cache = serve.PlanCache(dev, workers=2)
        seq = serve.summarize(serve.serve_sequential(cache, reqs(idx, sat)))
        cache.close()
        del cache
        torch.cuda.empty_cache()
        out[f"served_{name}"] = served
        out[f"sequential_{name}"] = seq
        print(f"[bench] serving {name}: served {served['volumes_per_s']:.1f} vol/s p50 "
              f"{served['p50_latency_ms']:.1f} p99 {served['p99_latency_ms']:.1f} ms | sequential "
              f"{seq['volumes_per_s']:.1f} vol/s p50 {seq['p50_latency_ms']:.1f} p99 "
              f"{seq['p99_latency_ms']:.1f} ms | hit rate {served['cache_hit_rate']:.3f}, plan "
              f"build {served['plan_build_ms_mean']:.1f} ms mean", file=sys.stderr, flush=True)
    del pool, sinos
    return out


def data_path_bench(sino, vol, ref_vol, reps=5):
    """Sec. III-C data path on the whole clinical sinogram (every 4th column kept, linear
    upsampling, Philox noise) and the Sec. IV metrics on the volume: per-call time with HIP
    events on the launch stream and the algorithmic HBM bytes of each call."""
    import torch

    import paper_2201_02309_amd as K
    step, cols = 4, sino.shape[-1]
    sp = sino[..., ::step].contiguous()                  # the sparse-detector acquisition
    up = torch.empty_like(sino)
    noisy = torch.empty_like(sino)
    d_max = torch.empty(1, dtype=torch.float32, device=sino.device)
    scratch = torch.empty(1 << 20, dtype=torch.uint8, device=sino.device)
    res = torch.empty(2, dtype=torch.float64, device=sino.device)
    n = sino.numel()
    calls = {
        "sparse_upsample": (lambda: K.sparse_upsample(sp, cols, step, out=up), 4 * (sp.numel() + n)),
        "max": (lambda: K.max_value(up, scratch=scratch, out=d_max), 4 * n),
        "add_noise": (lambda: K.add_noise(up, 1e5, 0.5, 7, d_max=d_max, out=noisy), 8 * n),
        "rmse_ssim": (lambda: K.rmse_ssim(vol, ref_vol, scratch=scratch, result=res),
                      2 * 2 * 4 * vol.numel()),
    }
    out = {"workload": f"clinical sinogram {tuple(sino.shape)} float32, sparse step {step}; "
                       f"metrics on the {tuple(vol.shape)} volume",
           "hbm_peak_GBps": 8000.0}
    for name, (fn, nbytes) in calls.items():
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[name] = {"ms": round(ms, 4), "algorithmic_GB": round(nbytes / 1e9, 4),
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(nbytes / (ms * 1e-3) / 8e12, 4)}
    del sp, up, noisy, scratch
    return out


def network_bench(steps=5, warmup=2):
    """One training step (batch 1, forward + backward + Adam, Sec. III-B) of the dual-domain
    network on one pitch of the paper's p = 7 pi workload: window sinogram of the 627 x 16
    detector -> 512 x 512 x 10 slices.  The sample is the sparse (every 4th column) and noisy
    input of Sec. III-C; labels are the noise-free window sinogram and the phantom."""
    import numpy as np
    import torch

    import paper_2201_02309_amd as K
    from paper_2201_02309_amd import network as N
    from synth import configs, gpu_projector, phantom

    dev = torch.device("cuda", 0)
    wl = configs.network_pitch()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    gw, _ = N.pitch_window_geometry(geom, gr)
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    g_gt = gpu_projector.project(ph, gw, device=dev)
    g_in = K.add_noise(K.sparse_upsample(g_gt[..., ::4].contiguous(), gw["det_cols"], 4), 1e5, 0.5, 11)
    z = gr["z_first"] + np.arange(gr["nz"]) * gr["dz"]
    y = gr["y_first"] + np.arange(gr["ny"]) * gr["dy"]
    x = gr["x_first"] + np.arange(gr["nx"]) * gr["dx"]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    f_gt = torch.from_numpy(phantom.density(ph, np.stack([X, Y, Z], -1)).astype(np.float32)).to(dev)
    plan = K.Plan(gw, gr, device=0)
    torch.manual_seed(0)
    net = N.DualDomainNet(plan).to(dev)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    g_in, g_gt, f_gt = g_in[None], g_gt[None], f_gt[None]

    # MIOpen compiles every convolution configuration on its first use (seconds to tens of
    # seconds each): warm the distinct ones up one by one, reporting each
    for name, sub, shape in (("sinogram", net.sino_net, tuple(g_in.shape[1:])),
                             ("image", net.image_net, tuple(f_gt.shape[1:]))):
        for label, conv, cin in (("first", sub.convs[0], 1), ("middle", sub.convs[1], 16),
                                 ("last", sub.out, 16)):
            x = torch.randn((1, cin) + shape, device=dev, requires_grad=True)
            conv(x).sum().backward()
            torch.cuda.synchronize()
            print(f"[bench] network: {name} subnetwork, {label} convolution compiled",
                  file=sys.stderr, flush=True)
    opt.zero_grad(set_to_none=True)

    def step():
        opt.zero_grad(set_to_none=True)
        gs, f = net(g_in)
        L = N.loss(gs, f, g_gt, f_gt)
        L.backward()
        opt.step()
        return L.detach()

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] network warm-up step {i + 1}/{warmup}", file=sys.stderr, flush=True)
    losses = []
    t0 = time.perf_counter()
    for _ in range(steps):
        losses.append(step())
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / steps
    # the Katsevich layer alone on the same plan: forward and adjoint
    gsino = g_in[0].contiguous()
    vol = K.recon(plan, gsino)
    gvol = torch.randn_like(vol)
    K.recon_backward(plan, gvol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        K.recon(plan, gsino, out=vol)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 200
    t0 = time.perf_counter()
    for _ in range(5):
        K.recon_backward(plan, gvol)
    torch.cuda.synchronize()
    bwd_ms = (time.perf_counter() - t0) * 200
    out = {"workload": f"one pitch of the p = 7 pi network workload: window sinogram "
                       f"{tuple(g_in.shape[1:])}, slices {tuple(f_gt.shape[1:])}, batch 1, "
                       f"16-channel 7-block subnetworks, Adam lr 1e-3",
           "step_s": round(step_s, 4), "layer_forward_ms": round(fwd_ms, 3),
           "layer_adjoint_ms": round(bwd_ms, 3),
           "loss_first_last": [round(float(losses[0]), 3), round(float(losses[-1]), 3)],
           "paper_step_s_other_hardware": "5-6 (RTX A6000, TensorFlow 2.5)"}
    plan.close()
    return out


def _measured_traffic():
    """HBM bytes per backprojection launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (scaled by a plain-copy calibration), or None when the kernel or
    plan sources changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "bp_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    h = hashlib.sha256()
    for src in tr.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return tr.get("bytes_per_launch") if h.hexdigest() == tr.get("source_sha256") else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-network", action="store_true",
                    help="skip the training step of the dual-domain network (MIOpen compiles "
                         "its convolutions on first use: about two minutes on a fresh machine)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving trace in seconds at 20 requests/s (0 skips it)")
    ap.add_argument("--bp-slices", type=int, default=0,
                    help="slices per backprojection register run (0: library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the reconstructor runs on one GPU; --gpus must be 1 "
                                   "(sharding by pitch ranges across GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2201_02309_amd as K
    from synth import configs, gpu_projector, phantom

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = configs.config2()
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    t0 = time.perf_counter()
    plan = K.Plan(geom, gr, device=0, bp_slices=args.bp_slices)
    t_plan = time.perf_counter() - t0
    # the same plan built on the GPU (katsevich_plan_device); warmed once
    K.Plan(geom, gr, gpu_plan=True, device=0, bp_slices=args.bp_slices).close()
    t0 = time.perf_counter()
    K.Plan(geom, gr, gpu_plan=True, device=0, bp_slices=args.bp_slices).close()
    t_plan_gpu = time.perf_counter() - t0
    info = plan.info
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    sino = gpu_projector.project(ph, geom, device=dev)          # whole scan, resident in HBM
    n_filt = plan.n_filtered
    gF = torch.empty(K.katsevich.filtered_shape(plan), dtype=torch.float32, device=dev)
    vol = torch.empty((gr["nz"], gr["ny"], gr["nx"]), dtype=torch.float32, device=dev)
    ws = plan.workspace()
    print(f"[bench] plan {t_plan:.2f} s, tables {info['table_bytes'] / 2**20:.0f} MiB, "
          f"workspace {info['workspace_bytes'] / 2**20:.0f} MiB, N_vv {info['n_vv']:.4e}, "
          f"filtered views {n_filt}", file=sys.stderr, flush=True)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        K.filter_views(plan, sino, out=gF, ws=ws)
        if ev is not None:
            ev[1].record()
        K.backproject(plan, gF, out=vol)
        if ev is not None:
            ev[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    filt_ms = [e[0].elapsed_time(e[1]) for e in events]
    bp_ms = [e[1].elapsed_time(e[2]) for e in events]
    ms_step = wall * 1e3 / args.steps
    n_vv = int(info["n_vv"])
    value = n_vv / (ms_step * 1e-3) / 1e9

    # plain katsevich_recon (the single-call entry point) for comparison
    for _ in range(2):
        K.recon(plan, sino, out=vol, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(max(3, args.steps // 2)):
        K.recon(plan, sino, out=vol, ws=ws)
    torch.cuda.synchronize()
    recon_ms = (time.perf_counter() - t1) * 1e3 / max(3, args.steps // 2)

    # the half-sample derivative option (KATS_FLAG_HALF_SAMPLE_DERIVATIVE), same workload
    plan_h = K.Plan(geom, gr, device=0, bp_slices=args.bp_slices, half_sample=True)
    ws_h = plan_h.workspace()
    for _ in range(2):
        K.recon(plan_h, sino, out=vol, ws=ws_h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        K.recon(plan_h, sino, out=vol, ws=ws_h)
    torch.cuda.synchronize()
    half_ms = (time.perf_counter() - t1) * 1e3 / 5
    plan_h.close()
    del plan_h, ws_h

    # the adjoint (katsevich_recon_backward: sinogram cotangent of a volume cotangent)
    gvol = torch.randn_like(vol)
    gsino = torch.empty_like(sino)
    K.recon_backward(plan, gvol, out=gsino, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        K.recon_backward(plan, gvol, out=gsino, ws=ws)
    torch.cuda.synchronize()
    adjoint_ms = (time.perf_counter() - t1) * 1e3 / 3
    del gvol, gsino

    bp_avg = float(np.mean(bp_ms))
    achieved = n_vv * BP_FLOP_PER_UPDATE / (bp_avg * 1e-3) / 1e12
    traffic = _measured_traffic()
    out = {
        "metric": "Gvoxel-view/s (512^2x128 clinical high-pitch Katsevich recon)",
        "value": round(value, 3),
        "unit": "Gvoxel-view/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ellipsoid phantom, closed-form FP64 line integrals)",
        "config": {"workload": wl.name, "grid": [gr["nx"], gr["ny"], gr["nz"]],
                   "voxel_mm": [gr["dx"], gr["dy"], round(gr["dz"], 6)],
                   "detector": [geom["det_cols"], geom["det_rows"]],
                   "views": geom["n_views"], "views_per_turn": geom["views_per_turn"],
                   "feed_mm_per_turn": geom["feed_per_turn"], "n_psi": info["n_psi"],
                   "pitches": info["n_pitches"], "slices_per_pitch": info["slices_per_pitch"],
                   "n_vv": n_vv, "filtered_views": n_filt,
                   "bp_slices": args.bp_slices or 16},
        "volumes_per_s": round(1e3 / ms_step, 3),
        "stage_ms": {"filter": round(float(np.mean(filt_ms)), 4), "backproject": round(bp_avg, 4)},
        "backproject_gvoxel_view_per_s": round(n_vv / (bp_avg * 1e-3) / 1e9, 3),
        "recon_call_ms": round(recon_ms, 4),
        "adjoint_call_ms": round(adjoint_ms, 3),
        "half_sample_recon_call_ms": round(half_ms, 4),
        "plan_build_s": round(t_plan, 3),
        "plan_build_gpu_s": round(t_plan_gpu, 4),
        "roofline": {"kernel": "k_bp_lds", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": traffic,
                     "flop_per_update": BP_FLOP_PER_UPDATE},
    }
    K.recon(plan, sino, out=vol, ws=ws)
    ref_vol = vol.clone()
    K.recon(plan, K.add_noise(sino, 1e5, 0.5, 3), out=vol, ws=ws)
    out["data_path"] = data_path_bench(sino, vol, ref_vol)
    del ref_vol
    if not args.no_network:
        print("[bench] dual-domain network training step", file=sys.stderr, flush=True)
        out["network"] = network_bench()
    if args.serve_seconds > 0:
        gF = ws = None
        plan.release_workspace()
        torch.cuda.empty_cache()
        out["serving"] = serving_bench(duration=args.serve_seconds)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a 16-slice slab on every host core "
              "(cpu_baseline)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, sino)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
