"""Benchmark: curvature-regularized NLOS reconstruction on one MI355X.

A step is one complete reconstruction of a 64x64x512 scene with the
dual-domain model (Algorithm 2): problem set-up (kernel spectrum H^, step
constants by power iteration), loading the measurement, 50 warm-start
iterations of Algorithm 1 and 200 iterations of Algorithm 2 with
backtracking, and reading the volume back.  The metric is voxel-ADMM-
iterations per second (64*64*512 voxels x 250 iterations per step, divided by
the step time), with reconstructions/s and the p50/p99 step latency.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# MI355X's published FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop
# (FMA) x 2 (packed or dual-issued FP32) x 2.4 GHz
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
# the same without the packed/dual-issue factor: the ceiling of this library,
# which is built with packed FP32 disabled
VALU_NONPACKED_TFLOPS = VALU_PEAK_TFLOPS / 2
# kernels whose bound is the vector ALU (rocprofv3 SQ counters), reported
# against VALU_PEAK_TFLOPS with their algorithmic flops
ALU_BOUND = ("plane_conv",)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium",
                    choices=["small", "medium", "large", "batch", "serve", "ablation", "nonconfocal"])
    ap.add_argument("--requests", type=int, default=96, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=50.0, help="serve: Poisson arrival rate (1/s)")
    ap.add_argument("--no-serve-baseline", action="store_true",
                    help="serve: the stream through the engine only (no one-at-a-time runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--profile-all", action="store_true",
                    help="print per-kernel event times of one extra reconstruction to stderr")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the rates of the other single-scene workloads")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-one-at-a-time comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (PMC byte-counter calibration)")
    return ap.parse_args()


WORKLOADS = {
    # name: (scene factory, model, warm-start iters, iters, parameters)
    "small": dict(scene="scene_small", model="object", init=0, iters=50,
                  params=dict(a_u=5e-5, b_u=5e-5, mu=0.1)),
    "medium": dict(scene="scene_medium", model="dual", init=50, iters=200,
                   params=dict(a_u=5e-4, b_u=5e-5, a_tau=3e-3, b_tau=5e-4, warm_a=1.5e-4,
                               warm_b=4e-5, mu=0.1, lam=200.0)),
    "large": dict(scene="scene_large", model="dual", init=50, iters=300,
                  params=dict(a_u=5e-4, b_u=3e-4, a_tau=5e-3, b_tau=1e-3, warm_a=1e-4,
                              warm_b=4e-5, mu=0.1, lam=150.0)),
}


# Uneven multi-scene mixes for the batched form: scan grids, time bins, mask
# densities 10-50% and both models; every time axis spans the same 2.46 m.
MIX_FULL = dict(grids=(32, 64, 128), bins=(256, 512, 1024), count=64, seed0=4000)
MIX_SMALL = dict(grids=(32, 64), bins=(256, 512), count=16, seed0=4500)
MIX_ITERS = dict(object=(0, 50), dual=(20, 60))      # (warm start, iterations)


def make_mix(mix):
    from paper_2301_00406_amd import scenes
    rng = np.random.Generator(np.random.PCG64(mix["seed0"]))
    out = []
    for i in range(mix["count"]):
        n = int(rng.choice(mix["grids"]))
        m = int(rng.choice(mix["bins"]))
        model = "dual" if i % 2 else "object"
        dens = float(rng.uniform(0.1, 0.5))
        peak = float(rng.integers(1, 51))
        sc = scenes.scene_custom(n, m, mix["seed0"] + i, wall=1.0, bin_ps=16.0 * 1024 / m,
                                 density=dens, n_planes=2, n_shells=1, peak=peak,
                                 background=0.01 * peak)
        out.append((sc, model))
    return out


def mix_config(C, sc, model):
    init, iters = MIX_ITERS[model]
    pr = WORKLOADS["medium"]["params"] if model == "dual" else WORKLOADS["small"]["params"]
    return C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                            bin_ps=sc.bin_ps, model=C.MODEL_DUAL if model == "dual" else C.MODEL_OBJECT,
                            max_iters=iters, init_iters=init, **pr)


def batched_comparison(torch, C, scenes, mix):
    """Reconstructions/s of an uneven scene mix, one scene at a time against
    the batched form (scenes grouped by shape and model, one launch per kernel
    per group, groups set up from their own host threads and overlapping on
    their own streams).  Both include create (H^, step constants),
    set_measurement, the run and the read-back."""
    dev = torch.device("cuda", 0)
    items = make_mix(mix)
    # measurements: literal-falloff forward model of the library + seeded Poisson noise
    raws, op = [], {}
    for sc, _ in items:
        key = (sc.n, sc.m)
        if key not in op:
            oc = C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                                  bin_ps=sc.bin_ps, model=C.MODEL_OPERATOR, falloff=C.FALLOFF_LITERAL)
            op[key] = C.Problem(oc, np.ones((sc.n, sc.n), np.uint8), device=dev)
        clean = op[key].apply_A(torch.tensor(sc.u_true.astype(np.float32), device=dev))
        r = scenes.poisson_counts(clean.double().cpu().numpy(), sc.peak, sc.background,
                                  np.random.Generator(np.random.PCG64(sc.seed)))
        raws.append(torch.tensor(r.astype(np.float32), device=dev))
    for P in op.values():
        P.close()
    cfgs = [mix_config(C, sc, model) for sc, model in items]
    voxel_iters = sum(sc.n * sc.n * sc.m * (c.init_iters * (c.model == C.MODEL_DUAL) + c.max_iters)
                      for (sc, _), c in zip(items, cfgs))

    def alone():
        vols = []
        for (sc, _), c, raw in zip(items, cfgs, raws):
            P = C.Problem(c, sc.mask, device=dev)
            P.set_measurement(raw)
            P.run()
            vols.append(P.volume())
            P.close()
        torch.cuda.synchronize()
        return vols

    def batched():
        groups = {}
        for i, ((sc, model), c) in enumerate(zip(items, cfgs)):
            groups.setdefault((sc.n, sc.m, model), []).append(i)

        # every group is set up from its own host thread on its own stream, so
        # the groups' set-up launches overlap on the device
        def make(idx):
            st = torch.cuda.Stream(device=dev)
            B = C.Batch([cfgs[i] for i in idx], [items[i][0].mask for i in idx], device=dev,
                        stream=st)
            with torch.cuda.stream(st):
                for mem, i in zip(B.members, idx):
                    mem.set_measurement(raws[i])
            return B, idx, st

        with ThreadPoolExecutor(max_workers=len(groups)) as ex:
            bs = list(ex.map(make, list(groups.values())))
        status, _ = C.run_many([b for b, _, _ in bs])
        if status != C.OK:
            raise RuntimeError(C.last_error())
        vols = [None] * len(items)
        for B, idx, st in bs:
            with torch.cuda.stream(st):
                for mem, i in zip(B.members, idx):
                    vols[i] = mem.volume()
            st.synchronize()
        for B, _, _ in bs:
            B.close()
        torch.cuda.synchronize()
        return vols

    alone()                                   # warm-up of both forms
    batched()
    t0 = time.perf_counter()
    va = alone()
    t_alone = time.perf_counter() - t0
    t0 = time.perf_counter()
    vb = batched()
    t_batch = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(va, vb))
    shapes = sorted({(sc.n, sc.m, mdl) for sc, mdl in items})
    return {
        "scenes": len(items),
        "mix": f"scan grids {sorted({sc.n for sc, _ in items})}, time bins "
               f"{sorted({sc.m for sc, _ in items})}, masks 10-50%, both models; object "
               f"{MIX_ITERS['object'][1]} iterations, dual {MIX_ITERS['dual'][0]} warm-start + "
               f"{MIX_ITERS['dual'][1]}",
        "groups": len(shapes),
        "one_at_a_time_rec_per_s": len(items) / t_alone,
        "batched_rec_per_s": len(items) / t_batch,
        "speedup": t_alone / t_batch,
        "batched_voxel_iters_per_s": voxel_iters / t_batch,
        "results_bitwise_equal": bool(same),
    }


def batched_metric(torch, C, scenes, count=8):
    """Batched against one scene at a time at the metric configuration itself:
    `count` seeded scenes of the 64x64x512 dual workload (50 + 200
    iterations), every step create + set_measurement + run + read volume."""
    dev = torch.device("cuda", 0)
    wl = WORKLOADS["medium"]
    scs = [scenes.scene_medium(201 + i) for i in range(count)]
    sc0 = scs[0]
    oc = C.default_config(nx=sc0.n, ny=sc0.n, nt=sc0.m, wall_w_m=sc0.wall_w, wall_h_m=sc0.wall_h,
                          bin_ps=sc0.bin_ps, model=C.MODEL_OPERATOR, falloff=C.FALLOFF_LITERAL)
    op = C.Problem(oc, np.ones((sc0.n, sc0.n), np.uint8), device=dev)
    raws = []
    for sc in scs:
        clean = op.apply_A(torch.tensor(sc.u_true.astype(np.float32), device=dev))
        r = scenes.poisson_counts(clean.double().cpu().numpy(), sc.peak, sc.background,
                                  np.random.Generator(np.random.PCG64(sc.seed)))
        raws.append(torch.tensor(r.astype(np.float32), device=dev))
    op.close()
    cfgs = [C.default_config(nx=sc.n, ny=sc.n, nt=sc.m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                             bin_ps=sc.bin_ps, model=C.MODEL_DUAL, max_iters=wl["iters"],
                             init_iters=wl["init"], **wl["params"]) for sc in scs]

    def alone():
        vols = []
        for sc, c, raw in zip(scs, cfgs, raws):
            P = C.Problem(c, sc.mask, device=dev)
            P.set_measurement(raw)
            P.run()
            vols.append(P.volume())
            P.close()
        torch.cuda.synchronize()
        return vols

    def batched():
        B = C.Batch(cfgs, [sc.mask for sc in scs], device=dev)
        for mem, raw in zip(B.members, raws):
            mem.set_measurement(raw)
        status, _ = B.run()
        if status != C.OK:
            raise RuntimeError(C.last_error())
        vols = [mem.volume() for mem in B.members]
        torch.cuda.synchronize()
        B.close()
        return vols

    alone()                                   # warm-up of both forms
    batched()
    t0 = time.perf_counter()
    va = alone()
    t_alone = time.perf_counter() - t0
    t0 = time.perf_counter()
    vb = batched()
    t_batch = time.perf_counter() - t0
    vi = count * sc0.n * sc0.n * sc0.m * (wl["init"] + wl["iters"])
    return {"scenes": count, "workload": "64x64x512 dual-domain (Algorithm 2), 50 + 200 iterations, "
                                          "seeded scenes 201..",
            "one_at_a_time_rec_per_s": count / t_alone, "batched_rec_per_s": count / t_batch,
            "speedup": t_alone / t_batch, "batched_voxel_iters_per_s": vi / t_batch,
            "results_bitwise_equal": bool(all(torch.equal(a, b) for a, b in zip(va, vb)))}


def _ssim(x, y, sigma=1.5, data_range=1.0):
    """Mean structural similarity of two images (Wang, Bovik, Sheikh and
    Simoncelli 2004): Gaussian window of width sigma (radius 3.5 sigma),
    constants K1 = 0.01, K2 = 0.03."""
    from scipy.ndimage import gaussian_filter
    f = lambda a: gaussian_filter(a, sigma, truncate=3.5, mode="reflect")
    c1, c2 = (0.01 * data_range) ** 2, (0.03 * data_range) ** 2
    mx, my = f(x), f(y)
    vx, vy, cxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    s = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return float(s.mean())


def image_quality(u, u_true):
    """Reconstruction quality against the ground truth on the front view (the
    maximum-intensity projection along depth, each normalized to a peak of 1):
    accuracy (1 - mean absolute error), RMSE, PSNR and SSIM, and the relative L2
    error of the volume after the best scalar scaling (the reconstruction is
    in normalized units)."""
    img = u.max(axis=2)
    ref = u_true.max(axis=2)
    img = img / img.max() if img.max() > 0 else img
    ref = ref / ref.max()
    err = img - ref
    rmse = float(np.sqrt(np.mean(err ** 2)))
    uu = float(np.sum(u * u))
    a = float(np.sum(u * u_true)) / uu if uu > 0 else 0.0
    vol = float(np.linalg.norm(a * u - u_true) / np.linalg.norm(u_true))
    return {"accuracy": 1.0 - float(np.mean(np.abs(err))), "rmse": rmse,
            "psnr_db": 20.0 * float(np.log10(1.0 / max(rmse, 1e-12))),
            "ssim": _ssim(img, ref), "volume_rel_err": vol}


def _trv_weights(pr):
    """TRV's phi = sqrt(a + b k^2) meets a at k = 0 and b|k| for large |k| when
    its weights are the squares of the TAC/TSC ones."""
    return {k: (v * v if k in ("a_u", "b_u", "a_tau", "b_tau", "warm_a", "warm_b") else v)
            for k, v in pr.items()}


def ablation(torch, C, scenes, n_scenes=4, seed=7000):
    """Curvature functions phi (TRV, TAC, TSC) and plain TV (b = 0) for both
    algorithms on synthetic scenes of the 64x64x512 geometry with known ground
    truth: two scene kinds (three solid planar patches; the benchmark's five
    point-sampled ellipsoid shells and a letter patch), each under two scan
    masks (a regular 6x6 grid of scan points, the sparse setting of the
    paper's curvature comparison, and 25% random points).  Every variant gets
    the same weights (squared for TRV).  Stands in for the paper's comparison
    on measured data, which is not available here."""
    dev = torch.device("cuda", 0)
    base = scenes.scene_medium()
    n, m = base.n, base.m
    pw = WORKLOADS["medium"]["params"]
    variants = [("TRV", C.PHI_TRV, False), ("TAC", C.PHI_TAC, False), ("TSC", C.PHI_TSC, False),
                ("TV", C.PHI_TSC, True)]
    models = [("Algorithm 1", C.MODEL_OBJECT, dict(a_u=pw["warm_a"], b_u=pw["warm_b"], mu=pw["mu"]),
               0, 250),
              ("Algorithm 2", C.MODEL_DUAL, pw, 50, 200)]
    kinds = [("planes", lambda s: scenes.scene_custom(n, m, s, wall=base.wall_w, bin_ps=base.bin_ps,
                                                       density=0.25, n_planes=3, n_shells=0,
                                                       peak=base.peak, background=base.background)),
             ("shells", scenes.scene_medium)]
    rows = {}
    t0 = time.perf_counter()
    for i, (kind, make) in ((i, k) for k in kinds for i in range(n_scenes)):
        sc = make(seed + i)
        opP = C.Problem(C.default_config(nx=n, ny=n, nt=m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                                         bin_ps=sc.bin_ps, model=C.MODEL_OPERATOR,
                                         falloff=C.FALLOFF_LITERAL),
                        np.ones((n, n), np.uint8), device=dev)
        clean = opP.apply_A(torch.tensor(sc.u_true.astype(np.float32), device=dev))
        opP.close()
        raw = scenes.poisson_counts(clean.double().cpu().numpy(), sc.peak, sc.background,
                                    np.random.Generator(np.random.PCG64(sc.seed)))
        raw = torch.tensor(raw.astype(np.float32), device=dev)
        grid = scenes.strided_dropout_mask(n, 11, 1.0, np.random.Generator(np.random.PCG64(0)))
        for mask_name, mask in (("6x6 grid", grid), ("25% random", sc.mask)):
            for mname, model, params, init, iters in models:
                for vname, phi, tv in variants:
                    pr = _trv_weights(params) if phi == C.PHI_TRV else dict(params)
                    if tv:
                        pr.update({k: 0.0 for k in ("b_u", "b_tau", "warm_b") if k in pr})
                    cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=sc.wall_w,
                                           wall_h_m=sc.wall_h, bin_ps=sc.bin_ps, phi=phi,
                                           model=model, max_iters=iters, init_iters=init, **pr)
                    P = C.Problem(cfg, mask, device=dev)
                    P.set_measurement(raw)
                    P.run()
                    u = P.volume().double().cpu().numpy()
                    P.close()
                    rows.setdefault((kind, mask_name, mname, vname), []).append(
                        image_quality(u, sc.u_true))
    table = []
    for (kind, mask_name, mname, vname), vals in rows.items():
        r = {"scene": kind, "mask": mask_name, "method": mname, "phi": vname}
        for k in vals[0]:
            r[k] = float(np.mean([v[k] for v in vals]))
        table.append(r)
    return {"scenes": n_scenes,
            "scene": f"{n}x{n}x{m}, {base.wall_w} m wall, {base.bin_ps:g} ps bins, "
                     f"{base.peak:g} photons at the peak, background {base.background / base.peak:.0%}",
            "iterations": {"Algorithm 1": 250, "Algorithm 2": "50 warm-start + 200"},
            "seconds": time.perf_counter() - t0, "table": table}


def serve_workload(torch, C, scenes, n_req, rate, seed=5000, baseline=True):
    """Poisson arrivals of requests drawn from the uneven size mix, each with
    its own mask, photon level U{1..50} and iteration budget U{100..300},
    served by the library's continuous-batching engine; latency is arrival to
    completion on the host clock.  With baseline: the same stream one request
    at a time through the plain solver, both forms' capacity (all requests
    present at the start), and both at 80 % of the engine's capacity.

    A request's measurement is drawn on the device when it arrives (up to 256
    requests: before the run) and dropped with its output when it completes;
    arrived requests wait on the host until the engine's own queue is short,
    so a long stream needs device memory only for what is in flight."""
    dev = torch.device("cuda", 0)
    rng = np.random.Generator(np.random.PCG64(seed))
    # a few base scenes per shape; requests vary mask, noise and budget
    base = {}
    reqs = []
    for i in range(n_req):
        n = int(rng.choice(MIX_FULL["grids"]))
        m = int(rng.choice(MIX_FULL["bins"]))
        model = "dual" if rng.random() < 0.5 else "object"
        key = (n, m)
        if key not in base:
            sc = scenes.scene_custom(n, m, seed + len(base), wall=1.0, bin_ps=16.0 * 1024 / m,
                                     density=0.5, n_planes=2, n_shells=1)
            oc = C.default_config(nx=n, ny=n, nt=m, wall_w_m=1.0, wall_h_m=1.0, bin_ps=sc.bin_ps,
                                  model=C.MODEL_OPERATOR, falloff=C.FALLOFF_LITERAL)
            P = C.Problem(oc, np.ones((n, n), np.uint8), device=dev)
            clean = P.apply_A(torch.tensor(sc.u_true.astype(np.float32), device=dev))
            P.close()
            # FP32 round-off of the literal r^-3 weight leaves negative values in
            # empty near-wall bins; like scenes.poisson_counts, rates are clipped at 0
            clean = torch.clamp(clean, min=0.0)
            base[key] = (sc, clean / clean.max())
        sc, _ = base[key]
        mask = scenes.density_mask(n, float(rng.uniform(0.1, 0.5)), rng)
        photons = float(rng.integers(1, 51))
        budget = int(rng.integers(100, 301))
        cfg = mix_config(C, sc, model)
        if model == "dual":
            cfg.init_iters = min(50, budget // 3)
            cfg.max_iters = budget - cfg.init_iters
        else:
            cfg.max_iters = budget
        reqs.append((cfg, mask, key, photons, n * n * m * budget))
    gaps = rng.exponential(1.0, size=n_req)       # unit-rate gaps, scaled per run
    vox = sum(r[4] for r in reqs)
    pre = n_req <= 256

    def measurement(i):
        _, _, key, photons, _ = reqs[i]
        g = torch.Generator(device=dev)
        g.manual_seed(int(seed * 7 + i))
        lam = base[key][1] * photons + 0.01 * photons
        return torch.poisson(lam, generator=g)

    raws = [measurement(i) for i in range(n_req)] if pre else None

    def arrivals(r):
        a = np.cumsum(gaps / r) if r > 0 else np.zeros(n_req)
        return a - a[0]

    def served(arrive, tag):
        """The stream through the continuous-batching engine."""
        S = C.Server(200 << 30, slots=8, rounds=4, device=dev)
        live = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, done, lat, queued = 0, 0, [], 0
        last = t0
        while done < n_req:
            now = time.perf_counter() - t0
            while nxt < n_req and arrive[nxt] <= now and queued < 32:
                cfg, mask, _, _, _ = reqs[nxt]
                raw = raws[nxt] if pre else measurement(nxt)
                out = torch.empty(tuple(raw.shape), dtype=torch.float32, device=dev)
                live[nxt] = (raw, out)
                S.submit(cfg, mask, raw, out, nxt)
                queued += 1
                nxt += 1
            active, queued = S.step()
            t = time.perf_counter() - t0
            for c in S.poll():
                if c["status"] != C.OK:
                    raise RuntimeError(f"request {c['id']} failed: {c['status']}")
                lat.append(1e3 * (t - arrive[c["id"]]))
                live.pop(c["id"], None)
                done += 1
            if time.perf_counter() - last > 20.0 or done == n_req:
                last = time.perf_counter()
                print(f"serve ({tag}): {done}/{n_req} done at {t:.1f} s", file=sys.stderr,
                      flush=True)
            if active == 0 and queued == 0 and nxt < n_req:
                time.sleep(max(0.0, arrive[nxt] - (time.perf_counter() - t0)))
        makespan = time.perf_counter() - t0
        S.close()
        return makespan, lat

    def one_at_a_time(arrive, tag):
        """The same stream through the plain solver, first come first served:
        each request runs alone (create + set_measurement + run + read) once it
        has arrived and the one before it has finished."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = []
        last = t0
        for i, (cfg, mask, _, _, _) in enumerate(reqs):
            wait = arrive[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            raw = raws[i] if pre else measurement(i)
            P = C.Problem(cfg, mask, device=dev)
            P.set_measurement(raw)
            P.run()
            out = P.volume()
            P.close()
            del out, raw
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - t0 - arrive[i]))
            if time.perf_counter() - last > 20.0 or i + 1 == n_req:
                last = time.perf_counter()
                print(f"one at a time ({tag}): {i + 1}/{n_req} done", file=sys.stderr, flush=True)
        return time.perf_counter() - t0, lat

    def stats(makespan, lat, r):
        return {"arrival_rate_per_s": r, "makespan_s": makespan,
                "reconstructions_per_s": n_req / makespan, "voxel_iters_per_s": vox / makespan,
                "latency_ms": {"p50": float(np.percentile(lat, 50)),
                               "p99": float(np.percentile(lat, 99))}}

    out = {"requests": n_req, "rate_per_s": rate,
           "mix": "scan grids 32/64/128, time bins 256/512/1024, masks 10-50%, both models, "
                  "photons U{1..50}, iteration budget U{100..300}",
           "arena_bytes": 200 << 30, "slots_per_group": 8}
    out["served"] = stats(*served(arrivals(rate), f"{rate:g}/s"), rate)
    if baseline:
        out["one_at_a_time"] = stats(*one_at_a_time(arrivals(rate), f"{rate:g}/s"), rate)
        # capacity: every request present at the start, so service is never idle
        cap_s = stats(*served(arrivals(0.0), "saturated"), None)
        cap_1 = stats(*one_at_a_time(arrivals(0.0), "saturated"), None)
        out["capacity_rec_per_s"] = {"served": cap_s["reconstructions_per_s"],
                                     "one_at_a_time": cap_1["reconstructions_per_s"]}
        # latency where the engine keeps up: arrivals at 80 % of its capacity
        r = 0.8 * cap_s["reconstructions_per_s"]
        out["at_sustainable_rate"] = {"served": stats(*served(arrivals(r), f"{r:.1f}/s"), r),
                                      "one_at_a_time": stats(*one_at_a_time(arrivals(r),
                                                                            f"{r:.1f}/s"), r)}
    # headline figures of the served run at the requested rate
    out.update({k: out["served"][k] for k in ("makespan_s", "reconstructions_per_s",
                                               "voxel_iters_per_s", "latency_ms")})
    return out


def hq_bytes(n, m, layout=False):
    """Bytes of the kernel spectrum H^ per convolution: the quarter (n + 1)^2
    of each kt plane that its evenness in kx and ky determines (the method's
    own bytes), or the full 2n x 2n plane the plane kernel reads, lane-ordered
    so that its loads coalesce (the layout's bytes)."""
    return (m + 1) * (4 * n * n if layout else (n + 1) * (n + 1)) * 8


def algorithmic_bytes(kind, n, m, dual):
    """Bytes a kernel kind must move per launch (inputs read once, outputs
    written once), averaged over its launches in one ADMM iteration."""
    V = n * n * m
    spec_c = m * n * n * 8                # convolution spectrum, complex64: kt = 1 .. m - 1
                                          # and the real planes kt = 0, m packed in one
    spec_s = (m // 2 + 1) * n * n * 8     # solve spectrum
    f = 4 * V
    if kind == "plane_conv":
        return 2 * spec_c + hq_bytes(n, m)
    if kind == "t_fwd_conv":       # the adjoint's first pass reads 3 volumes (the forward
        return spec_c + 3 * f      # operator's runs inside the u solve's last pass)
    if kind == "t_inv_conv":       # adjoint: with the u solve's first pass (reads ubar,
        adj = spec_c + 5 * f + spec_s  # Lambda (3), phi; writes the solve planes)
        if dual:                   # forward: writes A u+, reads A u^k, A u^{k-1}, and the
            fwd = spec_c + 3 * f + 7 * f + n * n + spec_s  # tau solve's first pass (taubar,
        else:                      # Lambda3, tau0, Lambda2 (3), phi_tau; solve planes)
            fwd = spec_c + 4 * f   # object: A u+, A u^k, A u^{k-1}, tau0
        return (fwd + adj) / 2
    if kind == "t_fwd_solve":      # standalone (both solves' first passes run inside the
        return spec_s + 8 * f + n * n  # convolutions' last passes in the iteration loop)
    if kind == "plane_solve":
        return 2 * spec_s
    if kind == "t_inv_solve":      # u solve: reads ubar, writes u+ and A u+'s first planes;
        u = spec_s + 2 * f + spec_c  # tau solve (dual): writes tau+
        return (u + spec_s + f) / 2 if dual else u
    # the splitting variables v, w, f are recomputed where they are used
    if kind == "post":           # object: 7 volumes in, 5 out; dual adds the tau side (10 in, 6 out)
        return 28 * f + n * n if dual else 12 * f
    return 0.0


def algorithmic_flops(kind, n, m):
    """Flops a kernel kind must do per launch: for the plane pass of the
    convolution, the pruned padded 2n x 2n transforms of m planes (n row and
    2n column transforms forward, the same inverse, 5 L log2 L flops per
    length-L complex transform) plus the complex product with H^."""
    if kind != "plane_conv":
        return 0.0
    L = 2 * n
    t = 5.0 * L * np.log2(L)
    return m * (6 * n * t + 6.0 * L * L)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("k_spectral.hip", "k_admm.hip", "fft_device.h", "cnlos_internal.h",
                 "stencil_device.h"):
        with open(os.path.join(ROOT, "paper_2301_00406_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kind, workload):
    """HBM bytes per launch measured with rocprofv3 PMC counters, if the
    committed measurement matches the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    e = d.get("kernels", {}).get(kind)
    return None if e is None else float(e["bytes_per_launch"])


def cpu_baseline(sc, wl, cpu_iters, single_worker=True):
    """The FP64 oracle on a bounded sample of the same workload, with every
    host core and (single_worker) again with one FFT worker."""
    from oracle import cnlos_oracle as O
    from paper_2301_00406_amd import scenes
    opL = O.make_operator(sc.n, sc.n, sc.m, sc.wall_w, sc.wall_h, sc.bin_ps, O.FALLOFF_LITERAL)
    raw = scenes.poisson_counts(O.apply_A(sc.u_true, opL), sc.peak, sc.background,
                                np.random.Generator(np.random.PCG64(sc.seed)))
    op = O.make_operator(sc.n, sc.n, sc.m, sc.wall_w, sc.wall_h, sc.bin_ps, mask=sc.mask)
    tau0, _ = O.normalize_measurement(raw, sc.mask, O.FALLOFF_COMPENSATED)
    pr = wl["params"]
    p = O.Params(a=pr.get("warm_a", pr["a_u"]), b=pr.get("warm_b", pr["b_u"]), mu=pr["mu"],
                 a_u=pr["a_u"], b_u=pr["b_u"], a_tau=pr.get("a_tau", 0.0),
                 b_tau=pr.get("b_tau", 0.0), lam=pr.get("lam", 200.0))
    # step constants from short power estimates (untimed; they only set the
    # scale): masked for Algorithm 1, unmasked for Algorithm 2's u-step, as
    # the GPU path does
    L0o = 2 * O.power_norm2(lambda x: O.apply_A(x, op, True), lambda y: O.apply_AT(y, op, True),
                            tau0.shape, 2)
    L0d = 2 * O.power_norm2(lambda x: O.apply_A(x, op, False),
                            lambda y: O.apply_AT(y, op, False), tau0.shape, 2)
    fwdD = lambda x: O.apply_A(x, op, True)
    adjD = lambda y: O.apply_AT(y, op, True)
    if wl["model"] == "dual":
        # one warm-start iteration of Algorithm 1 (untimed), then the timed
        # Algorithm-2 iterations: the steps of the oracle's run_alg2
        fwd = lambda x: O.apply_A(x, op, False)
        adj = lambda y: O.apply_AT(y, op, False)
        s1 = O.alg1_init(tau0.shape, p, L0o)
        O.alg1_step(s1, tau0, fwdD, adjD, p)
        s2 = O.alg2_init(s1.u, p, L0d)
        t0 = time.perf_counter()
        for _ in range(cpu_iters):
            O.alg2_step(s2, tau0, op.mask, fwd, adj, p)
        what = f"{cpu_iters} Algorithm-2 iteration(s) after a 1-iteration warm start (untimed)"
    else:
        s1 = O.alg1_init(tau0.shape, p, L0o)
        t0 = time.perf_counter()
        for _ in range(cpu_iters):
            O.alg1_step(s1, tau0, fwdD, adjD, p)
        what = f"{cpu_iters} Algorithm-1 iteration(s)"
    dt = time.perf_counter() - t0
    V = sc.n * sc.n * sc.m
    out = {"value": V * cpu_iters / dt, "unit": "voxel-ADMM-iters/s", "cores": int(O.WORKERS),
           "kind": "oracle",
           "sample": f"{what} of the same {sc.n}x{sc.n}x{sc.m} scene, FP64 NumPy/SciPy FFT "
                     f"with {O.WORKERS} workers, {dt:.1f} s"}
    if single_worker and wl["model"] == "dual":
        workers = O.WORKERS
        O.WORKERS = 1
        try:
            t0 = time.perf_counter()
            O.alg2_step(s2, tau0, op.mask, fwd, adj, p)
            d1 = time.perf_counter() - t0
        finally:
            O.WORKERS = workers
        out["single_worker"] = {"value": V / d1, "cores": 1,
                                "sample": f"the next Algorithm-2 iteration with one FFT worker, "
                                          f"{d1:.1f} s"}
    return out


class Workload:
    """One of the single-scene workloads, ready to be reconstructed again and
    again: the scene, its measurement (the library's own literal-falloff
    forward model + seeded Poisson noise, device-resident), the
    configuration and one workspace."""

    def __init__(self, torch, C, scenes, name):
        wl = WORKLOADS[name]
        self.torch, self.C, self.wl = torch, C, wl
        sc = self.sc = getattr(scenes, wl["scene"])()
        n, m = self.n, self.m = sc.n, sc.m
        self.V = n * n * m
        self.dual = wl["model"] == "dual"
        self.iters_per_rec = wl["init"] + wl["iters"]
        dev = self.dev = torch.device("cuda", 0)
        op_cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                                  bin_ps=sc.bin_ps, model=C.MODEL_OPERATOR,
                                  falloff=C.FALLOFF_LITERAL)
        opP = C.Problem(op_cfg, np.ones((n, n), np.uint8), device=dev)
        clean = opP.apply_A(torch.tensor(sc.u_true.astype(np.float32), device=dev))
        raw_np = scenes.poisson_counts(clean.double().cpu().numpy(), sc.peak, sc.background,
                                       np.random.Generator(np.random.PCG64(sc.seed)))
        opP.close()
        self.raw = torch.tensor(raw_np.astype(np.float32), device=dev)
        self.cfg = C.default_config(nx=n, ny=n, nt=m, wall_w_m=sc.wall_w, wall_h_m=sc.wall_h,
                                    bin_ps=sc.bin_ps,
                                    model=C.MODEL_DUAL if self.dual else C.MODEL_OBJECT,
                                    max_iters=wl["iters"], init_iters=wl["init"], **wl["params"])
        self.ws = torch.empty(C.workspace_bytes(self.cfg), dtype=torch.uint8, device=dev)
        self.out = torch.empty((n, n, m), dtype=torch.float32, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        # the launch plan of this shape, measured once before any timing; every
        # reconstruction below starts with it (plans never change a result)
        P = C.Problem(self.cfg, sc.mask, device=dev, stream=self.stream, workspace=self.ws)
        self.plan = P.tune()
        P.close()

    def reconstruct(self, kinds=None, loop_events=None, stage_events=None):
        """create + set_measurement + run + read volume.  loop_events: two
        events around the run; stage_events: three, around the warm-start and
        Algorithm-2 stages (two run calls)."""
        C, st = self.C, self.stream
        P = C.Problem(self.cfg, self.sc.mask, device=self.dev, stream=st, workspace=self.ws)
        if kinds:
            P.profile_enable(kinds)
        P.set_measurement(self.raw)
        if loop_events is not None:
            loop_events[0].record(st)
        if stage_events is not None:
            stage_events[0].record(st)
            P.run(self.wl["init"])
            stage_events[1].record(st)
            rep = P.run()
            stage_events[2].record(st)
        else:
            rep = P.run()
        if loop_events is not None:
            loop_events[1].record(st)
        self.out.copy_(P.volume())
        prof = P.profile_read() if kinds else None
        P.close()
        return rep, prof

    def timed(self, steps):
        """Whole reconstructions, wall time each, and the run's event time."""
        torch = self.torch
        torch.cuda.synchronize()
        lat, loop_ms = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            self.reconstruct(loop_events=ev)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ts) * 1e3)
            loop_ms.append(ev[0].elapsed_time(ev[1]))
        total_s = time.perf_counter() - t0
        return total_s, lat, loop_ms

    def stage_split(self):
        """Iteration rates of the two stages (dual model) from one more
        reconstruction with events between them."""
        torch = self.torch
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        self.reconstruct(stage_events=ev)
        torch.cuda.synchronize()
        a1, a2 = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        i1, i2 = self.wl["init"], self.wl["iters"]
        out = {"algorithm2_ms": a2, "algorithm2_iterations": i2,
               "algorithm2_voxel_iters_per_s": self.V * i2 / (a2 * 1e-3)}
        if i1:
            out.update({"algorithm1_warm_start_ms": a1, "algorithm1_iterations": i1,
                        "algorithm1_voxel_iters_per_s": self.V * i1 / (a1 * 1e-3)})
        return out

    def summary(self, steps, warmup):
        """Rates of this workload alone (no roofline): the other configurations."""
        for _ in range(max(warmup, 1)):
            self.reconstruct()
        total_s, lat, loop_ms = self.timed(steps)
        ms = total_s * 1e3 / steps
        loop = float(np.median(loop_ms))
        sc = self.sc
        out = {"workload": f"{self.n}x{self.n}x{self.m} "
                           f"{'dual-domain (Algorithm 2)' if self.dual else 'object-domain (Algorithm 1)'}, "
                           f"{int(sc.mask.sum())}/{self.n * self.n} scan points, "
                           f"{self.wl['init']} warm-start + {self.wl['iters']} iterations",
               "steps": steps, "ms_per_reconstruction": ms,
               "reconstructions_per_s": 1e3 / ms,
               "voxel_iters_per_s": self.V * self.iters_per_rec / (ms * 1e-3),
               "latency_ms": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99))},
               "iteration_loop_ms": loop,
               "iteration_loop_voxel_iters_per_s": self.V * self.iters_per_rec / (loop * 1e-3),
               "plan": self.plan}
        if self.dual:
            out["stages"] = self.stage_split()
        return out


def nonconfocal_rates(torch, C):
    """The non-confocal direct-sum operator (Section 2's general model) and its
    transpose: milliseconds per application and paths per second at two grid
    sizes (one application evaluates n^4 m detector-voxel paths)."""
    out = {}
    for (n, m) in ((32, 256), (64, 512)):
        g = C.nc_geometry(n, m, 1.0, 16.0 * 512 / m, (0.2, 0.1), True)
        gen = torch.Generator(device="cuda").manual_seed(n + m)
        x = torch.rand((n, n, m), device="cuda", generator=gen)
        y = torch.empty_like(x)
        row = {}
        for name, fn in (("forward", C.nc_apply), ("transpose", C.nc_apply_T)):
            fn(g, x, y)
            torch.cuda.synchronize()
            reps = 5 if n <= 32 else 2
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn(g, x, y)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            row[name] = {"ms": ms, "paths_per_s": n ** 4 * m / (ms * 1e-3)}
        out[f"{n}x{n}x{m}"] = row
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2301_00406_amd import cnlos as C
    from paper_2301_00406_amd import scenes

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batch":
        cmp = batched_comparison(torch, C, scenes, MIX_FULL)
        t_b = cmp["scenes"] / cmp["batched_rec_per_s"]
        print(json.dumps({
            "metric": "voxel-ADMM-iters/s at 64^2x512 + reconstructions/s, p50/p99 latency",
            "value": cmp["batched_voxel_iters_per_s"], "unit": "voxel-ADMM-iters/s",
            "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * t_b,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 (f64 reductions)", "data": "synthetic (seeded scenes, Poisson noise)",
            "config": {"workload": f"batched uneven mix of {cmp['scenes']} scenes ({cmp['mix']})",
                       "step": "every scene: create + set_measurement + run + read volume"},
            "reconstructions_per_s": cmp["batched_rec_per_s"],
            "batched": cmp, "roofline": None,
        }))
        return
    if args.workload == "serve":
        sv = serve_workload(torch, C, scenes, args.requests, args.rate,
                            baseline=not args.no_serve_baseline)
        print(json.dumps({
            "metric": "voxel-ADMM-iters/s at 64^2x512 + reconstructions/s, p50/p99 latency",
            "value": sv["voxel_iters_per_s"], "unit": "voxel-ADMM-iters/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * sv["makespan_s"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 (f64 reductions)", "data": "synthetic (seeded scenes, Poisson noise)",
            "config": {"workload": f"served Poisson stream of {sv['requests']} requests at "
                                   f"{sv['rate_per_s']:g}/s ({sv['mix']})"},
            "reconstructions_per_s": sv["reconstructions_per_s"],
            "latency_ms": sv["latency_ms"], "serving": sv, "roofline": None,
        }))
        return
    if args.workload == "nonconfocal":
        print(json.dumps({"metric": "non-confocal operator by direct summation",
                          "data": "synthetic (uniform random volumes)",
                          "nonconfocal": nonconfocal_rates(torch, C)}))
        return
    if args.workload == "ablation":
        ab = ablation(torch, C, scenes)
        for r in ab["table"]:
            print(f"{r['scene']:6s} {r['mask']:10s} {r['method']:12s} {r['phi']:4s} accuracy {r['accuracy']:.4f}  "
                  f"RMSE {r['rmse']:.4f}  PSNR {r['psnr_db']:6.2f} dB  SSIM {r['ssim']:.4f}  "
                  f"volume error {r['volume_rel_err']:.4f}", file=sys.stderr)
        print(json.dumps({"metric": "reconstruction quality by curvature function (ablation)",
                          "data": "synthetic (seeded scenes, Poisson noise)", "ablation": ab}))
        return
    wl = WORKLOADS[args.workload]
    W = Workload(torch, C, scenes, args.workload)
    sc, n, m, V, dual, iters_per_rec = W.sc, W.n, W.m, W.V, W.dual, W.iters_per_rec
    reconstruct = W.reconstruct

    for _ in range(max(args.warmup, 1)):
        rep, _ = reconstruct()
    assert rep["total_iters"] == iters_per_rec, rep

    print(f"bench: {args.workload} warm-up done", file=sys.stderr, flush=True)
    # one untimed profiled reconstruction picks the dominant kernel
    rep, prof_all = reconstruct(kinds=C.KERNEL_KINDS)
    dominant = max(prof_all, key=lambda k: prof_all[k][0])
    if args.profile_all:
        tot = sum(v[0] for v in prof_all.values())
        for k, (ms, cnt) in sorted(prof_all.items(), key=lambda kv: -kv[1][0]):
            b = algorithmic_bytes(k, n, m, dual)
            gbs = b * cnt / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
            print(f"{k:12s} {ms:9.3f} ms {100 * ms / tot:5.1f}%  {cnt:6d} launches "
                  f"{1e3 * ms / cnt:8.2f} us/launch  {gbs:8.1f} GB/s", file=sys.stderr)

    # timed region: K reconstructions, events around the dominant kernel only
    torch.cuda.synchronize()
    lat = []
    loop_ms = []
    dom_ms, dom_cnt = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        rep, prof = reconstruct(kinds=[dominant], loop_events=ev)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        loop_ms.append(ev[0].elapsed_time(ev[1]))
        dom_ms += prof[dominant][0]
        dom_cnt += prof[dominant][1]
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0

    ms_per_step = total_s * 1e3 / args.steps
    value = V * iters_per_rec / (ms_per_step * 1e-3)
    avg_us = 1e3 * dom_ms / dom_cnt
    abytes = algorithmic_bytes(dominant, n, m, dual)
    traffic = load_traffic(dominant, args.workload)
    if dominant in ALU_BOUND:
        aflops = algorithmic_flops(dominant, n, m)
        achieved = aflops / (avg_us * 1e-6) / 1e12
        layout_bytes = abytes - hq_bytes(n, m) + hq_bytes(n, m, layout=True)
        roof = {"bound": "alu", "kernel": dominant,
                "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "traffic": traffic, "avg_launch_us": avg_us,
                "peak_nonpacked": VALU_NONPACKED_TFLOPS,
                "frac_nonpacked": achieved / VALU_NONPACKED_TFLOPS,
                "algorithmic_flops_per_launch": aflops,
                "algorithmic_bytes_per_launch": abytes,
                "layout_bytes_per_launch": layout_bytes,
                "layout_over_algorithmic_bytes": layout_bytes / abytes,
                "hbm_GBs": abytes / (avg_us * 1e-6) / 1e9}
    else:
        roof = {"bound": "hbm", "kernel": dominant,
                "achieved": abytes / (avg_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "traffic": traffic, "avg_launch_us": avg_us,
                "algorithmic_bytes_per_launch": abytes}
    roof["frac"] = roof["achieved"] / roof["peak"]
    result = {
        "metric": "voxel-ADMM-iters/s at 64^2x512 + reconstructions/s, p50/p99 latency",
        "value": value,
        "unit": "voxel-ADMM-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 reductions)",
        "data": "synthetic (seeded scene, Poisson noise)",
        "config": {
            "workload": f"{n}x{n}x{m} {'dual-domain (Algorithm 2)' if dual else 'object-domain (Algorithm 1)'}, "
                        f"{int(sc.mask.sum())}/{n * n} scan points, {sc.bin_ps:g} ps bins, "
                        f"{sc.wall_w:g} m wall, {wl['init']} warm-start + {wl['iters']} iterations, "
                        "backtracking on",
            "nx": n, "ny": n, "nt": m, "iters_per_reconstruction": iters_per_rec,
            "step": "create (H^, power iterations) + set_measurement + run + read volume",
        },
        "reconstructions_per_s": 1e3 / ms_per_step,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "iteration_loop": {
            "ms_per_reconstruction": float(np.median(loop_ms)),
            "voxel_iters_per_s": V * iters_per_rec / (float(np.median(loop_ms)) * 1e-3),
            **(W.stage_split() if dual else {}),
        },
        "roofline": roof,
        "plan": W.plan,
        "context": {"paper_titan_rtx_alg2_seconds_64x64x512": 15.0},
    }
    print(f"bench: timed region done ({ms_per_step:.1f} ms per reconstruction)", file=sys.stderr,
          flush=True)
    if not args.no_other_workloads:
        # the other single-scene configurations, rates only
        result["other_workloads"] = {}
        for name, steps in (("small", 20), ("large", 2)):
            if name != args.workload:
                result["other_workloads"][name] = Workload(torch, C, scenes, name).summary(steps, 1)
                torch.cuda.empty_cache()
                print(f"bench: {name} workload done", file=sys.stderr, flush=True)
    if not args.no_batch:
        result["batched"] = batched_comparison(torch, C, scenes, MIX_SMALL)
        result["batched_metric_config"] = batched_metric(torch, C, scenes)
    if not args.no_other_workloads:
        result["nonconfocal"] = nonconfocal_rates(torch, C)
    if not args.no_cpu_baseline:
        print("bench: CPU baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(sc, wl, args.cpu_iters)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
