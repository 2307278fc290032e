#!/usr/bin/env python3
"""Open-pipe Poisson solves/s on one MI355X (FP32 and FP64 legs) with roofline and CPU baseline.

Workload: 128 x 128 x 512 mesh (padded 256 x 256 x 1024) in a 1 x 1 pipe,
z-integrated Green function (IGF), 256 x 256 modes, charge = three seeded
Gaussian sub-bunches sampled with 2^28 macroparticles and deposited by
cloud-in-cell.  One step = one full solve (all five kernels: z forward,
y forward, x forward + mixed product + x inverse, y inverse, z inverse) of
that charge, input already resident in HBM.  The Green spectra are built once
per plan before timing (the paper computes them once and reuses them).

Prints ONE JSON line on stdout; progress goes to stderr.
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
  python bench.py --copy-calibration   (a plain copy of known size, for counter scaling)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "open-pipe Poisson solves/s at 128x128x512 (FP32 vs FP64) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
PASS_NAMES = ["z_forward", "y_forward", "x_product", "y_inverse", "z_inverse"]
KERNEL_NAMES = ["z_r2c_kernel", "strided_kernel<fwd>", "xprod_kernel", "strided_kernel<inv>", "z_c2r_kernel"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_three_bunch_cic.json")
KERNEL_SOURCES = ["paper_1111_4971_amd/csrc/passes.hip", "paper_1111_4971_amd/csrc/xprod.hip",
                  "paper_1111_4971_amd/csrc/pass_common.h", "paper_1111_4971_amd/csrc/fft_engine.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(leg, kernel_index):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    e = t.get("legs", {}).get(leg, {}).get(PASS_NAMES[kernel_index])
    return None if e is None else float(e["bytes_per_launch"])


def copy_calibration(nbytes=1 << 30, reps=5):
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                      "reps": reps}))


def time_leg(pipe, torch, wl, precision, steps, warmup):
    import numpy as np
    log("[bench] %s: building plan" % precision)
    plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                          precision=precision, mx=wl.mx, my=wl.my)
    info = plan.info
    rho = torch.from_numpy(np.ascontiguousarray(wl.rho)).to(device="cuda", dtype=plan.dtype)
    phi = torch.empty_like(rho)
    ws = plan.workspace()
    for _ in range(warmup):
        plan.solve(rho, out=phi, workspace=ws)
    torch.cuda.synchronize()
    log("[bench] %s: timing %d steps" % (precision, steps))
    # timed region: K solves back to back, bracketed by device synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(rho, out=phi, workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    # the same K solves again with HIP events recorded on the solve stream
    # before, between and after the five kernels: per-kernel durations for the
    # roofline.  (The event markers themselves add a few microseconds of gap
    # per solve, which is why the throughput comes from the region above.)
    plan.timing_start(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        plan.solve(rho, out=phi, workspace=ws)
    torch.cuda.synchronize()
    ms_events = (time.perf_counter() - t2) * 1e3 / steps
    pass_ms, n = plan.timing_stop()
    out = phi.double().cpu().numpy()
    dom = max(range(5), key=lambda i: pass_ms[i])
    achieved = info.pass_bytes[dom] / (pass_ms[dom] * 1e-3) / 1e9
    traffic = measured_traffic(precision, dom)
    leg = {
        "value": steps / (t1 - t0),
        "ms_per_step": ms_step,
        "ms_per_step_with_events": ms_events,
        "events_recorded": n,
        "plan_build_ms": info.build_ms,
        "schedule": {"x_tile": info.xtile, "a2_row_pad": info.apad, "z_block_cap": info.zblocks,
                     "x_nontemporal_stores": info.xnt, "a1_row_pad": info.a1pad},
        "padded_lengths": [info.lx, info.ly, info.lz],
        "model_bytes_per_solve": info.model_bytes,
        "model_GBps_whole_solve": info.model_bytes / (ms_step * 1e-3) / 1e9,
        "hbm_frac_whole_solve": info.model_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "passes": {PASS_NAMES[i]: {"kernel": KERNEL_NAMES[i], "ms": pass_ms[i],
                                   "model_bytes": info.pass_bytes[i],
                                   "GBps": info.pass_bytes[i] / (pass_ms[i] * 1e-3) / 1e9,
                                   "hbm_frac": info.pass_bytes[i] / (pass_ms[i] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                   for i in range(5)},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": info.pass_bytes[dom], "avg_launch_ms": pass_ms[dom]},
    }
    plan.close()
    return leg, out


def batch_leg(pipe, torch, workloads, replays=20, warmup=3):
    """96 uneven IGF solves (seeded manifest of four mesh shapes): one replay of
    the captured batch graph vs the same solves issued one by one, FP32 and FP64."""
    import numpy as np
    man = workloads.batch_manifest()
    members = [workloads.batch_member(d) for d in man]
    log("[bench] batch: building %d FP32 and %d FP64 plans" % (len(members), len(members)))
    # batch members: padded lengths per mesh shape chosen by the plan-time
    # autotuner in throughput mode (timed once per shape); the FP64 plans of
    # the plain sequential comparison keep the default lengths
    mk = lambda w, prec: pipe.GreenPlan(w.nx, w.ny, w.nz, w.hx, w.hy, w.hz, w.a, w.b, kind=w.kind,
                                        precision=prec, mx=w.mx, my=w.my,
                                        autotune="batch" if prec == "fp32" else False)
    p32 = [mk(w, "fp32") for w in members]
    p64 = [mk(w, "fp64") for w in members]
    r32 = [torch.from_numpy(w.rho).to("cuda", torch.float32) for w in members]
    r64 = [torch.from_numpy(w.rho).to("cuda", torch.float64) for w in members]
    o32 = [torch.empty_like(r) for r in r32]
    o64 = [torch.empty_like(r) for r in r64]
    ws32 = [p.workspace() for p in p32]
    ws64 = [p.workspace() for p in p64]
    b = pipe.Batch(p32)
    bws = b.workspace()

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_batch = timed(lambda: b.solve(r32, o32, workspace=bws), replays)
    got = [o.double().cpu().numpy() for o in o32]
    t_seq32 = timed(lambda: [p.solve(r, out=o, workspace=w) for p, r, o, w in zip(p32, r32, o32, ws32)], replays)
    t_seq64 = timed(lambda: [p.solve(r, out=o, workspace=w) for p, r, o, w in zip(p64, r64, o64, ws64)], replays)
    ref = [o.double().cpu().numpy() for o in o64]
    err = max(float(np.linalg.norm(g - r) / np.linalg.norm(r)) for g, r in zip(got, ref))
    model = sum(p.info.model_bytes for p in p32)
    # the same solves' model bytes at the smallest padded lengths the Appendix
    # allows (L >= 2n - 1, a supported 2^p 3^q; lz even with lz/2 >= nz): one
    # plan per shape at those lengths, few modes (the bytes do not depend on them)
    smooth = sorted(2 ** p * 3 ** q for p in range(11) for q in range(7) if 8 <= 2 ** p * 3 ** q <= 1024)
    least = lambda need: next(v for v in smooth if v >= need)
    per_shape = {}
    for w in members:
        if w.shape not in per_shape:
            L = (least(2 * w.nx - 1), least(2 * w.ny - 1), 2 * least(w.nz))
            q = pipe.GreenPlan(w.nx, w.ny, w.nz, w.hx, w.hy, w.hz, w.a, w.b, kind=w.kind, precision="fp32",
                               mx=2, my=2, L=L)
            per_shape[w.shape] = q.info.model_bytes
            q.close()
    model_min = sum(per_shape[w.shape] for w in members)
    n = len(members)
    tuned = {}
    for w, p in zip(members, p32):
        tuned["%dx%dx%d" % w.shape] = "%dx%dx%d" % (p.info.lx, p.info.ly, p.info.lz)
    res = {"solves": n, "shapes": sorted({"%dx%dx%d" % w.shape for w in members}),
           "autotuned_padded_lengths_fp32": tuned,
           "batched_fp32_solves_per_s": n / t_batch, "batched_fp32_ms_per_batch": t_batch * 1e3,
           "sequential_fp32_solves_per_s": n / t_seq32, "sequential_fp64_solves_per_s": n / t_seq64,
           "speedup_batched_fp32_over_sequential_fp64": t_seq64 / t_batch,
           "speedup_batched_fp32_over_sequential_fp32": t_seq32 / t_batch,
           "model_bytes_per_batch": model, "batched_model_GBps": model / t_batch / 1e9,
           "batched_hbm_frac": model / t_batch / 8e12,
           "model_bytes_per_batch_smallest_lengths": model_min,
           "batched_hbm_frac_smallest_lengths": model_min / t_batch / 8e12,
           "max_member_rel_l2_fp32_vs_fp64": err}
    b.close()
    for p in p32 + p64:
        p.close()
    return res


def subregion_leg(pipe, torch, steps=50):
    """Sec. 5's thin-beam argument: mesh only a 64x64 sub-region around a thin
    beam instead of the full 256x256 cross-section at the same spacing (pipe
    1 x 1, 512 z nodes, IGF, FP32).  Both plans use the pipe's 512 x 512 modes;
    the charge lies inside the sub-region, so both give the same potential on
    the shared nodes."""
    import numpy as np
    from paper_1111_4971_amd import workloads
    NX, nz, n = 256, 512, 64
    h, hz = 1.0 / (NX + 1), 20.0 / (nz - 1)
    k0 = (NX - n) // 2
    rho = workloads.gaussian(n, n, nz, h, h, hz, ((n + 1) * h / 2, (n + 1) * h / 2, 0.0), (0.02, 0.02, 1.0))
    full = np.zeros((NX, NX, nz))
    full[k0:k0 + n, k0:k0 + n] = rho
    log("[bench] subregion: plans")
    pf = pipe.GreenPlan(NX, NX, nz, h, h, hz, 1.0, 1.0, kind=pipe.IGF_Z, precision="fp32", mx=2 * NX, my=2 * NX)
    ps = pipe.GreenPlan(n, n, nz, h, h, hz, 1.0, 1.0, kind=pipe.IGF_Z, precision="fp32", mx=2 * NX, my=2 * NX,
                        offset=(k0 * h, k0 * h))
    out = {}
    res = {}
    for name, plan, x in (("full_256x256x512", pf, full), ("subregion_64x64x512", ps, rho)):
        xt = torch.from_numpy(x).to("cuda", torch.float32)
        y = torch.empty_like(xt)
        ws = plan.workspace()
        for _ in range(5):
            plan.solve(xt, out=y, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.solve(xt, out=y, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        res[name] = {"solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3}
        out[name] = y.double().cpu().numpy()
    a = out["subregion_64x64x512"]
    b = out["full_256x256x512"][k0:k0 + n, k0:k0 + n]
    res["speedup_subregion_over_full"] = res["full_256x256x512"]["ms_per_solve"] / res["subregion_64x64x512"]["ms_per_solve"]
    res["rel_max_diff_on_shared_nodes"] = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    pf.close()
    ps.close()
    return res


def band_leg(pipe, torch, steps=50, tol=1e-6):
    """Eq. 17-18 on the paper's long bunch (Sec. 4: pipe 4 cm, 20 x 20 modes,
    sigma_z = 1.2 m, IGF): banded plans keeping the plane distances up to N
    (N = 0 is Eq. 17; "auto" is the N chosen from the mode-sum decay bound at
    tol) timed beside the full 3-D plan of the same mesh, per precision, with
    their deviation from the full FP64 solve."""
    import numpy as np
    from paper_1111_4971_amd import workloads

    def timed(plan, x):
        y = torch.empty_like(x)
        ws = plan.workspace()
        for _ in range(5):
            plan.solve(x, out=y, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.solve(x, out=y, workspace=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / steps * 1e3
        plan.timing_start(steps)
        for _ in range(steps):
            plan.solve(x, out=y, workspace=ws)
        pass_ms, _ = plan.timing_stop()
        return ms, pass_ms, y.double().cpu().numpy()

    res = {"tol": tol}
    for n, nz, bands in ((128, 256, (0, 1, 2, "auto")), (256, 1024, (0, 1, "auto"))):
        wl, _ = workloads.accuracy_study_bunch(n, nz, 120.0, kind=pipe.IGF_Z)
        key = "%dx%dx%d" % (n, n, nz)
        r = {}
        ref = None
        for prec in ("fp64", "fp32"):
            dt = torch.float32 if prec == "fp32" else torch.float64
            x = torch.from_numpy(wl.rho).to("cuda", dt)
            log("[bench] band %s %s: full plan" % (key, prec))
            plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                                  precision=prec, mx=wl.mx, my=wl.my)
            ms_full, pm, y = timed(plan, x)
            plan.close()
            if ref is None:
                ref = y
            r.setdefault("full", {})[prec] = {"ms_per_solve": ms_full, "kernel_ms": pm}
            for nb in bands:
                log("[bench] band %s %s: N = %s" % (key, prec, nb))
                plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                                      precision=prec, mx=wl.mx, my=wl.my, band=nb, band_tol=tol)
                ms, pm, y = timed(plan, x)
                pb = plan.info.pass_bytes
                e = r.setdefault("N_auto" if nb == "auto" else "N%d" % nb, {})
                e["N"] = plan.band
                e[prec] = {"ms_per_solve": ms, "kernel_ms": pm[:3], "speedup_over_full": ms_full / ms,
                           "build_time_ratio_3d_over_banded": plan.info.band_speedup,
                           "x_pass_GBps": pb[1] / (pm[1] * 1e-3) / 1e9,
                           "rel_max_vs_full_fp64": float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))}
                plan.close()
                if nb == "auto":
                    # the same request with band_fastest: the faster of the banded and 3-D plans
                    plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                                          precision=prec, mx=wl.mx, my=wl.my, band=nb, band_tol=tol,
                                          band_fastest=True)
                    ms_f, _, _ = timed(plan, x)
                    f = r.setdefault("N_auto_fastest", {})
                    f[prec] = {"returned": "banded N=%d" % plan.band if plan.band is not None else "3-D",
                               "ms_per_solve": ms_f, "speedup_over_full": ms_full / ms_f}
                    plan.close()
        res[key] = r
    return res


def same_plan_leg(pipe, torch, wl, members=8, replays=20):
    """Many charges, one cached Green function (Sec. 2 after Eq. 10: the spectra
    are computed once and reused): the benchmark plan repeated `members` times
    in one batch, each member with its own charge (the benchmark charge shifted
    along z by k planes).  The fused x pass runs the members of one (kz tile, ky)
    back to back, so the spectra tile comes from L2 for all but the first."""
    import numpy as np
    res = {"members": members}
    for prec in ("fp32", "fp64"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        log("[bench] same-plan batch %s: plan" % prec)
        plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                              precision=prec, mx=wl.mx, my=wl.my)
        rhos = [torch.from_numpy(np.roll(wl.rho, k, axis=2)).to("cuda", dt) for k in range(members)]
        b = pipe.Batch([plan] * members)
        outs = [torch.empty_like(r) for r in rhos]
        ws = b.workspace()
        for _ in range(3):
            b.solve(rhos, outs=outs, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(replays):
            b.solve(rhos, outs=outs, workspace=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / replays * 1e3
        single = plan.solve(rhos[-1])
        torch.cuda.synchronize()
        res[prec] = {"ms_per_batch": ms, "solves_per_s": members * 1e3 / ms,
                     "last_member_equals_single_solve": bool(torch.equal(outs[-1], single))}
        del b, outs, ws
        plan.close()
        torch.cuda.empty_cache()
    return res


def free_leg(pipe, torch, wl, steps=100):
    """Sec. 1, Eq. 5: the free-space (Hockney) solve on the benchmark's mesh and
    charge (G = 1/r, zero at zero separation), beside the pipe solve: the same
    five passes with a one-term spectrum."""
    res = {}
    for prec in ("fp32", "fp64"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        x = torch.from_numpy(wl.rho).to("cuda", dt)
        log("[bench] free space %s: plan" % prec)
        plan = pipe.FreePlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, 0.0, precision=prec)
        y = torch.empty_like(x)
        ws = plan.workspace()
        for _ in range(10):
            plan.solve(x, out=y, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.solve(x, out=y, workspace=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / steps * 1e3
        plan.timing_start(steps)
        for _ in range(steps):
            plan.solve(x, out=y, workspace=ws)
        torch.cuda.synchronize()
        pass_ms, _ = plan.timing_stop()
        info = plan.info
        res[prec] = {"ms_per_solve": ms, "solves_per_s": 1e3 / ms, "build_ms": plan.info.build_ms,
                     "spectra_bytes": info.spectra_bytes,
                     "passes": {PASS_NAMES[i]: {"ms": pass_ms[i], "model_bytes": info.pass_bytes[i],
                                                "hbm_frac": info.pass_bytes[i] / (pass_ms[i] * 1e-3) / 1e9
                                                / HBM_PEAK_GBS} for i in range(5)}}
        plan.close()
    return res


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(wl, min_seconds=10.0, max_solves=12):
    """The oracle's mode-space solve (FP64 numpy/scipy on the host cores) of the
    same 128x128x512 charge, mode kernel included, repeated until at least
    min_seconds have passed (at most max_solves); the rate is solves per second
    over those solves.  The oracle's literal Eq. 10 form needs its four Green
    spectra built first, which takes minutes at this size, so the mode-space
    form -- exact to rounding for this full-aperture mesh, and pinned to it --
    is the timed sample."""
    from oracle import modespace
    log("[bench] cpu baseline: oracle mode-space solves (at least %.0f s)" % min_seconds)
    t = time.perf_counter()
    n = 0
    while True:
        phi = modespace.solve(wl.rho, **wl.geometry())
        n += 1
        dt = time.perf_counter() - t
        log("[bench] cpu baseline: %d solve(s), %.1f s" % (n, dt))
        if dt >= min_seconds or n >= max_solves:
            break
    return {"value": n / dt, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": "%d full 128x128x512 IGF solve(s) (256x256 modes), FP64, by the oracle's mode-space "
                      "form (DST-I in x and y, per-mode z convolution, mode kernel built inside each timed "
                      "call), numpy/scipy on the host" % n,
            "seconds": dt, "solves": n, "host_cpus": os.cpu_count()}, phi


def cpu_o2_leg(wl, L, solves=3):
    """The oracle's literal Eq. 10 form (one forward transform of the padded
    charge, four products with the mixed-direction Green spectra, four inverse
    transforms; scipy.fft on the host cores) on the same charge at the GPU
    plan's padded lengths, median of `solves`.  Its four Green spectra are
    built once before the timed solves and reported separately (minutes at
    this size, so the leg is opt-in)."""
    import statistics
    import numpy as np
    from oracle import fourterm
    g = wl.geometry()
    log("[bench] cpu O2: building the four Green spectra at %s" % (L,))
    t = time.perf_counter()
    spectra = []
    for term in fourterm.TERMS:   # as fourterm.green_spectra, one term at a time with progress
        gdir = term[3]
        xi = fourterm.green_array(wl.rho.shape, L, (g["hx"], g["hy"], g["hz"]), (g["a"], g["b"], g["mx"], g["my"]),
                                  g["kind"], term[1], term[2])
        spectra.append(fourterm._F3(xi.astype(np.complex128), gdir))
        del xi
        log("[bench] cpu O2: spectrum %d of 4 built, %.1f s" % (len(spectra), time.perf_counter() - t))
    build = time.perf_counter() - t
    log("[bench] cpu O2: spectra built in %.1f s" % build)
    ts = []
    for i in range(solves):
        t = time.perf_counter()
        fourterm.solve(wl.rho, **g, L=L, spectra=spectra)
        ts.append(time.perf_counter() - t)
        log("[bench] cpu O2: solve %d of %d, %.1f s" % (i + 1, solves, ts[-1]))
    med = statistics.median(ts)
    return {"value": 1.0 / med, "unit": "solves/s", "kind": "oracle O2 (literal Eq. 10)", "median_s": med,
            "solves": solves, "seconds": ts, "spectra_build_s": build, "fft_workers": fourterm._WORKERS,
            "host_cpus": os.cpu_count(),
            "sample": "%d full %dx%dx%d solves (%dx%d modes), FP64, padded %dx%dx%d, spectra prebuilt"
                      % (solves, wl.nx, wl.ny, wl.nz, g["mx"], g["my"], L[0], L[1], L[2])}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--legs", default="fp32,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-o2", action="store_true",
                    help="also time the oracle's literal Eq. 10 form on the host (median of 3; minutes)")
    ap.add_argument("--mesh", default=None,
                    help="NXxNYxNZ: time a smooth bunch on this mesh instead of the benchmark charge "
                         "(profiling other sizes; implies --no-batch and --no-cpu-baseline)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1111_4971_amd import pipe, workloads
    pipe.lib()
    if args.mesh:
        nx, ny, nz = (int(v) for v in args.mesh.lower().split("x"))
        wl = workloads.gaussian_bunch(nx, ny, nz)
        wl.notes = {"n_particles": 0, "peak_rel_noise": 0.0}
        args.no_batch = args.no_cpu_baseline = True
        log("[bench] smooth bunch on %dx%dx%d" % (nx, ny, nz))
    else:
        log("[bench] generating the 128x128x512 three-bunch CIC charge")
        t = time.perf_counter()
        wl = workloads.three_bunch_cic()
        log("[bench] generated in %.1f s (%d macroparticles)" % (time.perf_counter() - t, wl.notes["n_particles"]))

    legs = {}
    outs = {}
    for prec in args.legs.split(","):
        legs[prec], outs[prec] = time_leg(pipe, torch, wl, prec, args.steps, args.warmup)
        log("[bench] %s: %.1f solves/s, %.3f ms/solve, dominant %s at %.0f GB/s" % (
            prec, legs[prec]["value"], legs[prec]["ms_per_step"], legs[prec]["roofline"]["kernel"],
            legs[prec]["roofline"]["achieved"]))

    primary = "fp32" if "fp32" in legs else list(legs)[0]
    res = {
        "metric": METRIC,
        "value": legs[primary]["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": legs[primary]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if primary == "fp32" else "f64",
        "data": "synthetic: three seeded Gaussian sub-bunches, 2^28 CIC macroparticles",
        "config": {"workload": ("three_bunch_cic 128x128x512 (padded 256x256x1024), pipe 1x1, IGF Green "
                                "function, 256x256 modes, h=1/129, hz=20/511") if not args.mesh else wl.name,
                   "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "lx": legs[primary]["padded_lengths"][0],
                   "ly": legs[primary]["padded_lengths"][1], "lz": legs[primary]["padded_lengths"][2],
                   "green": "IGF_Z", "modes": [wl.mx, wl.my], "n_particles": wl.notes["n_particles"],
                   "peak_node_rel_noise": wl.notes["peak_rel_noise"]},
        "roofline": legs[primary]["roofline"],
        "legs": legs,
    }
    if "fp32" in legs and "fp64" in legs:
        res["fp32_speedup_over_fp64"] = legs["fp32"]["value"] / legs["fp64"]["value"]
        d = outs["fp32"] - outs["fp64"]
        res["fp32_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(outs["fp64"]))
        res["fp32_vs_fp64_rel_max"] = float(np.max(np.abs(d)) / np.max(np.abs(outs["fp64"])))
    if not args.no_batch:
        res["batch"] = batch_leg(pipe, torch, workloads)
        log("[bench] batch: %.0f solves/s batched FP32, %.0f sequential FP32, %.0f sequential FP64" % (
            res["batch"]["batched_fp32_solves_per_s"], res["batch"]["sequential_fp32_solves_per_s"],
            res["batch"]["sequential_fp64_solves_per_s"]))
    if not args.no_batch:
        res["subregion"] = subregion_leg(pipe, torch)
        log("[bench] subregion: %.1fx faster than the full cross-section, max rel diff %.1e" % (
            res["subregion"]["speedup_subregion_over_full"], res["subregion"]["rel_max_diff_on_shared_nodes"]))
    if not args.no_batch:
        res["same_plan_batch"] = same_plan_leg(pipe, torch, wl)
        log("[bench] same-plan batch of %d: %.0f (FP32) / %.0f (FP64) solves/s" % (
            res["same_plan_batch"]["members"], res["same_plan_batch"]["fp32"]["solves_per_s"],
            res["same_plan_batch"]["fp64"]["solves_per_s"]))
        res["free_space"] = free_leg(pipe, torch, wl)
        log("[bench] free space: %.4f ms (FP32), %.4f ms (FP64) per solve" % (
            res["free_space"]["fp32"]["ms_per_solve"], res["free_space"]["fp64"]["ms_per_solve"]))
        res["banded"] = band_leg(pipe, torch)
        for k, v in res["banded"].items():
            if not isinstance(v, dict):
                continue
            for nm, e in v.items():
                if nm.startswith("N") and "N" in e:
                    log("[bench] banded %s %s (N=%d): %.2fx (FP32) / %.2fx (FP64) the full solve's speed, "
                        "max rel deviation %.1e" % (k, nm, e["N"], e["fp32"]["speedup_over_full"],
                                                    e["fp64"]["speedup_over_full"], e["fp64"]["rel_max_vs_full_fp64"]))
    if not args.no_cpu_baseline:
        cb, ophi = cpu_baseline(wl)
        if args.cpu_o2:
            cb["o2_literal_eq10"] = cpu_o2_leg(wl, tuple(res["legs"]["fp64" if "fp64" in res["legs"] else "fp32"]
                                                         ["padded_lengths"]))
        res["cpu_baseline"] = cb
        for prec in outs:
            d = outs[prec] - ophi
            res[prec + "_vs_oracle"] = {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ophi)),
                                        "rel_max": float(np.max(np.abs(d)) / np.max(np.abs(ophi)))}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
