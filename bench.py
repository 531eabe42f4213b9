"""Benchmark of the fused primal-dual sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one full solve of the 4096 x 4096 denoising workload: 2000
iterations of the fused sweep (gradient, dual prox, divergence, primal prox,
extrapolation), the duality gap reduced every 10 iterations, plus the solve's
init and read-out.  The input (seeded synthetic scene, 200 shapes, noise 0.1)
is resident in HBM before timing starts.  One JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BYTES_PER_PIXEL_ITER = 32      # one iteration as defined: reads f^k, f^{k-1}, p^k (2), g,
                               # writes f^{k+1}, p^{k+1} (2)
PASS_BYTES_PER_PIXEL = 28      # a launch of n iterations: reads f^k, p^k (2), g, writes
                               # f^{k+n}, p^{k+n} (2) (fbar^k is formed from f^k, g, p^k)
# Issue ceiling of the vector ALUs without packed fp32 math (which this build
# turns off): each CU has 4 SIMDs of 16 lanes, so one wave64 VALU instruction
# per CU and cycle; at 2.4 GHz over 256 CUs.  (The published 157.3 TFLOP/s
# counts a fused multiply-add as two operations and a packed pair as two.)
VALU_PEAK_WAVE_INSTR_S = 256 * 2.4e9
VALU_PEAK_TOPS = VALU_PEAK_WAVE_INSTR_S * 64 / 1e12      # 39.3 T lane-ops/s
# Texture-addresser ceiling of the gathers: 4 lane addresses per clock per
# CU, one wave64 buffer load per 16 cycles.

PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "sweep2d_xs5_denoise4096_traffic.txt")
SQ_FILE = os.path.join(PROFILES, "sweep2d_xs5_denoise4096_sq.txt")
TOMO_COUNTERS_FILE = os.path.join(PROFILES, "tomo_kernels_tomo2048x1000_counters.txt")
CSRC = os.path.join(ROOT, "paper_1608_03589_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, f)
               for f in ("kernels2d.hip", "tile2d.h", "tile2d_xs.h", "pointwise.h",
                         "finish.h", "sync.h")]
TOMO_SRCS = [os.path.join(CSRC, f)
             for f in ("tomo.hip", "tomo.h", "tile2d.h", "pointwise.h", "bst.hip", "lp.hip")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_hash() -> str:
    return source_hash(KERNEL_SRCS)


def read_kv(path):
    """key: value lines of a profile summary (comments start with #)."""
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def read_sweep_profile(path, key, tile):
    """A per-launch figure of the sweep from a committed rocprofv3 summary,
    or None when the kernel sources or the tile changed since it was taken."""
    kv = read_kv(path)
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    if kv.get("tile_th_wpb_order") != " ".join(str(v) for v in tile):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def read_traffic(pixels: int, tile):
    """HBM bytes per sweep launch (copy-calibrated FETCH_SIZE + WRITE_SIZE)."""
    return read_sweep_profile(TRAFFIC_FILE, "hbm_bytes_per_launch", tile)


def read_tomo_counters():
    """Per-dispatch counter figures of the tomography kernels, {kernel:
    {key: value}}, or {} when the sources changed since they were taken."""
    kv = read_kv(TOMO_COUNTERS_FILE)
    if kv.get("kernel_source_sha256_16") != source_hash(TOMO_SRCS):
        return {}
    out = {}
    for k, v in kv.items():
        if "." in k:
            kern, key = k.split(".", 1)
            try:
                out.setdefault(kern, {})[key] = float(v)
            except ValueError:
                pass
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def pass_schedule(iters, check_every, depth):
    """Iterations per launch of a solve, as the library schedules them: up
    to `depth` per pass, a gap check only on a pass's first iteration."""
    out, k = [], 0
    while k < iters:
        n = min(depth, iters - k)
        if check_every > 0:
            n = min(n, (k // check_every + 1) * check_every - k)
        out.append(n)
        k += n
    return out


def kernel_name(kernels, passes, pipelined=False):
    parts = []
    for n in kernels:
        nm = "sweep2d_pipe_kernel" if pipelined else f"sweep2d_xs_kernel<{n}>"
        parts.append(f"{nm} ({n} iteration{'s' if n > 1 else ''} per launch, "
                     f"{passes.count(n)} launches per solve)")
    return "; ".join(parts) + "; the launch at each 10th iteration also reduces the gap"


def cpu_baseline(g64, lam, s, budget_s=15.0, max_iter=30):
    """The FP64 oracle, untuned, on the host: as many iterations of the same
    4096^2 workload as fit in the budget (at least 2)."""
    import oracle
    f, f_prev, p = oracle.init_state(g64)
    n = 0
    t0 = time.perf_counter()
    while n < max_iter:
        if n >= 2 and time.perf_counter() - t0 > budget_s:
            break
        f_new, p = oracle.pdhg_iteration(f, f_prev, p, g64, lam, s, s)
        f_prev, f = f, f_new
        n += 1
        if n % 5 == 0:
            log(f"cpu baseline: {n} iterations, {time.perf_counter() - t0:.1f} s")
    t = time.perf_counter() - t0
    return n, t


def timed(fn, stream, reps=1):
    """Run fn reps times between HIP events on `stream`; returns ms/rep."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    out = None
    for _ in range(reps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def bench_denoise_256(dev):
    """The small parity workload (256^2, 1000 iterations, gap every 10) as a
    throughput case: its 2 MiB working set stays in the caches, so launch
    latency rather than HBM sets the time.  Direct launches and launches
    replayed from HIP graphs of 64 iterations."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, scene2d
    w = WORKLOADS["denoise_256"]
    _, g = scene2d(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    gt = torch.from_numpy(g.astype(np.float32)).to(dev)
    out = torch.empty_like(gt)
    solver = tv.PlainSolver(tuple(gt.shape), dev)
    stream = torch.cuda.current_stream(dev)
    s = 1.0 / math.sqrt(8.0)
    rec = {"workload": "denoise_256", "image": [w["H"], w["W"]],
           "iterations": w["iters"], "gap_check_every": 10,
           "launches_per_solve": len(pass_schedule(w["iters"], 10,
                                                   tv.pass_length(tuple(gt.shape))))}
    pix_its = w["H"] * w["W"] * w["iters"]
    for name, use_graph in (("direct", 0), ("graph", 1)):
        def run():
            return solver.solve(gt, w["lam"], tau=s, sigma=s, max_iter=w["iters"],
                                check_every=10, gap_tol=-1.0, use_graph=use_graph, out=out)
        run()
        ms, _ = timed(run, stream, 10)
        rec[f"{name}_ms"] = ms
        rec[f"mpix_its_{name}"] = pix_its / (ms * 1e-3) / 1e6
        rec[f"us_per_launch_{name}"] = ms * 1e3 / rec["launches_per_solve"]
    # latency of the small case against the pass depth and the band height:
    # a pass walks th + 2 depth - 1 rows serially, so small images favour
    # short bands
    sweep = []
    depth0 = tv.get_pass_depth()
    tile0 = tv.get_tile(tuple(gt.shape))
    try:
        for depth in (1, 2, 3, 4, 5):
            tv.set_pass_depth(depth)
            for th in (1, 2, 4, 8):
                tv.set_tile(tuple(gt.shape), th, 4, 0)
                def run():
                    return solver.solve(gt, w["lam"], tau=s, sigma=s, max_iter=w["iters"],
                                        check_every=10, gap_tol=-1.0, use_graph=1, out=out)
                run()
                ms, _ = timed(run, stream, 5)
                sweep.append({"depth": depth, "th": th, "ms": ms,
                              "mpix_its": pix_its / (ms * 1e-3) / 1e6})
    finally:
        tv.set_pass_depth(depth0)
        tv.set_tile(tuple(gt.shape), *tile0)
    rec["depth_band_sweep_graph"] = sweep
    best = min(sweep, key=lambda r: r["ms"])
    rec["best_depth_band"] = best
    # the stopping solve of the same image (relative gap 1e-4)
    def stop():
        return solver.solve(gt, w["lam"], tau=s, sigma=s, max_iter=w["iters"],
                            check_every=10, gap_tol=1e-4, out=out)
    stop()
    ms, (_, res) = timed(stop, stream, 10)
    rec["stopping_solve_ms"] = ms
    rec["stopping_solve_iters"] = res.iters
    log(f"denoise 256: direct {rec['direct_ms']:.3f} ms, graph {rec['graph_ms']:.3f} ms "
        f"per 1000 iterations; stopping solve {ms:.3f} ms ({res.iters} iterations); "
        f"best depth {best['depth']} band {best['th']}: {best['ms']:.3f} ms")
    return rec


def bench_batched(dev):
    """64 uneven images to relative gap 1e-4: one persistent launch, graph
    blocks, and the plain solver looping over the images."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, batch_scenes
    w = WORKLOADS["batch64_uneven"]
    data = batch_scenes(w["n"], w["seed"], w["n_shapes"])
    imgs = [torch.from_numpy(d[1].astype(np.float32)).to(dev) for d in data]
    stream = torch.cuda.current_stream(dev)
    b = tv.BatchedSolver([tuple(i.shape) for i in imgs], dev)
    b.pack(imgs)
    tile, _ = b.autotune()
    kw = dict(lam=w["lam"], max_iter=w["max_iter"], check_every=w["check_every"],
              gap_tol=w["gap_tol"])
    b.solve(None, mode="persistent", **kw)
    ms_p, (_, res) = timed(lambda: b.solve(None, mode="persistent", **kw), stream, 3)
    ms_g, (_, res_g) = timed(lambda: b.solve(None, mode="graph", **kw), stream, 2)
    solvers = [tv.PlainSolver(tuple(i.shape), dev) for i in imgs]
    outs = [torch.empty_like(i) for i in imgs]

    def loop():
        return [s.solve(i, out=o, **kw)[1] for s, i, o in zip(solvers, imgs, outs)]
    loop()
    ms_l, res_l = timed(loop, stream, 2)
    work = sum(int(i.numel()) * r.iters for i, r in zip(imgs, res))
    log(f"batched: persistent {ms_p:.1f} ms, graph {ms_g:.1f} ms, plain loop {ms_l:.1f} ms")
    return {
        "workload": "batch64_uneven",
        "images": len(imgs),
        "pixels": int(sum(int(i.numel()) for i in imgs)),
        "pixel_iters": work,
        "iters_min_max": [min(r.iters for r in res), max(r.iters for r in res)],
        "all_converged": all(r.converged for r in res),
        "max_rel_gap": max(r.rel_gap for r in res),
        "tile": list(tile),
        "persistent_ms": ms_p,
        "graph_blocks_ms": ms_g,
        "plain_loop_ms": ms_l,
        "mpix_its_persistent": work / (ms_p * 1e-3) / 1e6,
        "mpix_its_graph_blocks": work / (ms_g * 1e-3) / 1e6,
        "mpix_its_plain_loop": work / (ms_l * 1e-3) / 1e6,
        "effective_GBs_persistent": BYTES_PER_PIXEL_ITER * work / (ms_p * 1e-3) / 1e9,
        "speedup_vs_plain_loop": ms_l / ms_p,
        "same_iters_as_plain": all(a.iters == c.iters for a, c in zip(res, res_l)),
        "per_image_h_w_iters": [[int(i.shape[0]), int(i.shape[1]), int(r.iters)]
                                for i, r in zip(imgs, res)],
    }


def bench_unrolled_2d(dev, plain_mpix):
    """32 x 512^2, K = 20 unrolled iterations: forward, and forward plus the
    adjoint backward (store-all: ckpt_every = K)."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, scene2d
    w = WORKLOADS["unrolled_32x512"]
    pairs = [scene2d(w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"] + i)
             for i in range(w["B"])]
    g = torch.from_numpy(np.stack([p[1] for p in pairs]).astype(np.float32)).to(dev)
    clean = torch.from_numpy(np.stack([p[0] for p in pairs]).astype(np.float32)).to(dev)
    K = w["K"]
    c = tv.default_coeffs(K, 2, 0.1, dev)
    stream = torch.cuda.current_stream(dev)
    s = tv.UnrolledSolver(tuple(g.shape), K, K, 1.0, dev)
    f = s.forward(g, c)
    grad_f = 2 * (f - clean) / f.numel()
    s.backward(c, grad_f)
    ms_f, _ = timed(lambda: s.forward(g, c), stream, 5)

    def fb():
        s.forward(g, c)
        return s.backward(c, grad_f)
    ms_fb, _ = timed(fb, stream, 5)
    work = int(g.numel()) * K
    log(f"unrolled 2d: fwd {ms_f:.2f} ms, fwd+bwd {ms_fb:.2f} ms")
    return {
        "workload": "unrolled_32x512",
        "batch": w["B"], "image": [w["H"], w["W"]], "K": K, "ckpt_every": K,
        "fwd_ms": ms_f, "fwd_bwd_ms": ms_fb,
        "mpix_its_fwd": work / (ms_f * 1e-3) / 1e6,
        "mpix_its_fwd_bwd": work / (ms_fb * 1e-3) / 1e6,
        "fwd_vs_plain_4096": (work / (ms_f * 1e-3) / 1e6 / plain_mpix
                              if plain_mpix else None),
        "fwd_bwd_vs_plain_4096": (work / (ms_fb * 1e-3) / 1e6 / plain_mpix
                                  if plain_mpix else None),
    }


def bench_unrolled_3d(dev):
    """256^3, K = 100, checkpoint every 10: forward and forward + backward,
    with the peak device memory."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, scene3d
    w = WORKLOADS["unrolled_256cube"]
    clean, noisy = scene3d(w["D"], w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g = torch.from_numpy(noisy[None].astype(np.float32)).to(dev)
    cl = torch.from_numpy(clean[None].astype(np.float32)).to(dev)
    del clean, noisy
    K = w["K"]
    c = tv.default_coeffs(K, 3, 0.1, dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    base = torch.cuda.memory_allocated(dev)
    s = tv.UnrolledSolver(tuple(g.shape), K, w["ckpt_every"], 1.0, dev)
    f = s.forward(g, c)
    grad_f = 2 * (f - cl) / f.numel()
    s.backward(c, grad_f)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated(dev)
    ms_f, _ = timed(lambda: s.forward(g, c), stream, 2)

    def fb():
        s.forward(g, c)
        return s.backward(c, grad_f)
    ms_fb, _ = timed(fb, stream, 2)
    work = int(g.numel()) * K
    log(f"unrolled 3d: fwd {ms_f:.1f} ms, fwd+bwd {ms_fb:.1f} ms, peak {peak / 2**30:.2f} GiB")
    return {
        "workload": "unrolled_256cube",
        "volume": [w["D"], w["H"], w["W"]], "K": K, "ckpt_every": w["ckpt_every"],
        "fwd_ms": ms_f, "fwd_bwd_ms": ms_fb,
        "mvox_its_fwd": work / (ms_f * 1e-3) / 1e6,
        "mvox_its_fwd_bwd": work / (ms_fb * 1e-3) / 1e6,
        "peak_device_memory_GiB": peak / 2 ** 30,
        "memory_before_GiB": base / 2 ** 30,
        "workspace_GiB": s.nbytes / 2 ** 30,
    }


def bench_plain_3d(dev):
    """The plain solver on the 256^3 volume of the unrolled workload: 100
    fused 3D iterations (gap every 10), 40 algorithmic bytes per
    voxel-iteration."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, scene3d
    w = WORKLOADS["unrolled_256cube"]
    _, noisy = scene3d(w["D"], w["H"], w["W"], w["n_shapes"], w["noise"], w["seed"])
    g = torch.from_numpy(noisy.astype(np.float32)).to(dev)
    del noisy
    shape = tuple(g.shape)
    solver = tv.PlainSolver(shape, dev)
    stream = torch.cuda.current_stream(dev)
    iters = 100
    s3 = 1.0 / math.sqrt(12.0)

    def run():
        return solver.solve(g, 0.1, tau=s3, sigma=s3, max_iter=iters,
                            check_every=10, gap_tol=-1.0)
    run()
    ms, _ = timed(run, stream, 3)
    vox = int(g.numel())
    gbs = 40 * vox * iters / (ms * 1e-3) / 1e9
    log(f"plain 3d: {ms:.1f} ms per {iters} iterations")
    return {
        "workload": "plain_256cube",
        "volume": list(shape), "iterations": iters, "gap_check_every": 10,
        "tile_th_tz_wpb": list(tv.get_tile3d(shape)),
        "ms": ms,
        "mvox_its": vox * iters / (ms * 1e-3) / 1e6,
        "algorithmic_bytes_per_voxel_iteration": 40,
        "achieved_GBs": gbs,
        "frac_of_peak": gbs / HBM_PEAK_GBS,
    }


# Algorithmic fp32 operations per (pixel, angle) pair: the backprojection
# interpolates once (fraction, one multiply-add) and accumulates, with the
# position advanced by one add; the projection (as the transpose) forms the
# position, the fraction and two hat-weighted multiply-adds.
TOMO_FLOPS_BP = 5
TOMO_FLOPS_PROJ = 6
FP32_VECTOR_PEAK_TFLOPS = 157.3


def bench_tomo(dev):
    """Reconstruction of a 2048^2 slice from 1000 projections of 2048 rays
    (TV regulariser): 20 iterations of the primal-dual method, the two
    operators on their own, the regularised filtered backprojection with the
    exact backprojection and through the slice theorem, and the
    backprojection by the slice theorem."""
    import torch
    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, tomo_scene
    w = WORKLOADS["tomo_2048x1000"]
    H, W, na, nd = w["H"], w["W"], w["n_angles"], w["n_det"]
    img, _, g = tomo_scene(H, W, na, nd, w["n_ellipses"], w["noise"], w["seed"])
    gt = torch.from_numpy(g.astype(np.float32)).to(dev)
    ft = torch.from_numpy(img.astype(np.float32)).to(dev)
    solver = tv.TomoSolver(H, W, na, nd, dev)
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    L2 = solver.opnorm_sq(20)
    opnorm_s = time.perf_counter() - t0
    tau, sr, sp = tv.default_steps(L2, "tv")
    lam = w["lam"]
    iters = w["iters"]
    sino = torch.empty_like(gt)
    back = torch.empty_like(ft)
    solver.radon(ft, sino)
    solver.backproject(gt, back)
    ms_radon, _ = timed(lambda: solver.radon(ft, sino), stream, 5)
    ms_bp, _ = timed(lambda: solver.backproject(gt, back), stream, 5)
    solver.fbp(gt, 0.0, back)
    ms_fbp, _ = timed(lambda: solver.fbp(gt, 0.0, back), stream, 5)
    solver.bst(gt, back)
    ms_bst, _ = timed(lambda: solver.bst(gt, back), stream, 5)
    solver.fbp_bst(gt, 0.0, back)
    ms_fbp_bst, _ = timed(lambda: solver.fbp_bst(gt, 0.0, back), stream, 5)
    solver.logpolar(gt, back)                    # plans the log-polar workspace
    ms_lp, _ = timed(lambda: solver.logpolar(gt, back), stream, 5)
    n_rho, n_phi, L_rho, _, _ = solver.lp_mesh()

    def run():
        solver.init()
        solver.step(gt, iters, lam, tau, sr, sp, reg="tv")
    run()
    ms, _ = timed(run, stream, 2)
    pairs = H * W * na
    e = solver.energy(gt, lam, "tv")
    log(f"tomo: {ms / iters:.3f} ms per iteration, A {ms_radon:.3f} ms, "
        f"A^T {ms_bp:.3f} ms, regularised FBP {ms_fbp:.3f} ms, BST {ms_bst:.3f} ms, "
        f"regularised FBP through the BST {ms_fbp_bst:.3f} ms, log-polar {ms_lp:.3f} ms")
    tf_bp = pairs * TOMO_FLOPS_BP / (ms_bp * 1e-3) / 1e12
    tf_proj = pairs * TOMO_FLOPS_PROJ / (ms_radon * 1e-3) / 1e12
    cnt = read_tomo_counters()
    # the two fast backprojections: the least HBM traffic a pipeline from the
    # sinogram to the image can have (read g once, write the image once), the
    # traffic its kernels measured, and the VALU issue they measured
    io_bytes = 4 * (na * nd + H * W)

    def pipeline(ms_run, kernels):
        rec = {"ms": ms_run, "kernels": kernels,
               "algorithmic_bytes": io_bytes,
               "algorithmic_frac": io_bytes / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if all(k in cnt for k in kernels):
            byt = sum(cnt[k].get("hbm_bytes", 0.0) for k in kernels)
            valu = sum(cnt[k].get("valu_wave_instr", 0.0) for k in kernels)
            rec["traffic"] = byt
            rec["hbm_frac"] = byt / (ms_run * 1e-3) / 1e9 / HBM_PEAK_GBS
            rec["valu_frac"] = valu / (ms_run * 1e-3) / VALU_PEAK_WAVE_INSTR_S
            rec["bound"] = "alu" if rec["valu_frac"] > rec["hbm_frac"] else "hbm"
            rec["frac"] = max(rec["valu_frac"], rec["hbm_frac"])
        return rec

    # A's units from its counters (A alone, the first instance): VALU issue
    # against one wave64 instruction per CU and clock, the LDS and the
    # texture path's busy fractions; the binding one is the busiest
    proj = cnt.get("tomo_project_kernel#1", {})
    proj_units = None
    if proj.get("valu_wave_instr"):
        valu_s = proj["valu_wave_instr"] / (ms_radon * 1e-3)
        proj_units = {
            "valu_wave_instr_s": valu_s,
            "valu_frac": valu_s / VALU_PEAK_WAVE_INSTR_S,
            "lds_busy": proj.get("lds_busy"),
            "lds_bank_conflict": proj.get("lds_bank_conflict"),
            "ta_busy": proj.get("ta_busy"),
            "td_busy": proj.get("td_busy"),
            "vmem_rd_wave_instr": proj.get("vmem_rd_wave_instr"),
            "basis": "rocprofv3 SQ_INSTS_VALU per launch over the live launch time against "
                     "256 CUs x 2.4 GHz; SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT and "
                     "TA/TD busy per CU-cycle of the counter run"}
        units = {"alu": proj_units["valu_frac"],
                 "lds": proj_units["lds_busy"] or 0.0,
                 "ta": proj_units["ta_busy"] or 0.0}
        proj_units["bound"] = max(units, key=units.get)
    return {
        "workload": "tomo_2048x1000",
        "image": [H, W], "n_angles": na, "n_det": nd, "reg": "tv", "lam": lam,
        "iterations": iters,
        "ms_per_iteration": ms / iters,
        "opnorm_sq": L2, "opnorm_20_steps_s": opnorm_s,
        "steps_tau_sigma_r_sigma_p": [tau, sr, sp],
        "energy_after": list(e),
        "radon_ms": ms_radon,
        "backproject_ms": ms_bp,
        "fbp_ms": ms_fbp,
        "bst_backproject_ms": ms_bst,
        "fbp_bst_ms": ms_fbp_bst,
        "logpolar_backproject_ms": ms_lp,
        "logpolar_mesh": {"n_rho": n_rho, "n_phi": n_phi, "L": L_rho},
        "bst_pipeline": pipeline(ms_bst, ["bst_spectra_kernel", "bst_cartesian_rows_kernel",
                                          "bst_transpose_kernel", "bst_rows_inverse_kernel",
                                          "bst_extract_kernel"]),
        "logpolar_pipeline": pipeline(ms_lp, ["lp_rows_forward_kernel",
                                              "lp_angle_conv_kernel",
                                              "lp_rows_inverse_kernel",
                                              "lp_cartesian_kernel"]),
        "projection_units": proj_units,
        "gpairs_per_s_radon": pairs / (ms_radon * 1e-3) / 1e9,
        "gpairs_per_s_backproject": pairs / (ms_bp * 1e-3) / 1e9,
        "roofline": {
            "bound": proj_units["bound"] if proj_units else "alu",
            "kernel": "tomo_project_kernel (A, with the padded-copy kernel in the timing)",
            "achieved": proj_units["valu_wave_instr_s"] / 1e12 if proj_units else None,
            "peak": VALU_PEAK_WAVE_INSTR_S / 1e12,
            "unit": "T wave64 VALU instructions/s",
            "frac": proj_units["valu_frac"] if proj_units else None,
            "flops_achieved_tflops": tf_proj,
            "flops_frac_of_fp32_peak": tf_proj / FP32_VECTOR_PEAK_TFLOPS,
            "flops_per_pixel_angle": TOMO_FLOPS_PROJ,
            "backprojection_achieved": tf_bp,
            "backprojection_frac": tf_bp / FP32_VECTOR_PEAK_TFLOPS,
            "backprojection_flops_per_pixel_angle": TOMO_FLOPS_BP,
            "traffic": None,
        },
    }


def copy_bandwidth(dev):
    """Bandwidth of the library's plain copy kernel over 2 x 256 MiB (read
    and write counted), the attainable HBM figure beside the 8 TB/s peak."""
    import ctypes
    import torch
    from paper_1608_03589_amd import _lib
    n = 64 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)
    args = (ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
            ctypes.c_int64(n), ctypes.c_void_p(stream.cuda_stream))
    _lib.call("tvpd_stream_copy", *args)
    ms, _ = timed(lambda: _lib.call("tvpd_stream_copy", *args), stream, 20)
    del a, b
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def copy_calibration(dev):
    """Five copies of 256 MiB by the library's plain copy kernel
    (tvpd_copy_kernel: reads 256 MiB, writes 256 MiB): a transfer of known
    size against which the HBM byte counters are scaled.  (The runtime's own
    device copy is no reference: its counters read between 0.28 and 0.5 of
    the bytes on different boxes, part of it apparently moved outside the
    shader caches.)"""
    import ctypes
    import torch
    from paper_1608_03589_amd import _lib
    n = 64 * 1024 * 1024  # 256 MiB of float32
    a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev).cuda_stream
    for _ in range(5):
        _lib.call("tvpd_stream_copy", ctypes.c_void_p(a.data_ptr()),
                  ctypes.c_void_p(b.data_ptr()), ctypes.c_int64(n), ctypes.c_void_p(stream))
    torch.cuda.synchronize()
    log("copy calibration: 5 plain copies of 256 MiB done")


EXTRA_WORKLOADS = {
    "denoise_256": lambda dev: bench_denoise_256(dev),
    "batch64_uneven": lambda dev: bench_batched(dev),
    "unrolled_32x512": lambda dev, ref: bench_unrolled_2d(dev, ref),
    "unrolled_256cube": lambda dev: bench_unrolled_3d(dev),
    "plain_256cube": lambda dev: bench_plain_3d(dev),
    "tomo_2048x1000": lambda dev: bench_tomo(dev),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=None,
                    help="iterations per step (default: the workload's 2000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-blocking", action="store_true",
                    help="one iteration per launch (no temporal blocking)")
    ap.add_argument("--depth", type=int, default=None,
                    help="longest pass in iterations per launch (default: the library's)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and unrolled workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size "
                         "(for scaling HBM counters)")
    ap.add_argument("--only", default=None,
                    choices=sorted(EXTRA_WORKLOADS),
                    help="run only this secondary workload and print its record "
                         "(for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1608_03589_amd as tv
    from scenes import WORKLOADS, scene2d

    if args.only:
        dev = torch.device("cuda:0")
        fn = EXTRA_WORKLOADS[args.only]
        rec = fn(dev, None) if args.only == "unrolled_32x512" else fn(dev)
        if args.copy_calibration:
            copy_calibration(dev)
        print(json.dumps(rec), flush=True)
        return

    w = WORKLOADS["denoise_4096"]
    iters = args.iters or w["iters"]
    H, W = w["H"], w["W"]
    log(f"generating {H}x{W} scene (seed {w['seed']})")
    _, g = scene2d(H, W, w["n_shapes"], w["noise"], w["seed"])
    g32 = g.astype(np.float32)
    dev = torch.device("cuda:0")
    tv.set_blocking(not args.no_blocking)
    if args.depth is not None and not args.no_blocking:
        tv.set_pass_depth(args.depth)
    gt = torch.from_numpy(g32).to(dev)
    out = torch.empty_like(gt)
    solver = tv.PlainSolver((H, W), dev)
    s = 1.0 / math.sqrt(8.0)
    lam = w["lam"]

    def step():
        return solver.solve(gt, lam, tau=s, sigma=s, max_iter=iters,
                            check_every=10, gap_tol=-1.0, out=out)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    res = None
    for i in range(args.steps):
        _, res = step()
        log(f"step {i + 1}/{args.steps} done (gap {res.gap:.4e}, rel {res.rel_gap:.3e})")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    pix = H * W
    mpix_its = pix * iters * args.steps / (ms_total * 1e-3) / 1e6
    # Dominant kernel: the fused sweep.  The solver runs the iterations as
    # passes of up to `depth` iterations per launch, a pass ending before the
    # next gap check (every 10 iterations); replay that schedule to count the
    # launches (with passes of 10: 200 launches per solve).
    depth = tv.pass_length((H, W))
    passes = pass_schedule(iters, 10, depth)
    launches = args.steps * len(passes)
    its_per_launch = iters / len(passes)
    launch_s = ms_total * 1e-3 / launches
    alg_bytes = BYTES_PER_PIXEL_ITER * pix * its_per_launch
    achieved = alg_bytes / launch_s / 1e9
    # what a launch itself must move: reads f^k, p^k (2), g, writes f^{k+n},
    # p^{k+n} (2), whatever n
    pass_bytes = PASS_BYTES_PER_PIXEL * pix
    pass_achieved = pass_bytes / launch_s / 1e9
    kernels = sorted(set(passes))
    tile = tv.get_tile((H, W))
    traffic = read_traffic(pix, tile) if kernels == [depth] else None
    valu = (read_sweep_profile(SQ_FILE, "valu_wave_instr_per_launch", tile)
            if kernels == [depth] else None)
    hbm_bound = {
        "achieved": pass_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": pass_achieved / HBM_PEAK_GBS,
        "algorithmic_bytes_per_launch": pass_bytes,
        "basis": "what a launch of n iterations must move: reads f^k, p^k (2), g, "
                 "writes f^{k+n}, p^{k+n} (2), 28 B per pixel",
    }
    alu_bound = None
    if valu:
        ach = valu * 64 / launch_s / 1e12
        alu_bound = {
            "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": ach / VALU_PEAK_TOPS,
            "valu_wave_instructions_per_launch": valu,
            "basis": "VALU instructions the kernel issues per launch (rocprofv3 "
                     "SQ_INSTS_VALU, overlap margins included) x 64 lanes, against one "
                     "wave64 instruction per CU and cycle (256 CUs, 2.4 GHz, no packed fp32)",
        }
    if traffic:
        hbm_bound["measured_traffic_frac"] = traffic / launch_s / 1e9 / HBM_PEAK_GBS
    copy_gbs = copy_bandwidth(dev)
    hbm_bound["copy_kernel_GBs"] = copy_gbs
    hbm_bound["frac_of_copy"] = pass_achieved / copy_gbs
    if traffic:
        hbm_bound["measured_traffic_frac_of_copy"] = traffic / launch_s / 1e9 / copy_gbs
    # The binding unit is the one closer to saturation, HBM judged on the bytes
    # the launch actually moves (halo re-reads included) when they are known;
    # the reported fraction stays the algorithmic one of that unit.
    hbm_use = hbm_bound.get("measured_traffic_frac", hbm_bound["frac"])
    binding = alu_bound if alu_bound and alu_bound["frac"] > hbm_use else hbm_bound

    if args.copy_calibration:
        copy_calibration(dev)

    extra = {}
    if not args.no_extra:
        # release the main workload's buffers so that the peak memory of the
        # unrolled workloads is theirs alone
        del solver, gt, out
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        extra["denoise_256"] = bench_denoise_256(dev)
        extra["batched"] = bench_batched(dev)
        extra["unrolled_2d"] = bench_unrolled_2d(dev, mpix_its)
        extra["unrolled_3d"] = bench_unrolled_3d(dev)
        extra["plain_3d"] = bench_plain_3d(dev)
        extra["tomo"] = bench_tomo(dev)

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu, t_cpu = cpu_baseline(g32.astype(np.float64), lam, s)
        cpu = {
            "value": pix * n_cpu / t_cpu / 1e6,
            "unit": "Mpixel-iters/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{n_cpu} iterations of the 4096x4096 workload, numpy "
                      f"float64, single thread ({cpu_model()}, "
                      f"{os.cpu_count()} cores visible)",
        }

    line = {
        "metric": "Mpixel-iters/s (fused primal-dual TV sweep, 4096^2, fraction of HBM roofline)",
        "value": mpix_its,
        "unit": "Mpixel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "denoise_4096",
            "image": [H, W],
            "iterations_per_step": iters,
            "gap_check_every": 10,
            "lam": lam,
            "tau_sigma": s,
            "tile": list(tv.get_tile((H, W))),
            "iterations_per_launch": its_per_launch,
            "pass_depth": depth,
        },
        "roofline": {
            "bound": "alu" if binding is alu_bound else "hbm",
            "achieved": binding["achieved"],
            "peak": binding["peak"],
            "unit": binding["unit"],
            "frac": binding["frac"],
            "bounds": {"hbm": hbm_bound, "alu": alu_bound},
            "binding_basis": ("the unit closer to saturation: VALU issue against HBM on the "
                              "measured traffic (the algorithmic bytes when no traffic "
                              "profile matches the sources)"),
            "one_pass_equivalent_GBs": achieved,
            "one_pass_equivalent_basis": (
                "32 B per pixel-iteration (one HBM pass per iteration): the bandwidth a "
                "kernel without temporal blocking would need for this throughput"),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_vs_algorithmic": (traffic / pass_bytes) if traffic else None,
            "hbm_achieved_GBs": (traffic / launch_s / 1e9) if traffic else None,
            "kernel": kernel_name(kernels, passes, tile[2] == 2),
            "pixel_iterations_per_launch": pix * its_per_launch,
            "algorithmic_bytes_per_launch": pass_bytes,
            "avg_launch_us": launch_s * 1e6,
        },
        "cpu_baseline": cpu,
        **extra,
        "final_rel_gap": res.rel_gap if res else None,
        "wall_s": wall,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
