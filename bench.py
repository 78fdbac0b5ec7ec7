"""Benchmark: wavelet-domain FISTA deblurring on one MI355X.

One step = one whole solve of the 1024x1024 workload (db4, 6 levels, rotating
6/1 Gaussian PSF field, Theta_K with 20 nnz per pixel = 20,971,520 entries,
noise 0.005, lambda = 5e-4): forward wavelet transform of the blurred image,
FISTA iterations (two fused sparse kernels each) until the float64 relative
duality gap, checked every 20 iterations, is at most 1e-4, and the synthesis
Psi x.  Theta_K and its Lipschitz constant are built on the GPU before timing
(the paper treats Theta_K as computed offline, Sec. 5.5); their cost is
reported separately.

Prints one JSON line.  ``value`` is FISTA iterations per second of the whole
job; ``roofline`` is for one FISTA iteration (the residual kernel and the
transposed kernel with its proximal epilogue) timed inside the solve with HIP
events on the stream it runs on; ``cpu_baseline`` times the FP64 oracle's
Alg. 1 on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def layout_desc(layout, tile_shape):
    slice_h, group = layout
    if group == 3:
        return {"kind": "tiled", "tile": "8x8 coefficients", "waves_per_tile": tile_shape[0],
                "groups_in_flight": tile_shape[1], "values": "kept" if tile_shape[2] else "dense"}
    if group == 1:
        return {"kind": "circulant"}
    if group > 0:
        return {"kind": "csr", "lanes_per_row": group}
    return {"kind": "sliced_ell", "slice": slice_h}


def kernel_label(layout, waves=4, unroll=2, kept=0):
    slice_h, group = layout
    if group == 3:
        vals = ("kept values with a row mask per code" if kept else
                "dense values, zeros where a row lacks a code")
        return (f"k_res_tl<{waves}, {unroll}, {'true' if kept else 'false'}>",
                f"r = Theta_K y - x0, float32 tiled pattern storage (8x8 coefficient tiles, {vals}, "
                f"{waves} wavefronts per tile, {unroll} groups of 4 codes in flight)")
    if group > 0:
        return f"k_res_csr<{group}>", f"r = Theta_K y - x0, float32 CSR, {group} lanes per row"
    return "k_res", f"r = Theta_K y - x0, float32 sliced-ELL, {slice_h} rows per slice"


KERNEL_SOURCES = ("paper_1512_08401_amd/csrc/solve.hip", "paper_1512_08401_amd/csrc/tiled.hip",
                  "paper_1512_08401_amd/csrc/codes.hpp", "paper_1512_08401_amd/csrc/common.hpp",
                  "paper_1512_08401_amd/csrc/prox.hpp")


def layout_key(layout, tile_shape):
    """Text key of the iteration layout, as the profile summaries record it."""
    if layout[1] == 3:
        return (f"tiled waves={tile_shape[0]} unroll={tile_shape[1]} "
                f"values={'kept' if tile_shape[2] else 'dense'}")
    return f"slice={layout[0]} group={layout[1]}"


BATCHED_SOURCES = ("paper_1512_08401_amd/csrc/batch.hip", "paper_1512_08401_amd/csrc/codes.hpp",
                   "paper_1512_08401_amd/csrc/common.hpp", "paper_1512_08401_amd/csrc/prox.hpp")


def profiled_traffic(workload, kernel, key, sources=KERNEL_SOURCES):
    """HBM bytes per launch of ``kernel`` (for "fista_iteration": per iteration,
    both kernels) from a committed rocprofv3 counter summary under profiles/
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when no summary was
    taken on these kernel sources, layout and workload."""
    import glob
    import hashlib
    dig = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            dig.update(f.read())
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        fields = dict(line.strip().split(": ", 1) for line in text.splitlines()
                      if line.startswith("    ") and ": " in line)
        if (fields.get("source_sha256") == dig.hexdigest() and fields.get("kernel") == kernel
                and fields.get("layout") == key
                and fields.get("workload") == workload and "traffic_bytes_per_launch" in fields):
            return int(fields["traffic_bytes_per_launch"])
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(wl, seconds: float = 12.0):
    """FP64 oracle Alg. 1 iterations per second on a bounded sample: the
    seeded full-size stand-in operator of the workload's size and non-zero
    count (the oracle cannot build this Theta_K in bench time), same lambda."""
    import scipy.sparse as sp
    import synth
    from oracle import fista
    N = wl.n * wl.n
    rp, cc, vv = synth.local_operator(wl.n, wl.levels, float(wl.nnz_per_px), seed=77)
    A = sp.csr_matrix((vv, cc, rp), shape=(N, N))
    x0 = np.random.default_rng(78).standard_normal(N)
    # step 1 / (||A||_1 ||A||_inf), a cheap upper bound of ||A||_2^2, so the sample converges
    aa = abs(A)
    lam, tau = wl.lam, 1.0 / (float(aa.sum(axis=0).max()) * float(aa.sum(axis=1).max()))
    fista.fista(A, x0, lam, tau, 1)   # warm one iteration, then run until the time budget is spent
    iters, t0 = 0, time.perf_counter()
    x = None
    while time.perf_counter() - t0 < seconds:
        x, _, _ = fista.fista(A, x0, lam, tau, 2, x_init=x)
        iters += 2
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 oracle FISTA iterations (scipy CSR, single-threaded) in {dt:.1f} s on a "
                      f"{N}x{N} seeded stand-in operator with {A.nnz} non-zeros (the workload's Theta_K has "
                      f"{wl.nnz}), built by synth.local_operator with the workload's size, levels and "
                      f"non-zeros per pixel",
            "host_cpu": cpu_model(), "host_threads_visible": os.cpu_count()}


def ev_pair(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def copy_ceiling(torch, mib=512, reps=10):
    """Device copy rate (read + write bytes per second) of a plain copy kernel
    over `mib` MiB, above the 256 MB Infinity Cache."""
    src = torch.ones(mib * 1024 * 1024 // 4, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = ev_pair(torch)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * src.numel() * 4 / t / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale1024")
    ap.add_argument("--tol", type=float, default=None, help="relative duality gap of a step (default: workload's)")
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance measurement")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel layout")
    ap.add_argument("--tile", default=None, metavar="W,U,K",
                    help="run the tiled layout with W wavefronts per tile, U code groups in flight and "
                         "K = 1 kept values (0 dense) instead of the autotuner's choice (profiling runs, "
                         "whose timing would perturb the autotuner)")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "learned", "conv", "tuned", "exact", "cnn"],
                    help="plain: the single-problem solve (default); batched / learned: the extension workloads")
    ap.add_argument("--train-images", type=int, default=4096)
    ap.add_argument("--heldout-images", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=64)
    ap.add_argument("--target-tol", type=float, default=1e-6,
                    help="relative duality gap of the warm-start training targets (learned form)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1512_08401_amd import wdb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.form != "plain":
        res = {"batched": run_batched, "learned": run_learned, "conv": run_conv, "tuned": run_tuned,
               "exact": run_exact, "cnn": run_cnn}[args.form](args)
        print(json.dumps(res), flush=True)
        return
    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS[args.workload]
    tol = wl.tol if args.tol is None else args.tol
    n, N = wl.n, wl.n * wl.n
    stream = torch.cuda.current_stream()

    # ---- inputs (seeded), observation u0 = H u + b blurred on the GPU
    field = wl.psf()
    u = torch.as_tensor(wl.image().astype(np.float32), device=dev)
    b = torch.as_tensor(wl.noise().astype(np.float32), device=dev)
    u0 = (wdb.blur(field, u) + b).reshape(-1).contiguous()

    # ---- offline: Theta_K and L
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = wdb.build_theta(field, wl.wavelet, wl.levels, wl.nnz)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    if args.tile:
        tw, tu, tk = (int(v) for v in args.tile.split(","))
        th.set_kernel_layout(th.info()["slice"], 3)
        th.set_tile_shape(tw, tu)
        th.set_tile_values(tk)
    elif not args.no_autotune:
        th.autotune(reps=10)
    layout = (th.info()["slice"], th.info()["group"])
    tile_shape = (th.info()["tile_waves"], th.info()["tile_unroll"], th.info()["tile_kept"])
    t_tune = time.perf_counter() - t0
    t0 = time.perf_counter()
    lip = th.lipschitz_info(synth.power_start(N, wl.power_seed))
    L = lip["L"]
    t_lip = time.perf_counter() - t0
    info = th.info()
    nnz = info["nnz"]
    log(f"Theta_K built in {t_build:.2f} s (nnz {nnz}, stored {info['stored']}), L = {L:.12f} "
        f"({lip}) in {t_lip:.2f} s")

    x = torch.empty(N, device=dev, dtype=torch.float32)
    img = torch.empty((n, n), device=dev, dtype=torch.float32)
    last = {}

    def step():
        _, inf = th.solve(u0, wl.lam, args.max_iters, check_every=20, tol=tol, out=x, use_graph=True)
        th.synthesize(x, out=img)
        last.update(inf)
        return inf["iters"]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = ev_pair(torch)
    t0 = time.perf_counter()
    ev0.record(stream)
    total_iters = 0
    for i in range(args.steps):
        total_iters += step()
        log(f"step {i + 1}/{args.steps}: {last['iters']} iterations, rel gap {last['rel_gap']:.3e}")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    value = total_iters / (ms_per_step * args.steps / 1e3)

    # ---- roofline: one FISTA iteration inside the solve.  Eagerly launched
    # iterations of the real solve (no checks in between), timed with HIP
    # events on the solve's stream at two iteration counts; the slope is the
    # time of one iteration (transform and final check cancel).
    def timed_solve(k):
        th.solve(u0, wl.lam, k, check_every=0, out=x)
        e0, e1 = ev_pair(torch)
        e0.record(stream)
        th.solve(u0, wl.lam, k, check_every=0, out=x)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3
    k1, k2 = 100, 1100
    it_us = (timed_solve(k2) - timed_solve(k1)) / (k2 - k1)
    # algorithmic bytes of one iteration: each product streams its non-zeros'
    # values and indices once (8 B each); the residual kernel reads y and c and
    # writes r (12 B per coefficient); the transposed kernel gathers r, reads
    # x, y and the float64 anchor and writes x and y (28 B per coefficient)
    it_bytes = 16 * nnz + 40 * N
    achieved = it_bytes / (it_us * 1e-6) / 1e9
    copy_gbs = copy_ceiling(torch)

    # ---- the residual kernel alone, back to back (its operator copy stays in
    # the Infinity Cache between launches at this size: a secondary figure)
    y = torch.randn(N, device=dev, dtype=torch.float32)
    r = torch.empty(N, device=dev, dtype=torch.float32)
    th.apply(y, u0, out=r, repeat=20)
    reps = args.kernel_reps
    k0e, k1e = ev_pair(torch)
    k0e.record(stream)
    th.apply(y, u0, out=r, repeat=reps)
    k1e.record(stream)
    torch.cuda.synchronize()
    k_us = k0e.elapsed_time(k1e) * 1e3 / reps
    kname, kdesc = kernel_label(layout, *tile_shape)
    lkey = layout_key(layout, tile_shape)
    traffic = profiled_traffic(wl.name, "fista_iteration", lkey)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"one FISTA iteration inside the solve: {kname} ({kdesc}) + the transposed kernel "
                          f"with the proximal epilogue",
                "iteration_us": round(it_us, 2), "algorithmic_bytes": it_bytes,
                "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "layout": layout_desc(layout, tile_shape), "layout_key": lkey,
                "cached_loop": {"kernel": kname, "kernel_us": round(k_us, 2),
                                "algorithmic_bytes": 8 * nnz + 12 * N,
                                "gbs": round((8 * nnz + 12 * N) / (k_us * 1e-6) / 1e9, 1),
                                "note": "the same residual launch repeated back to back"}}

    # ---- 16-bit values: iteration rate and kernel times
    half = {}
    for vt in ("f16", "bf16"):
        th.set_precision(vt)
        th.autotune(reps=10)
        hi = th.info()
        th.apply(y, u0, out=r, repeat=20)
        h0, h1 = ev_pair(torch)
        h0.record(stream)
        th.apply(y, u0, out=r, repeat=reps)
        h1.record(stream)
        torch.cuda.synchronize()
        hk_us = h0.elapsed_time(h1) * 1e3 / reps
        th.solve(u0, wl.lam, 200, check_every=20, out=x, use_graph=True)
        e0, e1 = ev_pair(torch)
        e0.record(stream)
        th.solve(u0, wl.lam, 1000, check_every=20, out=x, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        half[vt] = {"iters_per_s": round(1000 / (e0.elapsed_time(e1) / 1e3), 1),
                    "k_res_us_cached_loop": round(hk_us, 2),
                    "layout": ({"tiled": {"waves": hi["tile_waves16"], "unroll": hi["tile_unroll16"]}}
                               if hi["group16"] == 3 else {"packed_lanes_per_row": hi["group16"]})}
    th.set_precision("f32")
    th.autotune(reps=10)

    ttt = None if args.no_ttt else time_to_tolerance(th, u0, wl, torch, wdb, synth, N, tol)
    E, rel_gap = last["objective"], last["rel_gap"]
    out = {
        "metric": "FISTA iters/s", "value": round(value, 1), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {n}x{n} piecewise-smooth image, {wl.wavelet} {wl.levels} levels, "
                               f"{wl.field} PSF field {wl.field_args}, noise {wl.noise_sigma}, Theta_K "
                               f"{wl.nnz_per_px} nnz/px ({nnz}), lambda {wl.lam}; one step = transform + FISTA "
                               f"to float64 relative duality gap {tol:g} checked every 20 iterations + synthesis",
                   "n": n, "nnz": nnz, "tol_rel_gap": tol,
                   "iters_per_step": total_iters / args.steps},
        "solve_to_tolerance": {"reached": bool(rel_gap <= tol), "iters": last["iters"], "rel_gap": rel_gap,
                               "objective": E, "seconds": round(ms_per_step / 1e3, 4)},
        "spmv_gbps": round(achieved, 1),
        "offline": {"theta_build_s": round(t_build, 3), "lipschitz_s": round(t_lip, 3),
                    "autotune_s": round(t_tune, 3), "lipschitz": lip},
        "roofline": roofline,
        "sixteen_bit": half,
    }
    if ttt is not None:
        out["time_to_rel_objective"] = ttt
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


def time_to_tolerance(th, u0, wl, torch, wdb, synth, N, tol, targets=(1e-4, 1e-6, 1e-8), cap=600):
    """Iterations and seconds to rho_k = (E(x_k) - E*)/E(0) <= target for each
    form, E(0) = ||x0||^2/2 (the same normaliser for every form), plus the
    float32 forms' time to the workload's duality-gap stop.

    E* is the objective of a long preconditioned solve run to a relative
    duality gap of 1e-8 (so E* is known to within that gap).  For each form,
    k* is located from a run that checks the float64 objective after every
    iteration (up to `cap`), then a clean solve of k* iterations (forward
    transform included, one float64 check at the end) is timed with HIP
    events.  The 16-bit forms are scored with the float64 objective of the
    float32 operator, like the others."""
    x0 = wdb.dwt(u0, wl.wavelet, wl.levels)
    E0 = 0.5 * float(torch.dot(x0.double(), x0.double()))
    th.set_precond("spai_scale", start=synth.power_start(N, wl.power_seed))
    _, inf = th.solve(u0, wl.lam, 40000, check_every=100, precond=True, tol=1e-8, use_graph=True)
    Estar = inf["objective"]
    res = {"E_star": Estar, "E_star_rel_gap": inf["rel_gap"], "E_star_converged": inf["converged"],
           "E_star_iters": inf["iters"], "rho_uncertainty": inf["rel_gap"] * Estar / E0, "E0": E0,
           "normaliser": "E(0) = ||x0||^2/2", "trace_every": 1}
    stream = torch.cuda.current_stream()
    x = torch.empty(N, device=u0.device)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def clean(k, pre, **kw):
        th.solve(u0, wl.lam, k, check_every=k, precond=pre, out=x, use_graph=True, **kw)   # warm (graph capture)
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record(stream)
        _, fin = th.solve(u0, wl.lam, k, check_every=k, precond=pre, out=x, use_graph=True, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, fin

    forms = (("plain_f32", False, "f32"), ("spai_scale_f32", True, "f32"), ("plain_f16", False, "f16"),
             ("spai_scale_f16", True, "f16"), ("plain_bf16", False, "bf16"), ("spai_scale_bf16", True, "bf16"))
    for form, pre, vt in forms:
        th.set_precision(vt)
        if vt != "f32":
            th.autotune(reps=10)   # the fastest 16-bit layout for this operator
        _, tr = th.solve(u0, wl.lam, cap, check_every=1, precond=pre, trace_cap=cap)
        rho = (tr["trace"][:, 1] - Estar) / E0
        res[form] = {"best_rel_objective": float(rho.min()), "gap_at_cap": float(tr["trace"][-1, 2])}
        for target in targets:
            hit = np.nonzero(rho <= target)[0]
            key = f"{target:.0e}"
            if hit.size == 0:
                res[form][key] = {"reached": False, "iters_checked": cap}
                continue
            k = int(tr["trace"][hit[0], 0])
            secs, fin = clean(k, pre)
            res[form][key] = {"reached": True, "iters": k, "seconds": secs,
                              "rel_objective": (fin["objective"] - Estar) / E0}
        if vt == "f32":   # the workload's own stop: float64 relative duality gap <= tol, checked every 20
            _, st = th.solve(u0, wl.lam, 20000, check_every=20, tol=tol, precond=pre, out=x, use_graph=True)
            e0, e1 = ev(), ev()
            e0.record(stream)
            _, st = th.solve(u0, wl.lam, 20000, check_every=20, tol=tol, precond=pre, out=x, use_graph=True)
            e1.record(stream)
            torch.cuda.synchronize()
            res[form][f"gap_{tol:g}"] = {"reached": st["converged"], "iters": st["iters"],
                                         "seconds": e0.elapsed_time(e1) / 1e3, "rel_gap": st["rel_gap"]}
        log(f"time to tolerance, {form}: {res[form]}")
    th.set_precision("f32")
    th.set_precond("none")
    return res


def _observe(wdb, torch, field, n, seed, noise_seed, sigma):
    img = torch.as_tensor(__import__("synth").piecewise_image(n, seed).astype(np.float32), device="cuda")
    b = torch.as_tensor(__import__("synth").noise(n, sigma, noise_seed).astype(np.float32), device="cuda")
    return (wdb.blur(field, img) + b).reshape(-1).contiguous()


def run_batched(args):
    """64 problems: 8 operators of uneven size (128..1024), 8 right-hand sides each,
    per-problem lambda; time to relative objective 1e-4 for the whole batch in
    one batched call vs 64 single solves, on the same GPU."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb
    groups = synth.batched_problems(41)
    probs, meta = [], []
    t0 = time.perf_counter()
    total_nnz = 0
    for gi, g in enumerate(groups):
        n = g["n"]
        kind, kw = g["field"]
        field = synth.psf_isotropic(n, **kw) if kind == "isotropic" else synth.psf_rotating(n, **kw)
        th = wdb.build_theta(field, "db4", g["levels"], g["nnz_per_px"] * n * n)
        th.lipschitz_lanczos(synth.power_start(n * n, 1000 + gi))
        th.autotune(reps=5)
        total_nnz += th.info()["nnz"]
        for j in range(8):
            u0 = _observe(wdb, torch, field, n, g["seeds"][j][0] % 100000, g["seeds"][j][1] % 100000, 0.01)
            probs.append([th, u0, g["lams"][j]])
            meta.append((gi, n))
        log(f"group {gi}: n={n} levels={g['levels']} nnz/px={g['nnz_per_px']} field={kind}")
    t_setup = time.perf_counter() - t0
    # one batched iteration (both phases over all packs): slope between two
    # fixed-length runs without checks, and its algorithmic bytes: per pack the
    # operator's values and indices once per product (16 B per non-zero) and
    # 8 right-hand sides x 40 B per coefficient (as in a single iteration)
    packs = {}
    for p in probs:
        packs[id(p[0])] = p[0]
    alg = sum(16 * t.info()["nnz"] + 8 * 40 * t.N for t in packs.values())
    plain = [p[:3] for p in probs]
    ts = []
    for its in (100, 300):
        wdb.solve_batched(plain, its, check_every=0)
        e0, e1 = ev_pair(torch)
        e0.record()
        wdb.solve_batched(plain, its, check_every=0)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    it_us = (ts[1] - ts[0]) / 200 * 1e6
    ach = alg / (it_us * 1e-6) / 1e9
    ceil = copy_ceiling(torch)
    log(f"batched iteration {it_us:.1f} us, {ach:.0f} GB/s algorithmic")
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(ach / 8000.0, 4),
            "traffic": profiled_traffic("batched", "batched_iteration", "packs of 8", BATCHED_SOURCES),
            "kernel": "one batched iteration: k_res_batched + k_prox_batched over the 8 packs of 8",
            "iteration_us": round(it_us, 2), "algorithmic_bytes": alg,
            "copy_ceiling_gbs": round(ceil, 1), "frac_of_copy": round(ach / ceil, 3)}
    config = {"workload": "batched: 8 operators (n in {128,256,512,1024}, db4, levels log2(n)-4, "
                          "20-40 nnz/px) x 8 right-hand sides, lambda logU[1e-4,1e-2]",
              "total_nnz": total_nnz}
    if args.no_ttt:
        return {"metric": "batched FISTA iteration, 64 problems", "value": round(1e6 / it_us, 1),
                "unit": "batched iters/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
                "data": "synthetic", "config": config, "roofline": roof, "setup_s": round(t_setup, 2)}
    # E* per problem: long batched run to a relative gap of 1e-8
    xs, inf = wdb.solve_batched([p[:3] for p in probs], 40000, check_every=100, tol=1e-8, use_graph=True)
    E0 = []
    for i, p in enumerate(probs):
        x0 = wdb.dwt(p[1], "db4", p[0].info()["levels"])
        E0.append(0.5 * float(torch.dot(x0.double(), x0.double())))
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {}
    for target in (1e-4, 1e-6):
        # stop target per problem: (E - E*)/E(0) <= target
        tg = [inf[i]["objective"] + target * E0[i] for i in range(len(probs))]
        batch = [(p[0], p[1], p[2], None, tg[i]) for i, p in enumerate(probs)]
        wdb.solve_batched(batch, 20000, check_every=10, use_graph=True)
        e0, e1 = ev(), ev()
        e0.record()
        _, binf = wdb.solve_batched(batch, 20000, check_every=10, use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        t_batched = e0.elapsed_time(e1) / 1e3
        e0, e1 = ev(), ev()
        e0.record()
        single_iters = []
        for i, p in enumerate(probs):
            _, r = p[0].solve(p[1], p[2], 20000, check_every=10, use_graph=True, target=tg[i])
            single_iters.append(r["iters"])
        e1.record()
        torch.cuda.synchronize()
        t_single = e0.elapsed_time(e1) / 1e3
        res[f"{target:.0e}"] = {"batched_s": round(t_batched, 4), "single_solves_s": round(t_single, 4),
                                "speedup": round(t_single / t_batched, 2),
                                "iters_batched_mean": float(np.mean([r["iters"] for r in binf])),
                                "iters_single_mean": float(np.mean(single_iters)),
                                # per operator (pack of 8): the pack iterates until its slowest problem stops
                                "iters_by_operator": [[int(binf[8 * g + j]["iters"]) for j in range(8)]
                                                      for g in range(len(groups))]}
        log(f"target {target:.0e}: batched {t_batched:.3f} s, 64 single solves {t_single:.3f} s")
    return {"metric": "time to rel. objective 1e-4, 64 problems (batched vs single)",
            "value": res["1e-04"]["batched_s"], "unit": "s", "higher_is_better": False, "n_gpus": 1,
            "dtype": "f32", "data": "synthetic",
            "config": config,
            "targets": res, "E_star_converged": all(r["converged"] for r in inf), "setup_s": round(t_setup, 2),
            "roofline": roof}


def run_learned(args):
    """Warm start: train on solver-generated targets (4096 images solved to a
    relative duality gap of 1e-6), then iterations and time to relative
    objective 1e-4 / 1e-6 / 1e-8 on 512 held-out images from the prediction
    (network inference included) vs from zero, located at iteration
    resolution for 1e-4 (float64 check after every iteration).  Both timed
    forms start from the images: the warm form transforms the batch once and
    hands the coefficients to the network and to the solver, the zero form
    hands the images to the solver, which transforms them."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb, warmstart
    wl = synth.WORKLOADS["learned256"]
    n, J, lam = wl.n, wl.levels, wl.lam
    field = wl.psf()
    th = wdb.build_theta(field, wl.wavelet, J, wl.nnz)
    th.lipschitz_lanczos(synth.power_start(n * n, wl.power_seed))
    th.autotune(reps=5)
    ntrain = args.train_images
    t0 = time.perf_counter()
    U = [_observe(wdb, torch, field, n, 50000 + i, 150000 + i, wl.noise_sigma) for i in range(ntrain)]
    X0 = wdb.dwt_batched(torch.stack(U), wl.wavelet, J)
    T = torch.empty_like(X0)
    tgt_iters, tgt_conv = [], []
    for b in range(0, ntrain, 512):
        # targets: the solver's own solutions, to the stated relative duality gap
        _, inf = wdb.solve_batched([(th, u, lam) for u in U[b:b + 512]], 40000, check_every=100,
                                   tol=args.target_tol, use_graph=True,
                                   outs=[T[i] for i in range(b, min(ntrain, b + 512))])
        tgt_iters += [r["iters"] for r in inf]
        tgt_conv += [r["converged"] for r in inf]
        log(f"targets {min(ntrain, b + 512)}/{ntrain}: mean {np.mean(tgt_iters):.0f} iterations, "
            f"converged {sum(tgt_conv)}/{len(tgt_conv)}")
    t_targets = time.perf_counter() - t0
    del U
    net = wdb.Cnn(n, J, 32, seed=1)
    t0 = time.perf_counter()
    hist = warmstart.train(net, X0, T, args.epochs, 32, 1e-3, seed=2, log=log, final_lr=1e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    nh = args.heldout_images
    Uh = [_observe(wdb, torch, field, n, 60000 + i, 160000 + i, wl.noise_sigma) for i in range(nh)]
    Ub = torch.stack(Uh)
    X0h = wdb.dwt_batched(Ub, wl.wavelet, J)
    xstar, star = wdb.solve_batched([(th, u, lam) for u in Uh], 40000, check_every=100, tol=1e-8, use_graph=True)
    E0 = 0.5 * (X0h.double() ** 2).sum(dim=1).cpu().numpy()
    Xs = torch.stack(xstar)
    pred_h = net.predict(X0h.reshape(-1).contiguous()).reshape(nh, -1)
    mse = {"zero": float((Xs ** 2).mean()), "x0": float(((X0h - Xs) ** 2).mean()),
           "network": float(((pred_h - Xs) ** 2).mean())}
    log(f"held-out MSE to the solution: {mse}")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {}
    for target, every in ((1e-4, 1), (1e-6, 5), (1e-8, 10)):
        tgt = [star[i]["objective"] + target * E0[i] for i in range(nh)]
        out[f"{target:.0e}"] = {"check_every": every}
        for form in ("zero", "warm"):
            for rep in range(2):   # the first run captures the graph
                e0, e1 = ev(), ev()
                torch.cuda.synchronize()
                e0.record()
                if form == "warm":
                    # x0 = Psi^* u once for the batch, shared by the network and the solver
                    X0t = wdb.dwt_batched(Ub, wl.wavelet, J)
                    init = net.predict(X0t.reshape(-1)).reshape(nh, -1)
                    _, r = wdb.solve_batched([(th, X0t[i], lam, init[i], tgt[i]) for i in range(nh)], 40000,
                                             check_every=every, use_graph=every > 1, coeffs=True)
                else:
                    _, r = wdb.solve_batched([(th, Uh[i], lam, None, tgt[i]) for i in range(nh)], 40000,
                                             check_every=every, use_graph=every > 1)
                e1.record()
                torch.cuda.synchronize()
            out[f"{target:.0e}"][form] = {"seconds": e0.elapsed_time(e1) / 1e3,
                                          "iters_mean": float(np.mean([x["iters"] for x in r])),
                                          "iters_median": float(np.median([x["iters"] for x in r]))}
        o = out[f"{target:.0e}"]
        o["speedup"] = round(o["zero"]["seconds"] / o["warm"]["seconds"], 3)
        log(f"target {target:.0e}: zero {o['zero']}, warm {o['warm']}")
    return {"metric": "time to rel. objective 1e-4, held-out images (warm start vs zero)",
            "value": round(out["1e-04"]["warm"]["seconds"], 4), "unit": "s", "higher_is_better": False, "n_gpus": 1,
            "dtype": "f32 solver, bf16 network", "data": "synthetic",
            "config": {"workload": f"learned256: {n}x{n}, db4 {J} levels, isotropic 1..3 field, {wl.nnz} nnz, "
                                   f"lambda {lam}; {ntrain} training images solved to relative gap "
                                   f"{args.target_tol:g} / {nh} held-out images; {args.epochs} epochs"},
            "targets": out, "heldout_mse_to_solution": mse,
            "training_targets": {"iters_mean": float(np.mean(tgt_iters)), "converged": int(sum(tgt_conv)),
                                 "of": len(tgt_conv), "tol_rel_gap": args.target_tol},
            "E_star_converged": int(sum(r["converged"] for r in star)),
            # the relative duality gap bounds E* - E_min relative to E, hence the uncertainty of every rho
            "E_star_rel_gap_max": float(max(r["rel_gap"] for r in star)),
            "rho_uncertainty_max": float(max(r["rel_gap"] * r["objective"] / E0[i] for i, r in enumerate(star))),
            "train_loss_first_last": [hist[0], hist[-1]], "targets_s": round(t_targets, 2),
            "train_s": round(t_train, 2)}


def _solve_rate(th, u0, lam, iters, torch, steps=3):
    x = torch.empty_like(u0)
    th.solve(u0, lam, iters, check_every=20, out=x, use_graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        _, info = th.solve(u0, lam, iters, check_every=20, out=x, use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    return iters * steps / (e0.elapsed_time(e1) / 1e3), info


def run_conv(args):
    """Stationary blur (a convolution): the Theta build by the fast path of
    Alg. 3 against the column-by-column build, then the solve rate."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb
    n, J, sig, lam = 1024, 6, 5.0, 5e-4
    field = synth.psf_stationary(n, sig, sig)
    K = 20 * n * n
    out = {}
    for name, general in (("fast", "0"), ("general", "1")):
        os.environ["WDB_BUILD_GENERAL"] = general
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = wdb.build_theta(field, "db4", J, K)
        torch.cuda.synchronize()
        out[name] = {"build_s": round(time.perf_counter() - t0, 3), "threshold": th.info()["threshold"],
                     "conv_build": th.info()["conv_build"]}
        log(f"{name} build: {out[name]}")
        if name == "general":
            del th
    os.environ.pop("WDB_BUILD_GENERAL", None)
    th = wdb.build_theta(field, "db4", J, K)
    th.autotune(reps=5)
    th.lipschitz_lanczos(synth.power_start(n * n, 22))
    u0 = _observe(wdb, torch, field, n, 21, 22, 0.005)
    rate, info = _solve_rate(th, u0, lam, 500, torch)
    return {"metric": "Theta build time, stationary blur (Alg. 3 fast path)", "value": out["fast"]["build_s"],
            "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64 build, f32 solve",
            "data": "synthetic",
            "config": {"workload": f"conv1024: {n}x{n}, db4 {J} levels, isotropic Gaussian sigma {sig} at every "
                                   f"pixel, Theta_K 20 nnz/px ({K}), lambda {lam}"},
            "builds": out, "speedup": round(out["general"]["build_s"] / out["fast"]["build_s"], 2),
            "fista_iters_per_s": round(rate, 1), "layout": [th.info()["slice"], th.info()["group"]]}


def cnn_flops(n, levels, F=32):
    """Algorithmic FLOPs per image of the warm-start network: (inference,
    training step).  Per position of a stack with C channels the three
    convolutions cost 2*9*C*F, 2*9*F*F and 2*9*F*C; a training step runs the
    forward pass, the stack's recomputed first two convolutions, both
    gradients of the last two and the weight gradient of the first."""
    sides = [n >> levels] + [n >> l for l in range(levels, 0, -1)]
    chans = [1] + [3] * levels
    inf = train = 0
    for s, C in zip(sides, chans):
        c1, c2, c3 = 18 * C * F, 18 * F * F, 18 * F * C
        inf += s * s * (c1 + c2 + c3)
        train += s * s * (3 * c1 + 4 * c2 + 3 * c3)
    return inf, train


def run_cnn(args):
    """The warm-start network's kernels alone, on the learned workload's
    shapes (256x256 coefficients, 4 levels, 32 channels) with a batch of 32:
    K timed Adam training steps, then K timed inference passes, inputs resident
    in HBM.  Roofline: the convolutions' algorithmic FLOPs per step over the
    step time, against the float32 matrix-core peak (the hidden 32 -> 32
    layers run on f32 MFMA; the 1- and 3-channel layers on the vector units)."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb
    wl = synth.WORKLOADS["learned256"]
    n, J, B = wl.n, wl.levels, 32
    net = wdb.Cnn(n, J, 32, seed=1)
    gen = torch.Generator(device="cuda").manual_seed(11)
    x0 = 0.1 * torch.randn(B * n * n, device="cuda", generator=gen)
    tgt = x0 + 0.01 * torch.randn(B * n * n, device="cuda", generator=gen)
    pred = torch.empty_like(x0)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for _ in range(max(args.warmup, 1)):
        net.train_step(x0, tgt, 1e-4)
        net.predict(x0, out=pred)
    torch.cuda.synchronize()
    e0, e1, e2 = ev(), ev(), ev()
    e0.record()
    for _ in range(args.steps):
        net.train_step(x0, tgt, 1e-4)
    e1.record()
    for _ in range(args.steps):
        net.predict(x0, out=pred)
    e2.record()
    torch.cuda.synchronize()
    t_train = e0.elapsed_time(e1) / 1e3 / args.steps
    t_inf = e1.elapsed_time(e2) / 1e3 / args.steps
    f_inf, f_train = cnn_flops(n, J)
    ach = B * f_train / t_train / 1e12
    log(f"train step {t_train * 1e3:.3f} ms, inference {t_inf * 1e3:.3f} ms (batch {B})")
    return {"metric": "warm-start network training steps/s", "value": round(1.0 / t_train, 2), "unit": "steps/s",
            "higher_is_better": True, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(t_train * 1e3, 4), "dtype": "bf16 weights, f32 compute", "data": "synthetic",
            "config": {"workload": f"cnn256: {n}x{n} coefficients, {J} levels, 32 channels, batch {B}"},
            "inference_ms": round(t_inf * 1e3, 4), "images_per_s_inference": round(B / t_inf, 1),
            "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": 157.3, "unit": "TFLOP/s",
                         "frac": round(ach / 157.3, 4), "traffic": None,
                         "kernel": "whole training step (convolution FLOPs / step time)",
                         "flops_per_step": B * f_train},
            "inference_tflops": round(B * f_inf / t_inf / 1e12, 3)}


def run_tuned(args):
    """The paper's own tuning on the 512x512 workload: Symmlet 6, the weighted
    thresholding rule sigma = 2^-k and l1 weights w[i] = j(i), against the
    plain db4 / naive / uniform setup: build time, FISTA rate and time to a
    relative objective for each."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb
    wl = synth.WORKLOADS["precision512"]
    n, lam = wl.n, wl.lam
    field = wl.psf()
    u0 = _observe(wdb, torch, field, n, wl.image_seed, wl.noise_seed, wl.noise_sigma)
    res = {}
    for form, wav, J, rule, weights in (("plain", "db4", 5, "naive", "uniform"), ("tuned", "sym6", 5, "scale", "scale")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = wdb.build_theta(field, wav, J, wl.nnz, rule=rule)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        th.autotune(reps=5)
        th.lipschitz_lanczos(synth.power_start(n * n, wl.power_seed))
        th.set_l1_weights(weights)
        rate, _ = _solve_rate(th, u0, lam, 500, torch)
        x0 = wdb.dwt(u0, wav, J)
        E0 = 0.5 * float(torch.dot(x0.double(), x0.double()))
        _, star = th.solve(u0, lam, 6000, check_every=100, trace_cap=60)
        Estar = float(star["trace"][:, 1].min())
        _, tr = th.solve(u0, lam, 3000, check_every=10, trace_cap=300)
        rho = (tr["trace"][:, 1] - Estar) / E0
        hit = {f"{t:.0e}": (int(tr["trace"][np.nonzero(rho <= t)[0][0], 0]) if np.any(rho <= t) else None)
               for t in (1e-4, 1e-6, 1e-7)}
        res[form] = {"wavelet": wav, "rule": rule, "weights": weights, "build_s": round(t_build, 3),
                     "fista_iters_per_s": round(rate, 1), "iters_to_rel_objective": hit,
                     "layout": [th.info()["slice"], th.info()["group"]]}
        log(f"{form}: {res[form]}")
        del th
    return {"metric": "FISTA iters/s with the paper's tuning (Symmlet 6, sigma = 2^-k thresholding, w = j(i))",
            "value": res["tuned"]["fista_iters_per_s"], "unit": "iters/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"precision512 field and image, {wl.nnz} nnz, lambda {lam}"}, "forms": res}


def run_exact(args):
    """The exact-operator baseline against Theta_K on the 1024x1024 workload:
    time per iteration of Alg. 1 with the exact gradient Psi^* H^* (H Psi y - u0)
    and with Theta_K (the sparsification speed-up of the paper's Tables 1-2),
    and iterations / seconds to relative objective 1e-4 and 1e-6 for each
    problem against its own E* (float64 objective after every iteration)."""
    import torch
    import synth
    from paper_1512_08401_amd import wdb
    wl = synth.WORKLOADS[args.workload]
    n, N = wl.n, wl.n * wl.n
    field = wl.psf()
    u0 = _observe(wdb, torch, field, n, wl.image_seed, wl.noise_seed, wl.noise_sigma)
    th = wdb.build_theta(field, wl.wavelet, wl.levels, wl.nnz)
    th.autotune(reps=5)
    lt = th.lipschitz_lanczos(synth.power_start(N, wl.power_seed))
    ex = wdb.Exact(field, wl.wavelet, wl.levels)
    le = ex.lipschitz(synth.power_start(N, wl.power_seed))
    log(f"L: Theta_K {lt}, exact {le}")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    x = torch.empty(N, device="cuda")

    def per_iter(solve, k1, k2):
        ts = []
        for k in (k1, k2):
            solve(k)
            e0, e1 = ev(), ev()
            e0.record()
            solve(k)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        return (ts[1] - ts[0]) / (k2 - k1)

    ex_us = per_iter(lambda k: ex.solve(u0, wl.lam, k, check_every=0, out=x), 10, 60)
    th_us = per_iter(lambda k: th.solve(u0, wl.lam, k, check_every=0, out=x), 100, 1100)
    log(f"per iteration: exact {ex_us:.1f} us, Theta_K {th_us:.1f} us")
    x0 = wdb.dwt(u0, wl.wavelet, wl.levels)
    E0 = 0.5 * float(torch.dot(x0.double(), x0.double()))
    res = {}
    for name, solve, long_iters in (("theta_k", lambda k, **kw: th.solve(u0, wl.lam, k, out=x, **kw), 20000),
                                    ("exact", lambda k, **kw: ex.solve(u0, wl.lam, k, out=x, **kw), 3000)):
        _, star = solve(long_iters, check_every=100, trace_cap=long_iters // 100)
        Estar = float(star["trace"][:, 1].min())
        cap = 300
        _, tr = solve(cap, check_every=1, trace_cap=cap)
        rho = (tr["trace"][:, 1] - Estar) / E0
        r = {"E_star": Estar, "E_star_iters": long_iters, "best_rel_objective": float(rho.min())}
        for target in (1e-4, 1e-6):
            hit = np.nonzero(rho <= target)[0]
            if hit.size == 0:
                r[f"{target:.0e}"] = {"reached": False, "iters_checked": cap}
                continue
            k = int(tr["trace"][hit[0], 0])
            solve(k, check_every=k)
            e0, e1 = ev(), ev()
            e0.record()
            solve(k, check_every=k)
            e1.record()
            torch.cuda.synchronize()
            r[f"{target:.0e}"] = {"reached": True, "iters": k, "seconds": e0.elapsed_time(e1) / 1e3}
        res[name] = r
        log(f"{name}: {r}")
    return {"metric": "time per FISTA iteration, exact operator vs Theta_K (sparsification speed-up)",
            "value": round(ex_us / th_us, 2), "unit": "x", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32 (exact: float64 PSF weights)", "data": "synthetic",
            "config": {"workload": f"{wl.name}: {n}x{n}, {wl.wavelet} {wl.levels} levels, {wl.field} field "
                                   f"{wl.field_args}, Theta_K {wl.nnz} nnz, lambda {wl.lam}"},
            "exact_iteration_us": round(ex_us, 1), "theta_k_iteration_us": round(th_us, 2),
            "lipschitz": {"theta_k": lt, "exact": le}, "time_to_rel_objective": res}


def th_x0(th, u0, wl, wdb):
    return wdb.dwt(u0, wl.wavelet, wl.levels)


if __name__ == "__main__":
    main()
