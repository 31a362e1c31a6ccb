#!/usr/bin/env python3
"""Time to k eigenpairs at relative residual 1e-6 on one MI355X.

Workload (one "step" = one complete solve, every hot-path stage included):
  wells48_k512 -- 13-point periodic finite-difference Kohn-Sham Hamiltonian on
  a 48^3 grid (n = 110592, h = 0.5) with 32 seeded Gaussian wells, k = 512
  wanted pairs, sub-block width 16, 16 buffer vectors, Rayleigh-Ritz every 5
  iterations, Jacobi preconditioner, random N(0,1) start block, tol 1e-6.
Both precisions are timed: the mixed FP32-bulk path (the value reported) and
the plain FP64 path (reported beside it).  Inputs are resident in HBM before
the timed region starts.

Prints ONE JSON line.  --gpus N with N > 1 exits: the solver runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to k eigenpairs @ resid 1e-6 (s), mixed/batched vs plain FP64; HBM GB/s"
PEAK = {"hbm": 8000.0, "f64": 78.6, "f32": 157.3}   # GB/s, TFLOP/s (MI355X datasheet, dense)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for fn in sorted(os.listdir(os.path.join(ROOT, "paper_1407_7506_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1407_7506_amd", "csrc", fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


F32_KERNELS = ("gram_proj", "update_proj", "stencil_f32")


STAGES = ("gemm", "ax", "rr", "cholqr", "small_eig", "other")


def is_f32(name, precision):
    return precision == "mixed" and name in F32_KERNELS


def hbm_rates(kt, precision):
    """Achieved HBM rate (algorithmic bytes / device time) of every kernel
    kind whose compulsory bytes at 8 TB/s take longer than its flops at the
    dtype's dense peak (HBM-bound by its own intensity), with the counter
    rate where the committed traffic summary covers it."""
    out = {}
    for name, (ms, cnt, fl, by) in kt.items():
        if cnt == 0 or by <= 0 or ms <= 0:
            continue
        pf = PEAK["f32"] if is_f32(name, precision) else PEAK["f64"]
        if fl / (pf * 1e12) > by / (PEAK["hbm"] * 1e9):
            continue
        d = {"algorithmic_GBps": round(by / (ms * 1e-3) / 1e9, 1), "frac": round(by / (ms * 1e-3) / 1e9 / PEAK["hbm"], 4),
             "avg_launch_us": round(ms / cnt * 1e3, 2)}
        t = traffic_for(name, precision)
        if t is not None:
            d["counter_GBps"] = round(t * cnt / (ms * 1e-3) / 1e9, 1)
            d["traffic_over_algorithmic"] = round(t * cnt / by, 3)
        out[name] = d
    return out


def solve_roofline(info):
    """Whole-solve roofline fraction: sum over the modelled launches of
    max(bytes / 8 TB/s, flops / MFMA peak), divided by the solve's wall time
    (kernels without a model -- eigensolves, pencils, Cholesky -- count 0)."""
    if not info.get("roofline_ms"):
        return None
    meas = info["time_s"] * 1e3
    return {"roofline_ms": round(info["roofline_ms"], 2), "measured_ms": round(meas, 2),
            "frac": round(info["roofline_ms"] / meas, 4)}


def stage_ms(info):
    return {k: round(v, 2) for k, v in zip(STAGES, info["stage_ms"])}


def roofline(kt, precision):
    """Dominant kernel (largest device time among kernels with an algorithmic
    model), placed on the roofline by its own arithmetic intensity: MFMA-bound
    when its flops at the dtype's dense peak take longer than its compulsory
    bytes at the HBM peak, else HBM-bound."""
    best = None
    for name, (ms, cnt, fl, by) in kt.items():
        if cnt == 0 or (fl <= 0 and by <= 0):
            continue
        if best is None or ms > best[1]:
            best = (name, ms, cnt, fl, by)
    if best is None:
        return None
    name, ms, cnt, fl, by = best
    f32 = is_f32(name, precision)
    pflops = PEAK["f32"] if f32 else PEAK["f64"]
    t_flop = fl / (pflops * 1e12)
    t_byte = by / (PEAK["hbm"] * 1e9)
    if t_flop >= t_byte:
        achieved = fl / (ms * 1e-3) / 1e12
        out = {"bound": "mfma", "achieved": round(achieved, 2), "peak": pflops, "unit": "TFLOP/s",
               "frac": round(achieved / pflops, 4)}
    else:
        achieved = by / (ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm"], "unit": "GB/s",
               "frac": round(achieved / PEAK["hbm"], 4)}
    out.update({"kernel": name, "dtype": "f32" if f32 else "f64", "launches": cnt,
                "avg_launch_us": round(ms / cnt * 1e3, 2),
                "algorithmic_flops_per_launch": fl / cnt, "algorithmic_bytes_per_launch": by / cnt,
                "traffic": traffic_for(name, precision)})
    return out


def traffic_path(precision):
    return os.path.join(ROOT, "profiles", f"traffic_wells48_{precision}.json")


def traffic_for(name, precision):
    """HBM bytes per launch of the kernel in a solve of the given precision,
    from the committed rocprofv3 counter summary of that precision, if it was
    taken on the current kernel sources; else None."""
    path = traffic_path(precision)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != kernel_source_sha() or d.get("precision") != precision:
        return None
    k = d.get("kernels", {}).get(name)
    return None if k is None else k.get("hbm_bytes_per_launch")


# logical kernel name -> (symbol prefix, call-site template argument or None)
TRAFFIC_KERNELS = {
    "gram_proj": ("ppcg::gram", "1"), "update_proj": ("ppcg::update", "1"), "gram_block": ("ppcg::block_gram_kernel", None),
    "stencil_f64": ("ppcg::stencil_kernel<double", None), "stencil_f32": ("ppcg::stencil_kernel<float", None),
    "block_update": ("ppcg::block_update_kernel", None), "block_pencil": ("ppcg::block_pencil_kernel", None),
}


def _symbol_matches(sym, prefix, site):
    if sym.startswith("void "):
        sym = sym[5:]
    if not sym.startswith(prefix):
        return False
    if site is None:
        return True
    return sym.rstrip().endswith(f", {site}>(ppcg::GramArgs)") or sym.rstrip().endswith(f", {site}>(ppcg::UpdateArgs)")


def write_traffic(fetch_db, write_db, launches, precision, path=None):
    """profiles/traffic_wells48_<precision>.json from two rocprofv3 --pmc
    databases (FETCH_SIZE, WRITE_SIZE) of `bench.py --steps 1 --warmup 1
    --only <precision> --calib-copy --no-cpu-baseline`:
    per logical kernel, the mean HBM bytes per dispatch over the last
    `launches[name]` dispatches (the timed solve), each counter scaled by the
    bytes it reports for the 1 GiB device copy of the calibration step."""
    import sqlite3

    def load(db, counter):
        c = sqlite3.connect(db)
        rows = c.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                         "where counter_name = ? order by dispatch_id", (counter,)).fetchall()
        return rows

    out = {"source_sha": kernel_source_sha(), "precision": precision, "kernels": {}, "calibration": {},
           "command": ("two rocprofv3 runs from the repository root, one per counter: rocprofv3 --pmc FETCH_SIZE "
                       "(then WRITE_SIZE) -d <dir> -o run -- python3 bench.py --steps 1 --warmup 1 --only "
                       f"{precision} --calib-copy --no-cpu-baseline; reduced by python3 bench.py --traffic-from "
                       f"<FETCH_DB> <WRITE_DB> --traffic-precision {precision} --traffic-launches "
                       "<launches_per_solve of the profiled run>")}
    per = {}
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        rows = load(db, counter)
        # the calibration copy (1 GiB device-to-device, a runtime blit kernel):
        # the copy dispatch with the largest count
        cal = [r for r in rows if "copyBuffer" in r[1]]
        if not cal:
            raise SystemExit(f"{db}: no calibration copy dispatch found")
        top = max(cal, key=lambda r: r[3])
        measured = top[3] * 1024.0
        factor = float(1 << 30) / measured
        out["calibration"][counter] = {"kernel": top[1][:80], "KiB": top[3], "factor": factor}
        for name, (prefix, site) in TRAFFIC_KERNELS.items():
            ks = [r for r in rows if _symbol_matches(r[1], prefix, site)]
            n = launches.get(name, 0)
            if n <= 0 or len(ks) < n:
                continue
            ks = ks[-n:]
            per.setdefault(name, {})[counter] = factor * 1024.0 * sum(r[3] for r in ks) / n
    for name, d in per.items():
        if "FETCH_SIZE" in d and "WRITE_SIZE" in d:
            out["kernels"][name] = {"fetch_bytes_per_launch": d["FETCH_SIZE"], "write_bytes_per_launch": d["WRITE_SIZE"],
                                    "hbm_bytes_per_launch": d["FETCH_SIZE"] + d["WRITE_SIZE"],
                                    "launches": launches[name]}
    path = path or traffic_path(precision)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {path}: {sorted(out['kernels'])}")


def cpu_baseline(p, gpu_iters, iters):
    """The oracle as it stands, on the host cores, for `iters` iterations of the
    same workload; extrapolated to the GPU's iteration count."""
    import numpy as np
    from oracle import ppcg_ref, stencil
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    g = p.grid
    A = lambda X: stencil.apply_h(X, p.V, g.N, g.h, g.order)
    T = 1.0 / stencil.diag_h(p.V, g.h, g.order)
    X0 = p.start()
    t0 = time.perf_counter()
    try:
        ppcg_ref.ppcg(A, T, X0, p.k, p.q, p.tol, p.rr_period, max_iter=iters)
    except ppcg_ref.NoConvergence:
        pass
    dt = time.perf_counter() - t0
    per_it = dt / iters
    return {"value": round(per_it * gpu_iters, 2), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} oracle iterations of the same solve ({dt:.1f} s incl. set-up and "
                      f"{iters // p.rr_period} Rayleigh-Ritz), scaled to the GPU's {gpu_iters} iterations",
            "sample_s": round(dt, 2), "s_per_iter": round(per_it, 3)}


def bench_batch(args):
    """64 independent 7-point problems of uneven size (grids 24^3..40^3,
    k 32..256, sbsize 8, tol 1e-6, FP64): one lockstep batched solve vs the
    same problems solved one after another."""
    import numpy as np
    import torch
    from paper_1407_7506_amd import binding as B
    from paper_1407_7506_amd import inputs as I

    ps = I.batch64()[:args.nprob]
    probs = [dict(V=torch.tensor(p.V, device="cuda"), N=p.grid.N, k=p.k,
                  X0=torch.tensor(p.start(), device="cuda"), order=2) for p in ps]
    hb = B.Handle("fp64", profile=True)
    hs = B.Handle("fp64")
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        hb.solve_batched(probs, 8, 1e-6, 5)
        for p, pr in zip(ps, probs):
            hs.solve(pr["V"], pr["N"], p.k, 8, 1e-6, 5, pr["X0"])
    torch.cuda.synchronize()
    hb.reset_kernel_times()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = hb.solve_batched(probs, 8, 1e-6, 5)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        seq = [hs.solve(pr["V"], pr["N"], p.k, 8, 1e-6, 5, pr["X0"]) for p, pr in zip(ps, probs)]
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / args.steps
    err = max(float(((r[0] - s_[0]).abs().max() / s_[0].abs().max()).item()) for r, s_ in zip(res, seq))
    kt = hb.kernel_times()
    log(f"batched {tb:.3f} s, sequential {ts:.3f} s, speedup {ts / tb:.2f}")
    for name, (ms, cnt, fl, by) in sorted(kt.items(), key=lambda x: -x[1][0])[:10]:
        log(f"   {name:14s} {ms / args.steps:9.1f} ms/solve {cnt // args.steps:6d} launches")
    out = {
        "metric": METRIC, "value": round(tb, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tb * 1e3, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch64: {len(ps)} 7-point problems, grids 24^3..40^3, k 32..256, sbsize 8, "
                               "rr_period 5, tol 1e-6, FP64, one lockstep batched solve",
                   "nprob": len(ps), "n_total": int(sum(p.grid.n for p in ps)), "k_total": int(sum(p.k for p in ps))},
        "sequential_s": round(ts, 4), "speedup_batched_vs_sequential": round(ts / tb, 3),
        "batched_vs_sequential_max_err": err,
        "iters_max": max(r[2]["iters"] for r in res), "statuses_ok": all(r[3] == "PPCG_OK" for r in res),
        "roofline": roofline(kt, "fp64"),
    }
    print(json.dumps(out), flush=True)


def bench_bloch(args):
    """The 96^3 complex Hermitian workload (Bloch vector (2 pi 0.25 / L, 0, 0),
    smoothed random potential in [-2, 0], 13-point stencil, k = 2048,
    sbsize 32, nbuf 64): one complete solve per precision (complex64 bulk
    with complex128 master, and plain complex128), fixed kernel plans (no
    autotuner warmup solve: a solve takes minutes).  Progress goes to stderr
    every 10 iterations.  The oracle cannot run at this size on the host (one
    n x K complex128 block is 30 GB and it keeps about ten), so no
    cpu_baseline is reported."""
    import numpy as np
    import torch
    from paper_1407_7506_amd import binding as B
    from paper_1407_7506_amd import inputs as I

    p = I.bloch96()
    g = p.grid
    V = torch.tensor(p.V, device="cuda")
    torch.cuda.synchronize()
    results = {}
    precs = ["mixed", "fp64"] if args.only == "both" else [args.only]
    for prec in precs:
        def prog(r, prec=prec):
            if r["iter"] % 10 == 0 or r["kind"] == "final_rr_failed":
                log(f"  {prec} iter {r['iter']:4d} rho {r['rho']:.3e} locked {r['n_locked']:5d} "
                    f"t {r['time_s']:8.1f} s")
        h = B.Handle(prec, profile=True, max_iter=args.max_iter, log=prog, seed=203,
                     orth="skip" if args.orth_skip else "cholqr")
        # (n, K) complex128 start block, 30 GB: from the host generator, or drawn
        # on the device (Philox, seed 203) with --device-x0
        X0 = None if args.device_x0 else torch.tensor(p.start(), device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, X, info = h.solve(V, g.N, p.k, p.q, p.tol, p.rr_period, X0, h=g.h, order=g.order, kpt=g.kpt,
                               check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del X0, X
        torch.cuda.empty_cache()
        kt = h.kernel_times()
        results[prec] = {"s": dt, "info": info, "lam": lam.cpu().numpy(), "kt": kt}
        if args.save_lam:
            np.save(f"{args.save_lam}_{prec}.npy", results[prec]["lam"])
        log(f"{prec}: {dt:.1f} s, status {info['status']}, iters {info['iters']}, rr {info['n_rr']}, "
            f"resid {info['resid_final']:.3e}")
        for name, (ms, cnt, fl, by) in sorted(kt.items(), key=lambda x: -x[1][0])[:16]:
            log(f"   {name:14s} {ms:10.1f} ms {cnt:6d} launches {ms / max(cnt, 1):9.2f} ms/launch")
        h.close()
    main_prec = "mixed" if "mixed" in results else "fp64"
    r = results[main_prec]
    out = {
        "metric": METRIC, "value": round(r["s"], 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(r["s"] * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64+c128 (mixed)" if main_prec == "mixed" else "c128", "data": "synthetic",
        "config": {"workload": "bloch96_k2048: 13-point 96^3 periodic FD Hamiltonian with Bloch vector "
                               "(2 pi 0.25/L, 0, 0), smoothed N(0,1) potential in [-2, 0], k=2048, sbsize=32, "
                               "nbuf=64, rr_period=5, tol=1e-6, Jacobi, N(0,1) start",
                   "n": g.n, "k": p.k, "sbsize": p.q, "K": p.K, "precision": main_prec, "max_iter": args.max_iter,
                   "start_block": "device Philox seed 203" if args.device_x0 else "host N(0,1) seed 203",
                   "orth": "skip" if args.orth_skip else "cholqr"},
        "status": r["info"]["status"], "iters": r["info"]["iters"], "n_rr": r["info"]["n_rr"],
        "resid_final": r["info"]["resid_final"], "orth_err": r["info"]["orth_err"],
        "n_locked": r["info"]["n_locked"],
        "roofline": roofline(r["kt"], main_prec), "solve_roofline": solve_roofline(r["info"]),
        "stage_ms": stage_ms(r["info"]), "hbm": hbm_rates(r["kt"], main_prec),
        "cpu_baseline": None,
    }
    if "fp64" in results and "mixed" in results:
        lf, lm = results["fp64"]["lam"], results["mixed"]["lam"]
        out["fp64_s"] = round(results["fp64"]["s"], 3)
        out["fp64_status"] = results["fp64"]["info"]["status"]
        out["fp64_iters"] = results["fp64"]["info"]["iters"]
        out["fp64_stage_ms"] = stage_ms(results["fp64"]["info"])
        out["speedup_mixed_vs_fp64"] = round(results["fp64"]["s"] / results["mixed"]["s"], 3)
        out["mixed_vs_fp64_max_err"] = float(np.abs(lm - lf).max() / np.abs(lf).max())
    print(json.dumps(out), flush=True)


def bench_scf(args):
    """The SCF-style sequence on the 48^3 workload's operator family (section
    6 of the paper): 15 potentials V_s = V + 0.5 * 0.7^s * dV; the first is
    solved to tol 1e-6, each of the 14 others gets two PPCG iterations without
    Cholesky-QR, warm-started from the previous step's 528 Ritz vectors.
    Timed: the 14 warm steps (inputs in HBM).  Reported beside them: the cold
    first solve, and a full solve of the last potential for the eigenvalue
    error of the last step."""
    import numpy as np
    import torch
    from paper_1407_7506_amd import binding as B
    from paper_1407_7506_amd import inputs as I

    p = I.wells48()
    g = p.grid
    Vs = [torch.tensor(V, device="cuda") for V in I.scf_potentials(p, steps=14, amp=0.5, decay=0.7)]
    X0 = torch.tensor(p.start(), device="cuda")
    out = {}
    for prec in (["mixed", "fp64"] if args.only == "both" else [args.only]):
        first = B.Handle(prec, return_buffers=True, autotune=not args.no_autotune, profile=True)
        step = B.Handle(prec, max_iter=2, orth="none", return_buffers=True, autotune=not args.no_autotune,
                        profile=True)
        t0 = time.perf_counter()
        lam, X, info0 = first.solve(Vs[0], g.N, p.k, p.q, p.tol, p.rr_period, X0, h=g.h, order=g.order)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        # warmup of the step handle (autotuner), on the first potential
        step.solve(Vs[0], g.N, p.k, p.q, p.tol, p.rr_period, X, h=g.h, order=g.order, check=False)
        torch.cuda.synchronize()
        step.reset_kernel_times()
        t0 = time.perf_counter()
        infos = []
        for V in Vs[1:]:
            lam, X, info = step.solve(V, g.N, p.k, p.q, p.tol, p.rr_period, X, h=g.h, order=g.order, check=False)
            infos.append(info)
        torch.cuda.synchronize()
        t_steps = time.perf_counter() - t0
        ref, _, rinfo = first.solve(Vs[-1], g.N, p.k, p.q, p.tol, p.rr_period, X0, h=g.h, order=g.order)
        lk, rk = lam[:p.k].cpu().numpy(), ref[:p.k].cpu().numpy()
        err = float(np.abs(lk - rk).max() / np.abs(rk).max())
        stages = np.sum([i["stage_ms"] for i in infos], axis=0)
        log(f"{prec}: first solve {t_first:.3f} s ({info0['iters']} iters); 14 warm steps {t_steps:.3f} s "
            f"({t_steps / 14 * 1e3:.1f} ms/step); last-step eigenvalue error {err:.2e}")
        out[prec] = {"steps_s": round(t_steps, 4), "ms_per_step": round(t_steps / 14 * 1e3, 2),
                     "first_solve_s": round(t_first, 3), "first_iters": info0["iters"],
                     "last_step_err_vs_full_solve": err, "last_step_rho_status": infos[-1]["status"],
                     "cholqr_in_steps": int(sum(i["n_cholqr"] for i in infos)),
                     "stage_ms_steps": {k: round(v, 2) for k, v in zip(STAGES, stages)}}
        first.close()
        step.close()
    main_prec = "mixed" if "mixed" in out else "fp64"
    r = out[main_prec]
    line = {"metric": METRIC, "value": r["steps_s"], "unit": "s", "n_gpus": 1, "steps": 14, "warmup": 1,
            "ms_per_step": r["ms_per_step"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64 (mixed)" if main_prec == "mixed" else "f64", "data": "synthetic",
            "config": {"workload": "scf48: 15 potentials V_s = V_wells48 + 0.5*0.7^s*dV (dV smoothed field seed 106); "
                                   "first solved to tol 1e-6, then 14 warm-started steps of 2 PPCG iterations "
                                   "without Cholesky-QR (k=512, sbsize=16, K=528)", "precision": main_prec},
            "results": out, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def eig_error_bound(h, V, g, lam, X):
    """A-posteriori accuracy of a returned solve (after the timed region):
    per-column residuals r_i = H x_i - lambda_i x_i from a fresh float64
    stencil product, and the quadratic bound |lambda_i - exact| <=
    |r_i|^2 / gap_i, gap_i the distance to the nearest other returned value,
    over the columns whose gap exceeds 1e-3 max|lambda| (within a cluster the
    bound says nothing); errors relative to max|lambda|."""
    import numpy as np
    import torch
    Xcm = X.t().contiguous()
    Y = h.apply_h(V, g.N, Xcm, h=g.h, order=g.order)
    rn = torch.linalg.norm(Y - lam[:, None] * Xcm, dim=1).cpu().numpy()
    del Y, Xcm
    lv = lam.cpu().numpy()
    scale = float(np.abs(lv).max())
    d = np.abs(lv[:, None] - lv[None, :])
    np.fill_diagonal(d, np.inf)
    gap = d.min(axis=1)
    sel = gap > 1e-3 * scale
    quad = rn[sel] ** 2 / gap[sel]
    return {"max_col_resid_rel": float(rn.max() / scale),
            "quadratic_bound_rel": float(quad.max() / scale) if sel.any() else None,
            "columns_with_gap": int(sel.sum()), "columns": int(lv.size)}


def bench_library_gemm(args):
    """The projection's two products at the wells48 shape (n = 110592 rows,
    K = 528 columns of X, 2m = 472 columns of [W P]: the timed solve's mean
    active width) through the vendor BLAS: Gram X^T [W P] and update
    [W P] - X G, float32 and float64, 20 timed repetitions each after 3 untimed
    ones.  Not part of the solver: a reference rate for its own kernels."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    n, K, m2 = 110592, 528, 472
    out = {"library_gemm": "torch.matmul / addmm (hipBLASLt or rocBLAS as torch dispatches), no TF32",
           "shape": {"n": n, "K": K, "2m": m2}, "results": []}
    for dt, tag, peak in ((torch.float32, "f32", 157.3), (torch.float64, "f64", 78.6)):
        Xcm = torch.randn(K, n, device="cuda", dtype=dt)     # X, column-major n x K
        Wcm = torch.randn(m2, n, device="cuda", dtype=dt)    # [W P], column-major n x 2m
        G = torch.randn(K, m2, device="cuda", dtype=dt)
        ops = (("gram", lambda: Xcm @ Wcm.t()),
               ("update", lambda: torch.addmm(Wcm, G.t(), Xcm, alpha=-1.0)))
        for name, f in ops:
            for _ in range(3):
                f()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                f()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / 20 * 1e3
            tf = 2.0 * n * K * m2 / us / 1e6
            out["results"].append({"op": name, "dtype": tag, "us": round(us, 1), "TFLOP/s": round(tf, 2),
                                   "peak": peak, "frac": round(tf / peak, 4)})
        del Xcm, Wcm, G
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain device copy of 1 GiB (counter calibration under rocprofv3)")
    ap.add_argument("--workload", choices=["wells48", "batch64", "bloch96", "scf48"], default="wells48")
    ap.add_argument("--no-autotune", action="store_true",
                    help="fixed kernel plans instead of the autotuner's (tuning happens in the warmup solve)")
    ap.add_argument("--nprob", type=int, default=64, help="problems of the batch64 workload")
    ap.add_argument("--max-iter", type=int, default=20000, help="iteration cap (bloch96)")
    ap.add_argument("--device-x0", action="store_true", help="bloch96: start block drawn on the device")
    ap.add_argument("--save-lam", default="",
                    help="bloch96: write the eigenvalues of each precision's solve to <path>_<precision>.npy")
    ap.add_argument("--orth-skip", action="store_true",
                    help="bloch96: omit Cholesky-QR while |X^H X - I|_F <= 0.1 (section 5.5)")
    ap.add_argument("--library-gemm", action="store_true",
                    help="time the vendor BLAS (torch.matmul, no TF32) on the wells48 projection shapes, "
                         "print one JSON line and exit: a reference for the projection kernels' MFMA rate")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic_wells48_<precision>.json from two rocprofv3 --pmc databases "
                         "and exit (no GPU use)")
    ap.add_argument("--traffic-precision", choices=["fp64", "mixed"], default="mixed",
                    help="precision of the solve the counter databases were taken on")
    ap.add_argument("--traffic-launches", default="",
                    help="name=count,... launches per timed solve (from the bench run under the profiler)")
    args = ap.parse_args()
    if args.traffic_from:
        launches = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.traffic_launches.split(",") if "=" in kv}
        return write_traffic(args.traffic_from[0], args.traffic_from[1], launches, args.traffic_precision)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.library_gemm:
        return bench_library_gemm(args)
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "bloch96":
        return bench_bloch(args)
    if args.workload == "scf48":
        return bench_scf(args)

    import numpy as np
    import torch
    from paper_1407_7506_amd import binding as B
    from paper_1407_7506_amd import inputs as I

    p = I.wells48()
    g = p.grid
    V = torch.tensor(p.V, device="cuda")
    X0 = torch.tensor(p.start(), device="cuda")
    torch.cuda.synchronize()
    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    results = {}
    precs = ["mixed", "fp64"] if args.only == "both" else [args.only]
    for prec in precs:
        h = B.Handle(prec, profile=True, autotune=not args.no_autotune)
        for _ in range(args.warmup):
            h.solve(V, g.N, p.k, p.q, p.tol, p.rr_period, X0, h=g.h, order=g.order)
        torch.cuda.synchronize()
        h.reset_kernel_times()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            lam, X, info = h.solve(V, g.N, p.k, p.q, p.tol, p.rr_period, X0, h=g.h, order=g.order)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = h.kernel_times()
        tune = h.tune_report()
        if tune:
            log(f"autotuner decisions ({prec}):")
            for line in tune.splitlines():
                log("   " + line)
        results[prec] = {"s": dt / args.steps, "info": infos[-1], "lam": lam.cpu().numpy(), "kt": kt,
                         "tune_classes": len(tune.splitlines()),
                         "eig_bound": eig_error_bound(h, V, g, lam, X)}
        log(f"{prec}: {dt / args.steps:.3f} s/solve, iters {infos[-1]['iters']}, rr {infos[-1]['n_rr']}, "
            f"resid {infos[-1]['resid_final']:.3e}, stages {stage_ms(infos[-1])}")
        top = sorted(kt.items(), key=lambda x: -x[1][0])[:24]
        for name, (ms, cnt, fl, by) in top:
            log(f"   {name:14s} {ms / args.steps:9.1f} ms/solve {cnt // args.steps:6d} launches "
                f"{ms / max(cnt, 1) * 1e3:9.1f} us/launch")
        h.close()

    main_prec = "mixed" if "mixed" in results else "fp64"
    r = results[main_prec]
    kt = r["kt"]
    tot_ms = sum(v[0] for v in kt.values())
    out = {
        "metric": METRIC,
        "value": round(r["s"], 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["s"] * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (mixed)" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "wells48_k512: 13-point 48^3 periodic FD Hamiltonian, 32 seeded Gaussian wells, "
                               "k=512, sbsize=16, nbuf=16, rr_period=5, tol=1e-6, Jacobi, N(0,1) start",
                   "n": g.n, "k": p.k, "sbsize": p.q, "K": p.K, "rr_period": p.rr_period, "tol": p.tol,
                   "precision": main_prec},
        "iters": r["info"]["iters"],
        "n_rr": r["info"]["n_rr"],
        "resid_final": r["info"]["resid_final"],
        "orth_err": r["info"]["orth_err"],
        "roofline": roofline(kt, main_prec),
        "solve_roofline": solve_roofline(r["info"]),
        "stage_ms": stage_ms(r["info"]),
        "eig_bound": r["eig_bound"],
        "hbm": hbm_rates(kt, main_prec),
        "kernel_share": {k: round(v[0] / tot_ms, 4) for k, v in sorted(kt.items(), key=lambda x: -x[1][0])[:8]},
        "launches_per_solve": {k: v[1] // args.steps for k, v in kt.items() if k in TRAFFIC_KERNELS},
        "autotune": {"enabled": not args.no_autotune, "shape_classes": r["tune_classes"],
                     "note": "candidates timed during the warmup solve; timed solves use the chosen plans"},
    }
    if "fp64" in results and "mixed" in results:
        lf, lm = results["fp64"]["lam"], results["mixed"]["lam"]
        rf = results["fp64"]
        out["fp64_s"] = round(rf["s"], 4)
        out["fp64_iters"] = rf["info"]["iters"]
        out["speedup_mixed_vs_fp64"] = round(rf["s"] / results["mixed"]["s"], 3)
        out["mixed_vs_fp64_max_err"] = float(np.abs(lm - lf).max() / np.abs(lf).max())
        out["eig_bound_fp64"] = rf["eig_bound"]
        out["roofline_fp64"] = roofline(rf["kt"], "fp64")
        out["solve_roofline_fp64"] = solve_roofline(rf["info"])
        out["stage_ms_fp64"] = stage_ms(rf["info"])
        out["hbm_fp64"] = hbm_rates(rf["kt"], "fp64")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, r["info"]["iters"], args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
