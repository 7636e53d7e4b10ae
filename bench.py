"""Benchmark of the contour-deformation G0W0 hot path on one MI355X.

Workload: the (H2O)10-shaped G0W0 problem (n_occ=50, n_virt=380, N_aux=1120,
64-point modified Gauss-Legendre grid, QP energies of HOMO-4..LUMO+4),
synthetic seeded inputs resident in HBM before timing starts.

One step = one gw_qp call with the W^c table cache dropped first, i.e. the
whole hot path: Pi(i xi) build on every grid point, Cholesky of 1 - Pi,
W^c table, imaginary-axis Sigma quadrature, batched MINRES residues and the
QP step tree, for all 10 states.  The headline value is the mixed-precision
path (BF16x3 Pi build and BF16x3 W^c contraction); the BF16x3-Pi-only path,
the plain FP64 path and the FP32 Pi path are timed the same way and reported
beside it, each with its error against the FP64 oracle's stored QP energies.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
# timed paths: name -> context options (Pi build precision, W^c contraction)
PATHS = {"bf16x3w": dict(pi_prec="bf16x3", wc_prec="bf16x3"),
         "bf16x3": dict(pi_prec="bf16x3", wc_prec="fp64"),
         "fp64": dict(pi_prec="fp64", wc_prec="fp64"),
         "fp32": dict(pi_prec="fp32", wc_prec="fp64")}
DTYPES = {"bf16x3w": "bf16x3 Pi and W^c (fp32 acc) + f64", "bf16x3": "bf16x3 Pi (fp32 acc) + f64",
          "fp64": "f64", "fp32": "f32 Pi + f64"}
MEV = 1e-3 / 27.211386245988


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pi_flops(n_aux, n_ov, G):
    """Algorithmic flops of the Pi build: N_aux (N_aux + 1) N_ov per grid point
    (the symmetric product counted once, multiply and add each one flop)."""
    return n_aux * (n_aux + 1) * n_ov * G


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter
    record, or None when the record is missing or the kernel's source file has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_h2o10_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["hbm_fetch_bytes"] + rec["hbm_write_bytes"]


def time_path(gwl, inp, states, grid, path, steps, warmup):
    import numpy as np
    import torch
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    c = gwl.Context.from_inputs(inp, qp_tol=1e-10, **PATHS[path])
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_setup)   # host -> HBM upload and setup
    with c:
        for _ in range(warmup):
            c.reset_cache()
            out = c.qp(states, grid)
        torch.cuda.synchronize()
        pi_ms, tot_ms, stages, each = [], [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            c.reset_cache()
            out = c.qp(states, grid)
            each.append(1e3 * (time.perf_counter() - t1))
            t = c.timing()
            pi_ms.append(t["pi_ms"])
            tot_ms.append(t["total_ms"])
            stages.append(t)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # the same call with the W^c table kept (a second molecule-independent
        # number: QP energies only, stage A cached)
        cached = []
        for _ in range(max(3, steps // 2)):
            t1 = time.perf_counter()
            c.qp(states, grid)
            cached.append(1e3 * (time.perf_counter() - t1))
    E = out[0]
    return dict(E=E, Z=out[2], status=out[3], wall_s=wall, ms_per_step=1e3 * wall / steps,
                median_ms=float(np.median(each)), p99_ms=float(np.percentile(each, 99)),
                setup_ms=setup_ms,
                cached_ms=float(np.median(cached)),
                pi_ms=float(np.mean(pi_ms)), total_ms=float(np.mean(tot_ms)),
                stages={k: float(np.mean([s[k] for s in stages])) for k in stages[0]})


def time_evgw(gwl, inp, states, grid, path, reps=2, n_cycles=3):
    """evGW0 and evGW, n_cycles cycles each, on the same workload: wall time
    per call (W^c built inside the call), QP rounds, and the last cycle's
    energies."""
    import numpy as np
    import torch
    out = {}
    with gwl.Context.from_inputs(inp, qp_tol=1e-10, **PATHS[path]) as c:
        for mode in ("evgw0", "evgw"):
            each, rounds = [], []
            for _ in range(reps + 1):        # the first call warms up
                c.reset_cache()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                E, S, Z, st, hist = c.evgw(states, grid, mode=mode, n_cycles=n_cycles)
                torch.cuda.synchronize()
                each.append(1e3 * (time.perf_counter() - t1))
                t = c.timing()
                rounds.append(t["qp_rounds"])
            out[mode] = dict(ms_per_call=float(np.median(each[1:])), cycles=int(hist.shape[0]),
                             qp_rounds=int(rounds[-1]), hist=hist, status=st,
                             stages={k: round(float(v), 3) for k, v in t.items()})
    return out


def time_core_spectrum(gwl, path, reps=2):
    """Every core level of the (H2O)20-shaped input (20 states, ~100 residue
    systems each per QP round), plain and with the cluster initial-guess
    layer; W^c table cached after the first call, so the calls time the QP
    stage (batched FP64 MINRES).  State 0 is checked against its oracle
    fixture."""
    import numpy as np
    import torch
    import gwgen
    cfg = gwgen.CONFIGS["h2o20_core"]
    n_core = 20
    inp = gwgen.make_inputs(cfg.shape, cfg.seed, list(range(n_core)))
    grid = gwl.Grid.gauss_legendre(cfg.grid_points)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "h2o20_core.json")))
    out = {"workload": f"(H2O)20-shaped, all {n_core} core levels: n_occ={cfg.shape.n_occ}, "
                       f"n_virt={cfg.shape.n_virt}, N_aux={cfg.shape.n_aux}, "
                       f"{cfg.grid_points}-point grid, seed {cfg.seed}", "path": path}
    for width in (0.0, 0.5):
        with gwl.Context.from_inputs(inp, qp_tol=1e-10, cluster_width=width,
                                     **PATHS[path]) as c:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            E, S, Z, st = c.qp(list(range(n_core)), grid)
            torch.cuda.synchronize()
            first = 1e3 * (time.perf_counter() - t1)
            each = []
            for _ in range(reps):
                t1 = time.perf_counter()
                E, S, Z, st = c.qp(list(range(n_core)), grid)
                torch.cuda.synchronize()
                each.append(1e3 * (time.perf_counter() - t1))
            t = c.timing()
        key = "clusters" if width > 0 else "plain"
        out[key] = {"cluster_width": width, "ms_first_call": round(first, 1),
                    "ms_cached_wtable": round(float(np.median(each)), 1),
                    "qp_per_s_cached_wtable": round(n_core / (np.median(each) / 1e3), 2),
                    "qp_rounds": t["qp_rounds"], "minres_systems": t["minres_systems"],
                    "minres_iters": t["minres_iters"], "minres_ms": round(t["minres_ms"], 1),
                    "status_nonzero": int(np.count_nonzero(st)),
                    "state0_err_mev_vs_oracle": float(abs(E[0] - gold["results"][0]["E"]) / MEV)}
        log(f"bench: core spectrum {key}: {json.dumps(out[key])}")
    return out


def crossover(gwl, ks, reps=3):
    """Spectral-decomposition route against contour deformation on the GPU
    for (H2O)_k-shaped inputs (HOMO and LUMO, 64-point grid for CD): wall
    time of a first call (decomposition or W^c table built inside) and of a
    cached call, per route."""
    import numpy as np
    import torch
    import gwgen
    rows = []
    for k in ks:
        shape = gwgen.cluster_shape(k)
        states = [shape.n_occ - 1, shape.n_occ]
        inp = gwgen.make_inputs(shape, 100 + k, states)
        grid = gwl.Grid.gauss_legendre(64)
        row = {"k": k, "n_ov": shape.n_ov, "n_aux": shape.n_aux}
        E = {}
        for route in ("sd", "cd_fp64", "cd_bf16x3"):
            prec = "bf16x3" if route == "cd_bf16x3" else "fp64"
            with gwl.Context.from_inputs(inp, pi_prec=prec, qp_tol=1e-10) as c:
                call = (lambda: c.qp_sd(states)) if route == "sd" else (lambda: c.qp(states, grid))
                times = []
                for rep in range(reps + 1):
                    if rep > 0:
                        c.reset_cache()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    out = call()
                    torch.cuda.synchronize()
                    times.append(1e3 * (time.perf_counter() - t1))
                t0 = time.perf_counter()
                call()
                torch.cuda.synchronize()
                cached = 1e3 * (time.perf_counter() - t0)
                tm = c.timing()
            E[route] = out[0]
            row[route] = {"ms": round(float(np.median(times[1:])), 3), "ms_cached": round(cached, 3)}
            if route == "sd":
                c2 = gwl.Context.from_inputs(inp)
                c2.qp_sd(states)
                row[route]["jacobi_sweeps"] = c2.timing()["sd_sweeps"]
                c2.close()
        row["max_abs_diff_sd_cd_fp64"] = float(np.max(np.abs(E["sd"] - E["cd_fp64"])))
        rows.append(row)
        log(f"bench: crossover k={k}: {json.dumps(row)}")
    return rows


def cpu_baseline(inp, states, G, gold):
    """Oracle timed on a bounded sample of the same workload (about 15 s of
    host work): the W^c table on three of the grid points (first, middle,
    last) and one Sigma^c evaluation (with its residues) each of the HOMO and
    the LUMO at their QP energies, scaled to the whole workload with the
    oracle's own iteration counts."""
    import numpy as np
    from oracle import cd, grid as ogrid
    try:
        from threadpoolctl import threadpool_info
        cores = max((i.get("num_threads", 1) for i in threadpool_info()), default=os.cpu_count())
    except Exception:
        cores = os.cpu_count()
    xi, z = ogrid.gauss_legendre(G)
    picks = sorted({0, G // 2, G - 1})
    t0 = time.perf_counter()
    for g in picks:
        cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi[g:g + 1])
    t_g = (time.perf_counter() - t0) / len(picks)
    homo = inp.n_occ - 1
    wt = np.zeros((inp.shape.n_mo, G))
    t_ev, nres = [], []
    for n in (homo, homo + 1):
        r = list(inp.row_ids).index(n)
        w = gold["results"][states.index(n)]["E"]
        t0 = time.perf_counter()
        _, _, k = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[r], wt, xi, z, w)
        t_ev.append(time.perf_counter() - t0)
        nres.append(k)
    t_eval = float(np.mean(t_ev))
    n_evals = sum(x["iters"] for x in gold["results"])
    total = G * t_g + n_evals * t_eval
    return {"value": len(states) / total, "unit": "QP energies/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"W^c table on {len(picks)} of {G} grid points ({t_g:.1f} s each) + one "
                       f"Sigma^c evaluation each of the HOMO and LUMO at their QP energies with "
                       f"{nres[0]} and {nres[1]} residues ({t_eval:.1f} s each); scaled to {G} grid "
                       f"points and {n_evals} evaluations"),
            "est_total_s": total}


def serve_bench(args):
    """Serving workload: water clusters of k ~ U{1..24} molecules (HOMO-2..LUMO+2,
    64-point grid) through gw_server.  Phase 1: closed loop with 8 requests
    outstanding, FP64 and the mixed form (BF16x3 Pi and W^c) -> saturated
    throughput of each.  Phase 2:
    Poisson arrivals at 0.8 x the FP64 saturated rate, for both paths ->
    throughput, p50 / p99 latency (done - submit) and the per-request energy
    difference between the paths."""
    import threading

    import numpy as np
    import gwgen
    import paper_2107_10423_amd as gwl

    stream = gwgen.serving_stream(n_requests=args.requests, k_max=args.kmax, seed=5000, rate=1.0)
    cache = {}
    log(f"serve: generating inputs for {len(set(r['k'] for r in stream))} cluster sizes")
    for r in stream:
        if r["k"] not in cache:
            cache[r["k"]] = gwgen.serving_inputs(r["k"], 1000 + r["k"])
    grid = gwl.Grid.gauss_legendre(64)

    def run(prec, arrivals, window=None):
        srv = gwl.Server(grid, n_streams=args.streams, **PATHS[prec])
        tickets, E = {}, {}
        lat, done_t, sub_t = [], [], []
        lock = threading.Lock()
        outstanding = threading.Semaphore(window) if window else None
        t0 = time.perf_counter()

        def producer():
            for i, r in enumerate(stream):
                if arrivals is not None:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                if outstanding:
                    outstanding.acquire()
                inp = cache[r["k"]]
                tk = srv.submit_inputs(inp, list(inp.row_ids))
                with lock:
                    tickets[tk] = i

        th = threading.Thread(target=producer)
        th.start()
        n_done = 0
        while n_done < len(stream):
            with lock:
                items = list(tickets.items())
            progressed = False
            for tk, i in items:
                out = srv.poll(tk)
                if out is None:
                    continue
                progressed = True
                with lock:
                    del tickets[tk]
                if outstanding:
                    outstanding.release()
                info = out[4]
                if info["rc"] != 0:
                    raise RuntimeError(f"request {i} failed with {info['rc']}")
                E[i] = out[0]
                lat.append(info["t_done"] - info["t_submit"])
                done_t.append(info["t_done"])
                sub_t.append(info["t_submit"])
                n_done += 1
                if n_done % 16 == 0:
                    log(f"serve: {prec}: {n_done}/{len(stream)} done")
            if not progressed:
                time.sleep(0.002)
        th.join()
        st = srv.stats()
        srv.close()
        span = max(done_t) - min(sub_t)
        lat = np.array(lat)
        return dict(E=E, span_s=span, req_per_s=len(stream) / span,
                    qp_per_s=sum(len(cache[r["k"]].row_ids) for r in stream) / span,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), peak_active=st["peak_active"],
                    peak_reserved_gb=st["peak_reserved_bytes"] / 2**30)

    sat = {}
    for prec in ("fp64", "bf16x3w"):
        log(f"serve: phase 1, {prec} closed loop (8 outstanding)")
        sat[prec] = run(prec, None, window=8)
    lam = 0.8 * sat["fp64"]["req_per_s"]
    arr = np.array([r["arrival_s"] for r in stream]) / lam
    res = {}
    for prec in ("fp64", "bf16x3w"):
        log(f"serve: phase 2, {prec}, Poisson arrivals at {lam:.2f} req/s")
        res[prec] = run(prec, arr)
    dE = max(float(np.max(np.abs(res["bf16x3w"]["E"][i] - res["fp64"]["E"][i])))
             for i in range(len(stream)))
    pick = lambda r: {k: (round(v, 4) if isinstance(v, float) else v)
                      for k, v in r.items() if k != "E"}
    out = {"metric": "serving: QP energies/s (saturated) and p50/p99 latency at a fixed Poisson "
                     "rate, mixed (BF16x3 Pi and W^c) vs FP64",
           "value": round(sat["bf16x3w"]["qp_per_s"], 3), "unit": "QP energies/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"{len(stream)} water clusters, k ~ U{{1..{args.kmax}}}, "
                                  "HOMO-2..LUMO+2, 64-point grid",
                      "poisson_rate_req_per_s": round(lam, 4), "streams": args.streams},
           "saturated": {p: pick(r) for p, r in sat.items()},
           "poisson": {p: pick(r) for p, r in res.items()},
           "max_abs_dE_mixed_vs_fp64_mev": dE / MEV,
           "mixed_over_fp64_saturated_qp_per_s":
               round(sat["bf16x3w"]["qp_per_s"] / sat["fp64"]["qp_per_s"], 3)}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-evgw", action="store_true", help="skip the evGW0 / evGW timing")
    ap.add_argument("--no-core", action="store_true", help="skip the full core spectrum timing")
    ap.add_argument("--crossover", default=None,
                    help="comma-separated cluster sizes k: time the SD and CD routes instead")
    ap.add_argument("--only", default=None, choices=list(PATHS),
                    help="time only this path (profiling)")
    ap.add_argument("--serve", action="store_true", help="run the serving workload instead")
    ap.add_argument("--requests", type=int, default=128)
    ap.add_argument("--kmax", type=int, default=24)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.serve:
        serve_bench(args)
        return
    if args.crossover:
        import paper_2107_10423_amd as gwl
        ks = [int(k) for k in args.crossover.split(",")]
        print(json.dumps({"metric": "G0W0 wall time per call, spectral decomposition vs "
                                    "contour deformation (HOMO, LUMO)", "unit": "ms",
                          "n_gpus": 1, "data": "synthetic", "rows": crossover(gwl, ks)}))
        return
    if args.copy_calibration:
        x = torch.ones(2**27, dtype=torch.float64, device="cuda")     # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8}))
        return
    import gwgen
    import paper_2107_10423_amd as gwl

    name = "h2o10"
    cfg = gwgen.CONFIGS[name]
    states = list(cfg.states)
    log(f"bench: generating {name} inputs")
    inp = gwgen.make_config(name)
    grid = gwl.Grid.gauss_legendre(cfg.grid_points)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", f"{name}.json")))
    E_ref = np.array([r["E"] for r in gold["results"]])
    n_aux, n_ov = cfg.shape.n_aux, cfg.shape.n_ov
    flops = pi_flops(n_aux, n_ov, cfg.grid_points)

    precs = [args.only] if args.only else list(PATHS)
    res = {}
    for prec in precs:
        log(f"bench: timing {prec} path, {args.warmup} warmup + {args.steps} steps")
        r = time_path(gwl, inp, states, grid, prec, args.steps, args.warmup)
        r["err_mev"] = float(np.max(np.abs(r["E"] - E_ref)) / MEV)
        r["qp_per_s"] = len(states) / (r["ms_per_step"] / 1e3)
        r["pi_tflops"] = flops / (r["pi_ms"] / 1e3) / 1e12
        res[prec] = r
        log(f"bench: {prec}: {r['ms_per_step']:.2f} ms/step, Pi {r['pi_ms']:.2f} ms "
            f"({r['pi_tflops']:.1f} TFLOP/s), max |E - oracle| = {r['err_mev']:.2e} meV, "
            f"stages {json.dumps({k: round(v, 3) for k, v in r['stages'].items()})}")

    head = precs[0]
    h = res[head]
    pi_prec, wc_prec = PATHS[head]["pi_prec"], PATHS[head]["wc_prec"]
    # roofline of the Pi build and of the W^c contraction (one launch each per
    # step at this size); the dominant one, by measured launch time, heads the line
    kname = {"bf16x3": "pi_bf16x3", "fp32": "pi_f32", "fp64": "pi_f64"}[pi_prec]
    tr_pi = recorded_traffic(kname)
    roof_pi = {"kernel": kname, "bound": "mfma", "achieved": round(h["pi_tflops"], 2),
               "peak": PEAK_TFLOPS[pi_prec], "unit": "TFLOP/s",
               "frac": round(h["pi_tflops"] / PEAK_TFLOPS[pi_prec], 4),
               "traffic": tr_pi,
               "flops_per_launch": flops, "launch_ms": round(h["pi_ms"], 4),
               # BF16x3 issues three bf16 products per algorithmic one
               "issued_frac": round(h["pi_tflops"] * (3 if pi_prec == "bf16x3" else 1)
                                    / PEAK_TFLOPS[pi_prec], 4),
               "traffic_gb_per_s": (round(tr_pi / (h["pi_ms"] / 1e3) / 1e9, 1) if tr_pi else None),
               "note": "achieved = algorithmic flops N_aux(N_aux+1)N_ov per grid point x 64 grid "
                       "points / launch time (HIP events on the context stream); BF16x3 issues 3 "
                       "bf16 MFMA products per algorithmic product, so its issued rate is 3x"}
    n_rows_mo = len(states) * (cfg.shape.n_occ + cfg.shape.n_virt)
    w_flops = float(n_rows_mo) * n_aux * n_aux * cfg.grid_points
    w_ms = h["stages"]["wtab_ms"]
    w_tf = w_flops / (w_ms / 1e3) / 1e12
    wname = "wc_bf16x3" if wc_prec == "bf16x3" else "w_gemm"
    tr_w = recorded_traffic(wname)
    roof_w = {"kernel": wname, "bound": "mfma", "achieved": round(w_tf, 2),
              "peak": PEAK_TFLOPS[wc_prec], "unit": "TFLOP/s",
              "frac": round(w_tf / PEAK_TFLOPS[wc_prec], 4), "traffic": tr_w,
              "flops_per_launch": w_flops, "launch_ms": round(w_ms, 4),
              "issued_frac": round(w_tf * (3 if wc_prec == "bf16x3" else 1)
                                   / PEAK_TFLOPS[wc_prec], 4),
              "traffic_gb_per_s": (round(tr_w / (w_ms / 1e3) / 1e9, 1) if tr_w else None),
              "note": "W^c_nm = |L^-1 b|^2 - |b|^2 for every supplied row and m: algorithmic "
                      "flops n_rows n_mo N_aux^2 per grid point (a triangular solve per b) x 64 "
                      "grid points / the W^c stage time (HIP events around the stage: the FP64 "
                      "GEMM with its squared-norm epilogue, or the F = L^-1 - I split and the "
                      "BF16x3 contraction with its 2 b^T y + |y|^2 epilogue, then the 10-us "
                      "reduction kernel)"}
    roof, other = (roof_w, roof_pi) if w_ms > h["pi_ms"] else (roof_pi, roof_w)
    roof = dict(roof)
    roof["other_kernel"] = other
    out = {
        # the headline metric of the workload; this line carries the QP energies/s and
        # Pi TFLOP/s of the mixed and FP64 paths (p50/p99 latency: the --serve line)
        "metric": "QP energies/sec + \u03a0(i\u03c9) TFLOP/s, mixed vs FP64 GPU at \u22641 meV; "
                  "p50/p99 latency",
        "value": round(h["qp_per_s"], 3), "unit": "QP energies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[head],
        "data": "synthetic",
        "config": {"workload": "(H2O)10-shaped G0W0: n_occ=50, n_virt=380, N_aux=1120, "
                               "64-point grid, HOMO-4..LUMO+4 (10 states), seed 2",
                   "n_occ": 50, "n_virt": 380, "n_aux": 1120, "grid_points": 64, "states": 10},
        "roofline": roof,
        # one molecule's request latency on an idle GPU (W^c table rebuilt, all
        # 10 states): the timed steps' distribution; loaded p50/p99 latency is
        # the --serve line's
        "latency_ms": {"p50": round(h["median_ms"], 3), "p99": round(h["p99_ms"], 3),
                       "samples": args.steps},
        "paths": {p: {"qp_per_s": round(r["qp_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 3),
                      "median_ms_per_step": round(r["median_ms"], 3),
                      "setup_ms": round(r["setup_ms"], 1),
                      "cached_wtable_qp_per_s": round(len(states) / (r["cached_ms"] / 1e3), 3),
                      "pi_ms": round(r["pi_ms"], 3), "pi_tflops": round(r["pi_tflops"], 2),
                      "pi_frac_of_peak": round(r["pi_tflops"] / PEAK_TFLOPS[PATHS[p]["pi_prec"]], 4),
                      "max_err_mev_vs_oracle": r["err_mev"],
                      "stages_ms": {k: round(v, 3) for k, v in r["stages"].items()}}
                  for p, r in res.items()},
    }
    if "fp64" in res and head != "fp64":
        out["mixed_over_fp64"] = {"qp_per_s": round(h["qp_per_s"] / res["fp64"]["qp_per_s"], 3),
                                  "pi_tflops": round(h["pi_tflops"] / res["fp64"]["pi_tflops"], 3)}
    if not args.no_evgw:
        log(f"bench: timing evGW0 / evGW (3 cycles) on the {head} path")
        evr = time_evgw(gwl, inp, states, grid, head)
        out["evgw"] = {}
        for mode, r in evr.items():
            d = {"ms_per_call": round(r["ms_per_call"], 3), "cycles": r["cycles"],
                 "qp_rounds": r["qp_rounds"],
                 "qp_per_s": round(len(states) / (r["ms_per_call"] / 1e3), 3),
                 "status_nonzero": int(np.count_nonzero(r["status"])),
                 "stages_ms": r["stages"]}
            p = os.path.join(ROOT, "tests", "golden", f"{name}_{mode}.json")
            if os.path.exists(p):
                ref = np.array(json.load(open(p))["cycles"])
                if ref.shape == r["hist"].shape:
                    d["max_err_mev_vs_oracle"] = float(np.max(np.abs(r["hist"] - ref)) / MEV)
            out["evgw"][mode] = d
            log(f"bench: {mode}: {json.dumps(d)}")
    if not args.no_core:
        log(f"bench: timing the full core spectrum on the {head} path")
        out["core_spectrum"] = time_core_spectrum(gwl, head)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(inp, states, cfg.grid_points, gold)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
