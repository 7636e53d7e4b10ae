"""Benchmark of the contour-deformation G0W0 hot path on one MI355X.

Headline workload: the (H2O)30-shaped G0W0 problem (n_occ=150, n_virt=1140,
N_aux=3360, 128-point modified Gauss-Legendre grid, QP energies of
HOMO-9..LUMO+9), synthetic seeded inputs resident in HBM before timing starts.

One step = one gw_qp call with the W^c table cache dropped first, i.e. the
whole hot path: Pi(i xi) build on every grid point, Cholesky of 1 - Pi,
W^c table, imaginary-axis Sigma quadrature, batched MINRES residues and the
QP step tree, for all 20 states.  The headline value is the mixed-precision
path (BF16x3 Pi build and BF16x3 W^c contraction), timed over exactly
--steps steps; the plain FP64 path, the BF16x3-Pi-only path and the FP32 Pi
path are timed beside it (fewer steps), each with its per-state error against
the FP64 oracle's stored QP energies.  The same line carries a (H2O)10 leg,
a bounded serving leg (p50/p99 latency of a Poisson request stream, mixed vs
FP64, batching on and off), evGW and core-spectrum legs, and the oracle timed
on a bounded sample of the headline workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload h2o30|h2o10] [--only PATH] [--no-serve] ...
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
# QP tolerance of the timed paths: the one the oracle fixtures were solved
# with, so that each path's error against them measures its arithmetic and
# not a different stopping point of the step tree (with 1e-10 Ha a Newton
# step may stop up to ~1e-10 Ha short of the root, ~1e-10 relative)
QP_TOL = 1e-12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pi_flops(n_aux, n_ov, G):
    """Algorithmic flops of the Pi build: N_aux (N_aux + 1) N_ov per grid point
    (the symmetric product counted once, multiply and add each one flop)."""
    return n_aux * (n_aux + 1) * n_ov * G


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from its committed
    rocprofv3 counter record, or None when the record is missing or the
    kernel's source file has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["hbm_fetch_bytes"] + rec["hbm_write_bytes"]


def time_path(gwl, inp, states, grid, path, steps, warmup, work_budget=0):
    import numpy as np
    import torch
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    c = gwl.Context.from_inputs(inp, qp_tol=QP_TOL, work_budget_bytes=work_budget, **PATHS[path])
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
        for _ in range(max(1, min(3, steps // 2))):
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
    with gwl.Context.from_inputs(inp, qp_tol=QP_TOL, **PATHS[path]) as c:
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
        with gwl.Context.from_inputs(inp, qp_tol=QP_TOL, cluster_width=width,
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
            with gwl.Context.from_inputs(inp, pi_prec=prec, qp_tol=QP_TOL) as c:
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


def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 1) for i in threadpool_info()), default=None)
    except Exception:
        return None


def cpu_baseline(inp, states, G, gold):
    """Oracle timed on a bounded sample of the headline workload: the W^c
    table on three grid points (Pi build, explicit inverse, contraction for
    every row) and three residue terms (explicit Pi(w) at a real frequency,
    inverse, W^c and its derivative) of the HOMO, then scaled to the whole workload
    with the oracle's own counts from its fixture (grid points, and residue
    terms summed over every Sigma evaluation of every state; states the
    fixture does not hold are counted at the mean of the occupied states it
    does hold).  The I-term quadrature itself is negligible next to these."""
    import numpy as np
    from oracle import cd, grid as ogrid
    xi, z = ogrid.gauss_legendre(G)
    pts = [G // 4, G // 2, (3 * G) // 4]
    t0 = time.perf_counter()
    cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi[pts])
    t_g = (time.perf_counter() - t0) / len(pts)
    homo = inp.n_occ - 1
    r = list(inp.row_ids).index(homo)
    have = {int(x["state"]): x for x in gold["results"]} if gold else {}
    E_h = have[homo]["E"] if homo in have else inp.eps[homo] - 0.3
    ms = [homo - 1, homo - 2, homo - 3]   # occupied levels: residue terms of the HOMO
    t0 = time.perf_counter()
    for m in ms:
        cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[r, m], inp.eps[m] - E_h)
    t_res = (time.perf_counter() - t0) / len(ms)
    occ_counts = [sum(x.get("n_residues", [])) for n, x in have.items() if n < inp.n_occ]
    mean_occ = float(np.mean(occ_counts)) if occ_counts else 0.0
    n_res = 0.0
    for n in states:
        if n in have:
            n_res += sum(have[n].get("n_residues", []))
        elif n < inp.n_occ:
            n_res += mean_occ
    total = G * t_g + n_res * t_res
    return {"value": len(states) / total, "unit": "QP energies/s", "cores": _cores(),
            "blas_threads": _blas_threads(), "kind": "oracle",
            "sample": (f"W^c table on {len(pts)} of {G} grid points ({t_g:.1f} s each: Pi "
                       f"build, explicit inverse, {inp.B_rows.shape[0]} x "
                       f"{inp.B_rows.shape[1]} rows) + {len(ms)} residue terms of the HOMO "
                       f"({t_res:.1f} s each: explicit Pi(w), inverse, W^c and derivative); "
                       f"scaled to {G} grid points and {n_res:.0f} residue terms (the "
                       f"oracle's own counts over all {len(states)} states)"),
            "sample_s": round(len(pts) * t_g + len(ms) * t_res, 1),
            "est_total_s": total}


def oracle_errors(E, states, gold):
    """Per-state |E - E_oracle| (meV) over the states the fixture holds."""
    import numpy as np
    if not gold:
        return {"states_checked": 0}
    ref = {int(x["state"]): x["E"] for x in gold["results"]}
    per = {int(n): float(abs(E[j] - ref[n]) / MEV) for j, n in enumerate(states) if n in ref}
    if not per:
        return {"states_checked": 0}
    rel = max(abs(E[j] - ref[n]) / abs(ref[n]) for j, n in enumerate(states) if n in ref)
    return {"states_checked": len(per), "max_err_mev_vs_oracle": max(per.values()),
            "max_rel_err_vs_oracle": float(rel),
            "per_state_err_mev": {str(k): float(f"{v:.3e}") for k, v in sorted(per.items())}}


def load_workload(name):
    import gwgen
    cfg = gwgen.CONFIGS[name]
    if name == "h2o30":      # block-wise recipe of the same distribution (its fixture's)
        inp = gwgen.make_inputs_blocked(cfg.shape, cfg.seed, cfg.states)
    else:
        inp = gwgen.make_config(name)
    p = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    gold = json.load(open(p)) if os.path.exists(p) else None
    return cfg, inp, gold


def serve_leg(gwl, n_requests, kmax, streams, small_k=6, n_burst=48):
    """Serving workload (bounded): the first n_requests requests of the stream
    (water clusters of k ~ U{1..kmax}, request r seeded 1000 + r, HOMO-2..LUMO+2,
    64-point grid) through gw_server.  Closed loop with 8 outstanding for FP64
    and for the mixed form -> saturated throughput; then Poisson arrivals at
    0.8 x the FP64 saturated rate for FP64, for the mixed form, and for the
    mixed form with batching off -> throughput and p50 / p99 latency (done -
    submit), also over the small requests (k <= small_k) alone.

    Small-request leg: the first n_burst requests of the same stream with
    k <= small_k (the sizes whose stage A is batched), mixed form, with and
    without batching: closed loop with 16 outstanding, then Poisson arrivals
    at 0.8 x the unbatched closed-loop rate."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import gwgen

    full = gwgen.serving_stream(n_requests=max(n_requests, 1024), k_max=kmax, seed=5000,
                                rate=1.0)
    stream = full[:n_requests]
    burst = [r for r in full if r["k"] <= small_k][:n_burst]
    # every request's inputs are generated before the timed runs and held in
    # host memory (generation is slower than the mixed path serves them);
    # refuse a request list whose inputs would not fit in about 160 GB
    held = sum(8 * r["shape"].n_aux * (r["shape"].n_ov + len(r["states"]) * r["shape"].n_mo)
               for r in stream + burst)
    if held > 160e9:
        raise SystemExit(f"serving leg: the inputs of {len(stream)} requests take "
                         f"{held / 1e9:.0f} GB of host memory; use fewer requests")
    log(f"serve: inputs of the timed requests: {held / 1e9:.1f} GB of host memory")
    log(f"serve: generating {len(stream)} + {len(burst)} requests (seed 1000 + r each)")
    with ThreadPoolExecutor(max_workers=min(16, _cores() or 1)) as ex:
        inputs = list(ex.map(lambda r: gwgen.serving_inputs(r["k"], r["seed"]), stream))
        b_inputs = list(ex.map(lambda r: gwgen.serving_inputs(r["k"], r["seed"]), burst))
    grid = gwl.Grid.gauss_legendre(64)

    def run(prec, arrivals, window=None, batch_max_aux=0, reqs=None):
        stream_, inputs_ = reqs if reqs is not None else (stream, inputs)
        return _serve_run(gwl, grid, streams, stream_, inputs_, small_k, prec, arrivals,
                          window, batch_max_aux)

    sat = {}
    for prec in ("fp64", "bf16x3w"):
        log(f"serve: {prec} closed loop (8 outstanding)")
        sat[prec] = run(prec, None, window=8)
    lam = 0.8 * sat["fp64"]["req_per_s"]
    arr = np.array([r["arrival_s"] for r in stream]) / lam
    res = {}
    for key, prec, lim in (("fp64", "fp64", 0), ("bf16x3w", "bf16x3w", 0),
                           ("bf16x3w_no_batching", "bf16x3w", -1)):
        log(f"serve: {key}, Poisson arrivals at {lam:.2f} req/s")
        res[key] = run(prec, arr, batch_max_aux=lim)
    dE = max(float(np.max(np.abs(res["bf16x3w"]["E"][i] - res["fp64"]["E"][i])))
             for i in range(len(stream)))
    # small requests alone: batching on and off
    b_sat, b_res = {}, {}
    for key, lim in (("batching", 0), ("no_batching", -1)):
        log(f"serve: small requests, mixed, {key}, closed loop (16 outstanding)")
        b_sat[key] = run("bf16x3w", None, window=16, batch_max_aux=lim, reqs=(burst, b_inputs))
    lam_b = 0.8 * b_sat["no_batching"]["req_per_s"]
    # arrival gaps of the burst requests' own Poisson process, rescaled
    gaps = np.diff([r["arrival_s"] for r in burst], prepend=burst[0]["arrival_s"])
    arr_b = np.cumsum(gaps) / np.mean(gaps[1:]) / lam_b
    for key, lim in (("batching", 0), ("no_batching", -1)):
        log(f"serve: small requests, mixed, {key}, Poisson arrivals at {lam_b:.1f} req/s")
        b_res[key] = run("bf16x3w", arr_b, batch_max_aux=lim, reqs=(burst, b_inputs))
    dEb = max(float(np.max(np.abs(b_res["batching"]["E"][i] - b_res["no_batching"]["E"][i])))
              for i in range(len(burst)))
    pick = lambda r: {k: (round(v, 4) if isinstance(v, float) else v)
                      for k, v in r.items() if k != "E"}
    return {"workload": f"first {len(stream)} requests of the serving stream: water clusters "
                        f"k ~ U{{1..{kmax}}}, request r seeded 1000 + r, HOMO-2..LUMO+2, "
                        f"64-point grid, {streams} pipelines",
            "small_k_max": small_k, "n_small": int(sum(r["k"] <= small_k for r in stream)),
            "poisson_rate_req_per_s": round(lam, 4),
            "saturated": {p: pick(r) for p, r in sat.items()},
            "poisson": {p: pick(r) for p, r in res.items()},
            "p50_s": {p: round(r["p50_s"], 4) for p, r in res.items()},
            "p99_s": {p: round(r["p99_s"], 4) for p, r in res.items()},
            "max_abs_dE_mixed_vs_fp64_mev": dE / MEV,
            "mixed_over_fp64_saturated_qp_per_s":
                round(sat["bf16x3w"]["qp_per_s"] / sat["fp64"]["qp_per_s"], 3),
            "small_requests": {
                "workload": f"the first {len(burst)} requests of the same stream with "
                            f"k <= {small_k}, mixed form",
                "poisson_rate_req_per_s": round(lam_b, 2),
                "saturated": {p: pick(r) for p, r in b_sat.items()},
                "poisson": {p: pick(r) for p, r in b_res.items()},
                "max_abs_dE_batching_vs_not_mev": dEb / MEV}}


def _serve_run(gwl, grid, streams, stream, inputs, small_k, prec, arrivals, window,
               batch_max_aux):
    """One pass of a request list through a fresh gw_server."""
    import threading

    import numpy as np
    ks = np.array([r["k"] for r in stream])
    srv = gwl.Server(grid, n_streams=streams, batch_max_aux=batch_max_aux, **PATHS[prec])
    tickets, E, lat = {}, {}, {}
    done_t, sub_t = [], []
    lock = threading.Lock()
    outstanding = threading.Semaphore(window) if window else None
    t0 = time.perf_counter()

    def producer():
        for i in range(len(stream)):
            if arrivals is not None:
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            if outstanding:
                outstanding.acquire()
            inp = inputs[i]
            tk = srv.submit_inputs(inp, list(inp.row_ids))
            with lock:
                tickets[tk] = i

    failed = []
    th = threading.Thread(target=producer, daemon=True)
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
                failed.append((i, info["rc"]))
            E[i] = out[0]
            lat[i] = info["t_done"] - info["t_submit"]
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
    if failed:
        raise RuntimeError(f"{prec}: requests failed (index, code): {failed}")
    span = max(done_t) - min(sub_t)
    L = np.array([lat[i] for i in range(len(stream))])
    small = L[ks <= small_k]
    # algorithmic Pi work of every request's W^c table: N_aux (N_aux + 1) N_ov
    # per grid point (the xi = 0 point of the preconditioner not counted)
    pi_flop = sum(float(x.shape.n_aux) * (x.shape.n_aux + 1) * x.shape.n_ov * grid.n
                  for x in inputs)
    return dict(E=E, span_s=span, req_per_s=len(stream) / span,
                qp_per_s=sum(len(x.row_ids) for x in inputs) / span,
                pi_tflops=pi_flop / span / 1e12,
                p50_s=float(np.percentile(L, 50)), p99_s=float(np.percentile(L, 99)),
                small_p50_s=float(np.percentile(small, 50)) if small.size else None,
                small_p99_s=float(np.percentile(small, 99)) if small.size else None,
                peak_active=st["peak_active"], batches=st["batches"],
                batched_requests=st["batched_requests"], graph_replays=st["graph_replays"],
                device_mallocs=st["device_mallocs"], cache_hits=st["cache_hits"],
                device_frees=st["device_frees"])


def roofline_objects(h, cfg, workload, states):
    """Roofline of the Pi build and of the W^c contraction of the timed path;
    the longer of the two heads, the other rides along."""
    n_aux, n_ov, G = cfg.shape.n_aux, cfg.shape.n_ov, cfg.grid_points
    pi_prec, wc_prec = h["pi_prec"], h["wc_prec"]
    Gx = G + 1                      # the xi = 0 point (preconditioner) is built too
    flops = pi_flops(n_aux, n_ov, G)
    kname = {"bf16x3": "pi_bf16x3", "fp32": "pi_f32", "fp64": "pi_f64"}[pi_prec]
    # algorithmic bytes of one step's Pi build(s): every operand element read
    # once in the kernel's own format (FP64: 8 B; FP32: 4 B; BF16x3: hi + lo of
    # the unscaled side and the FP32 scaled side, 8 B) plus the lower triangle
    # of 1 - Pi written once per grid point (FP64)
    opb = {"fp64": 8, "fp32": 4, "bf16x3": 8}[pi_prec]
    alg_pi = n_aux * n_ov * opb + Gx * n_aux * (n_aux + 1) // 2 * 8
    tr_pi = recorded_traffic(kname, workload)
    st = h["stages"]
    n_pi = max(1, round(st.get("pi_launches", 1)))
    pi_kms = st.get("pi_kernel_ms") or h["pi_ms"]       # the kernel's own launches
    pi_tf = flops / (pi_kms / 1e3) / 1e12
    roof_pi = {"kernel": kname, "bound": "mfma", "achieved": round(pi_tf, 2),
               "peak": PEAK_TFLOPS[pi_prec], "unit": "TFLOP/s",
               "frac": round(pi_tf / PEAK_TFLOPS[pi_prec], 4),
               "traffic": tr_pi, "algorithmic_bytes": alg_pi // n_pi,
               "traffic_over_algorithmic": round(tr_pi / (alg_pi / n_pi), 2) if tr_pi else None,
               "flops_per_launch": flops / n_pi, "launches_per_step": n_pi,
               "launch_ms": round(pi_kms / n_pi, 4), "stage_ms": round(h["pi_ms"], 4),
               "issued_frac": round(pi_tf * (3 if pi_prec == "bf16x3" else 1)
                                    / PEAK_TFLOPS[pi_prec], 4),
               "note": f"achieved = algorithmic flops N_aux(N_aux+1)N_ov per grid point x {G} "
                       "grid points per step / the Pi kernel's launch time (HIP events around "
                       "its launches on the context stream; the launch also builds the xi = 0 "
                       "point, not counted); BF16x3 issues 3 bf16 MFMA products per "
                       "algorithmic product, so its issued rate is 3x"}
    n_rows_mo = len(states) * (cfg.shape.n_occ + cfg.shape.n_virt)
    w_flops = float(n_rows_mo) * n_aux * n_aux * G
    w_ms = h["stages"]["wtab_ms"]
    n_w = max(1, round(st.get("wc_launches", 1)))
    w_kms = st.get("wc_kernel_ms") or w_ms
    w_tf = w_flops / (w_kms / 1e3) / 1e12
    wname = "wc_bf16x3" if wc_prec == "bf16x3" else "w_gemm"
    tr_w = recorded_traffic(wname, workload)
    # algorithmic bytes: the rows b = (P|nm) once and L^-1 (lower triangle)
    # once per grid point, in the operands' format, plus the table
    ob = 4 if wc_prec == "bf16x3" else 8
    alg_w = n_rows_mo * n_aux * ob + G * n_aux * (n_aux + 1) // 2 * ob + n_rows_mo * G * 8
    roof_w = {"kernel": wname, "bound": "mfma", "achieved": round(w_tf, 2),
              "peak": PEAK_TFLOPS[wc_prec], "unit": "TFLOP/s",
              "frac": round(w_tf / PEAK_TFLOPS[wc_prec], 4), "traffic": tr_w,
              "algorithmic_bytes": alg_w // n_w,
              "traffic_over_algorithmic": round(tr_w / (alg_w / n_w), 2) if tr_w else None,
              "flops_per_launch": w_flops / n_w, "launches_per_step": n_w,
              "launch_ms": round(w_kms / n_w, 4), "stage_ms": round(w_ms, 4),
              "issued_frac": round(w_tf * (3 if wc_prec == "bf16x3" else 1)
                                   / PEAK_TFLOPS[wc_prec], 4),
              "note": "W^c_nm = |L^-1 b|^2 - |b|^2 for every supplied row and m: algorithmic "
                      f"flops n_rows n_mo N_aux^2 per grid point x {G} / the launch time of "
                      "the FP64 GEMM or BF16x3 contraction (HIP events around its launches)"}
    roof, other = (roof_w, roof_pi) if w_kms > pi_kms else (roof_pi, roof_w)
    roof = dict(roof)
    roof["other_kernel"] = other
    return roof


def run_workload(gwl, name, head_path, args, side_paths, side_steps):
    cfg, inp, gold = load_workload(name)
    states = list(cfg.states)
    grid = gwl.Grid.gauss_legendre(cfg.grid_points)
    # one stage-A chunk holds every grid point (the whole build per launch)
    wb = 48 << 30 if name == "h2o30" else 0
    flops = pi_flops(cfg.shape.n_aux, cfg.shape.n_ov, cfg.grid_points)
    res = {}
    for path in [head_path] + [p for p in side_paths if p != head_path]:
        steps, warmup = (args.steps, args.warmup) if path == head_path else (side_steps, 1)
        log(f"bench: {name}: timing {path} path, {warmup} warmup + {steps} steps")
        r = time_path(gwl, inp, states, grid, path, steps, warmup, work_budget=wb)
        r.update(oracle_errors(r["E"], states, gold))
        r["qp_per_s"] = len(states) / (r["ms_per_step"] / 1e3)
        r["pi_tflops"] = flops / (r["pi_ms"] / 1e3) / 1e12
        r["pi_prec"], r["wc_prec"] = PATHS[path]["pi_prec"], PATHS[path]["wc_prec"]
        r["steps"] = steps
        res[path] = r
        log(f"bench: {name}: {path}: {r['ms_per_step']:.2f} ms/step, Pi {r['pi_ms']:.2f} ms "
            f"({r['pi_tflops']:.1f} TFLOP/s), oracle: {r.get('max_err_mev_vs_oracle')} meV over "
            f"{r.get('states_checked')} states, stages "
            f"{json.dumps({k: round(v, 3) for k, v in r['stages'].items()})}")
    return cfg, inp, gold, states, res


def path_summary(res, states):
    out = {}
    for p, r in res.items():
        d = {"qp_per_s": round(r["qp_per_s"], 4), "ms_per_step": round(r["ms_per_step"], 3),
             "steps": r["steps"], "median_ms_per_step": round(r["median_ms"], 3),
             "setup_ms": round(r["setup_ms"], 1),
             "cached_wtable_qp_per_s": round(len(states) / (r["cached_ms"] / 1e3), 3),
             "pi_ms": round(r["pi_ms"], 3), "pi_tflops": round(r["pi_tflops"], 2),
             "pi_frac_of_peak": round(r["pi_tflops"] / PEAK_TFLOPS[r["pi_prec"]], 4),
             "stages_ms": {k: round(v, 3) for k, v in r["stages"].items()}}
        for k in ("states_checked", "max_err_mev_vs_oracle", "max_rel_err_vs_oracle",
                  "per_state_err_mev"):
            if k in r:
                d[k] = r[k]
        out[p] = d
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="h2o30", choices=["h2o30", "h2o10"],
                    help="headline workload (default: the (H2O)30 shape)")
    ap.add_argument("--only", default=None, choices=list(PATHS),
                    help="time only this path of the headline workload (profiling)")
    ap.add_argument("--side-steps", type=int, default=1,
                    help="timed steps of each non-headline path of the headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-h2o10", action="store_true", help="skip the (H2O)10 leg")
    ap.add_argument("--no-evgw", action="store_true", help="skip the evGW0 / evGW timing")
    ap.add_argument("--no-core", action="store_true", help="skip the full core spectrum timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests of the serving leg (the first ones of the stream)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its object as the line")
    ap.add_argument("--core-only", action="store_true",
                    help="run only the (H2O)20 core-spectrum leg and print its object as the line")
    ap.add_argument("--kmax", type=int, default=24)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--crossover", default=None,
                    help="comma-separated cluster sizes k: time the SD and CD routes instead")
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
    import paper_2107_10423_amd as gwl
    if args.crossover:
        ks = [int(k) for k in args.crossover.split(",")]
        print(json.dumps({"metric": "G0W0 wall time per call, spectral decomposition vs "
                                    "contour deformation (HOMO, LUMO)", "unit": "ms",
                          "n_gpus": 1, "data": "synthetic", "rows": crossover(gwl, ks)}))
        return
    if args.core_only:
        print(json.dumps({"metric": "core spectrum: QP energies/s with the W^c table cached",
                          "n_gpus": 1, "data": "synthetic",
                          "core_spectrum": time_core_spectrum(gwl, "bf16x3w")}))
        return
    if args.serve_only:
        print(json.dumps({"metric": "serving: QP energies/s and p50/p99 request latency",
                          "n_gpus": 1, "data": "synthetic",
                          "serving": serve_leg(gwl, args.serve_requests, args.kmax,
                                               args.streams)}))
        return
    if args.copy_calibration:
        x = torch.ones(2**27, dtype=torch.float64, device="cuda")     # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8}))
        return

    name = args.workload
    head = args.only or "bf16x3w"
    side = [] if args.only else ["fp64", "bf16x3", "fp32"]
    log(f"bench: generating {name} inputs")
    cfg, inp, gold, states, res = run_workload(gwl, name, head, args, side, args.side_steps)
    h = res[head]
    sh = cfg.shape
    out = {
        "metric": "QP energies/sec + \u03a0(i\u03c9) TFLOP/s, mixed vs FP64 GPU at \u22641 meV; "
                  "p50/p99 latency",
        "value": round(h["qp_per_s"], 4), "unit": "QP energies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[head],
        "data": "synthetic",
        "config": {"workload": f"{'(H2O)30' if name == 'h2o30' else '(H2O)10'}-shaped G0W0: "
                               f"n_occ={sh.n_occ}, n_virt={sh.n_virt}, N_aux={sh.n_aux}, "
                               f"{cfg.grid_points}-point grid, {len(states)} states "
                               f"(HOMO-{sh.n_occ - 1 - states[0]}..LUMO+"
                               f"{states[-1] - sh.n_occ}), seed {cfg.seed}",
                   "n_occ": sh.n_occ, "n_virt": sh.n_virt, "n_aux": sh.n_aux,
                   "grid_points": cfg.grid_points, "states": len(states), "qp_tol_ha": QP_TOL},
        "roofline": roofline_objects(h, cfg, name, states),
        # one molecule's request latency on an idle GPU (the headline path's
        # timed steps); loaded latency under a request stream: "serving"
        "latency_ms": {"p50": round(h["median_ms"], 3), "p99": round(h["p99_ms"], 3),
                       "samples": args.steps},
        "paths": path_summary(res, states),
    }
    if "fp64" in res and head != "fp64":
        out["mixed_over_fp64"] = {"qp_per_s": round(h["qp_per_s"] / res["fp64"]["qp_per_s"], 3),
                                  "pi_tflops": round(h["pi_tflops"] / res["fp64"]["pi_tflops"], 3)}
    # free the headline inputs before the other legs
    del inp
    if name != "h2o10" and not args.no_h2o10 and not args.only:
        log("bench: (H2O)10 leg")
        ns = argparse.Namespace(**vars(args))
        ns.steps, ns.warmup = max(args.steps, 10), 2
        c2, inp2, gold2, st2, res2 = run_workload(gwl, "h2o10", "bf16x3w", ns, ["fp64"], 10)
        out["h2o10"] = {"paths": path_summary(res2, st2),
                        "mixed_over_fp64": {
                            "qp_per_s": round(res2["bf16x3w"]["qp_per_s"] /
                                              res2["fp64"]["qp_per_s"], 3),
                            "pi_tflops": round(res2["bf16x3w"]["pi_tflops"] /
                                               res2["fp64"]["pi_tflops"], 3)},
                        "roofline": roofline_objects(res2["bf16x3w"], c2, "h2o10", st2)}
        if not args.no_evgw:
            log("bench: timing evGW0 / evGW (3 cycles) on the (H2O)10 mixed path")
            grid2 = gwl.Grid.gauss_legendre(c2.grid_points)
            evr = time_evgw(gwl, inp2, st2, grid2, "bf16x3w")
            out["evgw"] = {"workload": "(H2O)10 shape, 3 cycles, mixed path"}
            for mode, r in evr.items():
                d = {"ms_per_call": round(r["ms_per_call"], 3), "cycles": r["cycles"],
                     "qp_rounds": r["qp_rounds"],
                     "qp_per_s": round(len(st2) / (r["ms_per_call"] / 1e3), 3),
                     "status_nonzero": int(np.count_nonzero(r["status"]))}
                pth = os.path.join(ROOT, "tests", "golden", f"h2o10_{mode}.json")
                if os.path.exists(pth):
                    ref = np.array(json.load(open(pth))["cycles"])
                    if ref.shape == r["hist"].shape:
                        d["max_err_mev_vs_oracle"] = float(np.max(np.abs(r["hist"] - ref)) / MEV)
                out["evgw"][mode] = d
        del inp2
    if not args.no_core and not args.only:
        log("bench: timing the full core spectrum on the mixed path")
        out["core_spectrum"] = time_core_spectrum(gwl, "bf16x3w")
    if not args.no_serve and not args.only:
        log("bench: serving leg")
        out["serving"] = serve_leg(gwl, args.serve_requests, args.kmax, args.streams)
        out["latency_p50_p99_s"] = {"mixed": [out["serving"]["p50_s"]["bf16x3w"],
                                              out["serving"]["p99_s"]["bf16x3w"]],
                                    "fp64": [out["serving"]["p50_s"]["fp64"],
                                             out["serving"]["p99_s"]["fp64"]]}
    if not args.no_cpu_baseline and not args.only:
        log("bench: timing the oracle on a bounded sample of the headline workload")
        _, inp, gold = load_workload(name)
        out["cpu_baseline"] = cpu_baseline(inp, states, cfg.grid_points, gold)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
