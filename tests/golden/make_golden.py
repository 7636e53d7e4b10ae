"""Write oracle fixtures for the named workloads (calls only oracle/ and gwgen).

    python tests/golden/make_golden.py monomer h2o10
    python tests/golden/make_golden.py h2o10:evgw0 h2o10:evgw     (3 cycles each)
    python tests/golden/make_golden.py --states 150,151,149 [--cache DIR] h2o30
    python tests/golden/make_golden.py --states 5,10,19 [--cache DIR] h2o20_core

The last two forms are incremental, for workloads whose oracle takes hours:
the fixture is rewritten after every state (states already in it are kept
and skipped), and with --cache each grid point's W^c table column is kept in
DIR as a .npy file, so an interrupted run resumes where it stopped.  The
(H2O)30 inputs use gwgen.make_inputs_blocked (the recipe its tests use), the
others gwgen.make_inputs with the union of the fixture's and the new states
as rows (a row's values do not depend on which other rows are drawn).

Each fixture is a JSON file tests/golden/<name>.json with the inputs' recipe
(seed, sizes, grid), the oracle's QP energies, Re Sigma^c at the root, Z,
status, iteration counts, Sigma^c at a few fixed frequencies, and the wall
time and thread count of the oracle run.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gwgen  # noqa: E402
from oracle import cd, ev, grid, qp  # noqa: E402


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        return os.cpu_count()


def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def make(name, qp_tol=1e-12):
    cfg = gwgen.CONFIGS[name]
    inp = gwgen.make_config(name)
    xi, z = grid.gauss_legendre(cfg.grid_points)
    t0 = time.time()
    wtab = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi)
    t_w = time.time() - t0
    res = []
    for k, n in enumerate(cfg.states):
        fe = qp.make_feval(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[k], wtab[k], xi, z, n)
        r = qp.step_tree(fe, inp.eps[n], tol=qp_tol)
        res.append(dict(state=n, E=r["E"], sigma_c=r["f"] - (inp.eps[n] - r["E"]), Z=r["Z"],
                        status=r["status"], iters=r["iters"],
                        steps=[t[2] for t in r["trace"]]))
    # Sigma^c at fixed frequencies (HOMO and LUMO rows): eps_n and eps_n -/+ 0.2
    fixed = []
    homo = inp.n_occ - 1
    for n in (homo, homo + 1):
        if n not in cfg.states:
            continue
        k = list(cfg.states).index(n)
        for w in (inp.eps[n], inp.eps[n] - 0.2, inp.eps[n] + 0.2):
            s, ds, nres = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[k], wtab[k], xi, z, w)
            fixed.append(dict(state=n, omega=w, sigma=s, dsigma=ds, n_res=nres))
    t_all = time.time() - t0
    out = dict(name=name, seed=cfg.seed, n_occ=cfg.shape.n_occ, n_virt=cfg.shape.n_virt,
               n_aux=cfg.shape.n_aux, grid_points=cfg.grid_points, x0=0.5, qp_tol=qp_tol,
               states=list(cfg.states), results=res, fixed=fixed,
               oracle_seconds=dict(w_table=t_w, total=t_all), threads=_threads(),
               note="written by tests/golden/make_golden.py from oracle/ only")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {t_all:.1f} s -> {path}")


def make_ev(name, mode, n_cycles=3, qp_tol=1e-12):
    """Fixture <name>_<mode>.json: the QP energies of every evGW0 / evGW cycle."""
    cfg = gwgen.CONFIGS[name]
    inp = gwgen.make_config(name)
    xi, z = grid.gauss_legendre(cfg.grid_points)
    t0 = time.time()
    res, cycles, hist = ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows,
                                list(cfg.states), xi, z, mode=mode, n_cycles=n_cycles,
                                tol=qp_tol)
    t_all = time.time() - t0
    out = dict(name=name, mode=mode, n_cycles=n_cycles, seed=cfg.seed, n_occ=cfg.shape.n_occ,
               n_virt=cfg.shape.n_virt, n_aux=cfg.shape.n_aux, grid_points=cfg.grid_points,
               x0=0.5, qp_tol=qp_tol, states=list(cfg.states),
               cycles=[[float(e) for e in E] for E in hist],
               results=[dict(state=int(r["state"]), E=r["E"], sigma_c=r["sigma_c"], Z=r["Z"],
                             status=r["status"]) for r in res],
               oracle_seconds=t_all, threads=_threads(),
               note="written by tests/golden/make_golden.py from oracle/ only")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_{mode}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name} {mode}: {t_all:.1f} s -> {path}")


BLOCKED = ("h2o30",)


def _w_table_cached(name, inp, xi, cache):
    """cd.w_table, one grid point at a time, each column kept in cache/."""
    n_rows, n_mo, _ = inp.B_rows.shape
    out = np.empty((n_rows, n_mo, len(xi)))
    for g, x in enumerate(xi):
        f = None if cache is None else os.path.join(cache, f"{name}_w{n_rows}_{g:03d}.npy")
        if f is not None and os.path.exists(f):
            out[:, :, g] = np.load(f)
            continue
        out[:, :, g] = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi[g:g + 1])[:, :, 0]
        if f is not None:
            np.save(f, out[:, :, g])
        print(f"  {name}: grid point {g + 1}/{len(xi)}", flush=True)
    return out


def make_incremental(name, new_states, cache=None, qp_tol=1e-12):
    """Fixture <name>.json extended state by state (see the module docstring)."""
    cfg = gwgen.CONFIGS[name]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    old = None
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
    done = {} if old is None else {int(r["state"]): r for r in old["results"]}
    t0 = time.time()
    if name in BLOCKED:
        recipe = "make_inputs_blocked"
        rows = list(cfg.states)
        inp = gwgen.make_inputs_blocked(cfg.shape, cfg.seed, rows)
    else:
        recipe = "make_inputs"
        rows = sorted(set(done) | set(int(n) for n in new_states))
        inp = gwgen.make_inputs(cfg.shape, cfg.seed, rows)
    print(f"{name}: inputs in {time.time() - t0:.1f} s", flush=True)
    xi, z = grid.gauss_legendre(cfg.grid_points)
    t1 = time.time()
    wtab = _w_table_cached(name, inp, xi, cache)
    t_w = time.time() - t1
    secs = {} if old is None else dict(old.get("oracle_seconds", {}))
    secs.setdefault("w_table", t_w)
    per_state = dict(secs.get("per_state", {}))
    for n in new_states:
        n = int(n)
        if n in done:
            continue
        if n not in rows:
            raise ValueError(f"state {n} is not among the rows {rows}")
        k = rows.index(n)
        t2 = time.time()
        calls = []
        fe = qp.make_feval(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[k], wtab[k], xi, z, n,
                           counter=calls)
        r = qp.step_tree(fe, inp.eps[n], tol=qp_tol)
        done[n] = dict(state=n, E=r["E"], sigma_c=r["f"] - (inp.eps[n] - r["E"]), Z=r["Z"],
                       status=r["status"], iters=r["iters"],
                       steps=[t[2] for t in r["trace"]], n_residues=[c[3] for c in calls])
        per_state[str(n)] = time.time() - t2
        secs["per_state"] = per_state
        out = dict(name=name, recipe=recipe, seed=cfg.seed, n_occ=cfg.shape.n_occ,
                   n_virt=cfg.shape.n_virt, n_aux=cfg.shape.n_aux,
                   grid_points=cfg.grid_points, x0=0.5, qp_tol=qp_tol,
                   states=sorted(done), results=[done[s] for s in sorted(done)],
                   fixed=[] if old is None else old.get("fixed", []),
                   oracle_seconds=secs, threads=_threads(), cores=_cores(),
                   note="written by tests/golden/make_golden.py from oracle/ only")
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)
        print(f"{name}: state {n} E = {r['E']:.12f} Z = {r['Z']:.6f} in "
              f"{per_state[str(n)]:.0f} s (residues per evaluation "
              f"{[c[3] for c in calls]})", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    states, cache = None, None
    while args and args[0].startswith("--"):
        opt = args.pop(0)
        if opt == "--states":
            states = [int(v) for v in args.pop(0).split(",")]
        elif opt == "--cache":
            cache = args.pop(0)
            os.makedirs(cache, exist_ok=True)
        else:
            raise SystemExit(f"unknown option {opt}")
    for nm in args or ["monomer"]:
        if states is not None:
            make_incremental(nm, states, cache)
        elif ":" in nm:
            base, mode = nm.split(":")
            make_ev(base, mode)
        else:
            make(nm)
