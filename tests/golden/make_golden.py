"""Write oracle fixtures for the named workloads (calls only oracle/ and gwgen).

    python tests/golden/make_golden.py monomer h2o10
    python tests/golden/make_golden.py h2o10:evgw0 h2o10:evgw     (3 cycles each)

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


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["monomer"]:
        if ":" in nm:
            base, mode = nm.split(":")
            make_ev(base, mode)
        else:
            make(nm)
