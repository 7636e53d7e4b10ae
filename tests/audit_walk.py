"""Walk every launch of the HIP path in launch-audit mode (no GPU needed).

Run as a separate process (audit mode is irreversible):
    python tests/audit_walk.py
Prints one line per case and exits non-zero if any launch guard refused a
launch or any entry point failed for another reason.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gwgen  # noqa: E402
import paper_2107_10423_amd as gwl  # noqa: E402

CASES = [
    # n_occ, n_virt, n_aux, rows, G, work_budget, minres cap
    (7, 45, 200, (4, 5, 6, 7, 8), 8, 0, 0),
    (5, 38, 112, (4, 5), 64, 0, 0),            # monomer shape
    (3, 20, 64, (1, 2), 5, 0, 0),              # n_aux = 64 < one Pi tile
    (1, 1, 1, (0, 1), 3, 0, 0),                # smallest possible
    (2, 3, 130, (1,), 4, 0, 1),                # N_aux just past a tile, fallback forced
    (11, 60, 300, tuple(range(0, 71)), 6, 0, 0),  # many rows (nR > 4000)
    (12, 70, 220, (0, 11), 32, 2 << 20, 0),    # chunked stage A
    (50, 380, 1120, tuple(range(45, 55)), 64, 0, 0),  # (H2O)10 shape
    (17, 63, 129, (16, 17, 40), 7, 0, 2),
    (3, 20, 2100, (1, 2), 4, 0, 0),            # N_aux past the wide tiles' threshold, ragged
]


def run_case(n_occ, n_virt, n_aux, rows, G, wb, cap):
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=1 if n_occ > 1 else 0)
    inp = gwgen.make_inputs(shape, 1, rows)
    g = gwl.Grid.gauss_legendre(G)
    for prec, wc in (("fp64", "fp64"), ("fp32", "fp64"), ("bf16x3", "fp64"),
                     ("bf16x3", "bf16x3")):
        kw = dict(pi_prec=prec, work_budget_bytes=wb, minres_max_iter=cap, wc_prec=wc)
        with gwl.Context.from_inputs(inp, **kw) as c:
            before = gwl.audit_launch_count()
            for call in (lambda: c.dielectric([0.1, 2.0]), lambda: c.cholesky([0.3]),
                         lambda: c.wtable(g),
                         lambda: c.sigma([rows[0]] * 3, [inp.eps[rows[0]], -21.0, 0.7], g),
                         lambda: c.residues([rows[0]] * 70, list(range(70 % (n_occ + n_virt))) *
                                            0 + [m % (n_occ + n_virt) for m in range(70)],
                                            np.linspace(-1, 22, 70)),
                         lambda: c.qp(list(rows), g),
                         lambda: c.evgw(list(rows), g, mode="evgw0", n_cycles=2),
                         lambda: c.evgw(list(rows), g, mode="evgw", n_cycles=2)) + (
                            (lambda: c.rpa_excitations(), lambda: c.qp_sd(list(rows)))
                            if n_occ * n_virt <= 16384 else ()):
                try:
                    call()
                except gwl.GWError as e:
                    if e.code != gwl.GW_EAUDIT:
                        raise
                else:
                    raise AssertionError("audit mode returned results")
            n = gwl.audit_launch_count() - before
        print(f"case {n_occ}/{n_virt}/{n_aux} rows={len(rows)} G={G} {prec}/wc {wc}: {n} launches checked",
              flush=True)


def run_budget_case(n_occ, n_virt, n_aux, G):
    """A context held to exactly its footprint: residue batches of 70, 150 and
    200 systems (MINRES capacities of 128, 192 and 256, whose split rules
    differ) must all stay inside it."""
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=1)
    rows = (n_occ - 1, n_occ)
    inp = gwgen.make_inputs(shape, 2, rows)
    n_mo = n_occ + n_virt
    fp = gwl.footprint(n_mo, n_occ, n_aux, len(rows), 1, G)
    g = gwl.Grid.gauss_legendre(G)
    with gwl.Context.from_inputs(inp, mem_budget_bytes=fp) as c:
        calls = [lambda: c.wtable(g)] + [
            (lambda k=k: c.residues([rows[0]] * k, [m % n_mo for m in range(k)],
                                    np.linspace(-1, 22, k))) for k in (70, 150, 200)]
        for call in calls:   # the W^c table's workspace first, as in a QP call
            try:
                call()
            except gwl.GWError as e:
                if e.code != gwl.GW_EAUDIT:
                    raise
    print(f"budget case {n_occ}/{n_virt}/{n_aux}: MINRES capacities 128, 192, 256 within "
          f"the footprint ({fp / 2**20:.0f} MiB)", flush=True)


def run_uhf_case(n_occ, n_virt, n_aux, rows, G):
    """Open-shell context: both spins' transitions stacked in one operator."""
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=1)
    inp = gwgen.make_inputs_uhf(shape, 2, rows)
    g = gwl.Grid.gauss_legendre(G)
    n_mo = inp.n_mo
    for prec in ("fp64", "bf16x3"):
        c = gwl.Context.from_inputs_uhf(inp, pi_prec=prec, wc_prec=prec)
        before = gwl.audit_launch_count()
        for call in (lambda: c.dielectric([0.1]), lambda: c.cholesky([0.3]),
                     lambda: c.wtable(g),
                     lambda: c.sigma([rows[0], rows[-1]], [inp.eps[0][1], -0.3], g),
                     lambda: c.residues([rows[-1]] * 5, [0, 1, 2, 3, n_mo - 1],
                                        np.linspace(-1, 2, 5)),
                     lambda: c.qp(list(rows), g), lambda: c.qp_sd(list(rows))):
            try:
                call()
            except gwl.GWError as e:
                if e.code != gwl.GW_EAUDIT:
                    raise
            else:
                raise AssertionError("audit mode returned results")
        n = gwl.audit_launch_count() - before
        c.close()
        print(f"uhf case {n_occ}/{n_virt}/{n_aux} rows={len(rows)} G={G} {prec}: {n} launches "
              f"checked", flush=True)


def run_group_case(ks, G):
    """The server's grouped stage A (several requests of one padded shape in
    one launch sequence), then each member's QP stage."""
    for prec, wc in (("fp64", "fp64"), ("fp32", "fp64"), ("bf16x3", "bf16x3")):
        ctxs = [gwl.Context.from_inputs(gwgen.serving_inputs(k, 1000 + j), pi_prec=prec, wc_prec=wc)
                for j, k in enumerate(ks)]
        g = gwl.Grid.gauss_legendre(G)
        before = gwl.audit_launch_count()
        try:
            gwl.group_stage_a(ctxs, g, use_graph=False)
        except gwl.GWError as e:
            if e.code != gwl.GW_EAUDIT:
                raise
        for c, k in zip(ctxs, ks):
            try:
                c.qp(list(c.row_ids), g)
            except gwl.GWError as e:
                if e.code != gwl.GW_EAUDIT:
                    raise
            c.close()
        n = gwl.audit_launch_count() - before
        print(f"group case k={ks} G={G} {prec}/wc {wc}: {n} launches checked", flush=True)


def run_server_case(reqs, G, prec, wc, streams):
    """The request server in audit mode: admission, batching by shape (grouped
    stage A through the block cache), QP stages; every request must end with
    GW_EAUDIT (all its launches checked), none with a refused launch."""
    g = gwl.Grid.gauss_legendre(G)
    before = gwl.audit_launch_count()
    with gwl.Server(g, pi_prec=prec, wc_prec=wc, n_streams=streams) as srv:
        ts = [srv.submit_inputs(r, list(r.row_ids)) for r in reqs]
        srv.drain()
        st = srv.stats()
        infos = [srv.poll(t)[4] for t in ts]
    rcs = [i["rc"] for i in infos]
    bad = [rc for rc in rcs if rc != gwl.GW_EAUDIT]
    if bad:
        raise AssertionError(f"server case {prec}/{wc}: request codes {rcs}: "
                             f"{gwl._lib.gw_last_error().decode()}")
    # admission reserves what gw_footprint states for the request's context
    # (the server's default work budget is 2 GiB)
    for r, i in zip(reqs, infos):
        want = gwl.footprint(r.shape.n_mo, r.n_occ, r.shape.n_aux, len(r.row_ids),
                             len(r.row_ids), G, prec, 2 << 30, wc_prec=wc)
        if i["footprint_bytes"] != want:
            raise AssertionError(f"server case {prec}/{wc}: footprint {i['footprint_bytes']} "
                                 f"against gw_footprint {want}")
    n = gwl.audit_launch_count() - before
    print(f"server case {len(reqs)} requests G={G} {prec}/wc {wc}: {n} launches checked, "
          f"{st['batches']} batches of {st['batched_requests']} requests", flush=True)


def run_wide_case(n_occ, n_virt, n_aux, rows, G, n_sys):
    """One MINRES batch of n_sys > 256 systems (padded to whole 128-row pass
    tiles)."""
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=1)
    inp = gwgen.make_inputs(shape, 1, rows)
    g = gwl.Grid.gauss_legendre(G)
    n_mo = n_occ + n_virt
    for prec, wc in (("fp64", "fp64"), ("bf16x3", "bf16x3")):
        with gwl.Context.from_inputs(inp, pi_prec=prec, wc_prec=wc, minres_batch=512) as c:
            before = gwl.audit_launch_count()
            for call in (lambda: c.cholesky([0.3, 1.0]), lambda: c.wtable(g),
                         lambda: c.residues([rows[0]] * n_sys, [m % n_mo for m in range(n_sys)],
                                            np.linspace(-1, 22, n_sys)),
                         lambda: c.qp(list(rows), g)):
                try:
                    call()
                except gwl.GWError as e:
                    if e.code != gwl.GW_EAUDIT:
                        raise
                else:
                    raise AssertionError("audit mode returned results")
            n = gwl.audit_launch_count() - before
        print(f"wide case {n_occ}/{n_virt}/{n_aux} G={G} systems={n_sys} {prec}/wc {wc}: "
              f"{n} launches checked", flush=True)


def main():
    gwl.audit_enable()
    small = []
    for k, seed in ((1, 11), (3, 12), (2, 13)):
        shape = gwgen.custom_shape(5 * k, 38 * k, 112 * k, n_core=k)
        small.append(gwgen.make_inputs(shape, seed, [5 * k - 1, 5 * k]))
    for prec, wc in (("bf16x3", "bf16x3"), ("fp64", "fp64")):
        run_server_case(small, 32, prec, wc, 2)
        run_server_case([gwgen.serving_inputs(k, 1000 + j) for j, k in
                         enumerate([1, 2, 1, 3, 1, 2, 9])], 16, prec, wc, 1)
    for case in CASES:
        run_case(*case)
    run_group_case([1, 1, 1], 64)
    run_group_case([3, 3], 16)
    run_group_case([6, 6, 6, 6], 8)
    run_budget_case(40, 900, 1152, 4)
    run_uhf_case(6, 40, 150, (3, 6, 46 + 4, 46 + 5), 6)
    run_uhf_case(1, 3, 20, (0, 4, 5), 3)
    run_wide_case(7, 45, 200, (4, 5, 6), 8, 300)
    run_wide_case(17, 63, 129, (16, 17, 40), 7, 257)
    run_wide_case(3, 20, 2100, (1, 2), 4, 390)
    print("audit ok")


if __name__ == "__main__":
    main()
