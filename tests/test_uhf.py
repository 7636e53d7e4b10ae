"""Parity of open-shell contexts (gw_setup_uhf, through the C-ABI) with the
FP64 open-shell oracle (oracle/uhf.py).

Tolerances as for closed shell: Pi 1e-12 relative, Sigma^c and QP energies
1e-10 relative in FP64, mixed-precision Pi within 1 meV."""
import numpy as np
import pytest

import gwgen
from oracle import cluster, grid, qp, uhf

pytestmark = pytest.mark.gpu

MEV = 1e-3 / 27.211386245988   # 1 meV in Hartree


def gwl():
    import paper_2107_10423_amd as m
    return m


def doublet(n_unpaired=1, same=False, seed=9):
    # N_aux = 200 (two Pi tiles, ragged); spin up carries the unpaired electron
    shape = gwgen.custom_shape(7, 45, 200, n_core=1)
    n_mo = shape.n_mo
    rows = [0, 5, 6, 7, 8, n_mo + 0, n_mo + 5, n_mo + 6, n_mo + 7, n_mo + 8]
    return gwgen.make_inputs_uhf(shape, seed, rows, n_unpaired=n_unpaired, same_spins=same)


def test_dielectric_open_shell():
    u = doublet()
    xis = np.array([1e-3, 0.4, 30.0])
    with gwl().Context.from_inputs_uhf(u) as c:
        got = c.dielectric(xis)
    for g, x in enumerate(xis):
        Pi = uhf.pi_imag(u.eps, u.n_occ, u.B_ov, x)
        ref = np.tril(np.eye(u.n_aux) - Pi)
        assert np.abs(got[g] - ref).max() <= 1e-12 * np.abs(Pi).max()


def test_qp_open_shell_matches_oracle():
    u = doublet()
    states = [int(p) for p in u.row_ids]
    xi, z = grid.gauss_legendre(48)
    ref = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, states, xi, z, tol=1e-12)
    with gwl().Context.from_inputs_uhf(u, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(states, gwl().Grid.gauss_legendre(48))
    for j, r in enumerate(ref):
        assert st[j] == r["status"], (states[j], st[j], r["status"])
        assert abs(E[j] - r["E"]) <= 1e-10 * abs(r["E"]), (states[j], E[j] - r["E"])
        assert abs(S[j] - r["sigma_c"]) <= 1e-10 * abs(r["sigma_c"]) + 1e-12
        assert abs(Z[j] - r["Z"]) <= 1e-9
    # the two spins of one orbital index differ (the unpaired electron)
    assert abs(E[1] - E[6]) > 1e-3


def test_sigma_fixed_omega_open_shell():
    u = doublet()
    n_mo = u.n_mo
    xi, z = grid.gauss_legendre(32)
    wt = uhf.w_table(u.eps, u.n_occ, u.B_ov, u.B_rows, xi)
    rows = [int(p) for p in u.row_ids]
    cases = [(rows[1], -0.9), (rows[6], -0.9), (rows[3], u.eps[0][7]), (rows[8], u.eps[1][8]),
             (rows[0], -20.3), (rows[5], 0.6)]
    with gwl().Context.from_inputs_uhf(u) as c:
        sg, dsg, nres = c.sigma([p for p, _ in cases], [w for _, w in cases],
                                gwl().Grid.gauss_legendre(32))
    for j, (p, w) in enumerate(cases):
        s, n = divmod(p, n_mo)
        r = rows.index(p)
        ref, dref, nr = uhf.sigma_c(u.eps, u.n_occ, u.B_ov, s, u.B_rows[r], wt[r], xi, z, w)
        assert nres[j] == nr
        assert abs(sg[j] - ref) <= 1e-10 * abs(ref) + 1e-13, (p, w)
        assert abs(dsg[j] - dref) <= 1e-9 * max(1.0, abs(dref)), (p, w)


def test_equal_spins_equal_the_closed_shell_path():
    u = doublet(n_unpaired=0, same=True)
    c_in = gwgen.make_inputs(gwgen.custom_shape(7, 45, 200, n_core=1), 9, [0, 5, 6, 7, 8])
    g = gwl().Grid.gauss_legendre(48)
    with gwl().Context.from_inputs(c_in, qp_tol=1e-12) as c:
        E0, S0, Z0, _ = c.qp([0, 5, 6, 7, 8], g)
    n_mo = u.n_mo
    with gwl().Context.from_inputs_uhf(u, qp_tol=1e-12) as c:
        E1, S1, Z1, _ = c.qp([0, 5, 6, 7, 8] + [n_mo + k for k in (0, 5, 6, 7, 8)], g)
    assert np.all(np.abs(E1[:5] - E0) <= 1e-10 * np.abs(E0))
    assert np.all(np.abs(E1[5:] - E0) <= 1e-10 * np.abs(E0))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_open_shell(prec):
    u = doublet()
    states = [int(p) for p in u.row_ids]
    xi, z = grid.gauss_legendre(48)
    ref = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, states, xi, z, tol=1e-12)
    with gwl().Context.from_inputs_uhf(u, pi_prec=prec, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(states, gwl().Grid.gauss_legendre(48))
    assert max(abs(E[j] - r["E"]) for j, r in enumerate(ref)) <= MEV


def test_cluster_layer_open_shell():
    """The cluster layer groups by the levels of each state's own spin."""
    u = doublet()
    n_mo = u.n_mo
    states = [int(p) for p in u.row_ids]
    xi, z = grid.gauss_legendre(48)
    wt = uhf.w_table(u.eps, u.n_occ, u.B_ov, u.B_rows, xi)
    fevals, starts = [], []
    for r, p in enumerate(states):
        s, n = divmod(p, n_mo)

        def fe(w, r=r, s=s, n=n):
            sg, ds, _ = uhf.sigma_c(u.eps, u.n_occ, u.B_ov, s, u.B_rows[r], wt[r], xi, z, w)
            return u.eps[s][n] + sg - w, ds - 1.0

        fevals.append(fe)
        starts.append(float(u.eps[s][n]))
    ref = cluster.solve_states(fevals, starts, 0.2, tol=1e-12)
    with gwl().Context.from_inputs_uhf(u, qp_tol=1e-12, cluster_width=0.2) as c:
        E, S, Z, st = c.qp(states, gwl().Grid.gauss_legendre(48))
    for j, r in enumerate(ref):
        assert st[j] == r["status"]
        assert abs(E[j] - r["E"]) <= 1e-10 * abs(r["E"]), (states[j], E[j] - r["E"])


def test_open_shell_refusals():
    u = doublet()
    g = gwl().Grid.gauss_legendre(8)
    with gwl().Context.from_inputs_uhf(u) as c:
        with pytest.raises(gwl().GWError):
            c.evgw([5], g)                      # evGW is closed-shell only
        with pytest.raises(gwl().GWError):
            c.qp([4], g)                        # spin-up orbital 4: no row supplied
