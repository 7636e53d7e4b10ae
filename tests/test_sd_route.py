"""Parity of the spectral-decomposition (Casida) route on the GPU (gw_qp_sd,
gw_rpa_excitations, through the C-ABI) with the oracle's Casida route
(oracle/sd.py), and agreement of the two GPU routes with each other.

Tolerances: excitation energies 1e-12 relative to the largest; QP energies
1e-10 relative (FP64 throughout); SD against CD on the GPU within the
128-point quadrature's error (1e-7 Ha)."""
import numpy as np
import pytest

import gwgen
from oracle import qp, sd

pytestmark = pytest.mark.gpu


def gwl():
    import paper_2107_10423_amd as m
    return m


def oracle_sd_qp(eps, n_occ, rho_rows, Omega, states, tol=1e-12):
    out = []
    for k, n in enumerate(states):
        def fe(w, k=k, n=n):
            s, ds = sd.sigma_c(eps, n_occ, rho_rows[k], Omega, w)
            return eps[n] + s - w, ds - 1.0
        out.append(qp.step_tree(fe, eps[n], tol=tol))
    return out


@pytest.mark.parametrize("shape", [None, (7, 45, 200), (3, 20, 64)])
def test_excitations_and_qp_match_the_oracle(shape):
    if shape is None:
        inp = gwgen.make_config("monomer")
    else:
        inp = gwgen.make_inputs(gwgen.custom_shape(*shape, n_core=1), 5,
                                list(range(shape[0] - 2, shape[0] + 2)))
    states = [int(r) for r in inp.row_ids]
    Omega, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    rho = [sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[k]) for k in range(len(states))]
    ref = oracle_sd_qp(inp.eps, inp.n_occ, rho, Omega, states)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp_sd(states)
        t = c.timing()
        om = c.rpa_excitations()
        E2, _, _, _ = c.qp_sd(states)            # decomposition kept in the context
        t2 = c.timing()
    print(f"N_ov {om.size}: {t['sd_sweeps']} Jacobi sweeps, {t['sd_ms']:.1f} ms", flush=True)
    assert np.abs(om - np.sort(Omega)).max() <= 1e-12 * Omega.max()
    for j, r in enumerate(ref):
        assert st[j] == r["status"] == 0
        assert abs(E[j] - r["E"]) <= 1e-10 * abs(r["E"]), (states[j], E[j] - r["E"])
        assert abs(Z[j] - r["Z"]) <= 1e-9
    assert np.array_equal(E, E2) and t2["sd_ms"] == 0.0


def test_sd_and_cd_routes_agree_on_the_gpu():
    inp = gwgen.make_inputs(gwgen.custom_shape(7, 45, 200, n_core=1), 5, [4, 5, 6, 7, 8])
    states = [4, 5, 6, 7, 8]
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E_sd, _, Z_sd, _ = c.qp_sd(states)
        E_cd, _, Z_cd, _ = c.qp(states, gwl().Grid.gauss_legendre(128))
    assert np.abs(E_sd - E_cd).max() < 1e-7
    assert np.abs(Z_sd - Z_cd).max() < 1e-6


def test_open_shell_sd_route():
    shape = gwgen.custom_shape(4, 20, 40, n_core=1)
    n_mo = shape.n_mo
    rows = [3, 4, 5, n_mo + 3, n_mo + 4]
    u = gwgen.make_inputs_uhf(shape, 7, rows)
    Omega, T, D, Bc = sd.casida_uhf(u.eps, u.n_occ, u.B_ov)
    with gwl().Context.from_inputs_uhf(u, qp_tol=1e-12) as c:
        om = c.rpa_excitations()
        E, S, Z, st = c.qp_sd(rows)
    assert np.abs(om - np.sort(Omega)).max() <= 1e-12 * Omega.max()
    for k, p in enumerate(rows):
        s, n = divmod(p, n_mo)
        rho = sd.pole_strengths_uhf(Bc, D, T, u.B_rows[k])

        def fe(w, s=s, n=n, rho=rho):
            sg, ds = sd.sigma_c(u.eps[s], u.n_occ[s], rho, Omega, w)
            return u.eps[s][n] + sg - w, ds - 1.0

        r = qp.step_tree(fe, u.eps[s][n], tol=1e-12)
        assert abs(E[k] - r["E"]) <= 1e-10 * abs(r["E"]), (p, E[k] - r["E"])


def test_large_systems_are_refused():
    inp = gwgen.make_config("h2o10", states=[49])       # N_ov = 19 000
    with gwl().Context.from_inputs(inp) as c:
        with pytest.raises(gwl().GWError):
            c.qp_sd([49])
