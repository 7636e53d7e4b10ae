"""Pins of the open-shell oracle (oracle/uhf.py), CPU only: equal spins
reduce to the closed-shell oracle; W^c and Sigma^c equal the spin-block
Casida route's closed forms (an independent formula); spin swap symmetry;
Pi is negative semidefinite."""
import numpy as np
import pytest

import gwgen
from oracle import cd, grid, qp, sd, uhf


def doublet(seed=7, n_unpaired=1, rows=(3, 4, 5), same=False):
    shape = gwgen.custom_shape(4, 20, 40, n_core=1)
    n_mo = shape.n_mo
    ids = list(rows) + [n_mo + r for r in rows]
    return gwgen.make_inputs_uhf(shape, seed, ids, n_unpaired=n_unpaired, same_spins=same)


def test_equal_spins_are_the_closed_shell():
    u = doublet(n_unpaired=0, same=True)
    c = gwgen.make_inputs(gwgen.custom_shape(4, 20, 40, n_core=1), 7, [3, 4, 5])
    assert np.array_equal(u.eps[0], c.eps) and np.array_equal(u.eps[1], c.eps)
    for x in (0.0, 0.3, 4.0):
        a = uhf.pi_imag(u.eps, u.n_occ, u.B_ov, x)
        b = cd.pi_imag(c.eps, c.n_occ, c.B_ov, x)
        assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()
    xi, z = grid.gauss_legendre(32)
    ref = qp.solve(c.eps, c.n_occ, c.B_ov, c.row_ids, c.B_rows, [3, 4, 5], xi, z, tol=1e-12)
    got = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, [3, 4, 5, 27, 28, 29], xi, z,
                    tol=1e-12)
    for k in range(3):
        for r in (got[k], got[k + 3]):
            assert abs(r["E"] - ref[k]["E"]) < 1e-12 and abs(r["Z"] - ref[k]["Z"]) < 1e-10


def test_pi_is_negative_semidefinite():
    u = doublet()
    for x in (0.0, 0.1, 2.0):
        assert np.linalg.eigvalsh(uhf.pi_imag(u.eps, u.n_occ, u.B_ov, x)).max() <= 1e-14


def test_w_and_sigma_match_the_spin_block_casida_route():
    u = doublet()
    Omega, T, D, Bc = sd.casida_uhf(u.eps, u.n_occ, u.B_ov)
    n_mo = u.n_mo
    xi = np.array([0.0, 0.05, 0.7, 9.0])
    wt = uhf.w_table(u.eps, u.n_occ, u.B_ov, u.B_rows, xi)
    gx, gz = grid.gauss_legendre(200)
    wtab = uhf.w_table(u.eps, u.n_occ, u.B_ov, u.B_rows, gx)
    for r, p in enumerate(u.row_ids):
        s, n = divmod(int(p), n_mo)
        rho = sd.pole_strengths_uhf(Bc, D, T, u.B_rows[r])
        for g, x in enumerate(xi):
            ref = sd.screened(rho, Omega, -x * x)
            scale = np.abs(np.sum(u.B_rows[r] ** 2, axis=-1)).max()
            assert np.abs(wt[r, :, g] - ref).max() <= 1e-12 * scale
        # real frequency (a residue frequency away from every Omega)
        w = 0.37 * Omega.min()
        wc, dwc = uhf.residue_value(u.eps, u.n_occ, u.B_ov, u.B_rows[r][2], w)
        ref_wc = sd.screened(rho[2], Omega, w * w)
        ref_dwc = -np.sum(rho[2] ** 2 * 2 * w / (Omega ** 2 - w * w) ** 2)
        assert abs(wc - ref_wc) < 1e-12 and abs(dwc - ref_dwc) < 1e-11
        # Sigma^c on a frequency grid (points within 0.05 Ha of a level of the
        # state's spin skipped: the quadrature of a/(a^2 + xi^2) needs |a| well
        # above the first nodes) and exactly at the levels (theta(0) = 1/2)
        poles = sd.poles(u.eps[s], u.n_occ[s], Omega)
        ws = [w for w in np.linspace(-1.6, 1.2, 15) if np.abs(w - u.eps[s]).min() > 0.05]
        ws += list(u.eps[s][2:7])
        for w in ws:
            if np.abs(poles - w).min() < 1e-3:
                continue
            sg, dsg, _ = uhf.sigma_c(u.eps, u.n_occ, u.B_ov, s, u.B_rows[r], wtab[r], gx, gz, w)
            ref_s, ref_d = sd.sigma_c(u.eps[s], u.n_occ[s], rho, Omega, w)
            assert abs(sg - ref_s) < 1e-10, (p, w, sg - ref_s)
            if w not in u.eps[s]:
                assert abs(dsg - ref_d) < 1e-8 * max(1, abs(ref_d)), (p, w)


def test_spin_swap():
    u = doublet()
    n_mo = u.n_mo
    sw = gwgen.InputsUHF(n_mo=n_mo, n_occ=u.n_occ[::-1], n_aux=u.n_aux, seed=u.seed,
                         eps=u.eps[::-1].copy(), B_ov=u.B_ov[::-1],
                         row_ids=np.array([(p + n_mo) % (2 * n_mo) for p in u.row_ids],
                                          dtype=np.int32),
                         B_rows=u.B_rows)
    a, b = uhf.pi_imag(u.eps, u.n_occ, u.B_ov, 0.4), uhf.pi_imag(sw.eps, sw.n_occ, sw.B_ov, 0.4)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(a).max()
    xi, z = grid.gauss_legendre(32)
    states = [4, n_mo + 4]
    a = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, states, xi, z, tol=1e-12)
    b = uhf.solve(sw.eps, sw.n_occ, sw.B_ov, sw.row_ids, sw.B_rows, [n_mo + 4, 4], xi, z,
                  tol=1e-12)
    for x, y in zip(a, b):
        assert abs(x["E"] - y["E"]) < 1e-12


def test_qp_energies_match_the_casida_route():
    u = doublet()
    n_mo = u.n_mo
    xi, z = grid.gauss_legendre(128)
    states = [int(p) for p in u.row_ids]
    got = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, states, xi, z, tol=1e-12)
    Omega, T, D, Bc = sd.casida_uhf(u.eps, u.n_occ, u.B_ov)
    for r, p in enumerate(states):
        s, n = divmod(p, n_mo)
        rho = sd.pole_strengths_uhf(Bc, D, T, u.B_rows[r])

        def fe(w, s=s, n=n, rho=rho):
            sg, ds = sd.sigma_c(u.eps[s], u.n_occ[s], rho, Omega, w)
            return u.eps[s][n] + sg - w, ds - 1.0

        ref = qp.step_tree(fe, u.eps[s][n], tol=1e-12)
        assert got[r]["status"] == 0 and ref["status"] == 0
        assert abs(got[r]["E"] - ref["E"]) < 1e-8, (p, got[r]["E"] - ref["E"])
    # the unpaired electron makes the spins differ
    assert abs(got[1]["E"] - got[4]["E"]) > 1e-3
