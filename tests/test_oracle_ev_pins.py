"""Pins of the eigenvalue-self-consistent oracle (oracle/ev.py), CPU only.

The contour-deformation evGW0 / evGW cycles are checked against the same
cycles run on the spectral-decomposition (Casida) route, whose Sigma^c has
the G poles written out explicitly (eps_m -/+ Omega_s) and whose W comes from
the Casida excitations of the energies in W: a plumbing mistake (updated
energies in the wrong place, W not rebuilt for evGW, the wrong constant term
of the QP equation) changes the CD energies but not the SD ones.
"""
import dataclasses

import numpy as np
import pytest

import gwgen
from oracle import cd, ev, grid, qp, sd


def small(seed=11):
    shape = gwgen.custom_shape(3, 12, 30, n_core=1)
    return gwgen.make_inputs(shape, seed, [2, 3])


def sd_cycles(inp, states, mode, n_cycles, tol=1e-12):
    """The evGW cycles on the SD route (independent of cd/ev)."""
    eps_ref = np.array(inp.eps, dtype=np.float64)
    eps_g = eps_ref.copy()
    rows = [int(r) for r in inp.row_ids]
    hist = []
    for cyc in range(n_cycles):
        eps_w = eps_ref if mode == "evgw0" else eps_g.copy()
        Omega, T, D = sd.casida(eps_w, inp.n_occ, inp.B_ov)
        E = []
        for n in states:
            rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[rows.index(n)])

            def fe(w, n=n, rho=rho):
                s, ds = sd.sigma_c(eps_g, inp.n_occ, rho, Omega, w)
                return eps_ref[n] + s - w, ds - 1.0

            E.append(qp.step_tree(fe, eps_g[n], tol=tol)["E"])
        E = np.array(E)
        hist.append(E)
        for k, n in enumerate(states):
            eps_g[n] = E[k]
    return hist


def test_one_cycle_is_g0w0():
    inp = small()
    xi, z = grid.gauss_legendre(48)
    res, cyc, hist = ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, [2, 3],
                             xi, z, mode="evgw0", n_cycles=1, tol=1e-12)
    ref = qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, [2, 3], xi, z,
                   tol=1e-12)
    assert cyc == 1
    # evGW integrates the static part of the I term exactly; one cycle differs
    # from G0W0's plain quadrature by that quadrature's error only
    for a, b in zip(res, ref):
        assert abs(a["E"] - b["E"]) < 1e-9 and abs(a["Z"] - b["Z"]) < 1e-9


def test_split_quadrature_near_a_pole():
    """Sigma^c with the static part split off matches the SD route next to the
    state's own G pole, where the plain quadrature is far off."""
    inp = small()
    xi, z = grid.gauss_legendre(128)
    rows = [int(r) for r in inp.row_ids]
    Omega, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    wtab = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi)
    w0 = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, np.zeros(1))[:, :, 0]
    worst_plain = 0.0
    for n in (2, 3):
        r = rows.index(n)
        rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[r])
        for d in (-1e-3, -1e-5, -1e-7, 1e-7, 1e-5, 1e-3):
            w = inp.eps[n] + d
            ref, dref = sd.sigma_c(inp.eps, inp.n_occ, rho, Omega, w)
            s, ds, _ = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[r], wtab[r], xi, z,
                                  w, w0_row=w0[r])
            p, _, _ = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[r], wtab[r], xi, z, w)
            assert abs(s - ref) < 1e-9
            assert abs(ds - dref) < 1e-6 * max(1.0, abs(dref))
            worst_plain = max(worst_plain, abs(p - ref))
    assert worst_plain > 1e-3


def test_zero_coupling_keeps_eigenvalues():
    inp = small()
    zero = dataclasses.replace(inp, B_ov=0 * inp.B_ov, B_rows=0 * inp.B_rows)
    xi, z = grid.gauss_legendre(16)
    for mode in ("evgw0", "evgw"):
        res, cyc, hist = ev.evgw(zero.eps, zero.n_occ, zero.B_ov, zero.row_ids, zero.B_rows,
                                 [2, 3], xi, z, mode=mode, n_cycles=3, tol=1e-13)
        for E in hist:
            np.testing.assert_allclose(E, zero.eps[[2, 3]], rtol=0, atol=1e-13)


@pytest.mark.parametrize("mode", ["evgw0", "evgw"])
def test_cycles_match_spectral_route(mode):
    inp = small()
    xi, z = grid.gauss_legendre(128)
    states = [2, 3]
    res, cyc, hist = ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states,
                             xi, z, mode=mode, n_cycles=3, tol=1e-12)
    ref = sd_cycles(inp, states, mode, 3)
    for c, (a, b) in enumerate(zip(hist, ref)):
        print(mode, c, a, a - b)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-8)
    # the cycles moved the energies (otherwise the comparison pins nothing)
    assert np.max(np.abs(hist[1] - hist[0])) > 1e-4
    if mode == "evgw":
        g0 = sd_cycles(inp, states, "evgw0", 3)
        assert np.max(np.abs(np.array(ref[2]) - np.array(g0[2]))) > 1e-5


def test_tolerance_stops_early():
    inp = small()
    xi, z = grid.gauss_legendre(48)
    res, cyc, hist = ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, [2, 3],
                             xi, z, mode="evgw0", n_cycles=20, ev_tol=1e-6, tol=1e-12)
    assert cyc < 20
    assert np.max(np.abs(hist[-1] - hist[-2])) < 1e-6
    assert np.max(np.abs(hist[-2] - hist[-3])) >= 1e-6
