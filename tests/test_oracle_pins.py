"""Pins of the FP64 oracle against things other than itself: closed forms,
the paper's literal complex-valued polarizability with an explicit spin sum,
the independent spectral-decomposition (Casida) route, invariants, a
two-level model solved as a polynomial, and brute-force root scans."""
import math

import numpy as np
import pytest

import gwgen
from oracle import cd, grid, qp, sd


def tiny(n_occ=3, n_virt=7, n_aux=11, seed=7, b_scale=1.0, n_core=1):
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=n_core)
    return gwgen.make_inputs(shape, seed, range(n_occ + n_virt), b_scale=b_scale)


# --- quadrature grid -------------------------------------------------------

@pytest.mark.parametrize("G,tol", [(64, 1e-10), (128, 1e-12), (200, 1e-12)])
def test_grid_lorentzian_closed_form(G, tol):
    # int_0^inf d xi / (Omega^2 + xi^2) = pi / (2 Omega)
    xi, z = grid.gauss_legendre(G)
    for om in np.logspace(np.log10(0.05), np.log10(25.0), 40):
        exact = math.pi / (2 * om)
        assert abs(np.sum(z / (om * om + xi * xi)) - exact) <= tol * exact


@pytest.mark.parametrize("G,tol", [(64, 1e-9), (128, 1e-12)])
def test_grid_sign_integral_and_pole_piece(G, tol):
    # (1/pi) int_0^inf a/(a^2+xi^2) d xi = sgn(a)/2 and
    # int_0^inf a/((a^2+xi^2)(W^2+xi^2)) d xi = (pi/2) sgn(a) / (W (W + |a|))
    xi, z = grid.gauss_legendre(G)
    for a in np.concatenate([-np.logspace(-2, 1.3, 15), np.logspace(-2, 1.3, 15)]):
        assert abs(np.sum(z * a / (a * a + xi * xi)) / math.pi - math.copysign(0.5, a)) < tol
        for W in (0.3, 1.0, 5.0, 22.0):
            ex = (math.pi / 2) * math.copysign(1, a) / (W * (W + abs(a)))
            got = np.sum(z * a / ((a * a + xi * xi) * (W * W + xi * xi)))
            assert abs(got - ex) <= 10 * tol * abs(ex)


def test_grid_range():
    xi, z = grid.gauss_legendre(64)
    assert np.all(np.diff(xi) > 0) and np.all(z > 0)
    assert 1.7e-4 < xi[0] < 1.8e-4 and 1.4e3 < xi[-1] < 1.5e3


# --- polarizability --------------------------------------------------------

def _pi_literal(eps, n_occ, B_ov, omega, eta=1e-13):
    """The paper's Pi_PQ(omega) typed as printed: complex frequency factors,
    an explicit loop over both spins and over i, a (pure Python)."""
    n_aux = B_ov.shape[0]
    n_virt = len(eps) - n_occ
    out = np.zeros((n_aux, n_aux), dtype=complex)
    for P in range(n_aux):
        for Q in range(n_aux):
            acc = 0j
            for _spin in (0, 1):
                for i in range(n_occ):
                    for a in range(n_virt):
                        ia = i * n_virt + a
                        ea, ei = eps[n_occ + a], eps[i]
                        fac = 1 / (omega - ea + ei + 1j * eta) + 1 / (-omega - ea + ei + 1j * eta)
                        acc += B_ov[P, ia] * fac * B_ov[Q, ia]
            out[P, Q] = acc
    return out


def test_pi_matches_literal_spin_summed_formula():
    inp = tiny(2, 3, 4)
    for xi in (0.0, 0.37, 4.0):
        lit = _pi_literal(inp.eps, inp.n_occ, inp.B_ov, 1j * xi)
        got = cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, xi)
        assert np.abs(lit.imag).max() < 1e-10
        np.testing.assert_allclose(got, lit.real, rtol=1e-12, atol=1e-14)
    for w in (0.1, 0.9):   # real frequency: principal value (eta -> 0+)
        lit = _pi_literal(inp.eps, inp.n_occ, inp.B_ov, w)
        got = cd.pi_real(inp.eps, inp.n_occ, inp.B_ov, w)
        np.testing.assert_allclose(got, lit.real, rtol=1e-9, atol=1e-12)


def test_pi_symmetric_negative_and_limits():
    inp = tiny(4, 9, 13)
    for xi in (1e-4, 0.2, 3.0, 1e3):
        P = cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, xi)
        assert np.abs(P - P.T).max() <= 1e-15 * np.abs(P).max()
        assert np.linalg.eigvalsh(P).max() < 1e-15      # Pi(i xi) <= 0: 1 - Pi is SPD
    # decays with xi, and vanishes for B = 0
    p1 = np.abs(cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, 10.0)).max()
    p2 = np.abs(cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, 1000.0)).max()
    assert p2 < 1e-3 * p1
    zero = tiny(4, 9, 13, b_scale=0.0)
    assert np.abs(cd.pi_imag(zero.eps, zero.n_occ, zero.B_ov, 0.3)).max() == 0.0


def test_pi_aux_rotation_covariance():
    inp = tiny(3, 8, 10)
    O, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((10, 10)))
    P = cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, 0.4)
    PO = cd.pi_imag(inp.eps, inp.n_occ, O @ inp.B_ov, 0.4)
    np.testing.assert_allclose(PO, O @ P @ O.T, atol=1e-14)


# --- screened interaction against the spectral decomposition ---------------

def test_wc_matches_casida_imaginary_and_real():
    inp = tiny(3, 8, 12)
    Om, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    b = inp.B_rows[2]                       # all (n=2, m) vectors
    rho = sd.pole_strengths(inp.B_ov, D, T, b)
    for xi in (0.0, 0.7, 25.0):
        got = cd.screened_from_pi(cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, xi), b)
        ref = sd.screened(rho, Om, -xi * xi)
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-15)
        assert np.all(got <= 0) and np.all(got >= -np.sum(b * b, axis=1) - 1e-15)
    for w in (0.2, 3.0, 10.0):
        got = np.array([cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b[m], w)[0]
                        for m in range(b.shape[0])])
        ref = sd.screened(rho, Om, w * w)
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-13)


def test_wc_derivative_matches_casida():
    inp = tiny(3, 8, 12)
    Om, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    b = inp.B_rows[1]
    rho = sd.pole_strengths(inp.B_ov, D, T, b)
    for w in (0.15, 2.0):
        for m in (0, 4, 9):
            got = cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b[m], w)[1]
            # d/dw [-rho^2 / (Om^2 - w^2)] = -2 w rho^2 / (Om^2 - w^2)^2
            ref = -np.sum(2 * w * rho[m] ** 2 / (Om * Om - w * w) ** 2)
            assert abs(got - ref) <= 1e-9 * abs(ref) + 1e-14


# --- self-energy: contour deformation against spectral decomposition -------

@pytest.mark.parametrize("seed", [11, 12])
def test_sigma_cd_matches_sd(seed):
    inp = tiny(4, 9, 14, seed=seed)
    xi, z = grid.gauss_legendre(128)
    Om, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    for n in (2, 3, 4, 5):
        wt = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[n:n + 1], xi)[0]
        rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[n])
        ws = list(np.linspace(-1.6, 1.2, 23)) + list(inp.eps[2:7])
        for w in ws:
            if np.min(np.abs(w - inp.eps)) < 1e-2 and w not in inp.eps:
                continue
            s_cd, ds_cd, _ = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[n], wt, xi, z, w)
            s_sd, ds_sd = sd.sigma_c(inp.eps, inp.n_occ, rho, Om, w)
            assert abs(s_cd - s_sd) < 1e-11, (n, w)
            if w not in inp.eps:
                assert abs(ds_cd - ds_sd) < 1e-9 * max(1, abs(ds_sd)), (n, w)


def test_sigma_exact_at_ks_level_needs_half_step():
    # at w = eps_n the residue of m = n enters with weight 1/2; dropping it
    # (theta(0) = 0) or taking it fully (theta(0) = 1) misses the SD value
    inp = tiny(3, 7, 10, seed=5)
    xi, z = grid.gauss_legendre(64)
    Om, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    n = 2
    wt = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[n:n + 1], xi)[0]
    w = inp.eps[n]
    s_cd, _, nres = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[n], wt, xi, z, w)
    s_sd, _ = sd.sigma_c(inp.eps, inp.n_occ, sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[n]), Om, w)
    assert abs(s_cd - s_sd) < 1e-11
    half = 0.5 * cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[n][n], 0.0)[0]
    assert abs(half) > 1e-3


def test_residue_weights_follow_residue_term():
    eps = np.array([-20.0, -1.0, -0.5, 0.2, 1.0])
    f = cd.residue_weights(eps, 3, -0.7)
    assert list(f) == [0, 0, -1, 0, 0]
    f = cd.residue_weights(eps, 3, 0.5)
    assert list(f) == [0, 0, 0, 1, 0]
    f = cd.residue_weights(eps, 3, -0.5)
    assert list(f) == [0, 0, -0.5, 0, 0]
    f = cd.residue_weights(eps, 3, -21.0)
    assert list(f) == [-1, -1, -1, 0, 0]


def test_sigma_invariant_under_aux_rotation():
    inp = tiny(3, 8, 10)
    xi, z = grid.gauss_legendre(64)
    O, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((10, 10)))
    Bo, Br = O @ inp.B_ov, inp.B_rows @ O.T
    for n in (2, 3):
        wt = cd.w_table(inp.eps, 3, inp.B_ov, inp.B_rows[n:n + 1], xi)[0]
        wto = cd.w_table(inp.eps, 3, Bo, Br[n:n + 1], xi)[0]
        for w in (-0.9, 0.4):
            a = cd.sigma_c(inp.eps, 3, inp.B_ov, inp.B_rows[n], wt, xi, z, w)
            b = cd.sigma_c(inp.eps, 3, Bo, Br[n], wto, xi, z, w)
            assert abs(a[0] - b[0]) < 1e-13 and abs(a[1] - b[1]) < 1e-11


# --- quasiparticle solver --------------------------------------------------

def _two_level(b, Bnm, e_occ=-0.6, e_vir=0.3):
    """n_occ = n_virt = N_aux = 1.  B_ov = b, B_rows[n][m] = Bnm[n][m]."""
    eps = np.array([e_occ, e_vir])
    B_ov = np.array([[b]])
    B_rows = np.array([[[Bnm[0][0]], [Bnm[0][1]]], [[Bnm[1][0]], [Bnm[1][1]]]])
    return eps, B_ov, B_rows


def test_two_level_model_roots_are_cubic_roots():
    b = 0.35
    Bnm = [[0.5, b], [b, 0.4]]
    eps, B_ov, B_rows = _two_level(b, Bnm)
    D = eps[1] - eps[0]
    Om = math.sqrt(D * (D + 4 * b * b))
    xi, z = grid.gauss_legendre(200)
    res = qp.solve(eps, 1, B_ov, [0, 1], B_rows, [0, 1], xi, z, tol=1e-13)
    for n, r in zip((0, 1), res):
        # Sigma = c0/(w - e0 + Om) + c1/(w - e1 - Om), c_m = 2 Bnm^2 b^2 D / Om
        c0 = 2 * Bnm[n][0] ** 2 * b * b * D / Om
        c1 = 2 * Bnm[n][1] ** 2 * b * b * D / Om
        p0, p1 = eps[0] - Om, eps[1] + Om
        # (e_n - w)(w - p0)(w - p1) + c0 (w - p1) + c1 (w - p0) = 0
        poly = np.polymul([-1, eps[n]], np.polymul([1, -p0], [1, -p1]))
        poly = np.polyadd(poly, np.polyadd(c0 * np.array([1, -p1]), c1 * np.array([1, -p0])))
        roots = np.roots(poly)
        roots = roots[np.abs(roots.imag) < 1e-12].real
        inwin = roots[(roots > p0) & (roots < p1)]
        assert len(inwin) == 1
        assert r["status"] == 0
        assert abs(r["E"] - inwin[0]) < 1e-9, (n, r["E"], inwin)
        # Z from the exact derivative
        dS = -c0 / (inwin[0] - p0) ** 2 - c1 / (inwin[0] - p1) ** 2
        assert abs(r["Z"] - 1 / (1 - dS)) < 1e-7
        assert 0 < r["Z"] < 1


def test_noninteracting_limit():
    inp = tiny(3, 6, 8, b_scale=0.0)
    xi, z = grid.gauss_legendre(64)
    res = qp.solve(inp.eps, 3, inp.B_ov, inp.row_ids, inp.B_rows, [1, 2, 3], xi, z)
    for n, r in zip([1, 2, 3], res):
        assert r["E"] == inp.eps[n] and r["sigma_c"] == 0.0 and r["Z"] == 1.0
        assert r["iters"] == 1


def test_dsig_x_shifts_reference():
    # with W = 0, E = eps + dsig_x exactly
    inp = tiny(3, 6, 8, b_scale=0.0)
    xi, z = grid.gauss_legendre(64)
    dx = np.linspace(-0.05, 0.05, 9)
    res = qp.solve(inp.eps, 3, inp.B_ov, inp.row_ids, inp.B_rows, [2, 3], xi, z, dsig_x=dx)
    for n, r in zip([2, 3], res):
        assert abs(r["E"] - (inp.eps[n] + dx[n])) < 1e-12


def test_step_tree_root_is_unique_scan_root_and_z_in_range():
    inp = tiny(4, 9, 14, seed=21)
    xi, z = grid.gauss_legendre(64)
    Om, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    poles = sd.poles(inp.eps, inp.n_occ, Om)
    for n in (3, 4):
        r = qp.solve(inp.eps, 4, inp.B_ov, inp.row_ids, inp.B_rows, [n], xi, z)[0]
        assert r["status"] == 0 and 0 < r["Z"] < 1
        wt = cd.w_table(inp.eps, 4, inp.B_ov, inp.B_rows[n:n + 1], xi)[0]
        fe = qp.make_feval(inp.eps, 4, inp.B_ov, inp.B_rows[n], wt, xi, z, n)
        lo = poles[poles < r["E"]].max()
        hi = poles[poles > r["E"]].min()
        roots, _ = qp.scan(fe, 0.5 * (lo + hi), half_width=0.5 * (hi - lo) - 2e-3, step=2e-3)
        assert len(roots) == 1 and abs(roots[0] - r["E"]) < 1e-9
        # between poles the exact df/dw < -1
        rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[n])
        assert sd.sigma_c(inp.eps, 4, rho, Om, r["E"])[1] < 0


def test_step_tree_branches_on_model_functions():
    # Newton path (Z = 1)
    r = qp.step_tree(lambda w: (-(w - 0.3), -1.0), 0.0, tol=1e-12)
    assert abs(r["E"] - 0.3) < 1e-12 and [t[2] for t in r["trace"]][:2] == ["residual", "newton"]
    # scaled Newton (Z = 0.2, no bracket): linear convergence, same root
    r = qp.step_tree(lambda w: (-5 * (w - 0.3), -5.0), 0.0, tol=1e-12)
    assert abs(r["E"] - 0.3) < 1e-12 and "scaled-newton" in [t[2] for t in r["trace"]]
    # Z = 0.05: residual steps of at most 0.1 Ha until f changes sign, then golden section
    r = qp.step_tree(lambda w: (-20 * (w - 0.47), -20.0), 0.0, tol=1e-10, max_iter=200)
    kinds = [t[2] for t in r["trace"]]
    assert abs(r["E"] - 0.47) < 1e-11 and "golden" in kinds
    steps = np.diff([t[0] for t in r["trace"]])
    assert np.all(np.abs(steps[:kinds.index("golden")]) <= 0.1 + 1e-15)


def test_step_tree_iteration_cap_returns_last_evaluated_point():
    """Reading of the paper's iterative QP solution at an iteration cap (the
    paper gives none): the answer is the last point at which f was evaluated,
    with f and Z from that evaluation, flagged.  Hand-computed sequence for
    f(w) = -20 (w - 0.47) from w = 0 (Z = 0.05 < 0.1, no bracket, so every
    step is a scaled residual alpha f with alpha = min(0.1, 0.1/|f|), i.e.
    exactly 0.1 Ha while |f| > 1): evaluations at 0, 0.1, 0.2; the step to 0.3
    computed after the third is not taken."""
    f = lambda w: (-20.0 * (w - 0.47), -20.0)
    r = qp.step_tree(f, 0.0, tol=1e-10, max_iter=3)
    assert [t[0] for t in r["trace"]] == pytest.approx([0.0, 0.1, 0.2], abs=1e-15)
    assert r["E"] == pytest.approx(0.2, abs=1e-15)
    assert r["f"] == pytest.approx(5.4, abs=1e-13)
    assert r["Z"] == pytest.approx(0.05, abs=1e-15)
    assert r["status"] == qp.STATUS_MAXITER | qp.STATUS_SMALL_Z and r["iters"] == 3
    # a cap of one evaluation returns the starting point itself
    r = qp.step_tree(f, 0.0, tol=1e-10, max_iter=1)
    assert r["E"] == 0.0 and r["f"] == pytest.approx(9.4, abs=1e-13)
    # Newton (Z = 1) converges on its second evaluation; with the cap there
    # the converged point is returned without the cap flag
    r = qp.step_tree(lambda w: (-(w - 0.3), -1.0), 0.0, tol=1e-12, max_iter=3)
    assert r["status"] == 0 and r["E"] == pytest.approx(0.3, abs=1e-15)


def test_bracket_rules():
    # proper sign change (f > 0 on the left end): a root bracket, s = end of smaller |f|
    assert qp._make_bracket(0.1, 0.5, 0.3, -0.2) == (0.3, -0.2, 0.1, 0.5)
    # f rises through zero going right: a pole lies between, no root bracket
    assert qp._make_bracket(0.1, -0.5, 0.3, 0.2) is None
    # same sign, growing, step taken along the residual: skipped root
    assert qp._make_bracket(0.1, 0.2, 0.3, 0.9) == (0.1, 0.2, 0.3, 0.9)
    # same sign, growing, but the step went against the residual: nothing
    assert qp._make_bracket(0.3, 0.2, 0.1, 0.9) is None
    # same sign, shrinking: nothing
    assert qp._make_bracket(0.1, 0.9, 0.3, 0.2) is None
    # shrinking a root bracket keeps opposite signs at the ends
    br = qp._shrink((0.3, -0.2, 0.1, 0.5), 0.2, 0.1)
    assert sorted([br[0], br[2]]) == [0.2, 0.3] and br[1] * br[3] < 0
    # skipped-root bracket (pole + root inside): a point on s's branch beyond s
    # (same sign, smaller |f|) replaces s; a point past the pole replaces e;
    # an opposite-sign point turns it into a root bracket with s
    assert qp._shrink((0.1, 0.2, 0.3, 0.9), 0.15, 0.1) == (0.15, 0.1, 0.3, 0.9)
    assert qp._shrink((0.1, 0.2, 0.3, 0.9), 0.25, 1.5) == (0.1, 0.2, 0.25, 1.5)
    assert qp._shrink((0.1, 0.2, 0.3, 0.9), 0.2, -0.05) == (0.2, -0.05, 0.1, 0.2)


def test_step_tree_golden_on_skipped_root():
    # f = -(w - r) * k + c / (w - p) has a root just left of the pole p; start
    # from a bracket-creating pair by forcing Z < 0.1 (steep f), then check the
    # solver lands on a root of f
    k, c, p = 30.0, 0.02, 0.45

    def f(w):
        return -k * (w - 0.43) + c / (w - p), -k - c / (w - p) ** 2
    r = qp.step_tree(f, 0.0, tol=1e-10, max_iter=400)
    assert r["status"] & qp.STATUS_MAXITER == 0
    assert abs(f(r["E"])[0]) < 1e-10
