"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: the FP64 path must match the oracle to 1e-10 relative on Pi,
Sigma^c at fixed frequencies and QP energies (W^c entries relative to
|b|^2, because |L^-1 b|^2 - |b|^2 cancels at large xi); every path, mixed
precision included, must match QP energies within 1 meV."""
import json
import os

import numpy as np
import pytest

import gwgen
from oracle import cd, grid, qp

pytestmark = pytest.mark.gpu

MEV = 1e-3 / 27.211386245988   # 1 meV in Hartree
HERE = os.path.dirname(os.path.abspath(__file__))


def gwl():
    import paper_2107_10423_amd as m
    return m


def ragged(seed=5, n_occ=7, n_virt=45, n_aux=200, rows=(4, 5, 6, 7, 8), b_scale=1.0):
    shape = gwgen.custom_shape(n_occ, n_virt, n_aux, n_core=1)
    return gwgen.make_inputs(shape, seed, rows, b_scale=b_scale)


def ctx(inp, **kw):
    return gwl().Context.from_inputs(inp, **kw)


# ---------------------------------------------------------------- stage A

@pytest.mark.parametrize("shape", [(7, 45, 200), (3, 20, 64), (11, 60, 300)])
def test_dielectric_fp64(shape):
    inp = ragged(n_occ=shape[0], n_virt=shape[1], n_aux=shape[2], rows=(1,))
    xis = np.array([1e-4, 0.3, 5.0, 1e3])
    with ctx(inp) as c:
        got = c.dielectric(xis)
    for g, x in enumerate(xis):
        Pi = cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, x)
        ref = np.tril(np.eye(inp.shape.n_aux) - Pi)
        err = np.abs(got[g] - ref).max() / np.abs(Pi).max()
        assert err < 1e-12, (x, err)


def test_cholesky_fp64():
    inp = ragged()
    xis = np.array([2e-4, 0.7, 40.0])
    with ctx(inp) as c:
        got = c.cholesky(xis)
    for g, x in enumerate(xis):
        A = np.eye(inp.shape.n_aux) - cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, x)
        L = np.linalg.cholesky(A)
        assert np.abs(got[g] - L).max() < 1e-12 * np.abs(L).max()


@pytest.mark.parametrize("G", [8, 64])
def test_wtable_fp64(G):
    inp = ragged()
    xi, z = grid.gauss_legendre(G)
    with ctx(inp) as c:
        got = c.wtable(gwl().Grid(xi, z))
    ref = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi)
    bn = np.sum(inp.B_rows ** 2, axis=2)[:, :, None]
    assert np.all(np.abs(got - ref) <= 1e-10 * bn + 1e-300)


def test_wtable_chunked_equals_unchunked():
    inp = ragged()
    xi, z = grid.gauss_legendre(16)
    g = gwl().Grid(xi, z)
    with ctx(inp) as c:
        a = c.wtable(g)
    with ctx(inp, work_budget_bytes=3 << 20) as c:
        b = c.wtable(g)
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- residues

def _residue_cases(inp):
    D = cd.transition_energies(inp.eps, inp.n_occ)
    ws = [0.0, 0.05, -0.3, 0.5 * D.min(), D.min() + 0.013, 2.7, -3.1, 21.3]
    st, ms = [], []
    rows = list(inp.row_ids)
    for j, w in enumerate(ws):
        st.append(rows[j % len(rows)])
        ms.append((3 * j + 1) % inp.shape.n_mo)
    return st, ms, ws


@pytest.mark.parametrize("fallback_only", [False, True])
def test_residues_match_direct_solve(fallback_only):
    inp = ragged()
    st, ms, ws = _residue_cases(inp)
    kw = dict(minres_max_iter=1) if fallback_only else {}
    with ctx(inp, **kw) as c:
        x, wc, dwc, it = c.residues(st, ms, ws)
    if fallback_only:
        assert np.all(it < 0)
    else:
        assert np.all(it > 0), it
    for j in range(len(ws)):
        b = inp.B_rows[list(inp.row_ids).index(st[j]), ms[j]]
        n = inp.shape.n_aux
        A = np.eye(n) - cd.pi_real(inp.eps, inp.n_occ, inp.B_ov, ws[j])
        xr = np.linalg.solve(A, b)
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(x[j] - xr) <= 1e-11 * kappa * np.linalg.norm(xr) + 1e-15
        w_ref, dw_ref = cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b, ws[j])
        scale = np.dot(b, b)
        assert abs(wc[j] - w_ref) <= 1e-10 * kappa * scale
        assert abs(dwc[j] - dw_ref) <= 1e-9 * kappa * max(abs(dw_ref), scale)


def test_fallback_batches_match_direct_solve():
    """More unconverged systems than one fallback batch (32), on an N_aux of
    five 128-column LU panels (ragged: 600 of 640): every x equals the dense
    solve of its own 1 - Pi(w), and W^c its residue value."""
    inp = ragged(seed=9, n_occ=6, n_virt=40, n_aux=600)
    rng = np.random.default_rng(3)
    k = 40
    rows = list(inp.row_ids)
    st = [rows[j % len(rows)] for j in range(k)]
    ms = [int(m) for m in rng.integers(0, inp.shape.n_mo, k)]
    D = cd.transition_energies(inp.eps, inp.n_occ)
    ws = list(rng.uniform(-1.5, 1.5, k) * D.min())
    with ctx(inp, minres_max_iter=1) as c:
        x, wc, dwc, it = c.residues(st, ms, ws)
        t = c.timing()
    assert np.all(it < 0) and t["fallback_systems"] == k
    n = inp.shape.n_aux
    for j in range(k):
        b = inp.B_rows[rows.index(st[j]), ms[j]]
        A = np.eye(n) - cd.pi_real(inp.eps, inp.n_occ, inp.B_ov, ws[j])
        xr = np.linalg.solve(A, b)
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(x[j] - xr) <= 1e-11 * kappa * np.linalg.norm(xr) + 1e-15, j
        w_ref, _ = cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b, ws[j])
        assert abs(wc[j] - w_ref) <= 1e-10 * kappa * np.dot(b, b), j


def test_fallback_solves_past_the_lds_vector():
    """N_aux 6200 (49 LU panels; the solve works on b in place, past the LDS
    size it uses below 6144): the forced-fallback solutions satisfy their
    systems to rounding."""
    inp = ragged(seed=11, n_occ=2, n_virt=10, n_aux=6200, rows=(1, 2))
    st, ms, ws = [1, 2, 1], [0, 5, 11], [0.05, -0.3, 0.7]
    with ctx(inp, minres_max_iter=1) as c:
        x, wc, dwc, it = c.residues(st, ms, ws)
    assert np.all(it < 0)
    rows = list(inp.row_ids)
    n = inp.shape.n_aux
    for j in range(3):
        b = inp.B_rows[rows.index(st[j]), ms[j]]
        A = np.eye(n) - cd.pi_real(inp.eps, inp.n_occ, inp.B_ov, ws[j])
        assert np.linalg.norm(A @ x[j] - b) <= 1e-12 * np.linalg.norm(b) * np.linalg.norm(A, 1), j


def test_many_residue_systems_in_one_batch():
    # more than one 64-system tile of systems
    inp = ragged()
    rng = np.random.default_rng(0)
    k = 150
    st = rng.choice(inp.row_ids, k)
    ms = rng.integers(0, inp.shape.n_mo, k)
    ws = rng.uniform(-0.4, 0.4, k)
    with ctx(inp) as c:
        x, wc, dwc, it = c.residues(st, ms, ws)
    for j in rng.choice(k, 12, replace=False):
        b = inp.B_rows[list(inp.row_ids).index(st[j]), ms[j]]
        w_ref, dw_ref = cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b, ws[j])
        assert abs(wc[j] - w_ref) <= 1e-10 * np.dot(b, b)
        assert abs(dwc[j] - dw_ref) <= 1e-9 * max(abs(dw_ref), np.dot(b, b))


# ---------------------------------------------------------------- Sigma

def test_sigma_fixed_omega_fp64():
    inp = ragged()
    xi, z = grid.gauss_legendre(64)
    wt = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi)
    states, oms = [], []
    for n in inp.row_ids:
        for w in (inp.eps[n], inp.eps[n] - 0.25, inp.eps[n] + 0.15, -21.0, 0.9):
            states.append(int(n))
            oms.append(float(w))
    with ctx(inp) as c:
        s, ds, nres = c.sigma(states, oms, gwl().Grid(xi, z))
    for j, (n, w) in enumerate(zip(states, oms)):
        r = list(inp.row_ids).index(n)
        rs, rds, rn = cd.sigma_c(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[r], wt[r], xi, z, w)
        assert nres[j] == rn
        assert abs(s[j] - rs) <= 1e-10 * abs(rs) + 1e-13, (n, w, s[j], rs)
        assert abs(ds[j] - rds) <= 1e-9 * abs(rds) + 1e-11, (n, w, ds[j], rds)


# ---------------------------------------------------------------- QP

def _oracle_qp(inp, states, G, tol=1e-12):
    xi, z = grid.gauss_legendre(G)
    return qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z, tol=tol)


def test_qp_fp64_ragged():
    inp = ragged()
    states = list(inp.row_ids)
    ref = _oracle_qp(inp, states, 64)
    with ctx(inp, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(states, gwl().Grid.gauss_legendre(64))
    for j, r in enumerate(ref):
        assert st[j] == 0
        assert abs(E[j] - r["E"]) <= 1e-10 * abs(r["E"]), (states[j], E[j], r["E"])
        assert abs(S[j] - r["sigma_c"]) <= 1e-10 * abs(r["sigma_c"]) + 1e-12
        assert abs(Z[j] - r["Z"]) <= 1e-9


def _golden(name):
    p = os.path.join(HERE, "golden", f"{name}.json")
    if not os.path.exists(p):
        pytest.skip(f"fixture {p} not written")
    return json.load(open(p))


@pytest.mark.parametrize("prec,tol", [("fp64", None), ("fp32", MEV), ("bf16x3", MEV)])
def test_qp_monomer_golden(prec, tol):
    gold = _golden("monomer")
    inp = gwgen.make_config("monomer")
    with ctx(inp, pi_prec=prec, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(gold["states"], gwl().Grid.gauss_legendre(gold["grid_points"]))
    for j, r in enumerate(gold["results"]):
        t = 1e-10 * abs(r["E"]) if tol is None else tol
        assert abs(E[j] - r["E"]) <= t, (prec, r["state"], E[j] - r["E"])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_pi_and_qp(prec):
    inp = ragged()
    xis = np.array([1e-3, 0.5, 20.0])
    with ctx(inp, pi_prec=prec, qp_tol=1e-12) as c:
        got = c.dielectric(xis)
        E, S, Z, st = c.qp(list(inp.row_ids), gwl().Grid.gauss_legendre(64))
    bound = 1e-6 if prec == "fp32" else 1e-4
    for g, x in enumerate(xis):
        Pi = cd.pi_imag(inp.eps, inp.n_occ, inp.B_ov, x)
        err = np.abs(got[g] - np.tril(np.eye(inp.shape.n_aux) - Pi)).max() / np.abs(Pi).max()
        assert err < bound, (prec, x, err)
    ref = _oracle_qp(inp, list(inp.row_ids), 64)
    for j, r in enumerate(ref):
        assert abs(E[j] - r["E"]) <= MEV, (prec, E[j] - r["E"])


def test_noninteracting_limit():
    inp = ragged(b_scale=0.0)
    with ctx(inp) as c:
        E, S, Z, st = c.qp(list(inp.row_ids), gwl().Grid.gauss_legendre(32))
    np.testing.assert_array_equal(E, inp.eps[inp.row_ids])
    np.testing.assert_array_equal(S, 0.0)
    np.testing.assert_array_equal(Z, 1.0)


def test_dsig_x_shift():
    inp = ragged(b_scale=0.0)
    dx = np.linspace(-0.03, 0.03, inp.shape.n_mo)
    with ctx(inp, dsig_x=dx, qp_tol=1e-13) as c:
        E, S, Z, st = c.qp([5, 6], gwl().Grid.gauss_legendre(16))
    np.testing.assert_allclose(E, inp.eps[[5, 6]] + dx[[5, 6]], rtol=0, atol=1e-13)


def test_cached_wtable_gives_identical_results():
    inp = ragged()
    g = gwl().Grid.gauss_legendre(32)
    with ctx(inp) as c:
        a = c.qp([5, 6], g)
        t1 = c.timing()
        b = c.qp([5, 6], g)
        t2 = c.timing()
        c.set_pi_prec("bf16x3")
        c.qp([5], g)
        t3 = c.timing()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert t1["wtab_cached"] == 0 and t2["wtab_cached"] == 1 and t3["wtab_cached"] == 0
    assert t1["qp_rounds"] >= 2 and t1["minres_systems"] > 0


def test_single_state_subset_and_errors():
    inp = ragged()
    g = gwl().Grid.gauss_legendre(16)
    with ctx(inp) as c:
        full = c.qp(list(inp.row_ids), g)
        one = c.qp([6], g)
        assert abs(one[0][0] - full[0][2]) <= 1e-12
        with pytest.raises(gwl().GWError) as e:
            c.qp([0], g)
        assert e.value.code == -1
        empty = c.qp([], g)
        assert all(len(a) == 0 for a in empty)


def test_core_level_residues_many_systems():
    # deepest level of a small cluster: every occupied level above E carries a residue
    shape = gwgen.custom_shape(12, 70, 220, n_core=3)
    inp = gwgen.make_inputs(shape, 44, [0, 11])
    ref = _oracle_qp(inp, [0], 32)
    with ctx(inp, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp([0], gwl().Grid.gauss_legendre(32))
        t = c.timing()
    assert abs(E[0] - ref[0]["E"]) <= 1e-10 * abs(ref[0]["E"])
    assert t["minres_systems"] >= 11


def test_minres_graph_replay_matches_eager():
    # MINRES iterations 2.. replay captured graphs (two parities, several padded
    # batch sizes across QP rounds, host work and synchronisation between the
    # replays); results must equal the eagerly launched ones bit for bit, on
    # the first call and on a second call that reuses the captured graphs
    shape = gwgen.custom_shape(12, 70, 220, n_core=3)
    inp = gwgen.make_inputs(shape, 44, [0, 5, 11, 12])
    g = gwl().Grid.gauss_legendre(32)
    states = [0, 5, 11, 12]
    with ctx(inp, qp_tol=1e-12, graphs=False) as c:
        ref = c.qp(states, g)
        t_ref = c.timing()
    with ctx(inp, qp_tol=1e-12) as c:
        first = c.qp(states, g)
        t_first = c.timing()
        c.reset_cache()
        second = c.qp(states, g)
    assert t_ref["minres_iters"] > 2 * t_ref["qp_rounds"]   # graphs were replayed
    assert t_first["minres_iters"] == t_ref["minres_iters"]
    for out in (first, second):
        for a, b in zip(out, ref):
            assert np.array_equal(a, b)


# ---------------------------------------------------------------- full size

@pytest.mark.parametrize("prec,tol", [("fp64", None), ("bf16x3", MEV), ("fp32", MEV)])
def test_h2o10_full_size_against_fixture(prec, tol):
    gold = _golden("h2o10")
    inp = gwgen.make_config("h2o10")
    with ctx(inp, pi_prec=prec, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(gold["states"], gwl().Grid.gauss_legendre(gold["grid_points"]))
        if prec == "fp64":
            fx = gold["fixed"]
            s, ds, nres = c.sigma([f["state"] for f in fx], [f["omega"] for f in fx],
                                  gwl().Grid.gauss_legendre(gold["grid_points"]))
            for j, f in enumerate(fx):
                assert nres[j] == f["n_res"]
                assert abs(s[j] - f["sigma"]) <= 1e-10 * abs(f["sigma"])
    for j, r in enumerate(gold["results"]):
        t = 1e-10 * abs(r["E"]) if tol is None else tol
        assert abs(E[j] - r["E"]) <= t, (prec, r["state"], E[j] - r["E"])


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-13), ("fp32", 2e-6), ("bf16x3", 1e-4)])
def test_pi_precision_h2o10_sampled_rows(prec, bound):
    # full (H2O)10 size; the oracle forms 40 sampled rows of Pi per frequency
    inp = gwgen.make_inputs(gwgen.CONFIGS["h2o10"].shape, 2, [49])
    xis = np.array([1e-3, 0.5, 20.0])
    with ctx(inp, pi_prec=prec) as c:
        got = c.dielectric(xis)
    rows = np.unique(np.r_[np.arange(0, 1120, 37), np.arange(1110, 1120)])
    D = cd.transition_energies(inp.eps, inp.n_occ)
    worst = 0.0
    for g, x in enumerate(xis):
        Pi_rows = -4.0 * (inp.B_ov[rows] * (D / (D * D + x * x))) @ inp.B_ov.T
        ref = np.eye(1120)[rows] - Pi_rows
        mask = np.arange(1120)[None, :] <= rows[:, None]       # lower triangle
        err = np.abs(np.where(mask, got[g][rows] - ref, 0.0)).max() / np.abs(Pi_rows).max()
        worst = max(worst, err)
    print(f"Pi precision {prec}: max |error| / max |Pi| = {worst:.3e}")
    assert worst < bound


@pytest.mark.parametrize("n_aux", [2100, 2200, 3360])
def test_pi_wide_tiles_cover_the_lower_triangle(n_aux):
    """The wide BF16x3 Pi build (N_aux padded to 2048 and up) stores every
    element of the lower triangle: 17, 18 and 27 blocks of 128 rows (an odd
    count packs the last block row into the diagonal tiles' spare halves).
    Two calls at different frequencies, so that a block left unwritten by
    the second would still hold the first call's values."""
    shape = gwgen.custom_shape(3, 20, n_aux, n_core=1)
    inp = gwgen.make_inputs(shape, 5, [2])
    D = cd.transition_energies(inp.eps, inp.n_occ)
    low = np.tril(np.ones((n_aux, n_aux), dtype=bool))
    with ctx(inp, pi_prec="bf16x3") as c:
        for xis in (np.array([0.05, 3.0]), np.array([0.4, 11.0])):
            got = c.dielectric(xis)
            for g, x in enumerate(xis):
                Pi = -4.0 * (inp.B_ov * (D / (D * D + x * x))) @ inp.B_ov.T
                ref = np.eye(n_aux) - Pi
                err = np.abs(np.where(low, got[g] - ref, 0.0)).max() / np.abs(Pi).max()
                assert err < 1e-4, (n_aux, x, err)


def test_setup_from_the_full_tensor():
    """gw_setup_full takes B [n_aux][n_mo][n_mo] and serves every state: the
    same energies as the row-supplied context, and states outside it."""
    inp = gwgen.make_config("monomer")
    B = gwgen.full_B(inp.shape, inp.seed)
    g = gwl().Grid.gauss_legendre(64)
    with ctx(inp, qp_tol=1e-12) as c:
        E0, S0, Z0, _ = c.qp([4, 5], g)
    with gwl().Context.full(inp.eps, inp.n_occ, B, qp_tol=1e-12) as c:
        E1, S1, Z1, _ = c.qp([4, 5], g)
        E2, _, _, st2 = c.qp([3, 6], g)
    assert np.all(np.abs(E1 - E0) <= 1e-12 * np.abs(E0))
    ref = _oracle_qp(gwgen.make_config("monomer", states=[3, 6]), [3, 6], 64)
    for j, r in enumerate(ref):
        assert abs(E2[j] - r["E"]) <= 1e-10 * abs(r["E"])


def test_preconditioned_minres_matches_plain_and_saves_iterations():
    """Residue systems below the lowest transition energy run MINRES
    preconditioned by 1 - Pi(0): the QP results agree with plain MINRES and
    with the oracle, in fewer iterations."""
    inp = ragged()
    states = list(inp.row_ids)
    g = gwl().Grid.gauss_legendre(64)
    out = {}
    for pre in (False, True):
        with ctx(inp, qp_tol=1e-12, precond=pre) as c:
            E, S, Z, st = c.qp(states, g)
            out[pre] = (E, Z, c.timing()["minres_iters"])
    assert np.all(np.abs(out[True][0] - out[False][0]) <= 1e-10 * np.abs(out[False][0]))
    assert np.all(np.abs(out[True][1] - out[False][1]) <= 1e-9)
    assert out[True][2] < out[False][2], (out[True][2], out[False][2])
    ref = _oracle_qp(inp, states, 64)
    for j, r in enumerate(ref):
        assert abs(out[True][0][j] - r["E"]) <= 1e-10 * abs(r["E"])


def test_preconditioned_residues_match_direct_solve():
    """After a W^c build the context holds the preconditioner 1 - Pi(0):
    residue systems below the lowest transition energy are then solved
    preconditioned, to the same accuracy against a direct solve."""
    inp = ragged()
    D = cd.transition_energies(inp.eps, inp.n_occ)
    # five frequencies inside the preconditioned window and one above every
    # transition energy (plain MINRES converges there; inside the transition
    # band it may need the fallback either way)
    ws = np.array([0.0, 0.05, -0.2, 0.5 * D.min(), -0.85 * D.min(), 1.5 * D.max()])
    st = [int(inp.row_ids[j % len(inp.row_ids)]) for j in range(len(ws))]
    ms = [(3 * j + 1) % inp.shape.n_mo for j in range(len(ws))]
    with ctx(inp) as c:
        c.qp([int(inp.row_ids[0])], gwl().Grid.gauss_legendre(16))   # builds M^-1
        x, wc, dwc, it = c.residues(st, ms, ws)
    with ctx(inp, precond=False) as c:
        _, _, _, it_plain = c.residues(st, ms, ws)
    assert np.all(it > 0) and np.all(it_plain > 0)
    # the systems inside the window converge in fewer iterations
    assert np.sum(it[:5]) < np.sum(it_plain[:5]), (it, it_plain)
    for j in range(len(ws)):
        b = inp.B_rows[list(inp.row_ids).index(st[j]), ms[j]]
        n = inp.shape.n_aux
        A = np.eye(n) - cd.pi_real(inp.eps, inp.n_occ, inp.B_ov, ws[j])
        xr = np.linalg.solve(A, b)
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(x[j] - xr) <= 1e-11 * kappa * np.linalg.norm(xr) + 1e-15, j
        w_ref, dw_ref = cd.residue_value(inp.eps, inp.n_occ, inp.B_ov, b, ws[j])
        assert abs(wc[j] - w_ref) <= 1e-10 * kappa * np.dot(b, b), j
