"""Parity of the eigenvalue self-consistent path (gw_evgw, through the C-ABI)
with the FP64 oracle (oracle/ev.py).

Tolerances: FP64 QP energies of every cycle within 1e-10 relative (as for
G0W0), Z within 1e-9; the mixed-precision Pi builds within 1 meV."""
import numpy as np
import pytest

import gwgen
from oracle import ev, grid, qp

pytestmark = pytest.mark.gpu

MEV = 1e-3 / 27.211386245988   # 1 meV in Hartree


def gwl():
    import paper_2107_10423_amd as m
    return m


def inputs(rows=(0, 4, 5, 6, 7, 8), seed=5):
    # N_aux = 200: two Pi tiles with a ragged tail; state 0 is a core level
    shape = gwgen.custom_shape(7, 45, 200, n_core=1)
    return gwgen.make_inputs(shape, seed, rows)


def oracle_cycles(inp, states, G, mode, n_cycles, ev_tol=0.0):
    xi, z = grid.gauss_legendre(G)
    return ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z,
                   mode=mode, n_cycles=n_cycles, ev_tol=ev_tol, tol=1e-12)


@pytest.mark.parametrize("mode", ["evgw0", "evgw"])
@pytest.mark.parametrize("states", [[5, 6, 7], [0, 6, 7]], ids=["valence", "core"])
def test_cycles_match_oracle_fp64(mode, states):
    inp = inputs()
    res, cycles, hist = oracle_cycles(inp, states, 48, mode, 4)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E, S, Z, st, h = c.evgw(states, gwl().Grid.gauss_legendre(48), mode=mode, n_cycles=4)
    assert h.shape == (cycles, len(states))
    for k in range(cycles):
        for j in range(len(states)):
            assert abs(h[k, j] - hist[k][j]) <= 1e-10 * abs(hist[k][j]), (mode, k, states[j])
    for j, r in enumerate(res):
        assert st[j] == r["status"] == 0
        assert E[j] == h[-1, j]
        assert abs(S[j] - r["sigma_c"]) <= 1e-10 * abs(r["sigma_c"]) + 1e-12
        assert abs(Z[j] - r["Z"]) <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_evgw(prec):
    inp = inputs()
    states = [0, 6, 7]
    res, cycles, hist = oracle_cycles(inp, states, 48, "evgw", 3)
    with gwl().Context.from_inputs(inp, pi_prec=prec, qp_tol=1e-12) as c:
        E, S, Z, st, h = c.evgw(states, gwl().Grid.gauss_legendre(48), mode="evgw", n_cycles=3)
    assert np.abs(h - np.array(hist)).max() <= MEV


def test_tolerance_stops_like_the_oracle():
    inp = inputs()
    states = [5, 6, 7]
    g = gwl().Grid.gauss_legendre(48)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        # a tolerance no change reaches stops after the second cycle
        E, S, Z, st, h = c.evgw(states, g, mode="evgw0", n_cycles=10, ev_tol=1.0)
        assert h.shape[0] == 2
        res, cycles, hist = oracle_cycles(inp, states, 48, "evgw0", 10, ev_tol=1e-6)
        changes = [np.abs(hist[k] - hist[k - 1]).max() for k in range(1, cycles)]
        # the comparison is decided well away from the threshold
        assert min(abs(np.log10(x / 1e-6)) for x in changes) > 0.01
        E, S, Z, st, h = c.evgw(states, g, mode="evgw0", n_cycles=10, ev_tol=1e-6)
        assert h.shape[0] == cycles < 10
        np.testing.assert_allclose(h, np.array(hist), rtol=1e-10, atol=0)


def test_one_cycle_is_g0w0_up_to_the_static_quadrature():
    inp = inputs()
    states = [0, 5, 6, 7]
    g = gwl().Grid.gauss_legendre(48)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E0, S0, Z0, st0 = c.qp(states, g)
        E1, S1, Z1, st1, h = c.evgw(states, g, mode="evgw", n_cycles=1)
    assert h.shape == (1, len(states))
    assert np.all(np.abs(E1 - E0) <= 1e-9 * np.abs(E0))
    # and the difference is the oracle's
    xi, z = grid.gauss_legendre(48)
    r0 = qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z, tol=1e-12)
    r1, _, _ = oracle_cycles(inp, states, 48, "evgw", 1)
    d_ref = np.array([b["E"] - a["E"] for a, b in zip(r0, r1)])
    assert np.all(np.abs((E1 - E0) - d_ref) <= 2e-10 * np.abs(E0))


def test_context_is_restored():
    """After evGW (energies moved in G and W) the context gives bitwise the
    G0W0 results and W^c table of a fresh context."""
    inp = inputs()
    states = [0, 6, 7]
    g = gwl().Grid.gauss_legendre(32)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        W_ref = c.wtable(g)
        E_ref, S_ref, Z_ref, _ = c.qp(states, g)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        c.evgw(states, g, mode="evgw", n_cycles=3)
        W = c.wtable(g)
        E, S, Z, _ = c.qp(states, g)
        c.evgw(states, g, mode="evgw0", n_cycles=2)
        E2, _, _, _ = c.qp(states, g)
    assert np.array_equal(W, W_ref)
    assert np.array_equal(E, E_ref) and np.array_equal(S, S_ref) and np.array_equal(Z, Z_ref)
    assert np.array_equal(E2, E_ref)


def test_bad_arguments():
    inp = inputs()
    g = gwl().Grid.gauss_legendre(8)
    with gwl().Context.from_inputs(inp) as c:
        for kw in (dict(mode=2), dict(n_cycles=0), dict(ev_tol=-1.0)):
            args = dict(mode="evgw0", n_cycles=2, ev_tol=0.0)
            args.update(kw)
            with pytest.raises(gwl().GWError):
                c.evgw([5], g, **args)
        with pytest.raises(gwl().GWError):
            c.evgw([3], g)   # not among the supplied rows


@pytest.mark.parametrize("mode", ["evgw0", "evgw"])
@pytest.mark.parametrize("prec,tol", [("fp64", None), ("bf16x3", MEV)])
def test_h2o10_full_size_against_fixture(mode, prec, tol):
    """The (H2O)10 workload, three cycles, against the oracle's cycles stored
    by tests/golden/make_golden.py."""
    import json
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"h2o10_{mode}.json")
    if not os.path.exists(p):
        pytest.skip(f"fixture {p} not written")
    gold = json.load(open(p))
    inp = gwgen.make_config("h2o10")
    with gwl().Context.from_inputs(inp, pi_prec=prec, qp_tol=gold["qp_tol"]) as c:
        E, S, Z, st, h = c.evgw(gold["states"], gwl().Grid.gauss_legendre(gold["grid_points"]),
                                mode=mode, n_cycles=gold["n_cycles"])
    ref = np.array(gold["cycles"])
    assert h.shape == ref.shape
    bound = 1e-10 * np.abs(ref) if tol is None else tol
    assert np.all(np.abs(h - ref) <= bound), np.abs(h - ref).max()
    assert np.all(st == [r["status"] for r in gold["results"]])
