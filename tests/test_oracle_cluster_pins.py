"""Pins of the cluster initial-guess layer (oracle/cluster.py), CPU only.

The layer only changes where each state's step tree starts, so its pins are:
the grouping and representative rules on hand-made energies; width 0 is the
plain solver; every root it returns is a root of the spectral-decomposition
(Casida) route's QP equation, an independent formula for the same Sigma^c,
and a sign change that the graphical scan also finds; members start at their
own energy plus the representative's QP shift."""
import numpy as np
import pytest

import gwgen
from oracle import cd, cluster, ev, grid, qp, sd


def core_rich(seed=3):
    # six core levels within 0.25 Ha of each other, two valence states
    shape = gwgen.custom_shape(10, 40, 150, n_core=6)
    return gwgen.make_inputs(shape, seed, list(range(8)))


def test_grouping_rules():
    e = [1.0, 0.0, 1.2, 5.0, 0.3]
    assert cluster.clusters(e, 0.25) == [[1], [4], [0, 2], [3]]
    # single linkage: a chain of small gaps is one cluster
    assert cluster.clusters([0.0, 0.2, 0.4, 0.6], 0.25) == [[0, 1, 2, 3]]
    # width 0 (or negative): every state alone, ties included
    assert cluster.clusters([0.5, 0.5, 0.1], 0.0) == [[2], [0], [1]]
    assert cluster.clusters([0.5, 0.5, 0.1], -1.0) == [[2], [0], [1]]
    # equal energies with a positive width share a cluster, first requested first
    assert cluster.clusters([0.5, 0.1, 0.5], 1e-9) == [[1], [0, 2]]


def test_representative_is_the_lower_median():
    assert cluster.representative([7]) == 7
    assert cluster.representative([3, 1]) == 3
    assert cluster.representative([3, 1, 4]) == 1
    assert cluster.representative([3, 1, 4, 0]) == 1


def test_width_zero_is_the_plain_solver():
    inp = core_rich()
    xi, z = grid.gauss_legendre(32)
    states = [0, 2, 4, 6, 7]
    a = qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z, tol=1e-12)
    b = cluster.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z, 0.0,
                      tol=1e-12)
    for x, y in zip(a, b):
        assert x["E"] == y["E"] and x["Z"] == y["Z"] and y["representative"]


def test_roots_are_roots_of_the_spectral_route_and_of_the_scan():
    inp = core_rich()
    xi, z = grid.gauss_legendre(128)
    states = list(range(8))
    res = cluster.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z,
                        0.5, tol=1e-12)
    Omega, T, D = sd.casida(inp.eps, inp.n_occ, inp.B_ov)
    wtab = cd.w_table(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows, xi)
    rows = [int(r) for r in inp.row_ids]
    for k, n in enumerate(states):
        r = res[k]
        assert r["status"] & qp.STATUS_MAXITER == 0, n
        rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[rows.index(n)])
        s, _ = sd.sigma_c(inp.eps, inp.n_occ, rho, Omega, r["E"])
        # G0W0 keeps the plain quadrature, whose error grows as a root comes
        # close to a pole of G (state 1 lands 4e-4 Ha below its own: 4.4e-7);
        # the roots the layer chooses between differ by > 5e-4
        assert abs(inp.eps[n] + s - r["E"]) < 1e-6, n
        fe = qp.make_feval(inp.eps, inp.n_occ, inp.B_ov, inp.B_rows[rows.index(n)],
                           wtab[rows.index(n)], xi, z, n)
        # (centred half a step off E, so that E itself is not a scan node)
        roots, _ = qp.scan(fe, r["E"] + 5e-5, half_width=2e-3, step=1e-4)
        assert min(abs(x - r["E"]) for x in roots) < 1e-9, n


def test_members_start_at_the_representatives_shift_and_save_evaluations():
    inp = core_rich()
    xi, z = grid.gauss_legendre(48)
    states = list(range(8))
    plain = qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z,
                     tol=1e-12)
    res = cluster.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states, xi, z,
                        0.5, tol=1e-12)
    groups = cluster.clusters([inp.eps[n] for n in states], 0.5)
    assert [len(g) for g in groups] == [6, 2]
    for g in groups:
        rep = cluster.representative(g)
        assert res[rep]["representative"] and res[rep]["w0"] == inp.eps[states[rep]]
        shift = res[rep]["E"] - inp.eps[states[rep]]
        for k in g:
            if k != rep:
                assert not res[k]["representative"]
                assert res[k]["w0"] == inp.eps[states[k]] + shift
    # on this input two core states exhaust the iteration cap from their own
    # energies and converge from the guess; the layer never costs evaluations
    assert sum(r["n_evals"] for r in res) < sum(r["n_evals"] for r in plain)
    assert sum(bool(r["status"] & qp.STATUS_MAXITER) for r in plain) == 2
    assert all(r["status"] == 0 for r in res)


@pytest.mark.parametrize("mode", ["evgw0", "evgw"])
def test_evgw_with_clusters_solves_each_cycle(mode):
    """Every cycle's energies are roots of that cycle's QP equation on the
    spectral route (energies in G and W as the cycle defines them)."""
    inp = core_rich()
    xi, z = grid.gauss_legendre(128)
    states = [0, 1, 2, 3, 6, 7]
    res, cycles, hist = ev.evgw(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states,
                                xi, z, mode=mode, n_cycles=3, tol=1e-12, cluster_width=0.5)
    rows = [int(r) for r in inp.row_ids]
    eps_g = np.array(inp.eps, dtype=np.float64)
    for c in range(cycles):
        eps_w = inp.eps if mode == "evgw0" else eps_g
        Omega, T, D = sd.casida(eps_w, inp.n_occ, inp.B_ov)
        for k, n in enumerate(states):
            rho = sd.pole_strengths(inp.B_ov, D, T, inp.B_rows[rows.index(n)])
            s, _ = sd.sigma_c(eps_g, inp.n_occ, rho, Omega, hist[c][k])
            assert abs(inp.eps[n] + s - hist[c][k]) < 1e-8, (c, n)
        eps_g = eps_g.copy()
        eps_g[states] = hist[c]
