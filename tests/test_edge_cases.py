"""Edge cases of the entry points, against the oracle where results exist:
empty state lists, the smallest shapes (one occupied, one auxiliary
function), repeated states, a one-electron spin channel."""
import numpy as np
import pytest

import gwgen
from oracle import grid, qp, uhf

pytestmark = pytest.mark.gpu


def gwl():
    import paper_2107_10423_amd as m
    return m


def test_empty_state_lists():
    inp = gwgen.make_config("monomer")
    g = gwl().Grid.gauss_legendre(16)
    with gwl().Context.from_inputs(inp) as c:
        for out in (c.qp([], g), c.qp_sd([]), c.evgw([], g, n_cycles=2)[:4]):
            assert all(len(a) == 0 for a in out)


@pytest.mark.parametrize("shape,rows", [((1, 1, 1), [0, 1]), ((1, 3, 5), [0, 1, 3]),
                                        ((2, 2, 130), [1, 2])])
def test_smallest_shapes_match_the_oracle(shape, rows):
    inp = gwgen.make_inputs(gwgen.custom_shape(*shape, n_core=0), 3, rows)
    xi, z = grid.gauss_legendre(24)
    ref = qp.solve(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, rows, xi, z, tol=1e-12)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(rows, gwl().Grid.gauss_legendre(24))
        E_sd, _, _, _ = c.qp_sd(rows)
        E128, _, _, _ = c.qp(rows, gwl().Grid.gauss_legendre(128))
    for j, r in enumerate(ref):
        assert st[j] == r["status"]
        assert abs(E[j] - r["E"]) <= 1e-10 * max(1.0, abs(r["E"])), (rows[j], E[j] - r["E"])
    # the exact pole form against CD on a grid fine enough for these strongly
    # coupled levels (24 points leave 1e-5 Ha where N_aux >> N_ov)
    assert np.all(np.abs(E_sd - E128) < 1e-8)


def test_repeated_states_give_identical_results():
    inp = gwgen.make_config("monomer")
    g = gwl().Grid.gauss_legendre(32)
    with gwl().Context.from_inputs(inp, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp([4, 5, 4, 5, 4], g)
    assert E[0] == E[2] == E[4] and E[1] == E[3]


def test_one_electron_spin_channel():
    # spin down has a single occupied level (the core), spin up two
    shape = gwgen.custom_shape(1, 12, 40, n_core=1)
    n_mo = shape.n_mo
    rows = [1, n_mo + 0, n_mo + 1]
    u = gwgen.make_inputs_uhf(shape, 5, rows, n_unpaired=1)
    assert u.n_occ == (2, 1)
    xi, z = grid.gauss_legendre(32)
    ref = uhf.solve(u.eps, u.n_occ, u.B_ov, u.row_ids, u.B_rows, rows, xi, z, tol=1e-12)
    with gwl().Context.from_inputs_uhf(u, qp_tol=1e-12) as c:
        E, S, Z, st = c.qp(rows, gwl().Grid.gauss_legendre(32))
    for j, r in enumerate(ref):
        assert abs(E[j] - r["E"]) <= 1e-10 * abs(r["E"]), (rows[j], E[j] - r["E"])
