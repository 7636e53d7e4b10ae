"""Serving loop (gw_server_*): each request's result is the same alone and in
the mix, admission never exceeds the memory budget, bad requests fail alone,
and latency stamps are ordered."""
import time

import numpy as np
import pytest

import gwgen

pytestmark = pytest.mark.gpu

MEV = 1e-3 / 27.211386245988


def gwl():
    import paper_2107_10423_amd as m
    return m


def requests(ks, seed0=1000):
    return [gwgen.serving_inputs(k, seed0 + i) for i, k in enumerate(ks)]


def alone(inp, prec, grid):
    with gwl().Context.from_inputs(inp, pi_prec=prec, qp_tol=1e-12) as c:
        return c.qp(list(inp.row_ids), grid)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_results_same_alone_and_in_the_mix(prec):
    grid = gwl().Grid.gauss_legendre(32)
    reqs = requests([1, 3, 2, 4, 1, 5, 2, 3, 1, 2])
    ref = [alone(r, prec, grid) for r in reqs]
    with gwl().Server(grid, pi_prec=prec, n_streams=3, qp_tol=1e-12) as srv:
        tickets = []
        for j, r in enumerate(reqs):        # staggered arrivals while others run
            tickets.append(srv.submit_inputs(r, list(r.row_ids)))
            if j % 3 == 2:
                time.sleep(0.02)
        srv.drain()
        st = srv.stats()
        outs = [srv.poll(t) for t in tickets]
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_active"] >= 2          # work of several requests overlapped
    worst = 0.0
    for (E, S, Z, status, info), (Ea, Sa, Za, sta) in zip(outs, ref):
        assert info["rc"] == 0
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        worst = max(worst, float(np.max(np.abs(E - Ea) / np.abs(Ea))))
        np.testing.assert_array_equal(status, sta)
    # stated tolerance of each path; the kernels are deterministic, so the
    # results are in fact expected to be identical
    assert worst <= 1e-10
    print(f"serving {prec}: max relative |E_mix - E_alone| = {worst:.3e}")


def test_admission_by_footprint_never_exceeds_budget():
    grid = gwl().Grid.gauss_legendre(16)
    reqs = requests([2, 3, 2, 3, 2])
    fp = [gwl().footprint(r.shape.n_mo, r.n_occ, r.shape.n_aux, 6, 6, 16, "fp64", 2 << 30)
          for r in reqs]
    budget = int(max(fp) * 1.5)           # never room for two of the larger ones
    with gwl().Server(grid, mem_budget_bytes=budget, n_streams=4) as srv:
        ts = [srv.submit_inputs(r, list(r.row_ids)) for r in reqs]
        srv.drain()
        st = srv.stats()
        infos = [srv.poll(t)[4] for t in ts]
    assert st["peak_reserved_bytes"] <= budget
    assert st["peak_active"] <= 2
    assert all(i["rc"] == 0 for i in infos)
    assert [i["footprint_bytes"] for i in infos] == fp
    # first come, first served: admission times follow submission order
    adm = [i["t_admit"] for i in infos]
    assert adm == sorted(adm)


def test_oversized_request_is_refused_and_bad_request_fails_alone():
    grid = gwl().Grid.gauss_legendre(16)
    r = requests([2])[0]
    with gwl().Server(grid, mem_budget_bytes=1 << 20) as srv:
        with pytest.raises(gwl().GWError) as e:
            srv.submit_inputs(r, list(r.row_ids))
        assert e.value.code == -2
    good = requests([1, 2])
    with gwl().Server(grid, n_streams=2, qp_tol=1e-12) as srv:
        t_bad = srv.submit(good[0].eps, good[0].n_occ, good[0].B_ov, good[0].row_ids,
                           good[0].B_rows, [0])          # state 0 has no row
        t_ok = srv.submit_inputs(good[1], list(good[1].row_ids))
        srv.drain()
        bad = srv.poll(t_bad)
        ok = srv.poll(t_ok)
    assert bad[4]["rc"] == -1 and ok[4]["rc"] == 0
    E_ref = alone(good[1], "fp64", grid)[0]
    np.testing.assert_array_equal(ok[0], E_ref)


def _burst(srv, head, reqs):
    """Submit `head` first (it keeps the one pipeline busy), then every request
    of `reqs` while it runs, so that requests of one shape queue together."""
    tickets = [srv.submit_inputs(head, list(head.row_ids))]
    tickets += [srv.submit_inputs(r, list(r.row_ids)) for r in reqs]
    srv.drain()
    return [srv.poll(t) for t in tickets]


@pytest.mark.parametrize("prec,wc", [("fp64", "fp64"), ("bf16x3", "bf16x3")])
def test_batched_stage_a_mixed_sizes_equals_solo_bitwise(prec, wc):
    """Water clusters of k = 1..24 on the 64-point grid, each seeded 1000 + r.
    The small shapes recur, so they queue behind the large head request and
    their stage A runs batched (one grouped launch sequence over all their grid
    points); every request's energies, Sigma^c, Z and status equal those of its
    own context run alone, bit for bit, in FP64 and in the mixed form."""
    grid = gwl().Grid.gauss_legendre(64)
    # the small requests first: their submissions (small host copies) are all
    # queued while the head runs; the large ones (up to 2 GB of input each)
    # follow, so that a slow copy cannot split a shape's queue
    ks = [1, 2, 1, 3, 2, 1, 4, 6, 5, 3, 1, 2, 6, 4, 9, 13, 18, 24]
    reqs = requests(ks)
    head = gwgen.serving_inputs(16, 999)
    solo = []
    for r in [head] + reqs:
        with gwl().Context.from_inputs(r, pi_prec=prec, wc_prec=wc, qp_tol=1e-12) as c:
            solo.append(c.qp(list(r.row_ids), grid))
    with gwl().Server(grid, pi_prec=prec, wc_prec=wc, n_streams=1, qp_tol=1e-12) as srv:
        outs = _burst(srv, head, reqs)
        st = srv.stats()
    assert st["completed"] == len(reqs) + 1 and st["failed"] == 0
    # k = 1 appears 4 times, 2 three times, 3, 4 and 6 twice: batches of 2-4
    # (a shape with one queued request runs alone and is not counted)
    assert st["batches"] >= 4 and st["batched_requests"] >= 12, st
    assert st["batched_requests"] > st["batches"]
    for j, ((E, S, Z, status, info), (Es, Ss, Zs, sts)) in enumerate(zip(outs, solo)):
        assert info["rc"] == 0
        np.testing.assert_array_equal(E, Es, err_msg=f"request {j}")
        np.testing.assert_array_equal(S, Ss, err_msg=f"request {j}")
        np.testing.assert_array_equal(Z, Zs, err_msg=f"request {j}")
        np.testing.assert_array_equal(status, sts, err_msg=f"request {j}")
    print(f"serving {prec}/{wc}: {st['batches']} batches of {st['batched_requests']} requests, "
          f"{st['graph_replays']} graph replays, identical to solo runs")


def test_recurring_shapes_reuse_memory_and_graphs():
    """Once warm, a wave of recurring shapes runs from the server's block cache
    (no new device or pinned allocation) and replays the graphs captured
    earlier; results equal the first wave's.  The first wave creates the
    shape groups, whose workspaces keep some blocks of size classes the
    requests also use, so the cache settles after the second wave."""
    grid = gwl().Grid.gauss_legendre(64)
    ks = [1, 1, 2, 2, 3, 3]
    reqs = requests(ks)
    head = gwgen.serving_inputs(12, 998)
    with gwl().Server(grid, pi_prec="bf16x3", wc_prec="bf16x3", n_streams=1,
                      qp_tol=1e-12) as srv:
        first = _burst(srv, head, reqs)
        _burst(srv, head, reqs)
        st2 = srv.stats()
        third = _burst(srv, head, reqs)
        st3 = srv.stats()
    print(f"device/pinned blocks from the runtime: {st2['device_mallocs']} after two waves, "
          f"{st3['device_mallocs']} after three; cache hits {st2['cache_hits']} -> "
          f"{st3['cache_hits']}; graph replays {st2['graph_replays']} -> "
          f"{st3['graph_replays']}", flush=True)
    assert st3["device_mallocs"] == st2["device_mallocs"], (st2, st3)
    assert st3["cache_hits"] > st2["cache_hits"]
    assert st3["graph_replays"] >= st2["graph_replays"] + 3, (st2, st3)
    for a, b in zip(first, third):
        np.testing.assert_array_equal(a[0], b[0])


def test_batching_off_gives_the_same_results():
    grid = gwl().Grid.gauss_legendre(32)
    reqs = requests([1, 1, 2, 2])
    head = gwgen.serving_inputs(8, 997)
    res = {}
    for lim in (0, -1):
        with gwl().Server(grid, pi_prec="bf16x3", n_streams=1, qp_tol=1e-12,
                          batch_max_aux=lim) as srv:
            res[lim] = _burst(srv, head, reqs)
            st = srv.stats()
        assert (st["batches"] > 0) == (lim == 0)
    for a, b in zip(res[0], res[-1]):
        np.testing.assert_array_equal(a[0], b[0])
