"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every function include/gw.h declares, and rejects bad input before touching
a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gw_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gw_setup", "gw_qp", "gw_free", "gw_last_error", "gw_grid_gauss_legendre"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2107_10423_amd as gwl
    lib = ctypes.CDLL(gwl.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(gwl.exported_symbols())


def test_grid_matches_oracle_grid():
    import paper_2107_10423_amd as gwl
    from oracle import grid
    for n in (1, 2, 7, 64, 128, 200):
        xi, w = gwl.grid_gauss_legendre(n, 0.5)
        xo, wo = grid.gauss_legendre(n, 0.5)
        # the map xi = x0 (1+t)/(1-t) amplifies the rounding of 1 - t near t = 1,
        # so the largest nodes' weights agree only to ~1e-11 between two
        # correct Gauss-Legendre implementations
        np.testing.assert_allclose(xi, xo, rtol=1e-11)
        np.testing.assert_allclose(w, wo, rtol=1e-10)
    with pytest.raises(gwl.GWError):
        gwl.grid_gauss_legendre(0)
    with pytest.raises(gwl.GWError):
        gwl.grid_gauss_legendre(8, -1.0)


def _small():
    import gwgen
    shape = gwgen.custom_shape(3, 5, 9)
    return gwgen.make_inputs(shape, 3, [2, 3])


@pytest.mark.parametrize("mutate,frag", [
    (lambda d: d.update(eps=d["eps"][::-1].copy()), "ascending"),
    (lambda d: d["eps"].__setitem__(1, np.nan), "finite"),
    (lambda d: d.update(n_occ=8), "sizes"),
    (lambda d: d.update(row_ids=np.array([2, 2])), "repeated"),
    (lambda d: d.update(row_ids=np.array([2, 99])), "range"),
    (lambda d: d["B_ov"].__setitem__((0, 0), np.inf), "non-finite"),
])
def test_setup_rejects_bad_input_before_device_work(mutate, frag):
    import paper_2107_10423_amd as gwl
    inp = _small()
    d = dict(eps=inp.eps.copy(), n_occ=3, B_ov=inp.B_ov.copy(), row_ids=inp.row_ids.copy(),
             B_rows=inp.B_rows.copy())
    mutate(d)
    with pytest.raises((gwl.GWError, ValueError)) as e:
        gwl.Context(d["eps"], d["n_occ"], d["B_ov"], d["row_ids"], d["B_rows"])
    if isinstance(e.value, gwl.GWError):
        assert e.value.code == -1 and frag in str(e.value)


@pytest.mark.parametrize("mutate,frag", [
    (lambda d: d["eps"].__setitem__((1, slice(None)), d["eps"][1][::-1].copy()), "ascending"),
    (lambda d: d["eps"].__setitem__((1, 2), np.nan), "finite"),
    (lambda d: d.update(row_ids=np.array([2, 2])), "repeated"),
    (lambda d: d.update(row_ids=np.array([2, 16])), "range"),
    (lambda d: d["B_dn"].__setitem__((0, 0), np.inf), "non-finite"),
])
def test_open_shell_setup_rejects_bad_input_before_device_work(mutate, frag):
    import gwgen
    import paper_2107_10423_amd as gwl
    u = gwgen.make_inputs_uhf(gwgen.custom_shape(3, 5, 9), 3, [2, 8 + 3])
    d = dict(eps=u.eps.copy(), B_up=u.B_ov[0].copy(), B_dn=u.B_ov[1].copy(),
             row_ids=u.row_ids.copy(), B_rows=u.B_rows.copy())
    mutate(d)
    if d["B_rows"].shape[0] != d["row_ids"].size:
        d["B_rows"] = np.zeros((d["row_ids"].size,) + d["B_rows"].shape[1:])
    with pytest.raises((gwl.GWError, ValueError)) as e:
        gwl.Context.uhf(d["eps"], u.n_occ, d["B_up"], d["B_dn"], d["row_ids"], d["B_rows"])
    if isinstance(e.value, gwl.GWError):
        assert e.value.code == -1 and frag in str(e.value), str(e.value)


def test_generator_is_reproducible_and_shaped():
    import gwgen
    a = gwgen.make_config("monomer")
    b = gwgen.make_config("monomer")
    assert np.array_equal(a.B_ov, b.B_ov) and np.array_equal(a.eps, b.eps)
    assert a.B_ov.shape == (112, 5 * 38) and a.B_rows.shape == (2, 43, 112)
    assert a.eps[0] == -20.5 and np.all(np.diff(a.eps) > 0)
    B = gwgen.full_B(a.shape, 1)
    np.testing.assert_array_equal(B, B.transpose(0, 2, 1))
    np.testing.assert_array_equal(B[:, :5, 5:].reshape(112, -1), a.B_ov)
    np.testing.assert_array_equal(B[:, [4, 5], :].transpose(1, 2, 0), a.B_rows)
    # variance of the recipe
    c = gwgen.make_config("h2o10", states=[49])
    assert abs(c.B_ov.std() / np.sqrt(0.25 / (50 * 380)) - 1) < 0.01
    assert np.sum(c.eps < -10) == 10 and np.sum(c.eps > 0) == 380


def test_full_setup_rejects_bad_input_before_device_work():
    import gwgen
    import paper_2107_10423_amd as gwl
    a = gwgen.make_inputs(gwgen.custom_shape(3, 5, 9), 3, [2])
    B = gwgen.full_B(a.shape, 3)
    bad = B.copy()
    bad[2, 1, 6] = np.nan
    with pytest.raises(gwl.GWError) as e:
        gwl.Context.full(a.eps, 3, bad)
    assert e.value.code == -1 and "non-finite" in str(e.value)
    with pytest.raises(gwl.GWError) as e:
        gwl.Context.full(a.eps, 8, B)
    assert e.value.code == -1 and "sizes" in str(e.value)


def test_setup_rejects_unknown_wc_prec_before_device_work():
    import paper_2107_10423_amd as gwl
    inp = _small()
    for bad in (1, 3, -1):   # only FP64 and the BF16x3 form exist for W^c
        with pytest.raises(gwl.GWError) as e:
            gwl.Context.from_inputs(inp, wc_prec=bad)
        assert e.value.code == -1 and "wc_prec" in str(e.value)


def test_footprint_counts_the_mixed_contraction_workspace():
    """The mixed W^c form adds the split R (4 Rp Np bytes) and the split
    F = L^-1 - I of every grid point of a chunk (4 Np^2 bytes each)."""
    import paper_2107_10423_amd as gwl
    n_mo, n_occ, n_aux, n_rows, G = 430, 50, 1120, 10, 64
    Np, Rp = 1152, 4352
    base = gwl.footprint(n_mo, n_occ, n_aux, n_rows, 10, G, pi_prec="bf16x3")
    mixed = gwl.footprint(n_mo, n_occ, n_aux, n_rows, 10, G, pi_prec="bf16x3", wc_prec="bf16x3")
    assert mixed - base == 4 * Rp * Np + (G + 1) * 4 * Np * Np
