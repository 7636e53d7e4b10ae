"""gw_dielectric_noalloc, the allocation-free form of gw_dielectric: through
the C-ABI its output equals gw_dielectric's (the same kernels in the same
order, so bit for bit) in FP64 and BF16x3, on two calls in a row, the second
on a smaller molecule with fewer grid points; sizes past its scratch array
are refused with an error naming the limit."""
import ctypes

import numpy as np
import pytest

import gwgen

pytestmark = pytest.mark.gpu


class _Hip:
    """Device buffers through the HIP runtime the library itself loaded (a
    second runtime in the process, such as torch's, would not see the GPU
    once the library's runtime holds it)."""

    def __init__(self):
        import paper_2107_10423_amd  # noqa: F401  (loads libgw and its runtime)
        path = None
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    path = line.split()[-1]
                    break
        assert path, "libamdhip64 not loaded"
        self.rt = ctypes.CDLL(path)
        self.rt.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.rt.hipFree.argtypes = [ctypes.c_void_p]
        self.rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_int]
        self.rt.hipDeviceSynchronize.argtypes = []

    def alloc(self, nbytes):
        p = ctypes.c_void_p()
        assert self.rt.hipMalloc(ctypes.byref(p), nbytes) == 0
        return p.value

    def free(self, p):
        assert self.rt.hipFree(ctypes.c_void_p(p)) == 0

    def put(self, dst, a):
        a = np.ascontiguousarray(a)
        assert self.rt.hipMemcpy(ctypes.c_void_p(dst), a.ctypes.data, a.nbytes, 1) == 0

    def get(self, src, a):
        assert self.rt.hipMemcpy(a.ctypes.data, ctypes.c_void_p(src), a.nbytes, 2) == 0
        return a

    def sync(self):
        assert self.rt.hipDeviceSynchronize() == 0


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_noalloc_dielectric_equals_dielectric(prec):
    import paper_2107_10423_amd as gwl
    hip = _Hip()
    cases = [(gwgen.cluster_shape(3), 7, [1e-3, 0.3, 2.0, 40.0, 900.0]),
             (gwgen.cluster_shape(1), 8, [0.05, 5.0])]
    for shape, seed, xis in cases:
        print(f"noalloc {prec}: n_aux={shape.n_aux} n_xi={len(xis)}", flush=True)
        inp = gwgen.make_inputs(shape, seed, [shape.n_occ - 1])
        with gwl.Context.from_inputs(inp, pi_prec=prec) as c:
            ref = c.dielectric(xis)    # also makes the split copies the mixed build reads
            Np = -(-shape.n_aux // 128) * 128
            ld = Np + 2                # rows longer than the matrix
            got = np.full((len(xis), Np, ld), np.nan)
            d_out = hip.alloc(got.nbytes)
            d_xi = hip.alloc(8 * len(xis))
            try:
                hip.put(d_out, got)
                hip.put(d_xi, np.array(xis))
                c.dielectric_noalloc(d_xi, len(xis), d_out, ld, Np * ld)
                hip.sync()
                hip.get(d_out, got)
            finally:
                hip.free(d_out)
                hip.free(d_xi)
        n = shape.n_aux
        for g in range(len(xis)):
            np.testing.assert_array_equal(np.tril(got[g, :n, :n]), np.tril(ref[g]))
            # padding rows and columns hold the identity's entries
            pad = got[g, n:Np, :Np]
            assert np.array_equal(np.tril(pad, n), np.tril(np.eye(Np)[n:Np], n))


def test_noalloc_dielectric_refuses_oversized_requests():
    """Refused before any launch: the buffers are never touched."""
    import paper_2107_10423_amd as gwl
    hip = _Hip()
    shape = gwgen.cluster_shape(2)
    inp = gwgen.make_inputs(shape, 9, [shape.n_occ - 1])
    d = hip.alloc(64)
    try:
        with gwl.Context.from_inputs(inp) as c:
            Np = 256
            with pytest.raises(gwl.GWError) as e:
                c.dielectric_noalloc(d, 100000, d, Np, Np * Np)
            assert e.value.code == -1 and "scratch" in str(e.value)
            with pytest.raises(gwl.GWError) as e:       # rows shorter than the padded matrix
                c.dielectric_noalloc(d, 1, d, Np - 2, Np * Np)
            assert e.value.code == -1
        with gwl.Context.from_inputs(inp, pi_prec="bf16x3") as c:
            with pytest.raises(gwl.GWError) as e:       # split copies not built yet
                c.dielectric_noalloc(d, 1, d, Np, Np * Np)
            assert e.value.code == -1 and "split copies" in str(e.value)
    finally:
        hip.free(d)
