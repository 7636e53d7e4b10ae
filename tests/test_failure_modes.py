"""Debug and failure modes, forced from the host (every kernel still exits
normally): GW_DEBUG_SYNC=1 synchronises after every launch and must not change
results; GW_TEST_INDEFINITE=1 turns 1 - Pi(i xi) into 1 + Pi(i xi) before the
Cholesky, which must end the call with GW_ENOTSPD and leave the context
usable.  Each mode runs in a child process (the variables are read once)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import gwgen

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import gwgen
import paper_2107_10423_amd as gwl
inp = gwgen.make_inputs(gwgen.custom_shape(5, 38, 112, n_core=1), 7, [4, 5], b_scale={bs})
out = {{}}
with gwl.Context.from_inputs(inp, qp_tol=1e-12, graphs=False) as c:
    try:
        E, S, Z, st = c.qp([4, 5], gwl.Grid.gauss_legendre(32))
        out["E"] = [float(x).hex() for x in E]
    except gwl.GWError as e:
        out["code"] = e.code
        out["msg"] = str(e)
        E, S, Z, st = c.qp_sd([4, 5])   # the context is still usable
        out["E_sd"] = [float(x) for x in E]
print("RESULT " + json.dumps(out))
"""


def run_child(env_extra, b_scale=1.0):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, bs=b_scale)], env=env,
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_debug_sync_gives_identical_results():
    import paper_2107_10423_amd as gwl
    inp = gwgen.make_inputs(gwgen.custom_shape(5, 38, 112, n_core=1), 7, [4, 5])
    with gwl.Context.from_inputs(inp, qp_tol=1e-12, graphs=False) as c:
        E, S, Z, st = c.qp([4, 5], gwl.Grid.gauss_legendre(32))
    out = run_child({"GW_DEBUG_SYNC": "1"})
    assert out["E"] == [float(x).hex() for x in E]


def test_indefinite_dielectric_matrix_is_reported():
    out = run_child({"GW_TEST_INDEFINITE": "1"}, b_scale=3.0)
    assert out["code"] == -4 and "not positive definite" in out["msg"]
    assert all(np.isfinite(out["E_sd"]))
