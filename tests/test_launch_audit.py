"""Every launch of the HIP path, walked on the CPU in launch-audit mode for a
range of shapes (ragged, tiny, chunked, many rows, the (H2O)10 shape), must
pass its host-side bounds guard."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def test_every_launch_stays_in_bounds():
    r = subprocess.run([sys.executable, os.path.join(HERE, "audit_walk.py")],
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "audit ok" in r.stdout
