"""The C-ABI from plain C: tests/c/abi_c_client.c includes only include/*.h,
must compile as strict C99 (-Wall -Wextra -Werror -pedantic), link against
libgw.so and run its calls in launch-audit mode (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_c_client_compiles_links_and_runs(tmp_path):
    gcc = shutil.which("gcc")
    lib_dir = os.path.join(ROOT, "paper_2107_10423_amd")
    if gcc is None:
        pytest.skip("gcc not installed")
    if not os.path.exists(os.path.join(lib_dir, "libgw.so")):
        pytest.skip("libgw.so not built")
    exe = str(tmp_path / "abi_c_client")
    cc = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                         "-I", os.path.join(ROOT, "include"),
                         os.path.join(HERE, "c", "abi_c_client.c"), "-L", lib_dir, "-lgw",
                         f"-Wl,-rpath,{lib_dir}", "-o", exe], capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c client ok" in r.stdout
