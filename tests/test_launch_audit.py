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


def test_launch_audit_under_host_sanitizers():
    """The same walk with the host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unchanged, nothing launched)."""
    import shutil
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        import pytest
        pytest.skip("ROCm compilers not installed")
    root = os.path.dirname(HERE)
    b = subprocess.run([sys.executable, os.path.join(root, "paper_2107_10423_amd", "build.py"),
                        "--host-sanitizers"], capture_output=True, text=True, timeout=900)
    assert b.returncode == 0, b.stdout[-2000:] + b.stderr[-2000:]
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", GW_LIB_VARIANT="hostsan")
    r = subprocess.run([sys.executable, os.path.join(HERE, "audit_walk.py")], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "audit ok" in r.stdout
