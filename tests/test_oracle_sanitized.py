"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's own pin tests (detection, forces, integration, the delayed
schedule with its judge, meshes, family tags) run again in a child process
on a build with both sanitizers, where any out-of-bounds access, use after
free or undefined operation aborts the run.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    try:
        p = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime() is None, reason="gcc's AddressSanitizer runtime is not available")
def test_oracle_pins_pass_under_sanitizers():
    env = dict(os.environ)
    env["DEM_ORACLE_SANITIZE"] = "1"
    env["LD_PRELOAD"] = _runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_mesh.py", "test_oracle_families.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests,
                        "-k", "not incline and not sliding and not restitution and not energy"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
