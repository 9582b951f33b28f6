"""Host-code sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer,
then ThreadSanitizer) of the library's host-only entry points: the worker
pool, the Givens planner, the MPO builder, input validation, the workspace
bound and the one-hot count (tests/sanitize/).  CPU only; about two minutes
of compilation, so it runs when TNQE_SANITIZE=1."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(os.environ.get("TNQE_SANITIZE") != "1", reason="set TNQE_SANITIZE=1 (two minutes of builds)")
def test_host_sanitizers(tmp_path):
    r = subprocess.run([os.path.join(HERE, "sanitize", "run_sanitizers.sh"), str(tmp_path)], capture_output=True,
                       text=True, timeout=1800)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert r.stdout.count("host driver: ok (0 failed checks)") == 2
