"""The oracle's C code under gcc's address and undefined-behaviour
sanitizers: a stand-alone driver (oracle/selftest.c) runs every stage of the
oracle on small meshes -- load, push, both collision processes, deposit,
Dirichlet and open-end solves, the elliptic insert at orders 1 and 3, cubic
shapes, the seed source, cross-section and anisotropy tables, moments, well
depth, diagnostics -- with electrons absorbed on the walls and the insert,
and checks the exact bookkeeping.  Any sanitizer report ends it with a
failure status."""
import os
import shutil
import subprocess

import pytest

from oracle import build


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_selftest_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = build.build_selftest(str(tmp_path / "selftest"))
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    lines = [l for l in r.stdout.splitlines() if "absorbed" in l]
    assert len(lines) == 5
    for l in lines:  # every run absorbed electrons and scattered some
        assert int(l.split(",")[-1].split()[0]) > 0 and int(l.split(" elastic")[0].split(",")[-1]) > 0, l
