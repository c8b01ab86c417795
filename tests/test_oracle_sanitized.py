"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle is rebuilt with -fsanitize=address,undefined (every report
fatal) and a child Python process, with the ASan runtime preloaded, drives
every exported routine on small grids, degenerate ones included (1 x 1 x 1,
extents of 1 and 2 where neighbours wrap onto the node itself): the step and
multi-step runs (BGK and MRT), the macroscopic fields, the ligament set-up on
every axis with noise, the diagnostics on every axis, the droplet labelling,
and a short coexistence run.  The child must end cleanly with no sanitizer
report.  (Leak detection is off: the Python interpreter itself keeps
allocations until exit.)
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle, workloads
for shape in [(1, 1, 1), (2, 1, 3), (5, 4, 3), (9, 7, 11)]:
    nz, ny, nx = shape
    f = workloads.random_populations(shape, seed=sum(shape), base=1.2, spread=0.4)
    g = oracle.step(f, 0.8, -5.5)
    g = oracle.run(g, 3, 0.9, -5.5)
    g = oracle.run(g, 2, 0.9, -5.5, mrt=dict(oracle.MRT_DEFAULT))
    fl = oracle.fields(g, -5.5)
    for axis in (0, 1, 2):
        d = oracle.diag(g, axis=axis)
        h = oracle.init_ligament(nx, ny, nz, axis=axis, R0=1.5, amp_rel=0.1, wavelength=4.0,
                                 rho_l=2.2, rho_v=0.1, noise_amp=1e-3, seed=3)
    count, lab = oracle.label(fl["rho"], float(np.median(fl["rho"])))
    assert np.all(np.isfinite(g)) and lab.shape == shape
co = oracle.coexistence(-5.5, 1.0, max_steps=3000, chunk=1000)
assert co.rho_l > co.rho_v > 0
print("SANITIZED_OK", oracle.num_threads())
"""


def test_oracle_is_clean_under_asan_and_ubsan():
    import oracle

    try:
        oracle.build(sanitize=True)
    except (subprocess.CalledProcessError, FileNotFoundError) as e:
        pytest.fail(f"sanitized oracle build failed: {e}")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.exists(asan), asan
    env = dict(os.environ, ORACLE_SANITIZED="1", LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True, timeout=600,
                       cwd=ROOT, env=env)
    report = r.stdout[-2000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "SANITIZED_OK" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
