"""The oracle's OpenMP timing build (the benchmark's CPU baseline) gives the
same bits as the single-threaded checker: its pragmas only split loops whose
iterations are independent."""
import os
import subprocess
import sys

import numpy as np

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CASE = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1407_5600_amd import inputs
w = inputs.random_suspension(5, 24, 30)
prm = oracle.params(w.L, rho=1.2, eta=0.8, dt=0.02)
v0 = 0.1 * np.random.default_rng(2).standard_normal((3, w.L, w.L, w.L))
r = oracle.step(prm, w.springs(), w.q, v0, w.Fext, 3)
np.savez(sys.argv[2], **r)
"""


def _run(lib, out, threads):
    env = dict(os.environ, MBO_ORACLE_LIB=lib, OMP_NUM_THREADS=str(threads))
    subprocess.run([sys.executable, "-c", _CASE, ROOT, out], check=True, env=env)
    return dict(np.load(out))


def test_openmp_build_is_bitwise_equal(tmp_path):
    serial = obuild.LIB if os.path.exists(obuild.LIB) else obuild.build()
    omp = obuild.LIB_OMP if os.path.exists(obuild.LIB_OMP) else obuild.build(openmp=True)
    a = _run(serial, str(tmp_path / "a.npz"), 1)
    b = _run(omp, str(tmp_path / "b.npz"), 4)
    assert set(a) == set(b)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
