"""The C ABI from a plain C program (tests/capi_demo.c, built by the package's
build step, no Python in the process): its fluxes and balance must equal,
bitwise, those of the same problem run through the Python binding, in time
steps and in steady state."""
import os
import subprocess

import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "tests", "capi_demo")


def _box():
    from paper_2511_16821_amd import workloads as W
    return W.c1(n_s=1, n_particles=10000, si_tol=1e-12, si_max_iter=400, w_cut_rel=1e-8,
                seed=20251116)


@pytest.mark.parametrize("mode", ["steps", "steady"])
def test_c_program_matches_binding(mode):
    assert os.path.exists(DEMO), "tests/capi_demo is built by __graft_entry__.build()"
    log("capi_demo", mode)
    args = [DEMO] + (["steady"] if mode == "steady" else [])
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = r.stdout.split()
    phi_c = np.array([float(v) for v in vals[:400]])
    emitted, absorbed, segments = float(vals[400]), float(vals[401]), int(vals[402])
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh as S
    p = dict(_box(), steady=(mode == "steady"))
    s = S.Solver(p)
    s.advance(1 if mode == "steady" else 3)
    phi = s.get_flux(0)
    b = s.get_balance(2)
    s.destroy()
    assert np.array_equal(phi, phi_c)
    assert b["emitted"] == emitted and b["absorbed"] == absorbed and b["segments"] == segments
    log("  C and Python agree bitwise; phi_R sum %.6e" % phi.sum())
