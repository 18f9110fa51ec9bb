"""GPU tests of the solvers' stopping rules on problems they cannot solve to tol.

A column whose residual stalls must stop after a bounded number of iterations
and be reported as SC_NOT_CONVERGED, instead of iterating to the default
iteration limit (100000):
  * tol = 1e-17 on the 32 x 32 Laplacian is below what the FP64 true residual
    can reach: mixed-precision CG stops when reliable updates stop reducing the
    true residual, FP64 CG after its bounded restarts;
  * an inconsistent system (a well-conditioned diagonal with one zero entry,
    b nonzero there): MINRES's residual reaches the least-squares residual
    |b_0| within a few dozen iterations and cannot fall further; it stops by
    the least-squares test (||A r|| tiny against ||A|| ||r||) there, before
    the later iterations let x grow without bound (they would push the true
    residual above the plateau while the rotated one drifts below it).
Each case also checks that the answer returned is still the best the solver
reached (true residual at the rounding floor, or at the plateau).
"""
import time

import numpy as np
import pytest
import torch

from paper_0810_0330_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def test_cg_stops_below_attainable_tol():
    op = api.Op.laplace2d(32, 32)
    B = synth.real_gaussian(1024, 3, synth.rng(60, 1))
    Bt = torch.from_numpy(B.T.copy()).to(DEV)
    for mixed in (True, False):
        _say("cg tol 1e-17 on laplace 32x32, mixed", mixed)
        t0 = time.time()
        X, its, rel, st = api.solve_cg(op, Bt, 1e-17, mixed=mixed, with_status=True)
        torch.cuda.synchronize()
        dt = time.time() - t0
        _say("  iters", its, "relres", rel, "status", st, f"{dt:.2f} s")
        assert st == 1
        assert max(its) < 3000
        assert dt < 60
        assert max(rel) < 1e-12


def test_stall_on_inconsistent_system():
    # A = diag(0, then values in [1, 2]): MINRES reaches the least-squares
    # residual |b_0| within a few dozen iterations and then cannot decrease
    n = 5000
    d = np.concatenate([[0.0], np.linspace(1.0, 2.0, n - 1)])
    dt_ = torch.from_numpy(d).to(DEV)
    op = api.Op.diag(dt_)
    B = synth.real_gaussian(n, 2, synth.rng(61, 1))
    Bt = torch.from_numpy(B.T.copy()).to(DEV)
    floor = np.abs(B[0]) / np.linalg.norm(B, axis=0)  # smallest attainable relative residual
    _say("minres on a singular diagonal")
    X, its, rel, st = api.solve_minres(op, Bt, 1e-10, with_status=True)
    _say("  iters", its, "relres", rel, "status", st)
    assert st == 1 and max(its) < 200
    for j in range(2):
        assert rel[j] < 1.0001 * floor[j]


def test_minres_stops_below_attainable_tol():
    op = api.Op.laplace2d(32, 32)
    B = synth.real_gaussian(1024, 2, synth.rng(62, 1))
    Bt = torch.from_numpy(B.T.copy()).to(DEV)
    _say("minres tol 1e-17 on laplace 32x32")
    X, its, rel, st = api.solve_minres(op, Bt, 1e-17, with_status=True)
    _say("  iters", its, "relres", rel, "status", st)
    assert st == 1 and max(its) < 5000 and max(rel) < 1e-12
