"""GPU checks on the 16^3 x 32 benchmark workload at its full size (n = 1572864
complex unknowns, Wilson D^H D, kappa 0.12, 12 point sources + 12 Z4 noise
right-hand sides, m = 1000, freq = 100, mixed precision, tol 1e-8), in the
launch configuration of the benchmark step.  The oracle cannot run the whole
solve at this size in seconds, so the checks are on outputs it computes one by
one and on properties that hold at any size:

- the benchmark step itself (the one-call single-seed driver): every column
  converged with m_done = m; the FP64 true relative residual of sampled columns
  recomputed on the host by the oracle's operator (<= 1.5 tol); the seeded CG
  counts of RHS 2..24 not above plain FP64 CG's counts for the same columns + 2
  (seeding projects out a part of the initial error, which cannot slow CG down
  by more than rounding noise);
- the 24-column FP32 D and D^H passes in the stencil shape the autotuner chose
  for that step, on three sampled columns, element-wise against the oracle to
  4e-6 of the largest element (the bar of the small-lattice stencil tests);
- the first Lanczos coefficients of the seed (alpha_1..3, beta_0..3; three
  oracle applications), FP32 operator with a complex64 basis, to 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import operators as ops
from oracle.seed import seed_lanczos as o_seed_lanczos
from paper_0810_0330_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def full():
    _say("full-size workload: building 16^3 x 32 inputs")
    w = synth.wilson_16x3x32()
    inp = synth.make_inputs(w)
    op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(DEV), w.kappa)
    B = torch.from_numpy(api.pack_field(np.ascontiguousarray(inp["B"].T))).to(DEV)
    return w, inp, op, B, ops.WilsonNormalOp(inp["U"], w.kappa)


def test_benchmark_step_full_size(full):
    w, inp, op, B, oop = full
    _say("full-size benchmark step: single-seed driver, 24 RHS, m", w.m)
    out = api.single_seed_solve(op, B, w.m, w.freq, w.tol, mixed=True)
    _say("iters", out["iters"], "status", out["status"], "max relres", max(out["relres"]))
    assert out["status"] == 0
    assert out["m_done"] == w.m
    assert max(out["relres"]) <= w.tol
    X = out["X"]
    for j in (0, 1, 11, 12, 23):
        x = api.unpack_field(X[j:j + 1].cpu().numpy())[0]
        b = inp["B"][:, j]
        rr = np.linalg.norm(b - oop(x)) / np.linalg.norm(b)
        _say("column", j, "oracle true residual %.3e" % rr)
        assert rr <= 1.5 * w.tol, (j, rr)
    plain = [api.solve_cg(op, B[j:j + 1], w.tol)[1][0] for j in range(1, w.nrhs)]
    _say("plain FP64 CG counts", plain)
    for j, p in enumerate(plain, start=1):
        assert out["iters"][j] <= p + 2, (j, out["iters"][j], p)


def test_stencil_full_size_tuned_shape(full):
    w, inp, op, B, oop = full
    k = w.nrhs
    # the step above (or this call, when run alone) tunes the shape for (lattice, FP32, 24 columns)
    X = B.to(torch.complex64)
    op.dslash(X, 0, single=True)
    variant, _ = op.tune_info(k, single=True)
    _say("full-size 24-column FP32 passes, tuned shape", variant)
    U = inp["U"]
    for which, f in [(0, ops.wilson_D), (1, ops.wilson_Ddag)]:
        Y = op.dslash(X, which, single=True)
        for j in (0, 5, 17):
            y = api.unpack_field(Y[j:j + 1].cpu().numpy())[0]
            ref = f(inp["B"][:, j].reshape(w.dims[::-1] + (4, 3)), U, w.kappa).reshape(-1)
            err = _rel(y, ref)
            _say("pass", which, "column", j, "rel err %.2e" % err)
            assert err < 4e-6, (which, j, err)


def test_seed_first_steps_full_size(full):
    w, inp, op, B, oop = full
    _say("full-size seed: first three Lanczos steps against the oracle")
    basis = api.seed_lanczos(op, B[0], 3, 0, v_dtype=op.single_dtype)
    ref = o_seed_lanczos(oop, inp["B"][:, :1], m=3, freq=0)
    a = basis.alpha.cpu().numpy()[:3]
    b = basis.beta.cpu().numpy()[:4]
    _say("alpha", a, "oracle", ref.alpha[:3])
    assert basis.m_done == 3
    assert np.abs(a - ref.alpha[:3]).max() <= 1e-6 * np.abs(ref.alpha[:3]).max()
    assert np.abs(b - ref.beta[:4]).max() <= 1e-6 * np.abs(ref.beta[:4]).max()
