"""GPU tests of the differentiable seeded solve (adjoint backward).

Bars: against the oracle gradient (dense solves) on a 4^4 lattice, dL/db and
dL/dkappa within 1e-8 relative (FP64 solves to 1e-12); on the 12^4 lattice
(point sources, kappa = 0.12), against the oracle gradient of two right-hand
sides (tight oracle CG solves, stored in tests/golden/oracle_grad12.json by
tests/golden/make_oracle_golden.py): L, dL/dkappa and dL/db at 256 sampled
entries within 1e-8 relative; with all 12, the central difference in kappa with
h = 1e-6 (FP64 solves to 1e-13, so the difference carries ~1e-13/1e-6 noise)
within 1e-5 relative, and the central difference along random directions of
b, which has no truncation error because L is linear in b, within 1e-8.  In
mixed precision (FP32 solves with FP64 reliable updates, tol 1e-10) on 4^4,
against the oracle gradient within 1e-7 (cond(A) tol bounds the solution errors).
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import grad as ograd
from paper_0810_0330_amd import api, synth
from paper_0810_0330_amd.autograd import seeded_solve

pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLDEN_GRAD12 = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                            "oracle_grad12.json")))


def _lib(Bnat):
    return torch.from_numpy(api.pack_field(np.ascontiguousarray(Bnat.T))).to(DEV)


def _nat(X):
    return api.unpack_field(X.detach().cpu().numpy()).T


def _loss(X, Eta):
    return (torch.conj(Eta) * X).real.sum()


def test_grad_matches_oracle_4x4():
    print("grad vs oracle 4^4", flush=True)
    dims = (4, 4, 4, 4)
    U = synth.su3_links(dims, synth.rng(31, 0))
    B = synth.point_sources(dims, synth.ALL_SPIN_COLOUR[:3])
    Eta = synth.complex_gaussian(B.shape[0], 3, synth.rng(31, 2))
    Lo, Xo, Lamo, gko = ograd.grads(U, 0.12, B, Eta, dense=True)
    Ul = torch.from_numpy(api.pack_links(U)).to(DEV)
    Bl = _lib(B).requires_grad_(True)
    kap = torch.tensor(0.12, dtype=torch.float64, device=DEV, requires_grad=True)
    X = seeded_solve(Bl, kap, Ul, dims, 60, 1, 1e-12)
    L = _loss(X, _lib(Eta))
    L.backward()
    assert abs(L.item() - Lo) <= 1e-10 * abs(Lo)
    gB = _nat(Bl.grad)
    assert np.abs(gB - Lamo).max() <= 1e-8 * np.abs(Lamo).max()
    assert abs(kap.grad.item() - gko) <= 1e-8 * abs(gko)


def test_grad_mixed_precision_4x4():
    # FP32 solves with FP64 reliable updates in the forward and the adjoint:
    # the FP64 true residuals at tol = 1e-10 bound the errors of X and of the
    # adjoint solutions by cond(A) tol (about 5e-9 here), hence 1e-7 on the gradients
    print("grad mixed precision 4^4", flush=True)
    dims = (4, 4, 4, 4)
    U = synth.su3_links(dims, synth.rng(32, 0))
    B = synth.point_sources(dims, synth.ALL_SPIN_COLOUR[:3])
    Eta = synth.complex_gaussian(B.shape[0], 3, synth.rng(32, 2))
    Lo, Xo, Lamo, gko = ograd.grads(U, 0.12, B, Eta, dense=True)
    Ul = torch.from_numpy(api.pack_links(U)).to(DEV)
    Bl = _lib(B).requires_grad_(True)
    kap = torch.tensor(0.12, dtype=torch.float64, device=DEV, requires_grad=True)
    X = seeded_solve(Bl, kap, Ul, dims, 60, 10, 1e-10, mixed=True)
    L = _loss(X, _lib(Eta))
    L.backward()
    assert abs(L.item() - Lo) <= 1e-7 * abs(Lo)
    gB = _nat(Bl.grad)
    assert np.abs(gB - Lamo).max() <= 1e-7 * np.abs(Lamo).max()
    assert abs(kap.grad.item() - gko) <= 1e-7 * abs(gko)


@pytest.fixture(scope="module")
def c4():
    w = synth.wilson_12x4(m=150)
    inp = synth.make_inputs(w)
    Eta = synth.complex_gaussian(w.n, w.nrhs, synth.rng(w.config_id, 2))
    return w, inp, Eta


def test_grad_12x4_against_oracle(c4):
    # the C4 lattice itself: two right-hand sides through the autograd path
    # (forward seeded solve, adjoint solves seeded from the forward basis)
    # against the oracle's gradient with tight CG solves
    w, inp, Eta = c4
    g = GOLDEN_GRAD12
    assert g["workload"] == w.name
    cols = g["cols"]
    print("grad vs oracle 12^4, columns", cols, flush=True)
    Ul = torch.from_numpy(api.pack_links(inp["U"])).to(DEV)
    Bl = _lib(inp["B"][:, cols]).requires_grad_(True)
    kap = torch.tensor(w.kappa, dtype=torch.float64, device=DEV, requires_grad=True)
    X = seeded_solve(Bl, kap, Ul, w.dims, w.m, w.freq, 1e-12)
    L = _loss(X, _lib(Eta[:, cols]))
    L.backward()
    gB = _nat(Bl.grad)
    idx = np.array(g["sample_index"])
    lam = np.stack([np.array([complex(a, b) for a, b in col]) for col in g["lambda_sample"]], axis=1)
    print(f"L {L.item():.15e} oracle {g['L']:.15e}; dL/dkappa {kap.grad.item():.15e} oracle {g['dL_dkappa']:.15e}",
          flush=True)
    assert abs(L.item() - g["L"]) <= 1e-8 * abs(g["L"])
    assert abs(kap.grad.item() - g["dL_dkappa"]) <= 1e-8 * abs(g["dL_dkappa"])
    assert np.abs(gB[idx] - lam).max() <= 1e-8 * np.abs(lam).max()
    for j in range(len(cols)):
        assert abs(np.linalg.norm(gB[:, j]) - g["lambda_norm"][j]) <= 1e-8 * g["lambda_norm"][j]


def test_grad_fd_12x4(c4):
    w, inp, Eta = c4
    print("grad FD 12^4", flush=True)
    Ul = torch.from_numpy(api.pack_links(inp["U"])).to(DEV)
    Bl = _lib(inp["B"]).requires_grad_(True)
    El = _lib(Eta)
    tol = 1e-13
    kap = torch.tensor(w.kappa, dtype=torch.float64, device=DEV, requires_grad=True)
    X = seeded_solve(Bl, kap, Ul, w.dims, w.m, w.freq, tol)
    L = _loss(X, El)
    L.backward()
    gk = kap.grad.item()
    h = 1e-6
    with torch.no_grad():
        lp = _loss(seeded_solve(Bl.detach(), torch.tensor(w.kappa + h, dtype=torch.float64), Ul, w.dims, w.m, w.freq,
                                tol), El).item()
        lm = _loss(seeded_solve(Bl.detach(), torch.tensor(w.kappa - h, dtype=torch.float64), Ul, w.dims, w.m, w.freq,
                                tol), El).item()
    fd = (lp - lm) / (2 * h)
    print(f"dL/dkappa analytic {gk:.12e} fd {fd:.12e}", flush=True)
    assert abs(fd - gk) <= 1e-5 * abs(gk)
    # L is linear in b: central differences along random directions are exact
    gen = synth.rng(w.config_id, 4)
    gB = Bl.grad.detach()
    with torch.no_grad():
        for _ in range(3):
            Ud = _lib(synth.complex_gaussian(w.n, w.nrhs, gen))
            t = 1e-3
            lp = _loss(seeded_solve(Bl.detach() + t * Ud, kap.detach(), Ul, w.dims, w.m, w.freq, tol), El).item()
            lm = _loss(seeded_solve(Bl.detach() - t * Ud, kap.detach(), Ul, w.dims, w.m, w.freq, tol), El).item()
            fdb = (lp - lm) / (2 * t)
            an = (torch.conj(gB) * Ud).real.sum().item()
            assert abs(fdb - an) <= 1e-8 * max(1.0, abs(an)), (fdb, an)
