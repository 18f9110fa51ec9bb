"""Write the oracle's expected values for the GPU tests whose oracle runs take
minutes on a host core (too long to repeat inside a test).

Every number written here comes from ``oracle/`` on inputs from the seeded
generators of ``paper_0810_0330_amd/synth.py``; nothing comes from the HIP
library.  Usage (from the repository root):

    python tests/golden/make_oracle_golden.py SECTION [SECTION ...]

Sections and the file each writes (tests/golden/oracle_<section>.json):
  mixed8   Wilson D^H D on 8^4 (12 point sources, m = 150, full
           reorthogonalization, tol 1e-8) through the mixed-precision
           emulation (oracle/mixed.py): per-RHS counts of the seeded solve,
           their range over 6 runs with b^1 changed by 1e-7 relative (the
           size of the single-precision rounding the GPU's own arithmetic
           makes), the FP64 oracle's counts and the per-RHS error of the
           emulation against the FP64 oracle; mixed CG from zero on the first
           4 columns; the mixed related-RHS solve of 5 related Gaussian
           right-hand sides (m = 60).
  tmarch   Wilson 16 x 16 x 4 x 8, 3 Gaussian columns, tol 1e-9: mixed CG counts.
  grad12   Wilson 12^4 (point sources (0,0) and (0,1), Gaussian eta): the
           oracle gradient with tight CG solves (tol 1e-13): L, dL/dkappa,
           and dL/db = lambda at 256 sampled entries per column with its norm.
  c3       Wilson 16^3 x 32 (the benchmark lattice): FP64 oracle CG counts of
           columns 0 and 12 at tol 1e-8, the mixed emulation's counts of the
           same, and tight solutions (tol 1e-12) of columns 0, 12 and 23 at
           512 sampled entries with their norms.
  c3all    the same lattice: the mixed emulation's plain-CG count (from zero,
           tol 1e-8) of every one of the 24 columns (4 worker processes).
  c3seed   the same lattice: the mixed emulation's single-seeded solve of all
           24 columns with m = 200, freq = 100 (counts per column), and the
           orthogonality of its complex64 basis, max |(V^H V - I)[i, j]| over
           j <= i, for the columns just before and just after the two
           reorthogonalization events (0-based 98..100 and 198..200).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import mixed  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle.cg import cg  # noqa: E402
from oracle.grad import grads  # noqa: E402
from oracle.seeded import seeded_solve  # noqa: E402
from paper_0810_0330_amd import synth  # noqa: E402


def _c(v):
    v = np.asarray(v)
    return [[float(z.real), float(z.imag)] for z in v.reshape(-1)]


def _say(*a):
    print(*a, flush=True)


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def mixed8():
    w = synth.wilson_8x4(m=150)
    inp = synth.make_inputs(w)
    op = ops.WilsonNormalOp(inp["U"], w.kappa)
    a32 = op.single()
    B = inp["B"]
    base = mixed.seeded_solve_mixed(op, a32, B, w.m, w.freq, w.tol)
    _say("mixed8 base", base["iters"])
    lo, hi = list(base["iters"]), list(base["iters"])
    for s in range(6):
        g = np.random.default_rng(200 + s)
        B2 = B.copy()
        nb = np.linalg.norm(B[:, 0])
        B2[:, 0] = B[:, 0] + (g.standard_normal(B.shape[0]) + 1j * g.standard_normal(B.shape[0])) * (
            1e-7 * nb / np.sqrt(2 * B.shape[0]))
        its = mixed.seeded_solve_mixed(op, a32, B2, w.m, w.freq, w.tol)["iters"]
        _say("mixed8 ensemble", s, its)
        lo = [min(a, b) for a, b in zip(lo, its)]
        hi = [max(a, b) for a, b in zip(hi, its)]
    ref = seeded_solve(op, B, w.m, w.freq, w.tol)
    err = [float(np.linalg.norm(base["X"][:, j] - ref["X"][:, j]) / np.linalg.norm(ref["X"][:, j]))
           for j in range(B.shape[1])]
    _, cg4, _ = mixed.cg_mixed_multi(op, a32, B[:, :4], tol=w.tol)
    _say("mixed8 cg4", cg4)
    Br = synth.related_rhs(synth.complex_gaussian(op.n, 5, synth.rng(1, 5)))
    _, rel_mv = mixed.related_rhs_solve_mixed(op, a32, Br, 60, 1, 1e-8)
    _say("mixed8 related", rel_mv)
    return {"workload": w.name, "m": w.m, "freq": w.freq, "tol": w.tol,
            "seeded_iters": base["iters"], "seeded_lo": lo, "seeded_hi": hi,
            "fp64_iters": ref["iters"], "err_vs_fp64": err,
            "cg4_iters": cg4, "related_m60_iters": rel_mv}


def tmarch():
    dims = (16, 16, 4, 8)
    U = synth.su3_links(dims, synth.rng(9, 0))
    op = ops.WilsonNormalOp(U, 0.12)
    B = synth.complex_gaussian(op.n, 3, synth.rng(9, 1))
    _, its, rel = mixed.cg_mixed_multi(op, op.single(), B, tol=1e-9)
    _say("tmarch", its, rel)
    return {"dims": dims, "tol": 1e-9, "cg_iters": its}


def grad12():
    w = synth.wilson_12x4(m=150)
    inp = synth.make_inputs(w)
    Eta = synth.complex_gaussian(w.n, w.nrhs, synth.rng(w.config_id, 2))
    cols = [0, 1]
    L, X, Lam, gk = grads(inp["U"], w.kappa, inp["B"][:, cols], Eta[:, cols], tol=1e-13)
    idx = _sample(w.n, 256, 12)
    _say("grad12 L", L, "dL/dkappa", gk)
    return {"workload": w.name, "cols": cols, "tol": 1e-13, "L": L, "dL_dkappa": gk,
            "sample_index": idx.tolist(),
            "lambda_sample": [_c(Lam[idx, j]) for j in range(len(cols))],
            "lambda_norm": [float(np.linalg.norm(Lam[:, j])) for j in range(len(cols))]}


def c3():
    w = synth.wilson_16x3x32()
    inp = synth.make_inputs(w)
    op = ops.WilsonNormalOp(inp["U"], w.kappa)
    B = inp["B"]
    out = {"workload": w.name, "tol": w.tol}
    fp64, mix = [], []
    for j in (0, 12):
        t = time.time()
        _, it, rel = cg(op, B[:, j], tol=w.tol)
        _say("c3 fp64 cg col", j, it, rel, f"{time.time() - t:.0f} s")
        fp64.append(it)
        t = time.time()
        _, itm, relm = mixed.cg_mixed(op, op.single(), B[:, j], tol=w.tol)
        _say("c3 mixed cg col", j, itm, relm, f"{time.time() - t:.0f} s")
        mix.append(itm)
    out["cols"] = [0, 12]
    out["fp64_cg_iters"] = fp64
    out["mixed_cg_iters"] = mix
    idx = _sample(op.n, 512, 3)
    out["sample_index"] = idx.tolist()
    out["x_cols"] = [0, 12, 23]
    out["x_tol"] = 1e-12
    out["x_sample"], out["x_norm"] = [], []
    for j in out["x_cols"]:
        t = time.time()
        x, it, rel = cg(op, B[:, j], tol=1e-12)
        _say("c3 tight col", j, it, rel, f"{time.time() - t:.0f} s")
        out["x_sample"].append(_c(x[idx]))
        out["x_norm"].append(float(np.linalg.norm(x)))
    return out


def _c3_mixed_col(j):
    w = synth.wilson_16x3x32()
    inp = synth.make_inputs(w)
    op = ops.WilsonNormalOp(inp["U"], w.kappa)
    _, it, rel = mixed.cg_mixed(op, op.single(), inp["B"][:, j], tol=w.tol)
    _say("c3all mixed cg col", j, it, rel)
    return it


def c3all():
    from multiprocessing import Pool
    w = synth.wilson_16x3x32()
    with Pool(4) as pool:
        its = pool.map(_c3_mixed_col, range(w.nrhs))
    return {"workload": w.name, "tol": w.tol, "mixed_cg_iters": its}


def basis_orthogonality(V, rows):
    """max |(V^H V - I)[i, j]| over j <= i for each 0-based column i of the basis V (n x m+1)."""
    out = {}
    for i in rows:
        vi = V[:, i].astype(np.complex128)
        g = V[:, : i + 1].astype(np.complex128).conj().T @ vi
        g[i] -= 1.0
        out[str(i)] = float(np.abs(g).max())
    return out


def c3seed():
    w = synth.wilson_16x3x32()
    inp = synth.make_inputs(w)
    op = ops.WilsonNormalOp(inp["U"], w.kappa)
    m, freq = 200, 100
    t = time.time()
    res = mixed.seeded_solve_mixed(op, op.single(), inp["B"], m, freq, w.tol)
    _say("c3seed mixed seeded iters", res["iters"], f"{time.time() - t:.0f} s")
    rows = [98, 99, 100, 198, 199, 200]
    orth = basis_orthogonality(res["seed"].V, rows)
    _say("c3seed basis orthogonality", orth)
    return {"workload": w.name, "m": m, "freq": freq, "tol": w.tol, "seeded_iters": res["iters"],
            "cg_iters": res["cg_iters"], "m_done": res["seed"].m_done, "basis_orth_rows": rows,
            "basis_orth": orth}


SECTIONS = {"mixed8": mixed8, "tmarch": tmarch, "grad12": grad12, "c3": c3, "c3all": c3all, "c3seed": c3seed}

if __name__ == "__main__":
    for name in sys.argv[1:]:
        t0 = time.time()
        res = SECTIONS[name]()
        res["generated_by"] = "tests/golden/make_oracle_golden.py " + name
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
            json.dump(res, f, indent=1)
        _say(name, "done in", f"{time.time() - t0:.0f} s")
