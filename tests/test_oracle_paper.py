"""Character pins of the oracle against the paper's diagonal examples (Section 2,
Examples 1-3, Table 2.1; Section 3, Examples 4-5, Table 3.1).

The paper's matrix and right-hand sides are random with unknown seeds, so the
printed counts (tests/golden/paper_tables.json) cannot be matched exactly
("parity unpinned" for the counts themselves).  What the paper's argument
fixes, and what a dropped term or wrong index in the seed recurrences would
break, is checked instead:
  * the unseeded CG count lies in a band around the paper's 617;
  * with reorthogonalization every 50 steps the second system's count falls
    monotonically as the first is run further past convergence, to well below
    a third of the unseeded count (Table 3.1, last column);
  * without reorthogonalization it does not keep falling (Table 3.1, middle);
  * total mvps: single seeding < multiple seeding < no seeding (Table 2.1);
  * multiple seeding helps the second system and then loses ground on the third
    (Example 1).
The run lengths of Table 3.1 are scaled by this matrix's own unseeded count
(the paper's 500..1500 over its 617).
"""
import json
import os

import numpy as np
import pytest

from oracle import operators as ops
from oracle.cg import cg
from oracle.seed import seed_lanczos
from oracle.seeded import multiple_seed_solve, related_rhs_solve, seeded_solve
from paper_0810_0330_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.fixture(scope="module")
def example():
    n = GOLDEN["example_1"]["n"]
    d = synth.diag_example(n, synth.rng(100, 0))
    B = synth.real_gaussian(n, GOLDEN["example_1"]["nrhs"], synth.rng(100, 1))
    return ops.DiagOp(d), B


def test_unseeded_count_band(example):
    op, B = example
    its = [cg(op, B[:, j], tol=GOLDEN["example_1"]["tol"])[1] for j in range(2)]
    ref = GOLDEN["example_1"]["rhs1_iterations"]
    for it in its:
        assert 0.55 * ref <= it <= 1.25 * ref


def _table_3_1(op, B, freq):
    t = GOLDEN["table_3_1"]
    k1 = cg(op, B[:, 0], tol=1e-8)[1]
    ms = [int(round(m * k1 / t["unseeded"])) for m in t["rhs1_mvps"]]
    rec = {}

    def cb(i, X):
        if i in ms:
            rec[i] = X[:, 1].copy()

    seed_lanczos(op, B[:, :2], m=max(ms), freq=freq, callback=cb)
    return [cg(op, B[:, 1], rec[m], tol=1e-8)[1] for m in ms], cg(op, B[:, 1], tol=1e-8)[1]


def test_table_3_1_with_reorthogonalization(example):
    op, B = example
    counts, unseeded = _table_3_1(op, B, GOLDEN["table_3_1"]["freq"])
    # beyond convergence of the first system, more seed steps never hurt
    assert all(b <= a for a, b in zip(counts[1:], counts[2:]))
    assert counts[-1] < counts[1]
    # at the paper's 1200 (index 5) the count is below 0.3x unseeded (paper: 64/617)
    assert counts[5] < 0.3 * unseeded


def test_table_3_1_without_reorthogonalization(example):
    op, B = example
    counts, unseeded = _table_3_1(op, B, 0)
    with_r, _ = _table_3_1(op, B, GOLDEN["table_3_1"]["freq"])
    # roundoff undoes the seeding: the count rises again past its minimum
    assert max(counts[2:]) > min(counts[:3]) + 50
    # and reorthogonalization is much better at the longest run
    assert counts[-1] > 2 * with_r[-1]


def test_table_2_1_ordering(example):
    op, B = example
    none = sum(cg(op, B[:, j], tol=1e-8)[1] for j in range(B.shape[1]))
    _, mult = multiple_seed_solve(op, B, 1e-8)
    k1 = cg(op, B[:, 0], tol=1e-8)[1]
    single = seeded_solve(op, B, k1, 0, 1e-8)["iters"]
    t = GOLDEN["table_2_1"]["mvps"]
    assert t["single"] < t["multiple"] < t["none"]
    assert sum(single) < sum(mult) < none
    # Example 1: the second system benefits, the third is pushed back up
    assert mult[1] < 0.85 * mult[0]
    assert mult[2] > mult[1]


def test_related_rhs_example_3(example):
    op, _ = example
    n = op.n
    gen = synth.rng(100, 3)
    u = synth.real_gaussian(n, 8, gen)
    B = np.zeros((n, 8))
    B[:, 0] = u[:, 0]
    for j in range(1, 8):
        B[:, j] = B[:, j - 1] + 0.2 ** j * u[:, j]
    k1 = cg(op, B[:, 0], tol=1e-8)[1]
    X, mv, before = related_rhs_solve(op, B, k1, 0, 1e-8)
    # the residual carried by step 3 stays the true residual of the carried guess
    # (up to the converged residual of the system projected over)
    for j in range(1, 8):
        xb, rb = before[j]
        assert np.linalg.norm(rb - (B[:, j] - op(xb))) <= 1e-7 * np.linalg.norm(B[:, j])
    rel = [np.linalg.norm(B[:, j] - op(X[:, j])) / np.linalg.norm(B[:, j]) for j in range(8)]
    assert max(rel) <= 1e-8
    # later systems start from increasingly small residuals (Example 3), and
    # projecting over the CG corrections beats single seeding alone
    assert mv[-1] < mv[1] < k1
    plain = seeded_solve(op, B, k1, 0, 1e-8)["iters"]
    assert mv[-1] < 0.5 * plain[-1]
