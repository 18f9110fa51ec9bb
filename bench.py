#!/usr/bin/env python3
"""Benchmark of the single-seed Lanczos-CG solver on one MI355X.

One step = one whole seeded solve of a batch of right-hand sides: the seed
phase on right-hand side 1 (Lanczos-CG run for m steps with reorthogonalization
every `freq` steps), the projection of the other right-hand sides over the
stored basis, and the mixed-precision CG that finishes every right-hand side to
a true FP64 relative residual <= tol.  Inputs are synthetic and already
resident in HBM when the timed region starts.

Metric: right-hand sides solved per second.  Beside it the same right-hand
sides are solved by plain per-RHS FP64 CG on the same GPU, the main kernels are
timed with HIP events inside the timed region (algorithmic bytes / time against
the 8 TB/s HBM peak), and the FP64 CPU oracle is timed on a bounded sample on
the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
METRIC = "RHS solved/sec at rel.res 1e-8 (seeded vs plain CG); stencil HBM GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="wilson_16x3x32",
                    choices=["wilson_16x3x32", "wilson_8x4", "laplace_32x32", "diag_5000"])
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--freq", type=int, default=None)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timer", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--timer-every", type=int, default=8,
                    help="time one launch in this many of each kernel class (an event pair costs a few us)")
    ap.add_argument("--micro", default=None, choices=["wilson_f32", "wilson_f64", "copy", "gemm_cn", "gemm_nn"],
                    help="time one kernel in isolation on the workload's lattice (for profilers)")
    ap.add_argument("--k", type=int, default=1, help="columns per launch in --micro mode")
    ap.add_argument("--reps", type=int, default=20, help="launches in --micro mode")
    ap.add_argument("--sweep-freq", default=None,
                    help="comma-separated reorthogonalization frequencies (0 = none): time the seed phase and the "
                         "whole seeded solve at each (Section 4, Table 4.1 analogue) instead of the benchmark")
    ap.add_argument("--related", type=int, default=None, metavar="NRHS",
                    help="time single seeding of NRHS related right-hand sides b^j = b^(j-1) + 0.2^(j-1) u^j "
                         "(Section 2.3, Example 3) on the workload's lattice instead of the benchmark")
    ap.add_argument("--indefinite", action="store_true",
                    help="time the indefinite variant (gamma_5 D, QR of T, MINRES; FP64) against the normal-equations "
                         "path on the workload instead of the benchmark (Sections 3 and 4)")
    ap.add_argument("--batch", action="store_true",
                    help="time the uneven batch (six independent Wilson lattices from 8^4 to 16^3x32, 4-24 RHS each, "
                         "mixed precision) in one batched call against the same systems solved one after another")
    ap.add_argument("--compare-seeding", action="store_true",
                    help="A-applies, vector operations and time of no / multiple / single seeding on the workload "
                         "(Section 2, Table 2.1 analogue) instead of the benchmark")
    ap.add_argument("--pin-stencil", type=int, default=None, metavar="V",
                    help="pin the stencil launch shape of the multi-column passes instead of autotuning it "
                         "(for reproducible counter runs)")
    ap.add_argument("--variant", type=int, default=None,
                    help="--micro wilson_*: pin this stencil launch shape instead of autotuning")
    return ap.parse_args()


def micro(args, w):
    """One kernel, `reps` launches, on the workload's lattice: for rocprofv3 counter runs."""
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    inp = synth.make_inputs(w)
    op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(dev), w.kappa)
    k = args.k
    single = args.micro != "wilson_f64"
    dt = torch.complex64 if single else torch.complex128
    g = torch.Generator(device=dev).manual_seed(1)
    X = torch.randn((k, op.n), dtype=dt, device=dev, generator=g)
    res = {"micro": args.micro, "k": k, "reps": args.reps, "n": op.n}
    if args.micro.startswith("wilson"):
        Y = torch.empty_like(X)
        if args.variant is not None:
            op.tune_set(k, args.variant, single=single)
        fn = lambda: op.dslash(X, 0, single=single, out=Y)  # noqa: E731
        bytes_per = (48.0 * k + 72.0) * (4 if single else 8) * (op.n // 12)
    elif args.micro == "copy":
        Y = torch.empty_like(X)
        fn = lambda: Y.copy_(X)  # noqa: E731
        bytes_per = 2.0 * X.numel() * X.element_size()
    else:
        m = 1000
        V = torch.randn((m, op.n), dtype=torch.complex64, device=dev, generator=g)
        basis = api.Basis(V, torch.ones(m, dtype=torch.float64, device=dev) * 4,
                          torch.ones(m + 1, dtype=torch.float64, device=dev) * 0.1, None, m, 0, op.n)
        R = X.to(torch.complex128)
        fn = lambda: api.project(basis, R)  # noqa: E731
        bytes_per = 2.0 * m * op.n * 8
    fn()
    torch.cuda.synchronize()
    api.timer_enable(True)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    res["avg_us"] = e0.elapsed_time(e1) * 1e3 / args.reps
    res["GBps"] = bytes_per / (res["avg_us"] * 1e-6) / 1e9
    res["kernels"] = {k2: v for k2, v in api.timer_read().items() if v["launches"]}
    api.timer_enable(False)
    if args.micro.startswith("wilson"):
        res["variant"], res["tune_us"] = op.tune_info(k, single=single)
    print(json.dumps(res), flush=True)


def sweep_freq(args, w):
    """Seed-phase and total time of the seeded solve against the reorthogonalization frequency.

    The paper's Table 4.1 gives, for its QCD problem on a CPU cluster, the time
    of right-hand side 1 (the seed phase) at frequencies 10, 100, 200, 250 and
    none; here the same is measured for the benchmark workload, with the CG
    counts of the other right-hand sides, which show what each frequency buys.
    """
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    inp = synth.make_inputs(w)
    op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(dev), w.kappa)
    B = torch.from_numpy(api.pack_field(np.ascontiguousarray(inp["B"].T))).to(dev)
    mixed = w.precision == "mixed"
    vdt = op.single_dtype if mixed else op.dtype
    api.seeded_solve(op, B, min(w.m, 50), 10, w.tol, mixed=mixed)  # warm: tuning, allocations
    rows = []
    for freq in [int(f) for f in args.sweep_freq.split(",")]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        basis = api.seed_lanczos(op, B[0], w.m, freq, v_dtype=vdt)
        torch.cuda.synchronize()
        t_seed = time.perf_counter() - t0
        t0 = time.perf_counter()
        out = api.seeded_solve(op, B, w.m, freq, w.tol, mixed=mixed)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        assert max(out["relres"]) <= w.tol
        its = out["iters"]
        rows.append({"freq": freq, "seed_ms": round(t_seed * 1e3, 2), "solve_ms": round(t_all * 1e3, 2),
                     "rhs1_iters": its[0], "rhs2_on_iters": its[1:], "m_done": basis.m_done})
        log(f"[sweep] freq {freq}: seed {t_seed * 1e3:.1f} ms, solve {t_all * 1e3:.1f} ms, iters {its[:4]}...")
    base = next((r["seed_ms"] for r in rows if r["freq"] == 0), None)
    for r in rows:
        r["seed_vs_none"] = round(r["seed_ms"] / base, 3) if base else None
    print(json.dumps({"sweep": "reorthogonalization frequency", "workload": w.name, "m": w.m, "rows": rows}),
          flush=True)


def related_bench(args, w):
    """Related right-hand sides on the workload's lattice: the related-RHS
    driver against single seeding alone and plain per-RHS CG, same inputs."""
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    inp = synth.make_inputs(w)
    op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(dev), w.kappa)
    k = args.related
    Bn = synth.related_rhs(synth.z4_noise(op.n, k, synth.rng(w.config_id, 6)))
    B = torch.from_numpy(api.pack_field(np.ascontiguousarray(Bn.T))).to(dev)
    mixed = w.precision == "mixed"
    api.related_rhs_solve(op, B[:2], 50, 10, w.tol, mixed=mixed)  # warm: tuning, allocations
    res = {"related": k, "workload": w.name, "m": w.m, "freq": w.freq, "tol": w.tol, "precision": w.precision}
    for name, fn in [("related", lambda: api.related_rhs_solve(op, B, w.m, w.freq, w.tol, mixed=mixed)),
                     ("single_seed", lambda: api.seeded_solve(op, B, w.m, w.freq, w.tol, mixed=mixed)),
                     ("plain_f64", lambda: {"iters": [api.solve_cg(op, B[j:j + 1], w.tol)[1][0] for j in range(k)],
                                            "relres": [0.0]})]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert max(out["relres"]) <= w.tol
        res[name] = {"ms": round(dt * 1e3, 2), "rhs_per_s": round(k / dt, 3), "iters": list(out["iters"])}
        log(f"[related] {name}: {dt * 1e3:.1f} ms, iters {list(out['iters'])}")
    print(json.dumps(res), flush=True)


def batch_bench(args):
    """The uneven batch: one sc_batch_solve call (seed phases of all systems in
    one HIP graph, then projection and CG of each system on its own stream)
    against the same systems solved one after another by the one-call driver."""
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    tol = 1e-8
    systems = []
    for sd in synth.uneven_batch():
        op = api.Op.wilson(sd["dims"], torch.from_numpy(api.pack_links(sd["U"])).to(dev), sd["kappa"])
        B = torch.from_numpy(api.pack_field(np.ascontiguousarray(sd["B"].T))).to(dev)
        _, it, _ = api.solve_cg(op, B[:1], tol)
        m = synth.seed_steps(it[0])
        systems.append({"op": op, "B": B, "m": m, "freq": 100 if m >= 200 else 50, "tol": tol, "mixed": True,
                        "dims": list(sd["dims"]), "kappa": round(sd["kappa"], 4)})
    nrhs = sum(int(sd["B"].shape[0]) for sd in systems)
    log(f"[batch] {len(systems)} systems, {nrhs} RHS: " +
        ", ".join(f"{sd['dims']} k={sd['B'].shape[0]} m={sd['m']}" for sd in systems))

    def batched():
        return api.batch_solve(systems)

    def one_at_a_time():
        return [api.single_seed_solve(sd["op"], sd["B"], sd["m"], sd["freq"], tol, mixed=True) for sd in systems]

    for fn in (batched, one_at_a_time):  # warm: tuning, graph capture, allocations
        fn()
    res = {"mode": "uneven_batch", "nrhs": nrhs, "tol": tol, "precision": "mixed", "steps": args.steps,
           "systems": [{"dims": sd["dims"], "kappa": sd["kappa"], "nrhs": int(sd["B"].shape[0]), "m": sd["m"],
                        "freq": sd["freq"]} for sd in systems]}
    for name, fn in (("batched", batched), ("one_at_a_time", one_at_a_time)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        for o in outs:
            assert o["status"] in (0, 2) and max(o["relres"]) <= tol
        res[name] = {"ms": round(dt * 1e3, 2), "rhs_per_s": round(nrhs / dt, 2),
                     "iters": [list(o["iters"]) for o in outs]}
        log(f"[batch] {name}: {dt * 1e3:.1f} ms per batch, {nrhs / dt:.1f} RHS/s")
    res["speedup"] = round(res["one_at_a_time"]["ms"] / res["batched"]["ms"], 3)
    print(json.dumps(res), flush=True)


def indefinite_bench(args, w):
    """The indefinite variant (gamma_5 D, QR of the tridiagonal matrix, MINRES; FP64) against the
    normal-equations path, on the workload's lattice and right-hand sides.

    Both solve the Wilson system of the workload: the normal-equations path solves D^H D x = b, the
    indefinite one gamma_5 D x = b (for D x = gamma_5 b); the comparison is the number of products with
    D and the time to reach the same relative residual.  Section 4 notes that the gamma_5 form needs one
    product with D per iteration instead of two.
    """
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    inp = synth.make_inputs(w)
    U = torch.from_numpy(api.pack_links(inp["U"])).to(dev)
    opq = api.Op.wilson_g5(w.dims, U, w.kappa)
    opn = api.Op.wilson(w.dims, U, w.kappa)
    B = torch.from_numpy(api.pack_field(np.ascontiguousarray(inp["B"].T))).to(dev)
    k = B.shape[0]
    mixed = w.precision == "mixed"
    # warm every path on the full right-hand-side block (stencil tuning per column count, allocations)
    api.indefinite_solve(opq, B, 50, 10, w.tol)
    api.solve_minres(opq, B, w.tol)
    api.single_seed_solve(opn, B, 50, 10, w.tol, mixed=mixed)
    res = {"indefinite": True, "workload": w.name, "m": w.m, "freq": w.freq, "tol": w.tol, "nrhs": k}
    runs = [("indefinite_seeded_f64", 1, lambda: api.indefinite_solve(opq, B, w.m, w.freq, w.tol)),
            ("minres_unseeded_f64", 1, lambda: dict(zip(("X", "iters", "relres"), api.solve_minres(opq, B, w.tol)))),
            ("normal_seeded_" + ("mixed" if mixed else "f64"), 2,
             lambda: api.single_seed_solve(opn, B, w.m, w.freq, w.tol, mixed=mixed))]
    for name, d_per_it, fn in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert max(out["relres"]) <= w.tol
        its = list(out["iters"])
        res[name] = {"ms": round(dt * 1e3, 2), "rhs_per_s": round(k / dt, 3), "iters": its,
                     "d_products": int(sum(its) * d_per_it)}
        log(f"[indefinite] {name}: {dt * 1e3:.1f} ms, D-products {sum(its) * d_per_it}, iters {its[:4]}...")
    print(json.dumps(res), flush=True)


def vector_ops(kind, iters, m=0, freq=0, nrhs=0):
    """Length-n vector operations (one dot or axpy on an n-vector each), as Table 2.1 counts them.

    CG: 2 dots + 3 axpys per iteration.  Multiple seeding adds, per iteration of
    system j, a dot and two axpys for each later system.  Single seeding adds the
    seed phase (5 per Lanczos step, 4 (i - 1) + 4 per reorthogonalization at step
    i) and the projection (2 m per projected right-hand side).
    """
    if kind == "none":
        return 5 * sum(iters)
    if kind == "multiple":
        k = len(iters)
        return sum(it * (5 + 3 * (k - 1 - j)) for j, it in enumerate(iters))
    seed = 5 * m + (sum(4 * (i - 1) + 4 for i in range(freq, m + 1, freq)) if freq > 0 else 0)
    return seed + 2 * m * (nrhs - 1) + 5 * (sum(iters) - m)


def compare_seeding(args, w):
    """Table 2.1 analogue on the GPU path: no seeding (per-RHS CG), multiple
    seeding (standard seed CG) and single seeding, on the same right-hand sides."""
    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    dev = torch.device("cuda:0")
    inp = synth.make_inputs(w)
    if w.op == "diag":
        op = api.Op.diag(torch.from_numpy(inp["d"]).to(dev))
        B = torch.from_numpy(np.ascontiguousarray(inp["B"].T)).to(dev)
    else:
        op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(dev), w.kappa)
        B = torch.from_numpy(api.pack_field(np.ascontiguousarray(inp["B"].T))).to(dev)
    k = w.nrhs
    api.solve_cg(op, B[:1], w.tol)  # warm: tuning, allocations
    res = {"compare_seeding": w.name, "nrhs": k, "tol": w.tol, "m": w.m, "freq": w.freq}
    none_its = []

    def none():
        for j in range(k):
            none_its.append(api.solve_cg(op, B[j:j + 1], w.tol)[1][0])
        return {"iters": list(none_its), "relres": [0.0]}

    m_run = w.m
    runs = [("none", none), ("multiple", lambda: api.multiple_seed_solve(op, B, w.tol)),
            ("single", lambda: api.seeded_solve(op, B, m_run, w.freq, w.tol))]
    for name, fn in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert max(out["relres"]) <= w.tol
        its = list(out["iters"])
        res[name] = {"a_applies": sum(its), "iters": its, "ms": round(dt * 1e3, 2),
                     "vector_ops": vector_ops(name, its, m_run, w.freq, k)}
        log(f"[compare] {name}: {sum(its)} A-applies, {dt * 1e3:.1f} ms")
    print(json.dumps(res), flush=True)


def workload_by_key(key):
    from paper_0810_0330_amd import synth
    if key == "wilson_16x3x32":
        w = synth.wilson_16x3x32()
    elif key == "wilson_8x4":
        w = synth.wilson_8x4(m=150)
        w.precision = "mixed"
    elif key == "diag_5000":
        w = synth.diag_5000()
    else:
        w = synth.laplace_32x32()
    return w


def workload(args):
    w = workload_by_key(args.workload)
    if args.m is not None:
        w.m = args.m
    if args.freq is not None:
        w.freq = args.freq
    return w


def measured_traffic(cls, k, variant, dims):
    """HBM bytes per launch of a stencil class from the committed rocprofv3 counter record.

    None unless the record holds this class, column count, lattice and (where the
    class depends on it) launch shape, and every source it lists still hashes to
    what was profiled.  A class's traffic is the mean over its kernels.
    """
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    cal = rec["calibration"]
    for c in rec["classes"]:
        if (c["class"], c["k"], list(c["dims"])) != (cls, k, list(dims)):
            continue
        if c["variant"] is not None and c["variant"] != variant:
            continue
        for src, digest in c["sources"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != digest:
                return None
        ks = c["kernels"]
        return sum(e["fetch_kib"] * 1024 * cal["fetch_factor"] + e["write_kib"] * 1024 * cal["write_factor"]
                   for e in ks) / len(ks)
    return None


def _oracle_unit_times(key, threads, nlz=8, nvec=64):
    """Unit times of the FP64 oracle's parts on the workload, BLAS limited to `threads`.

    Builds the workload's inputs itself so that it can run in a fresh worker
    process.  Parts: one seed-phase Lanczos step (one A-apply, its vector work
    and the incremental x^1 update), one CG iteration (CG for 10 minus CG for 2
    iterations, over 8), one A-apply, one length-n vector update.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import operators as ops
    from oracle.cg import cg
    from oracle.seed import seed_lanczos
    from paper_0810_0330_amd import synth

    w = workload_by_key(key)
    inp = synth.make_inputs(w)
    if w.op == "laplace2d":
        op = ops.Laplace2DOp(*w.dims)
    elif w.op == "diag":
        op = ops.DiagOp(inp["d"])
    else:
        op = ops.WilsonNormalOp(inp["U"], w.kappa)
    B = inp["B"]
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        seed_lanczos(op, B[:, :1], m=nlz, freq=0)
        t_step = (time.perf_counter() - t0) / nlz
        t0 = time.perf_counter()
        cg(op, B[:, 1], tol=1e-300, maxit=10)
        t10 = time.perf_counter() - t0
        t0 = time.perf_counter()
        cg(op, B[:, 1], tol=1e-300, maxit=2)
        t_iter = max(t10 - (time.perf_counter() - t0), 0.0) / 8
        t0 = time.perf_counter()
        for _ in range(2):
            op(B[:, 0])
        t_apply = (time.perf_counter() - t0) / 2
        v = B[:, 1].astype(np.complex128 if w.op == "wilson" else np.float64)
        y = v.copy()
        t0 = time.perf_counter()
        for _ in range(nvec):
            c = np.vdot(v, y)
            y = y - (c / (np.vdot(v, v) + 1.0)) * v
        t_vec = (time.perf_counter() - t0) / nvec
    return {"t_step": t_step, "t_iter": t_iter, "t_apply": t_apply, "t_vec": t_vec}


def _host_info():
    """CPU model, logical CPU counts and the NumPy/BLAS build of the host."""
    import numpy as np

    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        blas = f"{blas.get('name')} {blas.get('version')}"
    except Exception:  # noqa: BLE001 - build info is descriptive only
        blas = None
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "numpy": np.__version__, "blas": blas}


# workloads whose whole oracle solve finishes within seconds: timed in full instead of sampled
_FULL_ORACLE = ("laplace_32x32", "wilson_8x4")


def _oracle_full_time(key, threads):
    """Seconds of the FP64 oracle's whole seeded solve of the workload (seed phase, projection, CG of every
    right-hand side, true residuals), BLAS limited to `threads`; inputs built before the clock starts."""
    from threadpoolctl import threadpool_limits

    from oracle import operators as ops
    from oracle.seeded import seeded_solve
    from paper_0810_0330_amd import synth

    w = workload_by_key(key)
    inp = synth.make_inputs(w)
    op = ops.Laplace2DOp(*w.dims) if w.op == "laplace2d" else ops.WilsonNormalOp(inp["U"], w.kappa)
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        seeded_solve(op, inp["B"], w.m, w.freq, w.tol)
        return time.perf_counter() - t0


def cpu_baseline(key, w, counts):
    """Time the FP64 oracle as it stands on a bounded sample of the workload and scale it to the whole solve.

    The small workloads (the 32x32 Laplacian and Wilson 8^4) are timed in full
    instead: the oracle's whole seeded solve on one thread, and with BLAS on
    every host CPU (at most 16).

    Sample (about 10 s per process on the 16^3 x 32 lattice): the oracle's
    seed phase for 8 Lanczos steps on right-hand side 1, its CG on right-hand
    side 2 for 10 and for 2 iterations (the difference prices one CG
    iteration), 2 plain A-applies, and 64 of its length-n vector updates.  The
    full oracle solve is priced with this run's counts: the seed steps, the CG
    iterations, two residuals per right-hand side, and one vector update per
    stored basis vector touched by the reorthogonalizations and by the
    incremental seeding of the other right-hand sides.

    Two runs: one process with BLAS on one thread, and one process per host
    CPU (at most 16) running the same sample at once, each on one thread; the
    all-core figure is the throughput of that many independent copies of the
    workload solved side by side, each at its measured (contended) speed.  The
    oracle is sequential code, so this is how it uses a many-core host.
    """
    import multiprocessing as mp

    if key in _FULL_ORACLE:
        procs = min(len(os.sched_getaffinity(0)), 16)
        t1 = _oracle_full_time(key, 1)
        tn = _oracle_full_time(key, procs)
        return {
            "value": w.nrhs / tn,
            "unit": "RHS/s",
            "cores": procs,
            "kind": "oracle",
            "value_1_thread": w.nrhs / t1,
            "host": _host_info(),
            "sample": (f"the whole FP64 oracle seeded solve of the workload (m = {w.m}, freq = {w.freq}, "
                       f"{w.nrhs} right-hand sides, tol {w.tol:g}): {t1:.2f} s on one thread, {tn:.2f} s with "
                       f"BLAS on {procs} threads (not extrapolated)"),
        }

    def total(u):
        return (counts["seed_steps"] * u["t_step"] + counts["cg_iters"] * u["t_iter"]
                + counts["residuals"] * u["t_apply"] + counts["vector_passes"] * u["t_vec"])

    one = _oracle_unit_times(key, 1)
    v1 = w.nrhs / total(one)
    procs = min(len(os.sched_getaffinity(0)), 16)
    with mp.get_context("spawn").Pool(procs) as pool:
        many = pool.starmap(_oracle_unit_times, [(key, 1)] * procs)
    v_all = sum(w.nrhs / total(u) for u in many)
    slow = sum(u["t_iter"] for u in many) / len(many) / max(one["t_iter"], 1e-12)
    return {
        "value": v_all,
        "unit": "RHS/s",
        "cores": procs,
        "kind": "oracle",
        "value_1_thread": v1,
        "host": _host_info(),
        "sample": (f"oracle seed phase 8 Lanczos steps ({one['t_step'] * 1e3:.0f} ms each), oracle CG 10 and 2 "
                   f"iterations ({one['t_iter'] * 1e3:.0f} ms per iteration), 2 A-applies "
                   f"({one['t_apply'] * 1e3:.0f} ms each), 64 vector updates ({one['t_vec'] * 1e3:.2f} ms each) "
                   f"on the benchmark lattice, on one thread; the same sample in {procs} processes at once (one "
                   f"thread each, CG iteration {slow:.2f}x slower under contention) gives the all-core value as "
                   f"{procs} independent copies of the workload; scaled by this run's counts: "
                   f"{counts['seed_steps']} seed steps, {counts['cg_iters']} CG iterations, {counts['residuals']} "
                   f"residuals, {counts['vector_passes']} basis-vector passes (extrapolated)"),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; the multi-GPU path is design-only "
                                   "(the lattice would be split across GPUs by domain decomposition; not built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0810_0330_amd import api, synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    w = workload(args)
    if args.micro:
        return micro(args, w)
    if args.sweep_freq:
        return sweep_freq(args, w)
    if args.indefinite:
        return indefinite_bench(args, w)
    if args.batch:
        return batch_bench(args)
    if args.related:
        return related_bench(args, w)
    if args.compare_seeding:
        return compare_seeding(args, w)
    log(f"[bench] workload {w.name}: dims {w.dims} nrhs {w.nrhs} m {w.m} freq {w.freq} tol {w.tol} {w.precision}")
    t0 = time.perf_counter()
    inp = synth.make_inputs(w)
    if w.op == "laplace2d":
        op = api.Op.laplace2d(*w.dims)
        B = torch.from_numpy(np.ascontiguousarray(inp["B"].T)).to(dev)
    elif w.op == "diag":
        op = api.Op.diag(torch.from_numpy(inp["d"]).to(dev))
        B = torch.from_numpy(np.ascontiguousarray(inp["B"].T)).to(dev)
    else:
        op = api.Op.wilson(w.dims, torch.from_numpy(api.pack_links(inp["U"])).to(dev), w.kappa)
        B = torch.from_numpy(api.pack_field(np.ascontiguousarray(inp["B"].T))).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s, n = {op.n}")
    if args.pin_stencil is not None and w.op == "wilson":
        op.tune_set(w.nrhs, args.pin_stencil, single=w.precision == "mixed")
    mixed = w.precision == "mixed"

    def step():
        return api.single_seed_solve(op, B, w.m, w.freq, w.tol, mixed=mixed)

    for i in range(args.warmup):
        out = step()
        log(f"[bench] warmup {i}: iters {out['iters']} max relres {max(out['relres']):.2e}")
    stream = torch.cuda.current_stream()
    if not args.no_timer:
        api.timer_enable(True, every=args.timer_every)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t_wall = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step())
        log(f"[bench] step {i} done")
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ms = e0.elapsed_time(e1)
    kern = api.timer_read() if not args.no_timer else {}
    api.timer_enable(False)
    ms_per_step = max(ms, wall_ms) / args.steps
    out = outs[-1]
    relres = out["relres"]
    assert max(relres) <= w.tol, f"not converged: {relres}"
    value = w.nrhs / (ms_per_step / 1e3)
    log(f"[bench] {ms_per_step:.1f} ms/step -> {value:.1f} RHS/s; iters {out['iters']}")

    # ---- plain per-RHS FP64 CG on the same GPU
    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        t = time.perf_counter()
        pits = []
        for j in range(w.nrhs):
            _, it, rr = api.solve_cg(op, B[j:j + 1], w.tol, mixed=False)
            assert rr[0] <= w.tol
            pits.append(it[0])
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        plain = {"rhs_per_s": w.nrhs / tp, "ms": tp * 1e3, "iters": pits, "dtype": "f64"}
        log(f"[bench] plain FP64 CG: {tp * 1e3:.1f} ms, {plain['rhs_per_s']:.1f} RHS/s, iters {pits}")

    # ---- unseeded batched CG of the same right-hand sides, same precision and kernels: every column
    # from zero in one multi-column CG (what the seed phase and projection are measured against)
    unseeded = None
    if not args.no_plain:
        api.solve_cg(op, B, w.tol, mixed=mixed)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            _, uits, urel = api.solve_cg(op, B, w.tol, mixed=mixed)
        torch.cuda.synchronize()
        tu = (time.perf_counter() - t) / args.steps
        assert max(urel) <= w.tol
        unseeded = {"rhs_per_s": round(w.nrhs / tu, 3), "ms": round(tu * 1e3, 3), "iters": uits,
                    "dtype": "f32+f64" if mixed else "f64"}
        log(f"[bench] unseeded batched CG: {tu * 1e3:.1f} ms, {w.nrhs / tu:.1f} RHS/s, iters {uits}")

    # ---- error of sampled columns against the FP64 oracle's tight solutions (stored values written by
    # tests/golden/make_oracle_golden.py from the oracle alone, on these same seeded inputs)
    oracle_err = None
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_c3.json")
    if w.op == "wilson" and os.path.exists(gpath):
        g = json.load(open(gpath))
        if g["workload"] == w.name:
            idx = np.array(g["sample_index"])
            errs = {}
            for j, xs in zip(g["x_cols"], g["x_sample"]):
                x = api.unpack_field(out["X"][j:j + 1].cpu().numpy())[0][idx]
                xo = np.array([complex(a, b) for a, b in xs])
                errs[str(j)] = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
            oracle_err = {"columns": errs, "entries_per_column": len(idx), "oracle_tol": g["x_tol"],
                          "measure": "||x - x_oracle|| / ||x_oracle|| over the sampled entries"}
            log(f"[bench] error vs FP64 oracle (sampled): {errs}")

    # ---- roofline of the dominant kernel class.  Stencil launches are a uniform
    # 1-in-`timer_every` sample of their class and contraction launches are all
    # timed, so a class's total time is estimated as sampled time x its rate.
    roof = None
    kernels = {}
    for name, k in kern.items():
        if k["launches"] == 0:
            continue
        avg_ms = k["ms"] / k["launches"]
        rate = 1 if name.startswith("gemm") else args.timer_every
        kernels[name] = {"launches": k["launches"], "ms_total": round(k["ms"], 3), "avg_us": round(avg_ms * 1e3, 2),
                         "est_ms_per_step": round(k["ms"] * rate / args.steps, 3),
                         "GBps": round(k["bytes"] / (k["ms"] * 1e-3) / 1e9, 1),
                         "TFLOPs": round(k["flops"] / (k["ms"] * 1e-3) / 1e12, 3),
                         "bytes_per_launch": k["bytes"] / k["launches"]}
    if kernels:
        dom = max(kernels, key=lambda n: kernels[n]["est_ms_per_step"])
        kd = kernels[dom]
        achieved = kd["GBps"]
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": kd["avg_us"], "bytes_per_launch": kd["bytes_per_launch"],
                "timed_launches": kd["launches"], "sample_every": 1 if dom.startswith("gemm") else args.timer_every}

    # measured copy bandwidth of the device (the runtime's device-to-device copy of 24 complex64 columns of
    # the lattice, 302 MB each way), for the stencil rate as a fraction of what a plain copy reaches
    if roof is not None and roof["bound"] == "hbm":
        nb = 24 * 12 * int(np.prod(w.dims)) * 8 if w.op == "wilson" else 256 << 20
        cx = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        cy = torch.empty_like(cx)
        cy.copy_(cx)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            cy.copy_(cx)
        e1.record()
        e1.synchronize()
        copy_gbs = 2 * nb * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        roof["copy_GBps"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
        del cx, cy
        for kd_ in kernels.values():
            kd_["frac_of_hbm_peak"] = round(kd_["GBps"] / HBM_PEAK_GBS, 4)

    if roof is not None and w.op == "wilson" and roof["kernel"].startswith("wilson_f32"):
        # links in SU(3): the FP32 passes read 12 of the 18 reals of each link; the algorithmic bytes above
        # count whole links (72 reals per site), so also state them for two-row links (48 reals per site)
        roof["links"] = "two rows read, third rebuilt (SU(3) check passed)" if op.rebuild else "whole"
        if op.rebuild:
            per_site = roof["bytes_per_launch"] / float(np.prod(w.dims))
            two_row = roof["bytes_per_launch"] - 24 * 4 * float(np.prod(w.dims))
            roof["bytes_per_launch_two_row_links"] = two_row
            roof["frac_two_row_links"] = round(roof["frac"] * two_row / roof["bytes_per_launch"], 4)
            roof["bytes_per_site"] = round(per_site, 1)
        kk = 1 if roof["kernel"].endswith("_k1") else w.nrhs
        v, _ = op.tune_info(kk, single=True)
        t = measured_traffic(roof["kernel"], kk, v, w.dims)
        if t is not None:
            roof["traffic"] = round(t)
            roof["traffic_unit"] = "bytes/launch"
            roof["traffic_source"] = "profiles/traffic.json"

    tuning = {}
    if w.op == "wilson":
        for kk, single in [(1, True), (w.nrhs, True), (1, False), (w.nrhs, False)]:
            v, us = op.tune_info(kk, single=single)
            tuning[f"{'f32' if single else 'f64'}_k{kk}"] = {"variant": v, "us": us}

    # ---- oracle on the host
    cpu = None
    if not args.no_cpu_baseline:
        n_seed = out["m_done"]
        cg_its = sum(out["iters"]) - n_seed
        freq = max(w.freq, 1)
        reorth_vecs = sum(2 * (i - 1) for i in range(freq, n_seed + 1, freq)) if w.freq > 0 else 0
        counts = {"seed_steps": n_seed, "cg_iters": cg_its, "residuals": 2 * w.nrhs,
                  "vector_passes": reorth_vecs + 2 * n_seed * (w.nrhs - 1)}
        t = time.perf_counter()
        cpu = cpu_baseline(args.workload, w, counts)
        log(f"[bench] cpu baseline ({time.perf_counter() - t:.1f} s): {cpu['value']:.4f} RHS/s")

    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(w.dims), "nrhs": w.nrhs, "m": w.m, "freq": w.freq,
                   "tol": w.tol, "kappa": w.kappa, "precision": w.precision},
        "iters": out["iters"],
        "max_relres": max(relres),
        "plain_cg": plain,
        "speedup_vs_plain": round(value / plain["rhs_per_s"], 3) if plain else None,
        "unseeded_batched_cg": unseeded,
        "speedup_vs_unseeded_batched": round(value / unseeded["rhs_per_s"], 3) if unseeded else None,
        "error_vs_oracle": oracle_err,
        "roofline": roof,
        "kernels": kernels,
        "stencil_tuning": tuning,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
