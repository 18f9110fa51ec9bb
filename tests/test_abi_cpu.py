"""CPU checks of the boundary: the library loads and exports every symbol the
header declares, and host-side argument validation rejects bad calls without
touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seedcg.h")
LIB = os.path.join(ROOT, "paper_0810_0330_amd", "libseedcg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0810_0330_amd import build
        build.build()
    l = ctypes.CDLL(LIB)
    l.sc_last_error.restype = ctypes.c_char_p
    return l


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "sc_seed_lanczos" in names and "sc_project" in names and "sc_solve_cg" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_0810_0330_amd import api
    assert set(declared_functions()) == set(api._PROTOS)


def test_op_argument_errors(lib):
    out = ctypes.c_void_p()
    assert lib.sc_op_laplace2d(0, 4, ctypes.byref(out)) == -1
    assert b"nx and ny" in lib.sc_last_error()
    assert lib.sc_op_laplace2d(4, 4, None) == -1
    dims = (ctypes.c_int * 4)(4, 4, 0, 4)
    assert lib.sc_op_wilson_normal(dims, ctypes.c_void_p(256), None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.sc_op_wilson_normal(dims, None, None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    assert lib.sc_op_wilson_normal(dims, ctypes.c_void_p(264), None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    assert b"aligned" in lib.sc_last_error()
    assert lib.sc_op_wilson_normal(dims, ctypes.c_void_p(256), None, ctypes.c_double(float("nan")), 1,
                                   ctypes.byref(out)) == -1
    # the SU(3) check of the links: a Wilson operator only (refused on the host)
    dev = ctypes.c_double()
    rb = ctypes.c_int()
    assert lib.sc_op_wilson_check_su3(None, None, ctypes.byref(dev), ctypes.byref(rb)) == -1
    assert lib.sc_op_laplace2d(4, 4, ctypes.byref(out)) == 0
    assert lib.sc_op_wilson_check_su3(out, None, ctypes.byref(dev), ctypes.byref(rb)) == -1
    assert b"Wilson" in lib.sc_last_error()
    assert lib.sc_op_destroy(out) == 0


def test_op_create_info_destroy_on_host(lib):
    # creating an op only records pointers: no device access, so it works without a GPU
    out = ctypes.c_void_p()
    assert lib.sc_op_laplace2d(32, 16, ctypes.byref(out)) == 0
    n = ctypes.c_int64()
    dt = ctypes.c_int()
    assert lib.sc_op_info(out, ctypes.byref(n), ctypes.byref(dt)) == 0
    assert n.value == 512 and dt.value == 0
    nb = ctypes.c_size_t()
    assert lib.sc_workspace_size(out, 3, 4, 0, 0, ctypes.byref(nb)) == 0 and nb.value > 4 * 3 * 512 * 8
    assert lib.sc_workspace_size(out, 1, 1, 50, 0, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.sc_workspace_size(out, 10, 1, 50, 0, ctypes.byref(nb)) == -1  # unknown call id
    # seed: m < 1 and a NULL m_done are argument errors, caught before any launch
    md = ctypes.c_int()
    p = ctypes.c_void_p(4096)
    assert lib.sc_seed_lanczos(out, p, p, 0, 1, p, ctypes.c_int64(512), 0, p, p, ctypes.byref(md), p,
                               ctypes.c_size_t(1 << 30), None) == -1
    assert lib.sc_seed_lanczos(out, p, p, 10, 1, p, ctypes.c_int64(511), 0, p, p, ctypes.byref(md), p,
                               ctypes.c_size_t(1 << 30), None) == -1
    assert b"ldv" in lib.sc_last_error()
    # too small a workspace is reported as such
    assert lib.sc_seed_lanczos(out, p, p, 10, 1, p, ctypes.c_int64(512), 0, p, p, ctypes.byref(md), p,
                               ctypes.c_size_t(16), None) == -5
    # CG: tol <= 0 and k < 1
    it = (ctypes.c_int * 1)()
    rr = (ctypes.c_double * 1)()
    assert lib.sc_solve_cg(out, 0, p, ctypes.c_int64(512), p, ctypes.c_int64(512), 1, ctypes.c_double(0.0), 10, it, rr,
                           p, ctypes.c_size_t(1 << 30), None) == -1
    assert lib.sc_solve_cg(out, 0, p, ctypes.c_int64(512), p, ctypes.c_int64(512), 0, ctypes.c_double(1e-8), 10, it,
                           rr, p, ctypes.c_size_t(1 << 30), None) == -1
    # projection: mismatched real/complex dtypes
    assert lib.sc_project(ctypes.c_int64(512), p, ctypes.c_int64(512), 1, 10, p, p, 0, p, ctypes.c_int64(512), 1, p,
                          ctypes.c_int64(512), p, ctypes.c_size_t(1 << 30), None) == -1
    assert lib.sc_op_destroy(out) == 0


def test_seeded_driver_argument_errors(lib):
    # sc_seeded_solve validates on the host before any device call
    out = ctypes.c_void_p()
    assert lib.sc_op_laplace2d(32, 16, ctypes.byref(out)) == 0
    nb = ctypes.c_size_t()
    assert lib.sc_workspace_size(out, 7, 3, 50, 0, ctypes.byref(nb)) == 0 and nb.value > 51 * 512 * 8
    p = ctypes.c_void_p(4096)
    it = (ctypes.c_int * 3)()
    rr = (ctypes.c_double * 3)()
    md = ctypes.c_int()

    def call(op=out, k=3, m=50, freq=10, tol=1e-8, maxit=100, ldb=512, work=1 << 30, mdp=ctypes.byref(md)):
        return lib.sc_seeded_solve(op, 0, p, ctypes.c_int64(ldb), p, ctypes.c_int64(512), k, m, freq,
                                   ctypes.c_double(tol), maxit, it, rr, mdp, p, ctypes.c_size_t(work), None)

    assert call(op=None) == -1
    assert call(k=0) == -1
    assert call(m=0) == -1
    assert call(freq=-1) == -1
    assert call(tol=0.0) == -1 and b"tol" in lib.sc_last_error()
    assert call(tol=float("inf")) == -1
    assert call(maxit=0) == -1
    assert call(ldb=511) == -1 and b"ldb" in lib.sc_last_error()
    assert call(mdp=None) == -1
    assert call(work=16) == -5
    assert lib.sc_op_destroy(out) == 0


def test_indefinite_and_minres_argument_errors(lib):
    # the gamma_5 D constructor validates like the normal-operator one; the
    # MINRES and indefinite-variant calls validate on the host before any
    # device call
    out = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 0, 4)
    assert lib.sc_op_wilson_g5(dims, ctypes.c_void_p(256), None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.sc_op_wilson_g5(dims, None, None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    assert lib.sc_op_wilson_g5(dims, ctypes.c_void_p(264), None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == -1
    assert b"aligned" in lib.sc_last_error()
    assert lib.sc_op_wilson_g5(dims, ctypes.c_void_p(256), None, ctypes.c_double(0.12), 1, ctypes.byref(out)) == 0
    n = ctypes.c_int64()
    dt = ctypes.c_int()
    assert lib.sc_op_info(out, ctypes.byref(n), ctypes.byref(dt)) == 0 and n.value == 4 ** 4 * 12
    nb = ctypes.c_size_t()
    assert lib.sc_workspace_size(out, 8, 3, 0, dt.value, ctypes.byref(nb)) == 0 and nb.value > 3 * n.value * 16
    assert lib.sc_workspace_size(out, 9, 3, 40, dt.value, ctypes.byref(nb)) == 0 and nb.value > 41 * n.value * 16
    # both run in the op's own (FP64) type only
    assert lib.sc_workspace_size(out, 8, 3, 0, dt.value - 1, ctypes.byref(nb)) == -1
    p = ctypes.c_void_p(4096)
    it = (ctypes.c_int * 3)()
    rr = (ctypes.c_double * 3)()
    md = ctypes.c_int()
    ld = n.value

    def minres(k=3, tol=1e-8, maxit=100, ldb=ld, work=1 << 30, itp=it):
        return lib.sc_solve_minres(out, p, ctypes.c_int64(ldb), p, ctypes.c_int64(ld), k, ctypes.c_double(tol), maxit,
                                   itp, rr, p, ctypes.c_size_t(work), None)

    assert minres(k=0) == -1
    assert minres(tol=0.0) == -1 and b"tol" in lib.sc_last_error()
    assert minres(tol=float("nan")) == -1
    assert minres(maxit=0) == -1
    assert minres(ldb=ld - 1) == -1 and b"ldb" in lib.sc_last_error()
    assert minres(itp=None) == -1
    assert minres(work=16) == -5

    def indef(k=3, m=40, freq=10, tol=1e-8, maxit=100, ldb=ld, work=1 << 30, mdp=ctypes.byref(md)):
        return lib.sc_indefinite_solve(out, p, ctypes.c_int64(ldb), p, ctypes.c_int64(ld), k, m, freq,
                                       ctypes.c_double(tol), maxit, it, rr, mdp, p, ctypes.c_size_t(work), None)

    assert indef(k=0) == -1
    assert indef(m=0) == -1
    assert indef(freq=-1) == -1
    assert indef(tol=-1.0) == -1
    assert indef(maxit=0) == -1
    assert indef(ldb=ld - 1) == -1
    assert indef(mdp=None) == -1
    assert indef(work=16) == -5
    assert lib.sc_op_destroy(out) == 0


def test_timer_host_side(lib):
    # enabling, reading with no recorded launches and the class check need no device
    ms, nl, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    assert lib.sc_timer_enable(8) == 0
    for cls in range(6):
        assert lib.sc_timer_read(cls, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(by), ctypes.byref(fl)) == 0
        assert nl.value == 0 and ms.value == 0.0
    assert lib.sc_timer_read(6, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(by), ctypes.byref(fl)) == -1
    assert lib.sc_timer_read(0, None, ctypes.byref(nl), ctypes.byref(by), ctypes.byref(fl)) == -1
    assert lib.sc_timer_enable(0) == 0


def test_variant_count_matches_header():
    from paper_0810_0330_amd import api
    m = re.search(r"#define\s+SC_WILSON_VARIANTS\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == api.WILSON_VARIANTS


def test_tune_set_refuses_tmarch_on_other_lattices(lib):
    # pinning is host-only; the t-march shapes need an xy-plane of 256 sites
    out = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.sc_op_wilson_normal(dims, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_double(0.12), 1,
                                   ctypes.byref(out)) == 0
    assert lib.sc_wilson_tune_set(out, 1, 3, 32) == -1
    assert b"256" in lib.sc_last_error()
    assert lib.sc_wilson_tune_set(out, 1, 3, 31) == 0
    assert lib.sc_wilson_tune_set(out, 1, 3, 45) == -1  # 2 planes per block
    assert lib.sc_wilson_tune_set(out, 1, 3, 68) == -1  # 4 planes per block
    assert lib.sc_wilson_tune_set(out, 1, 3, 69) == -1  # out of range
    assert lib.sc_wilson_tune_set(out, 1, 3, 44) == 0
    assert lib.sc_wilson_tune_set(out, 1, 3, -1) == 0
    assert lib.sc_op_destroy(out) == 0
    dims = (ctypes.c_int * 4)(16, 16, 2, 2)
    assert lib.sc_op_wilson_normal(dims, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_double(0.12), 1,
                                   ctypes.byref(out)) == 0
    for v in (43, 45, 68):
        assert lib.sc_wilson_tune_set(out, 1, 3, v) == 0
    assert lib.sc_wilson_tune_set(out, 1, 3, -1) == 0
    assert lib.sc_op_destroy(out) == 0
