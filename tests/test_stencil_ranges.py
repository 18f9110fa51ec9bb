"""Host-side range check of the DPP-form stencil shapes (variants 69..86).

Their loads and stores go through buffer descriptors, which turn an access
outside the descriptor's record into a zero read or a dropped store instead of
a fault, so a mistake in the addressing would corrupt results silently.  The
library walks, on the CPU with the kernel's own index functions, every access
one pass makes and counts those outside their record
(``sc_wilson_range_check``).  Checked here for every DPP-form shape on the
lattices these shapes run on in the tests and batches (16^4, 16^3 x 32,
16 x 16 x 4 x 8) and on ragged and degenerate ones (Z = 1, T = 1, T not a
multiple of the segment length, an odd Z), for column counts that leave
partial column groups; and, as a planted mistake, with a leading dimension
smaller than a column, which the walk must flag.  No GPU is used.
"""
import ctypes

import pytest

from paper_0810_0330_amd import api

VARIANTS = range(69, 87)
LATTICES = [(16, 16, 16, 16), (16, 16, 16, 32), (16, 16, 4, 8), (16, 16, 1, 1), (16, 16, 3, 7), (16, 16, 5, 18)]


def _check(dims, v, k, ldx=None, ldy=None):
    n = 12 * dims[0] * dims[1] * dims[2] * dims[3]
    d = (ctypes.c_int * 4)(*dims)
    acc, bad = ctypes.c_int64(), ctypes.c_int64()
    st = api.lib().sc_wilson_range_check(d, v, k, n if ldx is None else ldx, n if ldy is None else ldy,
                                         ctypes.byref(acc), ctypes.byref(bad))
    return st, acc.value, bad.value


@pytest.mark.parametrize("dims", LATTICES)
def test_every_access_in_range(dims):
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    for v in VARIANTS:
        for k in (2, 3, 7, 24):
            st, acc, bad = _check(dims, v, k)
            assert st == 0
            # at least one link, one spinor and one store check per site and column group
            assert acc >= 3 * vol
            assert bad == 0, (dims, v, k, bad)
        # padded leading dimensions (columns further apart than their length)
        st, acc, bad = _check(dims, v, 5, ldx=12 * vol + 64, ldy=12 * vol + 8)
        assert st == 0 and bad == 0


def test_planted_short_leading_dimension_is_flagged():
    dims = (16, 16, 4, 8)
    n = 12 * 16 * 16 * 4 * 8
    st, acc, bad = _check(dims, 75, 6, ldx=n - 8)
    assert st == 0 and bad > 0
    st, acc, bad = _check(dims, 75, 6, ldy=n // 2)
    assert st == 0 and bad > 0


def test_rejects_other_shapes_and_lattices():
    assert _check((16, 16, 4, 8), 41, 4)[0] != 0       # a t-march shape: no descriptors
    assert _check((8, 8, 8, 8), 69, 4)[0] != 0         # X = Y = 16 only
