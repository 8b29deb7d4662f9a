"""The allocation-free DDC fraction threshold against the allocating entry
point, through the C ABI: two calls in a row on one device (the second on a
smaller operator, so the scratch array still holds the first call's theta
beyond the new row count), each bit for bit equal to
airg_ddc_fraction_threshold and to the oracle's fraction rule; sizes beyond
the scratch limit are refused before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from workloads import dg_square, p0_cube

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")


def pmisr_split(P):
    A = (P.rowptr, P.col, P.val)
    G = O.sym_graph(A, O.strength(A, 0.5))
    deg, h = O.pmisr_keys(G, P.seed, 0)
    cf0, _ = O.pmisr(G, deg, h, 3)
    return A, cf0


def test_noalloc_fraction_threshold_matches_allocating_entry_point():
    for P, frac in ((dg_square(256), 0.1), (p0_cube(12), 0.25), (dg_square(24), 0.1)):
        A, cf0 = pmisr_split(P)
        dA = airg.to_device(P.rowptr, P.col, P.val)
        dcf = torch.as_tensor(cf0, device="cuda")
        print("%s n=%d fraction %.2f" % (P.name, P.n, frac), flush=True)
        got = airg.airg_ddc_fraction_threshold_noalloc(dA, dcf, frac)
        again = airg.airg_ddc_fraction_threshold_noalloc(dA, dcf, frac)
        want = airg.airg_ddc_fraction_threshold(dA, dcf, frac)
        assert got == want == again, (P.name, got, want, again)
        assert got == O.ddc_fraction_threshold(A, cf0, frac), P.name


def test_noalloc_fraction_threshold_refuses_rows_beyond_the_limit():
    mx = airg.ddc_fraction_noalloc_max_rows()
    assert mx == 1 << 21
    P = dg_square(8)
    dA = airg.to_device(P.rowptr, P.col, P.val)
    dcf = torch.ones(P.n, dtype=torch.int8, device="cuda")
    out = C.c_double(-7.0)
    # n is checked on the host before any device work, so the small buffers
    # are never read
    st = airg.lib().airg_ddc_fraction_threshold_noalloc(mx + 1, P.nnz, dA[0].data_ptr(), dA[1].data_ptr(),
                                                        dA[2].data_ptr(), dcf.data_ptr(), 0.1, C.byref(out),
                                                        None)
    assert st == -8 and out.value == -7.0
    assert b"scratch limit" in airg.lib().airg_last_error()
    # the entry point still works after the refusal
    A, cf0 = pmisr_split(P)
    dcf = torch.as_tensor(cf0, device="cuda")
    assert airg.airg_ddc_fraction_threshold_noalloc(dA, dcf, 0.1) == O.ddc_fraction_threshold(A, cf0, 0.1)
