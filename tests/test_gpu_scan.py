"""The device-wide exclusive scan that builds every CSR row pointer, through
C-ABI calls whose output row pointers are plain prefix sums of per-row
counts:

* airg_drop with tau = 0 keeps every entry, so its row pointer must equal the
  input's (one scan of the kept counts);
* airg_transpose scans the column counts of A, compared with scipy's
  transpose;
* airg_extract scans three arrays in one launch (F, C and terminal ranks),
  compared with dense slicing.

Sizes straddle the single-workgroup limit (16,384 entries) and the 2,048-entry
tiles of the multi-workgroup scan, up to 2.5M rows (1,221 tiles), with empty
rows; calls alternate between two streams and repeat.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")

SIZES = [1, 2047, 2048, 2049, 16384, 16385, 18432, 18433, 123457, 2_500_001]


def random_csr(n, ncols, seed, maxlen=9):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxlen + 1, size=n)
    lens[rng.integers(0, n, size=max(1, n // 50))] = 0          # some empty rows
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    k = np.arange(rows.size) - np.repeat(np.cumsum(lens) - lens, lens)
    cols = (rows * 7919 + k * 3) % ncols
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    vals = rng.uniform(0.5, 2.0, size=rows.size) * rng.choice([-1.0, 1.0], size=rows.size)
    return rp.astype(np.int32), cols.astype(np.int32), vals


@pytest.mark.parametrize("n", SIZES)
def test_drop_keeping_everything_reproduces_the_row_pointer(n):
    rp, ci, v = random_csr(n, max(n, 64), seed=n)
    A = airg.to_device(rp, ci, v)
    s2 = torch.cuda.Stream()
    for rep in range(3):
        stream = s2 if rep % 2 else None
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            out = airg.airg_drop(A, max(n, 64), 0.0, False, stream=stream)
            got_rp, got_ci, got_v, _ = out.to_host()
        assert np.array_equal(got_rp, rp), (n, rep)
        assert np.array_equal(got_ci, ci) and np.array_equal(got_v, v), (n, rep)


@pytest.mark.parametrize("n", [16385, 40961, 300001])
def test_transpose_scans_column_counts(n):
    ncols = n + 4097
    rp, ci, v = random_csr(n, ncols, seed=7 * n)
    A = airg.to_device(rp, ci, v)
    got_rp, got_ci, got_v, nc = airg.airg_transpose(A, ncols).to_host()
    T = sp.csr_matrix((v, ci, rp), shape=(n, ncols)).T.tocsr()
    T.sort_indices()
    assert nc == n
    assert np.array_equal(got_rp, T.indptr) and np.array_equal(got_ci, T.indices)
    assert np.array_equal(got_v, T.data)


@pytest.mark.parametrize("n", [20000, 262145])
def test_extract_scans_three_arrays_in_one_launch(n):
    rp, ci, v = random_csr(n, n, seed=3 * n)
    # every row keeps a diagonal so that the blocks have the usual shape
    M = sp.csr_matrix((v, ci, rp), shape=(n, n)) + sp.identity(n, format="csr") * 4.0
    M.sort_indices()
    rp, ci, v = M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data
    cf = np.random.default_rng(n).choice(np.array([1, 2], np.int8), size=n, p=[0.6, 0.4])   # F = 1, C = 2
    A = airg.to_device(rp, ci, v)
    dcf = torch.as_tensor(cf, device="cuda")
    F, Cc = cf == 1, cf == 2
    for rs, cs, rsel, csel in ((F, F, 1, 1), (F, Cc, 1, 2), (Cc, F, 2, 1)):
        got_rp, got_ci, got_v, _ = airg.airg_extract(A, dcf, rsel, csel).to_host()
        want = M[rs][:, cs].tocsr()
        want.sort_indices()
        assert np.array_equal(got_rp, want.indptr) and np.array_equal(got_ci, want.indices)
        assert np.array_equal(got_v, want.data)
