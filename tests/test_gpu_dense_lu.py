"""The dense device LU of floor(W) (Sec. 2.2: factored densely when its sparse
factors would fill in), on given matrices through dp_dense_lu_test.

- Pivots and factors are those of plain column-by-column partial pivoting
  (largest modulus, the row swaps done at once), written out below in numpy:
  the device defers a panel's swaps to the panel's end, which must not change
  them.  Sizes span one and several 64-column panels with ragged tails.
- L U reproduces the rows of the matrix in the returned order.
- A zero or non-finite pivot column gives DP_ESINGULAR, and the library keeps
  working afterwards.
- At n = 8192 (blocks of four panels) the row order of a shuffled, diagonally
  dominant banded L0 U0 is recovered exactly, with factors L0 and U0.
"""
import numpy as np
import pytest

import paper_1408_1578_amd as dp

pytestmark = pytest.mark.gpu


def _eager(A0):
    """Partial pivoting one column at a time, swaps applied immediately."""
    A = A0.copy()
    n = A.shape[0]
    perm = np.arange(n)
    for c in range(n):
        p = c + int(np.argmax(np.abs(A[c:, c]) ** 2))
        A[[c, p], :] = A[[p, c], :]
        perm[[c, p]] = perm[[p, c]]
        A[c + 1:, c] /= A[c, c]
        A[c + 1:, c + 1:] -= np.outer(A[c + 1:, c], A[c, c + 1:])
    return A, perm


@pytest.fixture(scope="module")
def ctx():
    c = dp.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 129, 300])
def test_dense_lu_matches_partial_pivoting(ctx, n):
    rng = np.random.default_rng(n)
    A0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    rc, lu, perm = dp.dp_dense_lu_test(ctx, A0)
    assert rc == dp.DP_OK
    ref, pref = _eager(A0)
    assert np.array_equal(perm, pref)
    scale = np.abs(ref).max()
    assert np.abs(lu - ref).max() <= 1e-12 * n * scale
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    assert np.abs(L @ U - A0[perm]).max() <= 1e-13 * n * np.abs(A0).max()


def test_dense_lu_diagonally_dominant_keeps_order(ctx):
    # the largest entry of every column on the diagonal: no row moves
    n = 150
    rng = np.random.default_rng(3)
    A0 = 0.01 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) + 10 * np.eye(n)
    rc, lu, perm = dp.dp_dense_lu_test(ctx, A0)
    assert rc == dp.DP_OK
    assert np.array_equal(perm, np.arange(n))


@pytest.mark.parametrize("bad", ["zero_column", "nan_column", "zero_matrix"])
def test_dense_lu_singular_reports(ctx, bad):
    n = 100
    rng = np.random.default_rng(5)
    A0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if bad == "zero_column":
        A0[:, 70] = 0
    elif bad == "nan_column":
        A0[:, 37] = np.nan
    else:
        A0[:] = 0
    rc, _, _ = dp.dp_dense_lu_test(ctx, A0)
    assert rc == dp.DP_ESINGULAR
    assert "zero pivot" in dp.lib().dp_last_error().decode()
    # a regular matrix still factors afterwards
    B = rng.standard_normal((70, 70)) + 1j * rng.standard_normal((70, 70))
    rc, lu, perm = dp.dp_dense_lu_test(ctx, B)
    assert rc == dp.DP_OK
    L = np.tril(lu, -1) + np.eye(70)
    assert np.abs(L @ np.triu(lu) - B[perm]).max() <= 1e-12 * np.abs(B).max()


def test_dense_lu_four_panel_blocks_recover_row_order(ctx):
    # n = 8192 takes the blocks of four panels.  The rows of a diagonally
    # dominant banded product L0 U0 (unit L0 with entries ~0.01, U0 with
    # diagonal ~10 and entries ~0.1) are shuffled: at every step the row of the
    # next diagonal is the largest candidate by a wide margin, so partial
    # pivoting undoes the shuffle exactly and the factors are L0 and U0.
    import scipy.sparse as sp
    n, bw = 8192, 8
    rng = np.random.default_rng(9)

    def band(k, s):
        return s * (rng.standard_normal(n - k) + 1j * rng.standard_normal(n - k))

    L0 = sp.eye(n, dtype=np.complex128) + sp.diags([band(k, 0.01) for k in range(1, bw + 1)],
                                                   [-k for k in range(1, bw + 1)])
    U0 = sp.diags([10.0 + rng.random(n)] + [band(k, 0.1) for k in range(1, bw + 1)], list(range(bw + 1)))
    shuf = rng.permutation(n)
    A = (L0 @ U0).tocsr()[shuf].toarray()
    rc, lu, perm = dp.dp_dense_lu_test(ctx, A)
    del A
    assert rc == dp.DP_OK
    assert np.array_equal(shuf[perm], np.arange(n))
    ref = (L0 - sp.eye(n) + U0).toarray()
    assert np.abs(lu - ref).max() <= 1e-12 * 10
