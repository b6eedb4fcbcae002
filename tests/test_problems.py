"""The seeded workload generators (host only): the stand-ins of the paper's
Table I matrices have its n and nonzeros per row and are SPD banded
matrices; the batch of the batched solver is block diagonal with the
stated system sizes; every generator is deterministic."""
import numpy as np
import pytest

from paper_2510_13536_amd import problems as P


@pytest.mark.parametrize("name", [nm for nm, _, _ in P.TABLE1 if nm not in ("Hook_1498", "bone010")])
def test_table1_standins_have_the_tables_shape(name):
    n, nnz = {nm: (n, z) for nm, n, z in P.TABLE1}[name]
    A = P.table1_standin(name)
    assert A.n == n
    lens = np.diff(A.row_ptr)
    hb = (lens.max() - 1) // 2
    # 2 hb + 1 entries per interior row, hb rounded (+-1 per row); the first
    # and last hb rows lose up to hb entries (hb (hb + 1) / n per row)
    assert abs(A.nnz / A.n - nnz / n) <= 1.0 + hb * (hb + 1) / n
    assert A.nnz == (2 * hb + 1) * n - hb * (hb + 1)
    assert lens.min() == hb + 1 and lens.max() == 2 * hb + 1
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0                      # symmetric
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d > off)                                # strictly diagonally dominant, so SPD
    B = P.table1_standin(name)
    assert np.array_equal(A.val, B.val) and np.array_equal(A.col_idx, B.col_idx)


def test_batch_is_block_diagonal_with_its_offsets():
    B = P.batch_systems(nsys=16, seed=11, nmin=100, nmax=3000)
    off = np.asarray(B.sys_row_off)
    assert off[0] == 0 and off[-1] == B.A.n and np.all(np.diff(off) > 0)
    S = B.A.to_scipy().tocoo()
    sys_of = np.searchsorted(off, np.arange(B.A.n), side="right") - 1
    assert np.array_equal(sys_of[S.row], sys_of[S.col])  # no entry couples two systems
    for s in range(B.nsys):
        A_s, b_s = B.system(s)[:2]
        assert A_s.n == off[s + 1] - off[s]
        assert np.allclose(b_s, B.b[off[s]:off[s + 1]])
