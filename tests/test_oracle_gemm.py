"""Pins of the oracle's Cannon block product (ora_block_gemm, oracle.cannon; Sec. 4.4).

The oracle's block product is pinned against things other than itself: exact integer
arithmetic in pure Python on small ragged shapes (FP64 holds every partial sum of
these small integers exactly, so any correct summation gives the same bits), the
identity matrix, the transpose identity (A B)^T = B^T A^T (same products, same order:
equal bits), the FP64 error bound against an independent BLAS product, and, for the
Cannon schedule, the full product on P simulated ranks equal to the exact integer
product.  Planted mistakes in the C code (tests/test_oracle_mutations.py) fail these.
"""
import numpy as np
import pytest

import oracle as ora


def _py_product(A, B, C0=None):
    """Pure-Python integer product (no numpy arithmetic): C0 + A B."""
    m, k = len(A), len(A[0])
    n = len(B[0])
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            s = 0 if C0 is None else C0[i][j]
            for p in range(k):
                s += A[i][p] * B[p][j]
            row.append(s)
        out.append(row)
    return out


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (17, 9, 13), (2, 31, 1), (8, 1, 19)])
@pytest.mark.parametrize("accumulate", [False, True])
def test_block_gemm_exact_on_integers(m, n, k, accumulate):
    rng = np.random.default_rng(m * 100 + n * 10 + k)
    A = rng.integers(-50, 51, (m, k))
    B = rng.integers(-50, 51, (k, n))
    C0 = rng.integers(-1000, 1001, (m, n))
    # operands as row views of wider arrays: leading dimensions larger than the rows
    a = np.zeros((m, k + 3))
    a[:, :k] = A
    b = np.zeros((k, n + 5))
    b[:, :n] = B
    c = np.full((m, n + 2), 7.0)
    c[:, :n] = C0
    ora.block_gemm(a[:, :k], b[:, :n], c[:, :n], accumulate=accumulate)
    want = _py_product(A.tolist(), B.tolist(), C0.tolist() if accumulate else None)
    assert c[:, :n].tolist() == [[float(x) for x in row] for row in want]
    assert np.all(c[:, n:] == 7.0)  # nothing outside the block is written


def test_block_gemm_identity_and_empty_inner_dimension():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((9, 6))
    assert np.array_equal(ora.block_gemm(A, np.eye(6)), A)
    assert np.array_equal(ora.block_gemm(np.eye(9), A), A)
    C = rng.standard_normal((9, 4))
    keep = C.copy()
    ora.block_gemm(np.zeros((9, 0)), np.zeros((0, 4)), C, accumulate=True)
    assert np.array_equal(C, keep)
    ora.block_gemm(np.zeros((9, 0)), np.zeros((0, 4)), C, accumulate=False)
    assert np.all(C == 0.0)


def test_block_gemm_transpose_identity_is_bitwise():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((13, 7))
    B = rng.standard_normal((7, 11))
    ab = ora.block_gemm(A, B)
    btat = ora.block_gemm(np.ascontiguousarray(B.T), np.ascontiguousarray(A.T))
    assert np.array_equal(ab, btat.T)


def test_block_gemm_within_the_fp64_error_bound():
    """Against an independent BLAS product: |C - C_blas| <= 2 k u |A| |B| elementwise."""
    rng = np.random.default_rng(3)
    m, n, k = 40, 33, 257
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    C = ora.block_gemm(A, B)
    bound = 2 * k * np.finfo(np.float64).eps * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(C - A @ B) <= bound)


@pytest.mark.parametrize("N,P", [(6, 1), (6, 2), (6, 3), (10, 5), (12, 4)])
def test_cannon_on_P_ranks_is_the_product(N, P):
    rng = np.random.default_rng(N * 10 + P)
    A = rng.integers(-20, 21, (N, N))
    B = rng.integers(-20, 21, (N, N))
    C = ora.cannon(A.astype(np.float64), B.astype(np.float64), P)
    want = _py_product(A.tolist(), B.tolist())
    assert C.tolist() == [[float(x) for x in row] for row in want]


def test_cannon_order_visits_every_stripe_once():
    for P in (1, 2, 5, 8):
        for r in range(P):
            order = ora.cannon_order(r, P)
            assert order[0] == r and sorted(order) == list(range(P))
    with pytest.raises(ValueError):
        ora.cannon(np.zeros((6, 6)), np.zeros((6, 6)), 4)  # 6 is not divisible by 4
