"""Non-finite inputs on the GPU paths (IEEE semantics of Eq. (1) element
by element): a NaN or an infinity in row i of A reaches only row i of C,
one in column j of B only column j (op N); for op T, column i of A only
row i of C.  Whether an output is NaN, +inf, -inf or finite does not
depend on the summation order (inf + -inf is NaN in any order, inf plus a
finite value stays inf), so the class of every output is compared with the
oracle's exactly, and the finite outputs to the path's tolerance.  The
split-bfloat16 modes take the residual of an infinite element as
inf - inf = NaN, so there the rows (columns) that are not finite are
compared, not their class."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, dev, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def classes(C):
    return np.where(np.isnan(C), 3, np.where(np.isposinf(C), 1, np.where(np.isneginf(C), 2, 0)))


def check(C, ref, tol, what):
    assert np.array_equal(classes(C), classes(ref)), what
    fin = np.isfinite(ref)
    assert fin.any(), what
    assert_normwise(np.where(fin, C, 0.0), np.where(fin, ref, 0.0), tol, what)


def poison(A, B, f):
    A = A.copy()
    B = B.copy()
    A[5, 3] = np.nan
    A[77, 0] = np.inf
    A[78, 1] = -np.inf
    A[200, :] = np.inf  # a whole row
    B[2, 9 % B.shape[1]] = -np.inf
    return A.astype(f), B.astype(f)


@pytest.mark.parametrize("k,n", [(8, 8), (32, 32), (128, 128)])
def test_stream_binary64_keeps_non_finite_values_in_their_row_and_column(k, n):
    m = 1000
    A, B = poison(I.host_uniform((m, k), 810 + k, 1), I.host_uniform((k, n), 810 + k, 2), np.float64)
    C0 = I.host_uniform((m, n), 810 + k, 3)
    announce("non-finite op N f64", m, n, k)
    p = T.plan(m, n, k, "N", torch.float64)
    C = dev(C0, torch.float64)
    T.execute(p, dev(A, torch.float64), T.pack(dev(B, torch.float64)), C, 1.5, 0.5)
    check(host(C), oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12, p.describe())
    # the same bits from a tile with column groups, where one exists
    if n == 128:
        q = T.plan(m, n, k, "N", torch.float64).set_tile(kernel=T.KERNEL_STREAM, nsplit=1)
        C1 = dev(C0, torch.float64)
        T.execute(q, dev(A, torch.float64), T.pack(dev(B, torch.float64)), C1, 1.5, 0.5)
        assert torch.equal(torch.isnan(C1), torch.isnan(C))
        assert torch.equal(torch.nan_to_num(C1), torch.nan_to_num(C))


def test_op_t_keeps_non_finite_values_in_their_row():
    K, m, n = 4096, 64, 64
    A = I.host_normal((K, m), 820, 1)
    B = I.host_normal((K, n), 820, 2)
    A[100, 7] = np.nan
    A[4000, 9] = np.inf
    B[5, 30] = -np.inf
    announce("non-finite op T", K)
    p = T.plan(m, n, K, "T", torch.float64)
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    T.execute(p, dev(A, torch.float64), T.pack(dev(B, torch.float64), "T"), C, 1.0, 0.0)
    check(host(C), oracle.gemm_t(A, B), 1e-12, p.describe())


def test_column_major_keeps_non_finite_values_in_their_row_and_column():
    m, k, n = 1024, 32, 32
    A, B = poison(I.host_uniform((m, k), 830, 1), I.host_uniform((k, n), 830, 2), np.float64)
    devcol = lambda x: torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).cuda().t()
    announce("non-finite column-major")
    p = T.plan(m, n, k, "C", torch.float64)
    C = devcol(np.zeros((m, n)))
    T.execute(p, devcol(A), T.pack(devcol(B), "C"), C, 1.0, 0.0)
    assert p.info()["ran"] == "colmajor"
    check(host(C), oracle.gemm_n(A, B), 1e-12, p.describe())


def test_wide_binary32_keeps_non_finite_values_in_their_row_and_column():
    m, k, n = 3000, 64, 128
    A, B = poison(I.host_uniform((m, k), 840, 1, dtype=np.float32), I.host_uniform((k, n), 840, 2, dtype=np.float32),
                  np.float32)
    announce("non-finite wide f32")
    p = T.plan(m, n, k, "N", torch.float32).set_tile(kernel=T.KERNEL_WIDE)
    C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    T.execute(p, dev(A, torch.float32), T.pack(dev(B, torch.float32)), C, 1.0, 0.0)
    check(host(C), oracle.gemm_n(A, B), 1e-6, p.describe())


@pytest.mark.parametrize("mode", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("kernel", ["wide", "splitbf16"])
def test_split_modes_keep_non_finite_values_in_their_row(mode, kernel):
    # non-finite A only (a non-finite column of B has no power-of-two scale)
    m, k, n = 3000, 64, 128
    A = I.host_uniform((m, k), 850, 1, dtype=np.float32)
    B = I.host_uniform((k, n), 850, 2, dtype=np.float32)
    A[5, 3] = np.nan
    A[77, 0] = np.inf
    A[200, :] = -np.inf
    announce("non-finite split", mode, kernel)
    p = T.plan(m, n, k, "N", torch.float32).set_mode(mode)
    p.set_tile(kernel=T.KERNEL_WIDE if kernel == "wide" else T.KERNEL_SPLITBF16)
    C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    T.execute(p, dev(A, torch.float32), T.pack(dev(B, torch.float32), "N", mode), C, 1.0, 0.0)
    Ch = host(C)
    ref = oracle.gemm_n(A, B)
    bad = ~np.isfinite(ref)
    assert np.array_equal(~np.isfinite(Ch), bad), p.describe()
    assert set(np.nonzero(bad.any(axis=1))[0]) == {5, 77, 200}
    fin = ~bad
    assert_normwise(np.where(fin, Ch, 0.0), np.where(fin, ref, 0.0), 1e-6 if mode == "bf16x6" else 2e-5, mode)
