"""GPU parity of column-major operands (TSMM_COLMAJOR): C = alpha*A*B +
beta*C with A, B and C stored column by column, against the FP64 oracle on
the logical matrices; bit-exact on small integers."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def devcol(x, dtype):
    """A column-major device matrix holding x (the transpose of a
    contiguous tensor)."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).to(dtype).cuda().t()


def run(A, B, C0, alpha, beta, dtype, tile=None):
    m, k = A.shape
    n = B.shape[1]
    announce("colmajor", dtype, "m,n,k", m, n, k, tile)
    p = T.plan(m, n, k, "C", dtype)
    if tile:
        p.set_tile(**tile)
    pk = T.pack(devcol(B, dtype), "C")
    C = devcol(C0, dtype) if C0 is not None else devcol(np.zeros((m, n)), dtype)
    T.execute(p, devcol(A, dtype), pk, C, alpha, beta)
    return host(C), p, pk


SHAPES = [(4096, 16, 16), (1000, 8, 8), (3108, 33, 70), (65536, 256, 256), (20000, 128, 128), (300, 5, 3),
          (1001, 16, 16)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,k,n", SHAPES)
def test_colmajor_against_oracle(dtype, m, k, n):
    f = np.float64 if dtype == torch.float64 else np.float32
    seed = 7000 + m + k + n
    A = I.host_uniform((m, k), seed, 1, dtype=f)
    B = I.host_uniform((k, n), seed, 2, dtype=f)
    C0 = I.host_uniform((m, n), seed, 3, dtype=f)
    C, p, pk = run(A, B, C0, 1.5, 0.5, dtype)
    vw = 2 if dtype == torch.float64 else 4
    want_kernel = "colmajor" if (m % vw == 0 and k <= 256 and n <= 256) else "simple"
    assert p.info()["kernel"] == want_kernel, p.describe()
    assert_normwise(C, oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12 if dtype == torch.float64 else 1e-6)
    # the handle keeps B column-major
    assert np.array_equal(host(T.unpack(pk)), B.astype(np.float64))
    lo, hi = (-8, 8) if dtype == torch.float64 else (-4, 4)
    Ai = I.host_ints((m, k), seed, 4, lo, hi, dtype=f)
    Bi = I.host_ints((k, n), seed, 5, lo, hi, dtype=f)
    Ci = I.host_ints((m, n), seed, 6, lo, hi, dtype=f)
    Cs, _, _ = run(Ai, Bi, Ci, 1.5, 0.5, dtype)
    assert np.array_equal(Cs, oracle.gemm_n(Ai, Bi, Ci, 1.5, 0.5))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_colmajor_tiles_beta0_and_alignment(dtype):
    m, k, n = 8192, 64, 96
    f = np.float64 if dtype == torch.float64 else np.float32
    A = I.host_uniform((m, k), 71, 1, dtype=f)
    B = I.host_uniform((k, n), 71, 2, dtype=f)
    ref = oracle.gemm_n(A, B)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    base, _, _ = run(A, B, None, 1.0, 0.0, dtype)
    for tile in (dict(kernel=T.KERNEL_COLMAJOR, nsplit=2), dict(kernel=T.KERNEL_COLMAJOR, wg_per_cu=1),
                 dict(kernel=T.KERNEL_SIMPLE)):
        C, _, _ = run(A, B, None, 1.0, 0.0, dtype, tile)
        assert_normwise(C, ref, tol, str(tile))
        if tile["kernel"] == T.KERNEL_COLMAJOR:
            assert np.array_equal(C, base), tile  # same products, any tile
    # beta = 0 never reads C (NaN-safe)
    p = T.plan(m, n, k, "C", dtype)
    pk = T.pack(devcol(B, dtype), "C")
    Cn = devcol(np.full((m, n), np.nan), dtype)
    T.execute(p, devcol(A, dtype), pk, Cn, 1.0, 0.0)
    assert_normwise(host(Cn), ref, tol)
    # C not 16-byte aligned: the any-shape kernel on the transposed problem
    buf = torch.zeros(m * n + 1, dtype=dtype, device="cuda")
    Cu = buf[1:].view(n, m).t()
    T.execute(p, devcol(A, dtype), pk, Cu, 1.0, 0.0)
    assert_normwise(host(Cu), ref, tol)


def test_colmajor_rejects_row_major_and_other_types():
    with pytest.raises(ValueError):
        T.pack(torch.zeros((8, 8), dtype=torch.float64, device="cuda")[:, :4], "C")  # neither layout
    with pytest.raises(T.TsmmError) as e:
        T.plan(1000, 8, 8, "C", torch.bfloat16)
    assert e.value.status == T.NOT_SUPPORTED


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_colmajor_column_groups_in_and_across_workgroups(dtype):
    # k = n = 128: two column groups, as two groups of wavefronts in one
    # workgroup (rows_per_wave 2) or across workgroups (nsplit 2): the same
    # products, so the same bits
    m, k, n = 6000, 128, 128
    f = np.float64 if dtype == torch.float64 else np.float32
    A = I.host_uniform((m, k), 73, 1, dtype=f)
    B = I.host_uniform((k, n), 73, 2, dtype=f)
    C0 = I.host_uniform((m, n), 73, 3, dtype=f)
    inside, p, _ = run(A, B, C0, 1.5, 0.5, dtype, dict(kernel=T.KERNEL_COLMAJOR, rows_per_wave=2, nsplit=1))
    assert p.get_tile()["rows_per_wave"] == 2
    across, q, _ = run(A, B, C0, 1.5, 0.5, dtype, dict(kernel=T.KERNEL_COLMAJOR, rows_per_wave=1, nsplit=2))
    assert q.get_tile()["nsplit"] == 2
    assert np.array_equal(inside, across)
    assert_normwise(inside, oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12 if dtype == torch.float64 else 1e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_small_times_wide_row_major_through_colmajor(dtype):
    # row-major C (m x n) = A (m x k, small) * B (k x n, wide) is, on the
    # same memory, the column-major problem C^T = B^T A^T: the wide B is the
    # column-major "A" (n x k), the small A the packed column-major "B"
    # (k x m), C the column-major n x m result
    m, k, n = 24, 32, 100000
    f = np.float64 if dtype == torch.float64 else np.float32
    A = I.host_uniform((m, k), 81, 1, dtype=f)
    B = I.host_uniform((k, n), 81, 2, dtype=f)
    C0 = I.host_uniform((m, n), 81, 3, dtype=f)
    Ad = torch.from_numpy(A).to(dtype).cuda()        # row-major m x k
    Bd = torch.from_numpy(B).to(dtype).cuda()        # row-major k x n
    Cd = torch.from_numpy(C0).to(dtype).cuda()       # row-major m x n
    p = T.plan(n, m, k, "C", dtype)
    pk = T.pack(Ad.t(), "C")                         # A^T: column-major k x m
    announce("small x wide", dtype)
    T.execute(p, Bd.t(), pk, Cd.t(), 1.5, 0.5)       # B^T: column-major n x k; C^T: column-major n x m
    assert p.info()["kernel"] == "colmajor"
    assert_normwise(host(Cd), oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12 if dtype == torch.float64 else 1e-6)
