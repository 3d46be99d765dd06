"""GPU parity of the k-slab kernel (op N with a long shared dimension, the
paper's square-A x tall-skinny-B workload): against the FP64 oracle on the
same seeded inputs, bit-exact on small integers, at every k split, and on
sampled rows at the full 25600 x 25600 x 240 size."""
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


def npdt(dtype):
    return np.float64 if dtype == torch.float64 else np.float32


def tol(dtype, k):
    """binary64: the target 1e-12.  binary32: the matrix cores accumulate k
    terms in binary32; for terms of random sign the relative rounding error
    grows like u * sqrt(k) (u = 2^-24), which exceeds 1e-6 past k of about
    280: the bound is the larger of the two."""
    return 1e-12 if dtype == torch.float64 else max(1e-6, 2.0 ** -24 * np.sqrt(k))


def run(A, B, C0, alpha, beta, dtype, tile=None):
    m, k = A.shape
    n = B.shape[1]
    announce("slab", dtype, "m,n,k", m, n, k, "tile", tile)
    p = T.plan(m, n, k, "N", dtype)
    p.set_tile(kernel=T.KERNEL_SLAB, **(tile or {}))  # also for k within the streaming classes
    Cd = dev(C0, dtype) if C0 is not None else torch.zeros((m, n), dtype=dtype, device="cuda")
    T.execute(p, dev(A, dtype), T.pack(dev(B, dtype)), Cd, alpha, beta)
    return host(Cd), p


SHAPES = [(300, 1000, 40), (1000, 2048, 256), (515, 777, 66), (64, 4096, 8), (2100, 640, 240), (17, 33, 32)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,k,n", SHAPES)
def test_slab_against_oracle(dtype, m, k, n):
    seed = 5000 + m + k + n
    f = npdt(dtype)
    A = I.host_uniform((m, k), seed, 1, dtype=f)
    B = I.host_uniform((k, n), seed, 2, dtype=f)
    C0 = I.host_uniform((m, n), seed, 3, dtype=f)
    C, p = run(A, B, C0, 1.5, 0.5, dtype)
    assert p.info()["kernel"] == "slab", p.describe()
    assert_normwise(C, oracle.gemm_n(A, B, C0, 1.5, 0.5), tol(dtype, k))
    # small integers: every partial sum is exact, so every split gives the
    # oracle's result bit for bit
    lo, hi = (-8, 8) if dtype == torch.float64 else (-4, 4)
    Ai = I.host_ints((m, k), seed, 4, lo, hi, dtype=f)
    Bi = I.host_ints((k, n), seed, 5, lo, hi, dtype=f)
    Ci = I.host_ints((m, n), seed, 6, lo, hi, dtype=f)
    want = oracle.gemm_n(Ai, Bi, Ci, 1.5, 0.5)
    nsl = (k + 31) // 32
    for sk in sorted({1, 2, 3, min(7, nsl), nsl if nsl <= 64 else 64}):
        if sk > nsl:
            continue
        Cs, q = run(Ai, Bi, Ci, 1.5, 0.5, dtype, tile=dict(splitk=sk))
        assert q.get_tile()["splitk"] == sk
        assert np.array_equal(Cs, want), ("splitk", sk)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_slab_splits_repeatable_and_within_tolerance(dtype):
    m, k, n = 700, 3000, 128
    f = npdt(dtype)
    A = I.host_uniform((m, k), 91, 1, dtype=f)
    B = I.host_uniform((k, n), 91, 2, dtype=f)
    ref = oracle.gemm_n(A, B)
    for sk in (1, 4, 13):
        C1, _ = run(A, B, None, 1.0, 0.0, dtype, tile=dict(splitk=sk))
        C2, _ = run(A, B, None, 1.0, 0.0, dtype, tile=dict(splitk=sk))
        assert np.array_equal(C1, C2), sk  # fixed-order second pass
        assert_normwise(C1, ref, tol(dtype, k), "splitk %d" % sk)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_slab_blas_conventions_and_alignment(dtype):
    m, k, n = 400, 600, 64
    f = npdt(dtype)
    A = I.host_uniform((m, k), 92, 1, dtype=f)
    B = I.host_uniform((k, n), 92, 2, dtype=f)
    p = T.plan(m, n, k, "N", dtype)
    assert p.info()["kernel"] == "slab"
    pk = T.pack(dev(B, dtype))
    Ad = dev(A, dtype)
    # beta = 0 never reads C (NaN-safe), with and without a k split
    for sk in (1, 5):
        p.set_tile(kernel=T.KERNEL_SLAB, splitk=sk)
        C = torch.full((m, n), float("nan"), dtype=dtype, device="cuda")
        announce("slab nan C", dtype, sk)
        T.execute(p, Ad, pk, C, -0.75, 0.0)
        assert_normwise(host(C), oracle.gemm_n(A, B, None, -0.75, 0.0), tol(dtype, k))
    # C not 16-byte aligned: the plan runs the any-shape kernel
    buf = torch.zeros(m * n + 1, dtype=dtype, device="cuda")
    Cu = buf[1:].view(m, n)
    announce("slab unaligned C", dtype)
    T.execute(p, Ad, pk, Cu, 1.0, 0.0)
    assert_normwise(host(Cu), oracle.gemm_n(A, B), tol(dtype, k))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_paper_workload_sampled(dtype):
    # square A 25600 x 25600 times B 25600 x 240 (the default plan: k split
    # in parts), checked on 48 sampled rows
    m = k = 25600
    n = 240
    announce("slab paper workload", dtype)
    A = I.device_uniform((m, k), I.BASE_SEED, 51, dtype)
    B = I.device_uniform((k, n), I.BASE_SEED, 52, dtype)
    C0 = I.device_uniform((m, n), I.BASE_SEED, 53, dtype)
    C = C0.clone()
    p = T.plan(m, n, k, "N", dtype)
    assert p.info()["kernel"] == "slab" and p.get_tile()["splitk"] > 1
    T.execute(p, A, T.pack(B), C, 1.5, 0.5)
    rows = torch.from_numpy(I.sample_rows(m, 48, 11)).cuda()
    ref = oracle.gemm_n(host(A[rows]), host(B), host(C0[rows]), 1.5, 0.5)
    err = assert_normwise(host(C[rows]), ref, tol(dtype, k))
    print("paper workload", dtype, "sampled normwise error %.3e" % err)
