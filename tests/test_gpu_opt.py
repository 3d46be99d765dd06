"""GPU parity of the op T path (C = alpha*A^T*B + beta*C over a long shared
dimension, split-k with an ordered second pass) against the FP64 oracle."""
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


def run_t(A, B, C0, alpha, beta, splitk=None, reps=1):
    K, m = A.shape
    n = B.shape[1]
    announce("op T m,n,K", m, n, K, "splitk", splitk)
    Ad, Bd = dev(A, torch.float64), dev(B, torch.float64)
    p = T.plan(m, n, K, "T", torch.float64)
    if splitk:
        p.set_tile(kernel=T.KERNEL_SPLITK, splitk=splitk)
    pk = T.pack(Bd, "T")
    outs = []
    for _ in range(reps):
        Cd = dev(C0, torch.float64) if C0 is not None else torch.zeros((m, n), dtype=torch.float64, device="cuda")
        T.execute(p, Ad, pk, Cd, alpha, beta)
        outs.append(host(Cd))
    return outs if reps > 1 else outs[0]


SHAPES_T = [(1, 64, 64), (3, 5, 70), (100, 16, 16), (4101, 64, 64), (1000, 100, 33), (65536, 64, 64),
            (2048, 1, 1), (777, 20, 7)]


@pytest.mark.parametrize("K,m,n", SHAPES_T)
def test_op_t_small_integers_bit_exact(K, m, n):
    seed = 4000 + K + m + n
    A = I.host_ints((K, m), seed, 1, -8, 8)
    B = I.host_ints((K, n), seed, 2, -8, 8)
    C0 = I.host_ints((m, n), seed, 3, -8, 8)
    C = run_t(A, B, C0, 1.5, 0.5)
    assert np.array_equal(C, oracle.gemm_t(A, B, C0, 1.5, 0.5))


@pytest.mark.parametrize("K,m,n", SHAPES_T)
def test_op_t_normal_normwise(K, m, n):
    seed = 5000 + K + m + n
    A = I.host_normal((K, m), seed, 1)
    B = I.host_normal((K, n), seed, 2)
    C = run_t(A, B, None, 1.0, 0.0)
    assert_normwise(C, oracle.gemm_t(A, B), 1e-12)


@pytest.mark.parametrize("P", [1, 7, 64, 512, 3000])
def test_op_t_any_split_count(P):
    K, m, n = 20000, 64, 64
    A = I.host_normal((K, m), 6, 1)
    B = I.host_normal((K, n), 6, 2)
    C0 = I.host_normal((m, n), 6, 3)
    C = run_t(A, B, C0, 0.5, -1.0, splitk=P)
    assert_normwise(C, oracle.gemm_t(A, B, C0, 0.5, -1.0), 1e-12)


def test_op_t_bitwise_repeatable():
    K, m, n = 100000, 64, 64
    A = I.host_normal((K, m), 7, 1)
    B = I.host_normal((K, n), 7, 2)
    outs = run_t(A, B, None, 1.0, 0.0, reps=10)
    for o in outs[1:]:
        assert o.tobytes() == outs[0].tobytes()


def test_op_t_stacked_identity_exact():
    reps, d = 1024, 64
    A = np.tile(np.eye(d), (reps, 1))
    C = run_t(A, A, None, 1.5, 0.0)
    assert np.array_equal(C, reps * 1.5 * np.eye(d))
    C = run_t(np.ones((4096, 64)), np.ones((4096, 64)), np.full((64, 64), 2.0), 0.5, 0.25)
    assert np.all(C == 4096 * 0.5 + 0.5)


def test_op_t_conventions():
    K, m, n = 5000, 64, 64
    A = I.host_normal((K, m), 8, 1)
    B = I.host_normal((K, n), 8, 2)
    C = run_t(A, B, np.full((m, n), np.nan), 1.0, 0.0)
    assert np.all(np.isfinite(C))
    C0 = I.host_normal((m, n), 8, 3)
    C = run_t(np.full((K, m), np.nan), B, C0, 0.0, 2.0)
    assert np.array_equal(C, 2.0 * C0)


def test_op_t_full_size_2pow22():
    # the reduction workload at full size: A, B 2^22 x 64, normal(0, 1)
    K, m, n = 1 << 22, 64, 64
    announce("op T full size")
    A = I.device_normal((K, m), I.BASE_SEED, 21, torch.float64)
    B = I.device_normal((K, n), I.BASE_SEED, 22, torch.float64)
    p = T.plan(m, n, K, "T", torch.float64)
    pk = T.pack(B, "T")
    C = torch.empty((m, n), dtype=torch.float64, device="cuda")
    T.execute(p, A, pk, C, 1.0, 0.0)
    C2 = torch.empty_like(C)
    T.execute(p, A, pk, C2, 1.0, 0.0)
    got, got2 = host(C), host(C2)
    assert got.tobytes() == got2.tobytes()
    ref = oracle.gemm_t(host(A), host(B))
    assert_normwise(got, ref, 1e-12)
