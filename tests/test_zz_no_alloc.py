"""The allocation-free execute (tsmm_execute_noalloc) through the C ABI:
split-k plans run on the library's static device scratch instead of a
workspace and give tsmm_execute's results bit for bit (same plan, same
kernels, same partial sums), which in turn meet the FP64 oracle's bar
(Eq. (1); 1e-12 normwise in binary64).  Two calls in a row, the second
with a smaller problem, so the scratch holds the first call's partials
when the second starts."""
import ctypes

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


def lib():
    L = T._lib()
    f = L.tsmm_execute_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_double] * 2
    return L


def both(p, A, pk, C0, alpha, beta):
    """(C from tsmm_execute, C from tsmm_execute_noalloc) on copies of C0."""
    L = lib()
    C1 = C0.clone()
    C2 = C0.clone()
    T.execute(p, A, pk, C1, alpha, beta)
    torch.cuda.synchronize()
    assert L.tsmm_plan_set_stream(p.handle, T._stream()) == T.SUCCESS
    st = L.tsmm_execute_noalloc(p.handle, T._ptr(A), pk.handle, T._ptr(C2), alpha, beta)
    assert st == T.SUCCESS, L.tsmm_last_error()
    torch.cuda.synchronize()
    return host(C1), host(C2)


def test_op_t_two_calls_second_smaller():
    cases = [(1 << 20, 64, 64, 512), (1 << 15, 40, 24, 64)]  # (K, m, n, split-k parts)
    for K, m, n, P in cases:
        announce("noalloc op T", K, m, n, P)
        A = I.host_normal((K, m), 61, K + m)
        B = I.host_normal((K, n), 61, K + n)
        C0 = I.host_normal((m, n), 61, 3)
        p = T.plan(m, n, K, "T", torch.float64)
        p.set_tile(kernel=T.KERNEL_SPLITK, rows_per_wave=2, waves_per_wg=4, wg_per_cu=1, splitk=P)
        assert p.workspace_bytes() == P * m * n * 8 <= 32 << 20
        pk = T.pack(dev(B, torch.float64), "T")
        c1, c2 = both(p, dev(A, torch.float64), pk, dev(C0, torch.float64), 1.5, 0.5)
        assert c1.tobytes() == c2.tobytes()
        assert_normwise(c2, oracle.gemm_t(A, B, C0, 1.5, 0.5), 1e-12)


def test_slab_parts_two_calls_second_smaller():
    # the k-slab kernel with parts of the k range (binary64 partials)
    for m, k, n, parts in ((2000, 2048, 64, 8), (300, 1024, 40, 3)):
        announce("noalloc k-slab", m, k, n, parts)
        A = I.host_uniform((m, k), 62, m)
        B = I.host_uniform((k, n), 62, k)
        C0 = I.host_uniform((m, n), 62, n)
        p = T.plan(m, n, k, "N", torch.float64)
        p.set_tile(kernel=T.KERNEL_SLAB, splitk=parts)
        assert 0 < p.workspace_bytes() <= 32 << 20
        pk = T.pack(dev(B, torch.float64))
        c1, c2 = both(p, dev(A, torch.float64), pk, dev(C0, torch.float64), -0.75, 1.25)
        assert c1.tobytes() == c2.tobytes()
        assert_normwise(c2, oracle.gemm_n(A, B, C0, -0.75, 1.25), 1e-12)


def test_plans_without_scratch_and_errors():
    # an op N streaming plan needs no scratch: same bits as tsmm_execute
    m, k, n = 5000, 32, 32
    A = I.host_uniform((m, k), 63, 1)
    B = I.host_uniform((k, n), 63, 2)
    C0 = I.host_uniform((m, n), 63, 3)
    p = T.plan(m, n, k, "N", torch.float64)
    assert p.workspace_bytes() == 0
    c1, c2 = both(p, dev(A, torch.float64), T.pack(dev(B, torch.float64)), dev(C0, torch.float64), 1.5, 0.5)
    assert c1.tobytes() == c2.tobytes()
    # a plan whose partial sums exceed the static scratch is refused
    L = lib()
    K, mm, nn = 1 << 16, 64, 64
    q = T.plan(mm, nn, K, "T", torch.float64)
    q.set_tile(kernel=T.KERNEL_SPLITK, rows_per_wave=2, waves_per_wg=4, wg_per_cu=1, splitk=2048)
    assert q.workspace_bytes() > 32 << 20
    At = torch.zeros((K, mm), dtype=torch.float64, device="cuda")
    pk = T.pack(torch.zeros((K, nn), dtype=torch.float64, device="cuda"), "T")
    C = torch.zeros((mm, nn), dtype=torch.float64, device="cuda")
    st = L.tsmm_execute_noalloc(q.handle, T._ptr(At), pk.handle, T._ptr(C), 1.0, 0.0)
    assert st == T.NOT_SUPPORTED and b"static scratch" in L.tsmm_last_error()
    # batched plans have their own entry point
    bp = T.plan_batched([100], [8], [8], torch.float32)
    assert L.tsmm_execute_noalloc(bp.handle, T._ptr(At), pk.handle, T._ptr(C), 1.0, 0.0) == T.INVALID_VALUE
