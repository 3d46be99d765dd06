"""GPU checks of the runtime performance evaluator (tsmm_plan_tune): it
keeps a tile that runs, the result of the tuned plan still matches the
FP64 oracle, and later plans of the same shape class start from it."""
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
    T.tune_cache_clear()
    yield
    T.tune_cache_clear()


CASES = [
    ("N", torch.float64, 1 << 18, 64, 64, 1e-12),     # streaming kernel
    ("N", torch.float64, 2000, 64, 1000, 1e-12),      # k-slab kernel (long k)
    ("N", torch.float32, 20000, 128, 64, 1e-6),       # streaming and wide kernels
    ("T", torch.float64, 64, 64, 1 << 16, 1e-12),     # op T split-k
]


@pytest.mark.parametrize("layout,dtype,m,n,k,tol", CASES)
def test_tune_keeps_a_correct_tile(layout, dtype, m, n, k, tol):
    f = np.float64 if dtype == torch.float64 else np.float32
    seed = 300 + m + n + k
    A = I.host_uniform((m, k) if layout == "N" else (k, m), seed, 1, dtype=f)
    B = I.host_uniform((k, n), seed, 2, dtype=f)
    C0 = I.host_uniform((m, n), seed, 3, dtype=f)
    want = (oracle.gemm_n(A, B, C0, 1.5, 0.5) if layout == "N" else oracle.gemm_t(A, B, C0, 1.5, 0.5))
    Ad, pk = dev(A, dtype), T.pack(dev(B, dtype), layout)
    p = T.plan(m, n, k, layout, dtype)
    C = torch.zeros((m, n), dtype=dtype, device="cuda")
    announce("tune", layout, dtype, m, n, k)
    ms = p.tune(Ad, pk, C, reps=2)
    assert ms > 0 and p.info()["table"] == "2", p.describe()
    # the evaluator leaves A*B in C
    assert_normwise(host(C), oracle.gemm_n(A, B) if layout == "N" else oracle.gemm_t(A, B), tol)
    Cd = dev(C0, dtype)
    T.execute(p, Ad, pk, Cd, 1.5, 0.5)
    assert_normwise(host(Cd), want, tol)
    # a new plan of the same class starts from the tuned tile
    q = T.plan(m, n, k, layout, dtype)
    assert q.info()["table"] == "2" and q.get_tile() == p.get_tile()
    Cq = dev(C0, dtype)
    T.execute(q, Ad, pk, Cq, 1.5, 0.5)
    assert np.array_equal(host(Cq), host(Cd))


def test_cache_clear_and_validation():
    m, n, k = 4096, 16, 16
    A = I.device_uniform((m, k), 7, 1, torch.float64)
    pk = T.pack(I.device_uniform((k, n), 7, 2, torch.float64))
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    p = T.plan(m, n, k)
    p.tune(A, pk, C, reps=1)
    assert T.plan(m, n, k).info()["table"] == "2"
    T.tune_cache_clear()
    assert T.plan(m, n, k).info()["table"] != "2"
    with pytest.raises(T.TsmmError) as e:
        p.tune(A, pk, C, reps=0)
    assert e.value.status == T.INVALID_VALUE
    wrong = T.pack(I.device_uniform((k, 8), 7, 3, torch.float64))
    tile = p.get_tile()
    with pytest.raises(T.TsmmError) as e:
        p.tune(A, wrong, C, reps=1)
    assert e.value.status == T.SHAPE_MISMATCH
    assert p.get_tile() == tile  # an error leaves the plan's tile
