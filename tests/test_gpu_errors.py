"""Error paths and handle lifetimes on the device: allocation failures
reported as TSMM_ERROR_OUT_OF_MEMORY (forced from the host through the
library's TSMM_FAIL_ALLOC switch, so that no kernel ever sees a bad
pointer), and the binding's workspace handling across re-tiling and the
runtime evaluator."""
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


@pytest.fixture
def fail_alloc(monkeypatch):
    def set_(what):
        monkeypatch.setenv("TSMM_FAIL_ALLOC", what)
    yield set_
    monkeypatch.delenv("TSMM_FAIL_ALLOC", raising=False)


def test_pack_out_of_memory(fail_alloc):
    B = dev(I.host_uniform((16, 16), 3, 1), torch.float64)
    fail_alloc("pack")
    announce("forced pack allocation failure")
    with pytest.raises(T.TsmmError) as e:
        T.pack(B)
    assert e.value.status == T.OUT_OF_MEMORY and "hipMalloc" in str(e.value)
    fail_alloc("")
    pk = T.pack(B)  # the library is still usable
    assert torch.equal(T.unpack(pk), B)


def test_pack_a_out_of_memory(fail_alloc):
    A = dev(I.host_uniform((64, 32), 3, 2, dtype=np.float32), torch.float32)
    fail_alloc("pack_a")
    with pytest.raises(T.TsmmError) as e:
        T.pack_a(A, "bf16x6", 1.0)
    assert e.value.status == T.OUT_OF_MEMORY


def test_workspace_out_of_memory_leaves_the_plan_usable(fail_alloc):
    # the op T plan's lazily allocated workspace (no caller workspace)
    K, m, n = 1 << 14, 64, 64
    A = I.host_normal((K, m), 4, 1)
    B = I.host_normal((K, n), 4, 2)
    Ad, Bd = dev(A, torch.float64), dev(B, torch.float64)
    pk = T.pack(Bd, "T")
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    p = T.plan(m, n, K, "T", torch.float64)
    assert p.workspace_bytes() > 0
    lib = T._lib()
    fail_alloc("workspace")
    announce("forced workspace allocation failure")
    st = lib.tsmm_execute(p.handle, T._ptr(Ad), pk.handle, T._ptr(C), 1.0, 0.0)
    assert st == T.OUT_OF_MEMORY and b"workspace" in lib.tsmm_last_error()
    fail_alloc("")
    assert lib.tsmm_execute(p.handle, T._ptr(Ad), pk.handle, T._ptr(C), 1.0, 0.0) == T.SUCCESS
    assert_normwise(host(C), oracle.gemm_t(A, B), 1e-12)


def test_batched_plan_out_of_memory(fail_alloc):
    fail_alloc("batched")
    with pytest.raises(T.TsmmError) as e:
        T.plan_batched([100, 200], [8, 16], [8, 16], torch.float32)
    assert e.value.status == T.OUT_OF_MEMORY
    fail_alloc("")
    T.plan_batched([100, 200], [8, 16], [8, 16], torch.float32)


def test_workspace_survives_retile_and_tune():
    # execute -> tune -> tune and execute -> set_tile -> tune on an op T
    # plan: the binding must detach its workspace tensor from the C plan
    # before releasing it, so no pass-1 partials land in memory that torch
    # has handed to another tensor (a canary allocated in between)
    K, m, n = 1 << 16, 64, 64
    A = I.host_normal((K, m), 5, 1)
    B = I.host_normal((K, n), 5, 2)
    Ad, Bd = dev(A, torch.float64), dev(B, torch.float64)
    pk = T.pack(Bd, "T")
    ref = oracle.gemm_t(A, B)
    for second in ("tune", "set_tile"):
        announce("workspace lifetime", second)
        p = T.plan(m, n, K, "T", torch.float64)
        C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
        T.execute(p, Ad, pk, C)
        torch.cuda.synchronize()
        if second == "tune":
            p.tune(Ad, pk, C, reps=1)
        else:
            p.set_tile(kernel=T.KERNEL_SPLITK, rows_per_wave=2, waves_per_wg=4, wg_per_cu=1, splitk=256)
        # the freed workspace is free for the caching allocator to reuse
        canaries = [torch.full((p.workspace_bytes() // 8 + 4096,), 7.0, dtype=torch.float64, device="cuda")
                    for _ in range(4)]
        p.tune(Ad, pk, C, reps=1)
        T.execute(p, Ad, pk, C)
        torch.cuda.synchronize()
        for c in canaries:
            assert bool((c == 7.0).all()), "a canary tensor was overwritten (%s)" % second
        assert_normwise(host(C), ref, 1e-12)
