"""Single-shape executes captured in a HIP graph (torch.cuda.CUDAGraph on
the capture stream): no allocation or memset happens inside an execute
whose workspace is attached, so every replay equals the eager result."""
import numpy as np
import pytest
import torch

from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


CASES = [("N", torch.float64, 100000, 32, 32), ("N", torch.float32, 50000, 256, 256),
         ("T", torch.float64, 64, 64, 1 << 16), ("N", torch.float64, 3000, 64, 2000), ("C", torch.float64, 20000, 16, 16)]


@pytest.mark.parametrize("layout,dtype,m,n,k", CASES)
def test_graph_replays_match_eager(layout, dtype, m, n, k):
    if layout == "N":
        A = I.device_uniform((m, k), 31, 1, dtype)
        B = I.device_uniform((k, n), 31, 2, dtype)
        C = torch.zeros((m, n), dtype=dtype, device="cuda")
    elif layout == "T":
        A = I.device_uniform((k, m), 31, 1, dtype)
        B = I.device_uniform((k, n), 31, 2, dtype)
        C = torch.zeros((m, n), dtype=dtype, device="cuda")
    else:
        A = I.device_uniform((k, m), 31, 1, dtype).t()
        B = I.device_uniform((n, k), 31, 2, dtype).t()
        C = torch.zeros((n, m), dtype=dtype, device="cuda").t()
    pk = T.pack(B, layout)
    p = T.plan(m, n, k, layout, dtype)
    announce("graph single", layout, dtype, m, n, k, p.describe())
    C0 = torch.rand(C.shape, dtype=dtype, device="cuda")
    if layout == "C":
        C0 = C0.t().contiguous().t()
    C.copy_(C0)
    T.execute(p, A, pk, C, 1.5, 0.5)  # eager (also attaches any workspace)
    eager = C.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.copy_(C0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            T.execute(p, A, pk, C, 1.5, 0.5)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        C.copy_(C0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, eager), (rep, p.describe())
        # eager work between replays
        T.execute(p, A, pk, C, 1.5, 0.5)
        torch.cuda.synchronize()


@pytest.mark.parametrize("mode,m,n,k", [("bf16x6", 60000, 48, 64), ("bf16x3", 30000, 128, 128), ("native", 50000, 32, 32)])
def test_packed_a_graph_replays_match_eager(mode, m, n, k):
    # the packed-A execute launches kernels only, so it can be captured too
    A = I.device_uniform((m, k), 32, 1, torch.float32)
    B = I.device_uniform((k, n), 32, 2, torch.float32)
    p = T.plan(m, n, k, "N", torch.float32)
    if mode != "native":
        p.set_mode(mode)
    pk = T.pack(B, "N", mode)
    pa = T.pack_a(A, mode, 0.5)
    C0 = torch.rand((m, n), dtype=torch.float32, device="cuda")
    C = C0.clone()
    announce("graph packed A", mode, m, n, k)
    T.execute_packed_a(p, pa, pk, C, 0.5)
    eager = C.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.copy_(C0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            T.execute_packed_a(p, pa, pk, C, 0.5)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        C.copy_(C0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, eager), (rep, mode)
        T.execute_packed_a(p, pa, pk, C, 0.5)
        torch.cuda.synchronize()
