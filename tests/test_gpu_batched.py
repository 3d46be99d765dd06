"""GPU parity of the batched persistent launch and its graph replay: every
instance against the FP64 oracle, bitwise against the single-instance
execute (same matrix-core sequence), and every graph replay against the
eager result."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, dev, dev_bf16_bits, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def make_case(count, seed, dtype, m_hi=5000):
    ms, ns, ks = I.batched_shapes(count, seed, 1, m_hi)
    # a few odd sizes and an empty instance
    ks[0], ns[0] = 5, 33
    ks[1], ns[1] = 127, 7
    ms[2] = 0
    ms[3] = 1
    As, Bs, Ahost, Bhost = [], [], [], []
    for b in range(count):
        m, n, k = int(ms[b]), int(ns[b]), int(ks[b])
        if dtype == torch.bfloat16:
            a = I.host_bf16_uniform((m, k), seed, 10 * b + 1)
            bb = I.host_bf16_uniform((k, n), seed, 10 * b + 2)
            As.append(dev_bf16_bits(a))
            Bs.append(dev_bf16_bits(bb))
        else:
            a = I.host_uniform((m, k), seed, 10 * b + 1, dtype=np.float32)
            bb = I.host_uniform((k, n), seed, 10 * b + 2, dtype=np.float32)
            As.append(dev(a, torch.float32))
            Bs.append(dev(bb, torch.float32))
        Ahost.append(a)
        Bhost.append(bb)
    return ms, ns, ks, As, Bs, Ahost, Bhost


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batched_against_oracle_and_single(dtype):
    count = 40
    ms, ns, ks, As, Bs, Ah, Bh = make_case(count, 70, dtype)
    announce("batched", dtype, count)
    packs = [T.pack(b) for b in Bs]
    Cs = [torch.full((int(ms[b]), int(ns[b])), 7.0, dtype=torch.float32, device="cuda") for b in range(count)]
    C0 = [host(c) for c in Cs]
    alphas = [1.5] * count
    betas = [0.5 if b % 2 else 0.0 for b in range(count)]
    bp = T.plan_batched(ms, ns, ks, dtype)
    bp.execute(As, packs, Cs, alphas, betas)
    tol = 1e-6 if dtype == torch.float32 else 1e-5
    for b in range(count):
        got = host(Cs[b])
        ref = oracle.gemm_n(Ah[b], Bh[b], C0[b], alphas[b], betas[b])
        if ref.size:
            assert_normwise(got, ref, tol, "instance %d" % b)
        # the same instance through the single-shape path, with the same
        # matrix-core product (the wide kernels would sum in another order)
        single = torch.full_like(Cs[b], 7.0)
        sp = T.plan(int(ms[b]), int(ns[b]), int(ks[b]), "N", dtype)
        if dtype == torch.float32:
            sp.set_tile(kernel=T.KERNEL_STREAM)
        T.execute(sp, As[b], packs[b], single, alphas[b], betas[b])
        assert torch.equal(single, Cs[b]), "instance %d differs from the single execute" % b


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_graph_replays_match_eager(dtype):
    count = 24
    ms, ns, ks, As, Bs, Ah, Bh = make_case(count, 71, dtype)
    packs = [T.pack(b) for b in Bs]
    Cs = [torch.zeros((int(ms[b]), int(ns[b])), dtype=torch.float32, device="cuda") for b in range(count)]
    bp = T.plan_batched(ms, ns, ks, dtype)
    announce("graph eager", dtype)
    bp.execute(As, packs, Cs)
    eager = [c.clone() for c in Cs]
    g = bp.graph()
    for rep in range(4):
        for c in Cs:
            c.zero_()
        # fresh A between replays: the graph reads the bound buffers
        if rep == 2:
            for a in As:
                a.mul_(2)
        announce("graph replay", rep)
        g.launch()
        torch.cuda.synchronize()
        for b in range(count):
            exp = eager[b] * (2.0 if rep >= 2 else 1.0)
            assert torch.equal(Cs[b], exp), (rep, b)
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_chunk_size_does_not_change_results(dtype):
    # the chunk size only changes which workgroup computes which rows; each
    # row runs the same code, so the results are bitwise the same
    count = 24
    ms, ns, ks, As, Bs, Ah, Bh = make_case(count, 72, dtype, m_hi=9000)
    packs = [T.pack(b) for b in Bs]
    Cs = [torch.zeros((int(ms[b]), int(ns[b])), dtype=torch.float32, device="cuda") for b in range(count)]
    bp = T.plan_batched(ms, ns, ks, dtype)
    t = bp.get_tile()
    assert t["kernel"] == T.KERNEL_BATCHED and t["chunk_rows"] >= 256
    assert "kernel=batched" in bp.describe()
    announce("chunk default", dtype, t["chunk_rows"])
    bp.execute(As, packs, Cs)
    ref = [c.clone() for c in Cs]
    for chunk, wpc in ((256, 1), (1024, 1), (65536, 1), (1024, 2), (256, 4)):
        announce("chunk", dtype, chunk, "wg_per_cu", wpc)
        try:
            bp.set_chunk_rows(chunk, wpc)
        except T.TsmmError as e:
            # more copies of the largest packed B than the LDS holds
            assert wpc > 1 and e.status == T.INVALID_VALUE, e
            continue
        t = bp.get_tile()
        assert t["chunk_rows"] == chunk and t["wg_per_cu"] == wpc
        assert "wg_per_cu=%d" % wpc in bp.describe()
        for c in Cs:
            c.zero_()
        bp.execute()
        for b in range(count):
            assert torch.equal(Cs[b], ref[b]), (chunk, wpc, b)
    # the workgroup count stays when only the chunk size changes
    bp.set_chunk_rows(1024, 1)
    bp.set_chunk_rows(2048)
    assert bp.get_tile()["wg_per_cu"] == 1
    with pytest.raises(T.TsmmError) as e:
        bp.set_chunk_rows(1024, 3)
    assert e.value.status == T.INVALID_VALUE
    for b in range(count):
        if ms[b]:
            assert_normwise(host(Cs[b]), oracle.gemm_n(Ah[b], Bh[b]), 1e-6 if dtype == torch.float32 else 1e-5)
    # a graph fixes the chunk list it captured
    g = bp.graph()
    with pytest.raises(T.TsmmError) as e:
        bp.set_chunk_rows(2048)
    assert e.value.status == T.INVALID_VALUE
    del g
    bp.set_chunk_rows(2048)
    for bad in (300, 128, 1 << 17):
        with pytest.raises(T.TsmmError) as e:
            bp.set_chunk_rows(bad)
        assert e.value.status == T.INVALID_VALUE
    with pytest.raises(T.TsmmError) as e:
        T._set_tile(bp.handle, kernel=T.KERNEL_STREAM)
    assert e.value.status == T.NOT_SUPPORTED


def test_batched_validation():
    bp = T.plan_batched([100, 200], [8, 16], [8, 16], torch.float32)
    A = [torch.zeros((100, 8), device="cuda"), torch.zeros((200, 16), device="cuda")]
    C = [torch.zeros((100, 8), device="cuda"), torch.zeros((200, 16), device="cuda")]
    wrong = [T.pack(torch.zeros((8, 8), device="cuda")), T.pack(torch.zeros((16, 8), device="cuda"))]
    with pytest.raises(T.TsmmError) as e:
        bp.execute(A, wrong, C)
    assert e.value.status == T.SHAPE_MISMATCH
    with pytest.raises(T.TsmmError) as e:
        T.plan_batched([10], [300], [8], torch.float32)
    assert e.value.status == T.NOT_SUPPORTED
    with pytest.raises(T.TsmmError) as e:
        T.plan_batched([10], [8], [8], torch.float64)
    assert e.value.status == T.NOT_SUPPORTED
