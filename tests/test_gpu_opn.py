"""GPU parity of the op N path (C = alpha*A*B + beta*C; AutoTSMM Eq. (1),
Algorithm 1) in binary64 and binary32 against the FP64 oracle.

Bars: small-integer inputs are bit-exact (every partial sum is an integer
below 2^53, or 2^24 for binary32, and alpha, beta are dyadic); closed forms
are exact; otherwise binary64 agrees to a normwise relative error of 1e-12
and binary32 to 1e-6."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, dev, host, need_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 8, 8), (16, 2, 3), (17, 4, 4), (130, 5, 7), (1000, 8, 8), (333, 16, 16),
          (257, 17, 9), (64, 31, 32), (1000, 32, 32), (77, 33, 17), (513, 64, 48), (300, 127, 128),
          (1029, 128, 128), (129, 200, 100), (200, 256, 256), (50, 3, 256), (40, 256, 3)]


def run(A, B, C0, alpha, beta, dtype=torch.float64, tile=None, layout="N"):
    m = A.shape[0] if layout == "N" else A.shape[1]
    k = A.shape[1] if layout == "N" else A.shape[0]
    n = B.shape[1]
    announce("op", layout, dtype, "m,n,k", m, n, k, "tile", tile)
    Ad, Bd = dev(A, dtype), dev(B, dtype)
    Cd = dev(C0, dtype) if C0 is not None else torch.zeros((m, n), dtype=dtype, device="cuda")
    p = T.plan(m, n, k, layout, dtype)
    if tile:
        p.set_tile(**tile)
    pk = T.pack(Bd, layout)
    T.execute(p, Ad, pk, Cd, alpha, beta)
    return host(Cd), p


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_small_workload_4096x16():
    # 4096 x 16 times 16 x 16, alpha 1.5, beta 0.5, uniform [-1, 1]
    m, k, n = 4096, 16, 16
    A = I.host_uniform((m, k), I.BASE_SEED, 1)
    B = I.host_uniform((k, n), I.BASE_SEED, 2)
    C0 = I.host_uniform((m, n), I.BASE_SEED, 3)
    C, p = run(A, B, C0, 1.5, 0.5)
    assert p.info()["kernel"] == "stream"
    ref = oracle.gemm_n(A, B, C0, 1.5, 0.5)
    assert_normwise(C, ref, 1e-12)
    gam = k * 2.0 ** -53 / (1 - k * 2.0 ** -53)
    assert np.all(np.abs(C - ref) <= 2 * (gam * 1.5 * (np.abs(A) @ np.abs(B))) + 4 * 2.0 ** -53 * np.abs(ref))


@pytest.mark.parametrize("m,k,n", SHAPES)
def test_small_integers_bit_exact_f64(m, k, n):
    seed = 1000 + m + 3 * k + 7 * n
    A = I.host_ints((m, k), seed, 1, -8, 8)
    B = I.host_ints((k, n), seed, 2, -8, 8)
    C0 = I.host_ints((m, n), seed, 3, -8, 8)
    C, _ = run(A, B, C0, 1.5, 0.5)
    assert np.array_equal(C, oracle.gemm_n(A, B, C0, 1.5, 0.5))


@pytest.mark.parametrize("m,k,n", SHAPES)
def test_uniform_f64_normwise(m, k, n):
    seed = 2000 + m + 3 * k + 7 * n
    A = I.host_uniform((m, k), seed, 1)
    B = I.host_uniform((k, n), seed, 2)
    C0 = I.host_uniform((m, n), seed, 3)
    C, _ = run(A, B, C0, -0.75, 1.25)
    assert_normwise(C, oracle.gemm_n(A, B, C0, -0.75, 1.25), 1e-12)


@pytest.mark.parametrize("m,k,n", [(1000, 4, 4), (999, 8, 8), (1024, 32, 32), (515, 64, 16), (300, 128, 128),
                                   (130, 256, 256), (77, 12, 20), (65, 7, 33)])
def test_f32_native(m, k, n):
    seed = 3000 + m + k + n
    A = I.host_uniform((m, k), seed, 1, dtype=np.float32)
    B = I.host_uniform((k, n), seed, 2, dtype=np.float32)
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32)
    C, p = run(A, B, C0, 1.5, 0.5, dtype=torch.float32)
    assert_normwise(C, oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-6)
    Ai = I.host_ints((m, k), seed, 4, -4, 4, dtype=np.float32)
    Bi = I.host_ints((k, n), seed, 5, -4, 4, dtype=np.float32)
    Ci = I.host_ints((m, n), seed, 6, -4, 4, dtype=np.float32)
    C2, _ = run(Ai, Bi, Ci, 1.5, 0.5, dtype=torch.float32)
    assert np.array_equal(C2, oracle.gemm_n(Ai, Bi, Ci, 1.5, 0.5))


@pytest.mark.parametrize("dtype,m,k,n", [(torch.float64, 777, 32, 34), (torch.float64, 1000, 64, 100),
                                         (torch.float64, 515, 16, 126), (torch.float64, 300, 8, 66),
                                         (torch.float32, 777, 32, 64), (torch.float32, 1000, 64, 96),
                                         (torch.float32, 515, 16, 124), (torch.float32, 300, 128, 68),
                                         (torch.float32, 301, 40, 66)])
def test_interleaved_columns(dtype, m, k, n):
    # n a multiple of the 16-byte vector width and at least that many column
    # tiles: the fragments interleave columns and C moves in vectors, also
    # for a ragged last group (n = 66 binary32: plain order)
    seed = 4000 + m + k + n
    f32 = dtype == torch.float32
    A = I.host_ints((m, k), seed, 1, -4, 4, dtype=np.float32 if f32 else np.float64)
    B = I.host_ints((k, n), seed, 2, -4, 4, dtype=np.float32 if f32 else np.float64)
    C0 = I.host_ints((m, n), seed, 3, -4, 4, dtype=np.float32 if f32 else np.float64)
    C, p = run(A, B, C0, 1.5, 0.5, dtype=dtype, tile=dict(kernel=T.KERNEL_STREAM))
    assert np.array_equal(C, oracle.gemm_n(A, B, C0, 1.5, 0.5))
    A = I.host_uniform((m, k), seed, 4, dtype=np.float32 if f32 else np.float64)
    B = I.host_uniform((k, n), seed, 5, dtype=np.float32 if f32 else np.float64)
    C, _ = run(A, B, None, -0.75, 0.0, dtype=dtype, tile=dict(kernel=T.KERNEL_STREAM))
    assert_normwise(C, oracle.gemm_n(A, B, None, -0.75, 0.0), 1e-6 if f32 else 1e-12)


@pytest.mark.parametrize("k,n", [(8, 8), (32, 32), (128, 128)])
def test_every_tile_gives_the_same_bits(k, n):
    m = 2000
    A = I.host_uniform((m, k), 77, 1)
    B = I.host_uniform((k, n), 77, 2)
    C0 = I.host_uniform((m, n), 77, 3)
    ref, _ = run(A, B, C0, 1.5, 0.5)
    for rt in (1, 2, 4):
        for waves in (1, 2, 4):
            for wpc in (1, 8):
                try:
                    C, _ = run(A, B, C0, 1.5, 0.5, tile=dict(kernel=T.KERNEL_STREAM, rows_per_wave=rt,
                                                                waves_per_wg=waves, wg_per_cu=wpc))
                except T.TsmmError as e:
                    assert e.status == T.NOT_SUPPORTED
                    continue
                assert np.array_equal(C, ref), (rt, waves, wpc)
    # column groups (nsplit): each group of a row block is its own
    # workgroup; the per-element order of the products does not change
    for ns in (2, 4, 8):
        if ns > (n + 15) // 16:
            continue
        for rt in (1, 2):
            try:
                C, p = run(A, B, C0, 1.5, 0.5, tile=dict(kernel=T.KERNEL_STREAM, rows_per_wave=rt, waves_per_wg=4,
                                                            wg_per_cu=1, nsplit=ns))
            except T.TsmmError as e:
                # no instantiation, or a split through a column interleave group
                assert e.status in (T.NOT_SUPPORTED, T.INVALID_VALUE), e
                continue
            assert p.info()["nsplit"] == str(ns)
            assert np.array_equal(C, ref), ("nsplit", ns, rt)
    C, _ = run(A, B, C0, 1.5, 0.5, tile=dict(kernel=T.KERNEL_SIMPLE))
    assert_normwise(C, oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12)


def test_blas_conventions():
    m, k, n = 300, 16, 16
    A = I.host_uniform((m, k), 5, 1)
    B = I.host_uniform((k, n), 5, 2)
    C0 = I.host_uniform((m, n), 5, 3)
    # beta == 0: C is never read
    C, _ = run(A, B, np.full((m, n), np.nan), 2.0, 0.0)
    assert np.all(np.isfinite(C))
    assert_normwise(C, oracle.gemm_n(A, B, None, 2.0, 0.0), 1e-12)
    # alpha == 0: A and B are never read
    C, _ = run(np.full((m, k), np.nan), np.full((k, n), np.nan), C0, 0.0, 0.5)
    assert np.array_equal(C, 0.5 * C0)
    C, _ = run(np.full((m, k), np.nan), B, C0, 0.0, 0.0)
    assert not C.any()
    # k == 0: C = beta*C
    C, _ = run(np.zeros((m, 0)), np.zeros((0, n)), C0, 3.0, -2.0)
    assert np.array_equal(C, -2.0 * C0)
    # m == 0 and n == 0 are no-ops
    run(np.zeros((0, k)), B, np.zeros((0, n)), 1.0, 1.0)
    run(A, np.zeros((k, 0)), np.zeros((m, 0)), 1.0, 1.0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_closed_forms(dtype):
    npdt = np.float64 if dtype == torch.float64 else np.float32
    m, k = 1000, 32
    C0 = I.host_uniform((m, k), 6, 3, dtype=npdt)
    C, _ = run(np.ones((m, k), npdt), np.ones((k, k), npdt), C0, 1.5, 0.5, dtype=dtype)
    assert np.array_equal(C, (k * 1.5 + 0.5 * C0.astype(np.float64)).astype(npdt).astype(np.float64))
    A = I.host_uniform((m, k), 6, 1, dtype=npdt)
    C, _ = run(A, np.eye(k, dtype=npdt), C0, 1.5, 0.5, dtype=dtype)
    exp = (1.5 * A.astype(np.float64) + 0.5 * C0.astype(np.float64)).astype(npdt).astype(np.float64)
    assert np.array_equal(C, exp)


def offset_rows(x, off, ld):
    """x (r x c) binary64 as a row-major view with row stride ld whose first
    element lies off elements into its buffer (off 1: 8-byte aligned only);
    the padding holds 777."""
    r, c = x.shape
    buf = torch.full((off + r * ld,), 777.0, dtype=torch.float64, device="cuda")
    v = buf[off:].view(r, ld)
    v[:, :c] = dev(x, torch.float64)
    return buf, v[:, :c]


@pytest.mark.parametrize("m,k,n", [(1000, 8, 8), (777, 8, 2), (515, 16, 16), (300, 5, 6), (2049, 32, 14),
                                   (129, 128, 10), (33, 256, 4), (999, 4, 12), (17, 64, 16)])
def test_lane_pair_c_vectors(m, k, n):
    # binary64 with one column tile and n even: lanes j and j ^ 1 swap half
    # of their accumulators and C moves in 16-byte vectors when C is
    # 16-byte aligned with an even stride; otherwise element by element.
    # Both give the oracle's small-integer results exactly, the same bits on
    # uniform data, and leave the padding of C alone.
    seed = 4100 + m + k + n
    for data in ("ints", "uniform"):
        if data == "ints":
            A = I.host_ints((m, k), seed, 1, -4, 4, dtype=np.float64)
            B = I.host_ints((k, n), seed, 2, -4, 4, dtype=np.float64)
            C0 = I.host_ints((m, n), seed, 3, -4, 4, dtype=np.float64)
        else:
            A = I.host_uniform((m, k), seed, 4)
            B = I.host_uniform((k, n), seed, 5)
            C0 = I.host_uniform((m, n), seed, 6)
        pk = T.pack(dev(B, torch.float64))
        want = oracle.gemm_n(A, B, C0, 1.5, 0.5)
        outs = []
        for rt in (0, 1, 2, 4, 8):
            for off, pad in ((0, 0), (0, 2), (1, 0), (0, 1), (2, 4)):
                try:
                    p = T.plan(m, n, k, "N", torch.float64).set_tile(kernel=T.KERNEL_STREAM, rows_per_wave=rt)
                except T.TsmmError as e:
                    assert e.status == T.NOT_SUPPORTED and rt > 1, e  # no instantiation
                    break
                buf, Cv = offset_rows(C0, off, n + pad)
                announce("lane pairs", m, n, k, data, "rt", rt, "offset", off, "pad", pad)
                T.execute(p, dev(A, torch.float64), pk, Cv, 1.5, 0.5)
                assert p.info()["ran"] == "stream", p.describe()
                C = host(Cv)
                if data == "ints":
                    assert np.array_equal(C, want), (rt, off, pad)
                else:
                    assert_normwise(C, want, 1e-12, p.describe())
                outs.append(C)
                full = buf[off:].view(m, n + pad)
                assert bool((full[:, n:] == 777.0).all()) and (off == 0 or float(buf[0]) == 777.0)
        assert all(np.array_equal(o, outs[0]) for o in outs)
    # beta = 0 reads no C (NaN in C stays out)
    A = I.host_uniform((m, k), seed, 7)
    p = T.plan(m, n, k, "N", torch.float64)
    Cd = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    T.execute(p, dev(A, torch.float64), pk, Cd, -0.75, 0.0)
    assert_normwise(host(Cd), oracle.gemm_n(A, B, None, -0.75, 0.0), 1e-12)


@pytest.mark.parametrize("m,k,n", [(2049, 8, 8), (1000, 16, 16), (777, 32, 32), (515, 64, 64), (300, 8, 2),
                                   (129, 32, 64), (1000, 16, 34), (33, 64, 16)])
def test_beta0_store_variants(m, k, n):
    # beta = 0 on the memory-bound binary64 classes runs kernel variants of
    # their own (default-policy C stores): small-integer results exact for
    # every tile, NaN in C never read, and the same values as beta = 1 on a
    # zero C (the streaming-store variants)
    seed = 4200 + m + k + n
    A = I.host_ints((m, k), seed, 1, -4, 4, dtype=np.float64)
    B = I.host_ints((k, n), seed, 2, -4, 4, dtype=np.float64)
    want = oracle.gemm_n(A, B, None, 1.5, 0.0)
    pk = T.pack(dev(B, torch.float64))
    Ad = dev(A, torch.float64)
    for rt in (0, 1, 2, 4, 8):
        for wpc in (1, 8):
            try:
                p = T.plan(m, n, k, "N", torch.float64).set_tile(kernel=T.KERNEL_STREAM, rows_per_wave=rt,
                                                                  wg_per_cu=wpc)
            except T.TsmmError as e:
                assert e.status == T.NOT_SUPPORTED and rt > 1, e
                continue
            announce("beta 0 stores", m, n, k, "rt", rt, "wpc", wpc)
            C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
            T.execute(p, Ad, pk, C, 1.5, 0.0)
            assert np.array_equal(host(C), want), (rt, wpc, p.describe())
            C1 = torch.zeros((m, n), dtype=torch.float64, device="cuda")
            T.execute(p, Ad, pk, C1, 1.5, 1.0)
            assert np.array_equal(host(C1), want), (rt, wpc)


def test_misaligned_A_still_correct():
    m, k, n = 500, 32, 32
    A = I.host_uniform((m, k), 8, 1)
    B = I.host_uniform((k, n), 8, 2)
    big = torch.zeros(m * k + 1, dtype=torch.float64, device="cuda")
    big[1:] = dev(A, torch.float64).reshape(-1)
    Av = big[1:].view(m, k)  # 8-byte aligned, not 16
    p = T.plan(m, n, k, "N", torch.float64)
    pk = T.pack(dev(B, torch.float64))
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    announce("misaligned A")
    T.execute(p, Av, pk, C, 1.0, 0.0)
    assert_normwise(host(C), oracle.gemm_n(A, B), 1e-12)
    # the plan says which kernel the execute ran: the any-shape kernel here,
    # the plan's own kernel again for an aligned A
    info = p.info()
    assert info["kernel"] == "stream" and info["ran"] == "simple", p.describe()
    T.execute(p, dev(A, torch.float64), pk, C, 1.0, 0.0)
    assert p.info()["ran"] == "stream", p.describe()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_pack_round_trip(dtype):
    for k, n in [(8, 8), (33, 17), (256, 256), (300, 5)]:
        B = torch.from_numpy(I.host_uniform((k, n), 9, k + n)).to(dtype).cuda()
        announce("pack", dtype, k, n)
        pk = T.pack(B)
        pk2 = T.pack(B)
        assert torch.equal(T.unpack(pk), B) and torch.equal(T.unpack(pk2), B)
        assert pk.nbytes() == pk2.nbytes() > 0


def test_argument_errors_on_device():
    B = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    pk = T.pack(B)
    p = T.plan(100, 8, 16, "N", torch.float64)
    A = torch.zeros((100, 16), dtype=torch.float64, device="cuda")
    C = torch.zeros((100, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(T.TsmmError) as e:
        T.execute(p, A, pk, C)
    assert e.value.status == T.SHAPE_MISMATCH
    with pytest.raises(TypeError):
        T.execute(T.plan(100, 8, 8, "N", torch.float64), A[:, :8].float().contiguous(), pk, C)


def test_large_sampled_rows_2pow23_k8():
    # m = 2^23, k = n = 8: the streaming workload at full size, checked on
    # sampled rows against the oracle (rows are independent)
    m, k, n = 1 << 23, 8, 8
    announce("large m=2^23 k=n=8")
    A = I.device_uniform((m, k), I.BASE_SEED, 11, torch.float64)
    Bh = I.host_uniform((k, n), I.BASE_SEED, 12)
    C = I.device_uniform((m, n), I.BASE_SEED, 13, torch.float64)
    rows = I.sample_rows(m, 4096, 5)
    idx = torch.from_numpy(rows).cuda()
    C0s = host(C[idx])
    p = T.plan(m, n, k, "N", torch.float64)
    pk = T.pack(dev(Bh, torch.float64))
    T.execute(p, A, pk, C, 1.0, 1.0)
    ref = oracle.gemm_n(host(A[idx]), Bh, C0s, 1.0, 1.0)
    assert_normwise(host(C[idx]), ref, 1e-12)


@pytest.mark.parametrize("m,k,n", [(1, 8, 16), (63, 16, 32), (65, 64, 64), (1000, 128, 128), (777, 256, 256),
                                   (200, 24, 48), (4099, 128, 32)])
def test_valu64_kernel(m, k, n):
    # the binary64 vector-ALU kernel: ascending-l FMA chains per output, so
    # small integers are exact; uniform inputs agree to 1e-12
    seed = 6000 + m + k + n
    A = I.host_ints((m, k), seed, 1, -8, 8)
    B = I.host_ints((k, n), seed, 2, -8, 8)
    C0 = I.host_ints((m, n), seed, 3, -8, 8)
    for nb in (16, 32):
        if n % nb:
            continue
        tile = dict(kernel=T.KERNEL_VALU64, rows_per_wave=nb, waves_per_wg=4, wg_per_cu=2)
        C, p = run(A, B, C0, 1.5, 0.5, tile=tile)
        assert p.info()["kernel"] == "valu64"
        assert np.array_equal(C, oracle.gemm_n(A, B, C0, 1.5, 0.5))
        Au = I.host_uniform((m, k), seed, 4)
        Bu = I.host_uniform((k, n), seed, 5)
        Cu, _ = run(Au, Bu, None, -0.5, 0.0, tile=tile)
        assert_normwise(Cu, oracle.gemm_n(Au, Bu, None, -0.5, 0.0), 1e-12)
