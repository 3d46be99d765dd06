"""GPU parity of the packed big operand (Algorithm 1's PACKA, alpha folded
into A; the reused-operand case): tsmm_pack_a + tsmm_execute_packed_a
against the FP64 oracle, bit for bit where the arithmetic is exact (the
pre-split terms read back through an identity B, small integers) and
against the fresh-A execute on the same kernel geometry, which must give
the same bits when the terms are the same values."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, dev, host, need_gpu

pytestmark = pytest.mark.gpu

TERMS = {"bf16x3": 2, "bf16x6": 3}
TOL = {"bf16x3": 2e-5, "bf16x6": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def split_plan(m, n, k, mode, force_splitbf16=False):
    p = T.plan(m, n, k, "N", torch.float32).set_mode(mode)
    if force_splitbf16:
        p.set_tile(kernel=T.KERNEL_SPLITBF16)
    return p


def strided(A, dtype, pad=8):
    """A device copy of A whose rows sit `pad` elements apart beyond k."""
    m, k = A.shape
    buf = torch.zeros((m, k + pad), dtype=dtype, device="cuda")
    buf[:, :k] = dev(A, dtype)
    return buf[:, :k]


SPLIT_SHAPES = [(1000, 37, 20), (517, 64, 48), (4096, 256, 16), (300, 128, 128), (2050, 200, 256), (33, 8, 8)]


@pytest.mark.parametrize("mode", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("m,k,n", SPLIT_SHAPES)
def test_packed_split_is_bitwise_the_fresh_split(mode, m, k, n):
    seed = 7000 + m + k + n
    A = I.host_uniform((m, k), seed, 1, dtype=np.float32)
    B = I.host_uniform((k, n), seed, 2, dtype=np.float32)
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32)
    pk = T.pack(dev(B, torch.float32), "N", mode)
    Ad = dev(A, torch.float32)
    for alpha in (1.0, 0.5):  # powers of two scale every term exactly
        announce("packed A split", mode, m, k, n, "alpha", alpha)
        p = split_plan(m, n, k, mode)
        # the packed path runs the plan's wide kernel on RN32(alpha*A) where
        # the plan has one (k % 8 == 0), else the split-bf16 kernel on the
        # pre-split terms: the fresh reference runs the same kernel
        wide = p.info()["kernel"] == "wide" and k % 8 == 0
        Cf = dev(C0, torch.float32)
        T.execute(split_plan(m, n, k, mode, not wide), Ad, pk, Cf, alpha, 0.5)
        pa = T.pack_a(Ad, mode, alpha)
        Cp = dev(C0, torch.float32)
        T.execute_packed_a(p, pa, pk, Cp, 0.5)
        assert p.info()["ran"] == ("wide" if wide else "splitbf16"), p.describe()
        assert torch.equal(Cp, Cf), (mode, alpha)
        assert_normwise(host(Cp), oracle.gemm_n(A, B, C0, alpha, 0.5), TOL[mode], mode)
    # a scale that is not a power of two rounds alpha*a to binary32 first:
    # within the mode's tolerance of the exact product
    pa = T.pack_a(strided(A, torch.float32), mode, -2.7)
    Cp = dev(C0, torch.float32)
    T.execute_packed_a(split_plan(m, n, k, mode), pa, pk, Cp, 0.5)
    assert_normwise(host(Cp), oracle.gemm_n(A, B, C0, -2.7, 0.5), TOL[mode], mode)


@pytest.mark.parametrize("mode", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("m,k,n", [(2050, 200, 256), (3000, 256, 256), (777, 64, 128)])
def test_packed_a_through_the_eight_wavefront_wide_tile(mode, m, k, n):
    # a plan on the wide kernel with eight wavefronts per workgroup (one row
    # tile each) runs the packed call on RN32(alpha*A) with that tile: the
    # same bits as the fresh call of the same plan
    seed = 7100 + m + k + n
    A = I.host_uniform((m, k), seed, 1, dtype=np.float32)
    B = I.host_uniform((k, n), seed, 2, dtype=np.float32)
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32)
    pk = T.pack(dev(B, torch.float32), "N", mode)
    Ad = dev(A, torch.float32)
    p = split_plan(m, n, k, mode).set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=1, waves_per_wg=8)
    for alpha in (1.0, 0.5):
        announce("packed A eight-wavefront wide", mode, m, k, n, "alpha", alpha)
        Cf = dev(C0, torch.float32)
        T.execute(p, Ad, pk, Cf, alpha, 0.5)
        Cp = dev(C0, torch.float32)
        T.execute_packed_a(p, T.pack_a(Ad, mode, alpha), pk, Cp, 0.5)
        assert p.info()["ran"] == "wide" and p.info()["waves"] == "8", p.describe()
        assert torch.equal(Cp, Cf), (mode, alpha)
        assert_normwise(host(Cp), oracle.gemm_n(A, B, C0, alpha, 0.5), TOL[mode], mode)


@pytest.mark.parametrize("mode", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("m,k", [(1000, 37), (70, 64), (129, 256)])
def test_pre_split_terms_through_identity(mode, m, k):
    # B = I: each output is the sum of the terms of one packed element,
    # summed exactly (hi alone, then the lower terms, which have at most 16
    # significand bits together), so C is the oracle's split of RN32(alpha*a)
    # added up, bit for bit
    A = I.host_uniform((m, k), 8000 + m + k, 1, -3.0, 3.0, dtype=np.float32)
    alpha = 1.37
    announce("packed A identity", mode, m, k)
    pa = T.pack_a(strided(A, torch.float32), mode, alpha)
    pk = T.pack(torch.eye(k, dtype=torch.float32, device="cuda"), "N", mode)
    C = torch.full((m, k), float("nan"), dtype=torch.float32, device="cuda")
    T.execute_packed_a(split_plan(m, k, k, mode), pa, pk, C, 0.0)
    planes = oracle.pack_a(A, alpha, TERMS[mode])
    want = sum((planes[t].astype(np.uint32) << 16).view(np.float32).astype(np.float64) for t in range(TERMS[mode]))
    assert np.array_equal(host(C), want.astype(np.float32).astype(np.float64))
    planes_bytes = TERMS[mode] * ((m + 15) // 16 * 16) * ((k + 7) // 8 * 8) * 2
    # k % 8 == 0: RN32(alpha*A) itself follows the planes (for wide plans)
    a32 = (planes_bytes + 255) // 256 * 256 - planes_bytes + m * k * 4 if k % 8 == 0 else 0
    assert pa.nbytes() == planes_bytes + a32


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,k,n", [(5000, 32, 32), (777, 8, 8), (3000, 128, 128), (1024, 600, 64), (100, 3, 5)])
def test_native_packed_a(dtype, m, k, n):
    f = np.float64 if dtype == torch.float64 else np.float32
    seed = 9000 + m + k + n
    A = I.host_uniform((m, k), seed, 1, dtype=f)
    B = I.host_uniform((k, n), seed, 2, dtype=f)
    C0 = I.host_uniform((m, n), seed, 3, dtype=f)
    pk = T.pack(dev(B, dtype))
    announce("packed A native", dtype, m, k, n)
    # alpha = 0.5: the packed copy is A/2 exactly, so the plan's kernel
    # gives the fresh execute's bits
    Cf = dev(C0, dtype)
    T.execute(T.plan(m, n, k, "N", dtype), dev(A, dtype), pk, Cf, 0.5, 1.5)
    Cp = dev(C0, dtype)
    T.execute_packed_a(T.plan(m, n, k, "N", dtype), T.pack_a(dev(A, dtype), "native", 0.5), pk, Cp, 1.5)
    assert torch.equal(Cp, Cf)
    # alpha = 3 (rounded into the copy), strided A at pack time
    Cp = dev(C0, dtype)
    T.execute_packed_a(T.plan(m, n, k, "N", dtype), T.pack_a(strided(A, dtype), "native", 3.0), pk, Cp, 1.5)
    ref = oracle.gemm_n(A, B, C0, 3.0, 1.5)
    tol = 1e-12 if dtype == torch.float64 else max(1e-6, 2.0 ** -24 * np.sqrt(k))
    assert_normwise(host(Cp), ref, tol)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_native_packed_a_from_an_unaligned_A(dtype):
    # A one element past a 16-byte boundary: the element-wise packing path
    # (the vector path needs 16-byte rows), same values as the aligned one
    m, k, n = 999, 32, 16
    f = np.float64 if dtype == torch.float64 else np.float32
    A = I.host_uniform((m, k), 9100, 1, dtype=f)
    B = I.host_uniform((k, n), 9100, 2, dtype=f)
    buf = torch.zeros(m * k + 1, dtype=dtype, device="cuda")
    buf[1:] = dev(A, dtype).reshape(-1)
    announce("packed A unaligned", dtype)
    pk = T.pack(dev(B, dtype))
    Cs = []
    for Ad in (buf[1:].view(m, k), dev(A, dtype)):
        C = torch.full((m, n), float("nan"), dtype=dtype, device="cuda")
        T.execute_packed_a(T.plan(m, n, k, "N", dtype), T.pack_a(Ad, "native", 3.0), pk, C, 0.0)
        Cs.append(C)
    assert torch.equal(Cs[0], Cs[1])
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    assert_normwise(host(Cs[0]), oracle.gemm_n(A, B, None, 3.0, 0.0), tol)


@pytest.mark.parametrize("mode", ["native", "bf16x3", "bf16x6"])
def test_packed_a_small_integers_exact(mode):
    # every product and partial sum is exact: the result equals the oracle
    m, k, n = 1500, 96, 40
    A = I.host_ints((m, k), 95, 1, -4, 4, dtype=np.float32)
    B = I.host_ints((k, n), 95, 2, -4, 4, dtype=np.float32)
    C0 = I.host_ints((m, n), 95, 3, -4, 4, dtype=np.float32)
    announce("packed A integers", mode)
    p = T.plan(m, n, k, "N", torch.float32)
    if mode != "native":
        p.set_mode(mode)
    C = dev(C0, torch.float32)
    T.execute_packed_a(p, T.pack_a(dev(A, torch.float32), mode, 0.25), T.pack(dev(B, torch.float32), "N", mode),
                       C, 0.5)
    assert np.array_equal(host(C), oracle.gemm_n(A, B, C0, 0.25, 0.5))


@pytest.mark.parametrize("mode", ["native", "bf16x6"])
def test_packed_a_blas_conventions(mode):
    m, k, n = 300, 16, 24
    A = I.host_uniform((m, k), 96, 1, dtype=np.float32)
    B = I.host_uniform((k, n), 96, 2, dtype=np.float32)
    B[3, 5] = np.inf  # alpha = 0 must not read B
    C0 = I.host_uniform((m, n), 96, 3, dtype=np.float32)
    p = T.plan(m, n, k, "N", torch.float32)
    if mode != "native":
        p.set_mode(mode)
    pk = T.pack(dev(B, torch.float32), "N", mode)
    announce("packed A alpha 0", mode)
    C = dev(C0, torch.float32)
    T.execute_packed_a(p, T.pack_a(dev(A, torch.float32), mode, 0.0), pk, C, 0.5)
    assert np.array_equal(host(C), oracle.gemm_n(A, np.zeros_like(B), C0, 0.0, 0.5))
    # beta = 0 never reads C (NaN-safe)
    B[3, 5] = 0.25
    pk = T.pack(dev(B, torch.float32), "N", mode)
    C = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
    T.execute_packed_a(p, T.pack_a(dev(A, torch.float32), mode, 1.0), pk, C, 0.0)
    assert_normwise(host(C), oracle.gemm_n(A, B), 1e-6)
    # k = 0: C = beta*C; m = 0: nothing happens
    p0 = T.plan(m, n, 0, "N", torch.float32)
    if mode != "native":
        p0.set_mode(mode)
    C = dev(C0, torch.float32)
    T.execute_packed_a(p0, T.pack_a(torch.zeros((m, 0), device="cuda"), mode, 2.0),
                       T.pack(torch.zeros((0, n), device="cuda"), "N", mode), C, 0.5)
    assert np.array_equal(host(C), oracle.gemm_n(np.zeros((m, 0)), np.zeros((0, n)), C0, 2.0, 0.5))
    pm = T.plan(0, n, k, "N", torch.float32)
    if mode != "native":
        pm.set_mode(mode)
    T.execute_packed_a(pm, T.pack_a(torch.zeros((0, k), device="cuda"), mode, 1.0), pk,
                       torch.zeros((0, n), device="cuda"), 0.0)


def test_packed_a_handles_are_checked():
    m, k, n = 64, 32, 16
    A = dev(I.host_uniform((m, k), 97, 1, dtype=np.float32), torch.float32)
    pk = T.pack(dev(I.host_uniform((k, n), 97, 2, dtype=np.float32), torch.float32), "N", "bf16x6")
    pa = T.pack_a(A, "bf16x6", 1.0)
    C = torch.zeros((m, n), device="cuda")
    with pytest.raises(T.TsmmError) as e:  # plan of another m
        T.execute_packed_a(split_plan(m + 16, n, k, "bf16x6"), pa, pk, torch.zeros((m + 16, n), device="cuda"))
    assert e.value.status == T.SHAPE_MISMATCH
    with pytest.raises(T.TsmmError) as e:  # mode differs from the handle's
        T.execute_packed_a(T.plan(m, n, k, "N", torch.float32), pa, pk, C)
    assert e.value.status == T.SHAPE_MISMATCH
    with pytest.raises(T.TsmmError) as e:  # a packed A where the packed B goes
        T._check(T._lib().tsmm_execute(split_plan(m, n, k, "bf16x6").handle, T._ptr(A), pa.handle, T._ptr(C),
                                       1.0, 0.0), "tsmm_execute")
    assert e.value.status == T.INVALID_VALUE


def test_packed_a_full_size_sampled():
    # binary32 A of 2^23 x 32 in the three-term split mode, n = 32, checked
    # on sampled rows
    m, k, n = 1 << 23, 32, 32
    announce("packed A full size", m, k, n)
    A = I.device_uniform((m, k), I.BASE_SEED, 61, torch.float32)
    B = I.device_uniform((k, n), I.BASE_SEED, 62, torch.float32)
    C0 = I.device_uniform((m, n), I.BASE_SEED, 63, torch.float32)
    p = split_plan(m, n, k, "bf16x6")
    pa = T.pack_a(A, "bf16x6", 1.5)
    C = C0.clone()
    T.execute_packed_a(p, pa, T.pack(B, "N", "bf16x6"), C, 0.5)
    rows = torch.from_numpy(I.sample_rows(m, 64, 12)).cuda()
    ref = oracle.gemm_n(host(A[rows]), host(B), host(C0[rows]), 1.5, 0.5)
    assert_normwise(host(C[rows]), ref, 1e-6)
