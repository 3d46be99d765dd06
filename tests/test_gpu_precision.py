"""GPU parity of the precision variants of op N for binary32 inputs:
binary32 matrix-core products, and the two- / three-term bfloat16 splits
(with binary32 accumulation and a binary64 epilogue), plus bfloat16 inputs.
Every result is compared with the FP64 oracle on the same (widened) inputs.
The packed split planes are compared bit for bit with the oracle's split."""
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


def run_f32(A, B, C0, alpha, beta, mode):
    m, k = A.shape
    n = B.shape[1]
    announce("f32", mode, m, n, k)
    p = T.plan(m, n, k, "N", torch.float32)
    if mode != "native":
        p.set_mode(mode)
    pk = T.pack(dev(B, torch.float32), "N", mode)
    C = dev(C0, torch.float32) if C0 is not None else torch.zeros((m, n), dtype=torch.float32, device="cuda")
    T.execute(p, dev(A, torch.float32), pk, C, alpha, beta)
    return host(C), pk


@pytest.mark.parametrize("mode", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("k,n", [(8, 8), (32, 16), (33, 40), (256, 256), (100, 3)])
def test_split_planes_match_oracle_split(mode, k, n):
    terms = 2 if mode == "bf16x3" else 3
    B = (I.host_uniform((k, n), 30, k + n, dtype=np.float32) *
         np.float32(2.0) ** I.host_ints((1, n), 30, 7, -20, 20, dtype=np.float32))
    B = B.astype(np.float32)
    announce("split planes", mode, k, n)
    pk = T.pack(dev(B, torch.float32), "N", mode)
    planes, exps = T.split_planes(pk)
    planes = planes.cpu().numpy().view(np.uint16)
    exps = exps.cpu().numpy()
    e_ref = oracle.column_scale_exp(B)
    assert np.array_equal(exps, e_ref)
    scaled = np.ldexp(B.astype(np.float64), -e_ref[None, :].astype(np.int64)).astype(np.float32)
    assert np.array_equal(planes, oracle.split_bf16(scaled, terms))
    if terms == 3:
        assert torch.equal(T.unpack(pk).cpu(), torch.from_numpy(B))


def precision_inputs(m, k, n, seed):
    A = I.col_scaled_uniform(m, k, seed, 1)
    B = I.host_uniform((k, n), seed, 2, dtype=np.float32)
    return A, B


@pytest.mark.parametrize("m,k,n", [(4096, 256, 256), (3000, 64, 64), (517, 32, 48), (1000, 128, 16)])
def test_precision_against_fp64(m, k, n):
    A, B = precision_inputs(m, k, n, 31 + k)
    ref = oracle.gemm_n(A, B)
    e_native = assert_normwise(run_f32(A, B, None, 1.0, 0.0, "native")[0], ref, 1e-6, "f32 native")
    e6 = assert_normwise(run_f32(A, B, None, 1.0, 0.0, "bf16x6")[0], ref, 1e-6, "bf16x6")
    e3 = assert_normwise(run_f32(A, B, None, 1.0, 0.0, "bf16x3")[0], ref, 2e-5, "bf16x3")
    print("normwise errors: native %.2e bf16x6 %.2e bf16x3 %.2e" % (e_native, e6, e3))


def test_split_with_beta_and_alpha():
    m, k, n = 2000, 64, 32
    A, B = precision_inputs(m, k, n, 40)
    C0 = I.host_uniform((m, n), 40, 3, dtype=np.float32)
    C, _ = run_f32(A, B, C0, -1.5, 0.5, "bf16x6")
    assert_normwise(C, oracle.gemm_n(A, B, C0, -1.5, 0.5), 1e-6)


@pytest.mark.parametrize("mode", ["native", "bf16x6"])
def test_split_closed_forms(mode):
    m, k = 1000, 64
    A = I.host_uniform((m, k), 41, 1, dtype=np.float32)
    C0 = I.host_uniform((m, k), 41, 3, dtype=np.float32)
    C, _ = run_f32(A, np.eye(k, dtype=np.float32), C0, 1.5, 0.5, mode)
    exp = (1.5 * A.astype(np.float64) + 0.5 * C0.astype(np.float64)).astype(np.float32).astype(np.float64)
    assert np.array_equal(C, exp)
    C, _ = run_f32(np.ones((m, k), np.float32), np.ones((k, k), np.float32), C0, 1.5, 0.5, mode)
    assert np.array_equal(C, (k * 1.5 + 0.5 * C0.astype(np.float64)).astype(np.float32).astype(np.float64))


def test_bf16x3_misses_identity_by_the_dropped_term():
    # two terms keep 16 significand bits: identity B reproduces A only to
    # within 2^-16 relative, which is what tells the two readings apart
    m, k = 500, 32
    A = I.host_uniform((m, k), 42, 1, dtype=np.float32)
    C, _ = run_f32(A, np.eye(k, dtype=np.float32), None, 1.0, 0.0, "bf16x3")
    d = np.abs(C - A.astype(np.float64))
    assert np.all(d <= 2.0 ** -16 * np.abs(A)) and d.max() > 0


@pytest.mark.parametrize("m,k,n", [(1000, 32, 32), (777, 64, 16), (129, 128, 128), (300, 256, 256),
                                   (50, 8, 8), (33, 12, 20)])
def test_bf16_inputs(m, k, n):
    seed = 60 + m + k
    Ab = I.host_bf16_uniform((m, k), seed, 1)
    Bb = I.host_bf16_uniform((k, n), seed, 2)
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32)
    announce("bf16 inputs", m, n, k)
    p = T.plan(m, n, k, "N", torch.bfloat16)
    pk = T.pack(dev_bf16_bits(Bb))
    C = dev(C0, torch.float32)
    T.execute(p, dev_bf16_bits(Ab), pk, C, 1.5, 0.5)
    # products of bf16 values are exact in binary32; only the binary32
    # accumulation rounds
    assert_normwise(host(C), oracle.gemm_n(Ab, Bb, C0, 1.5, 0.5), 1e-5)
    Ai = I.f32_to_bf16_bits(I.host_ints((m, k), seed, 4, -8, 8, dtype=np.float32))
    Bi = I.f32_to_bf16_bits(I.host_ints((k, n), seed, 5, -8, 8, dtype=np.float32))
    C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    T.execute(T.plan(m, n, k, "N", torch.bfloat16), dev_bf16_bits(Ai), T.pack(dev_bf16_bits(Bi)), C, 1.0, 0.0)
    assert np.array_equal(host(C), oracle.gemm_n(Ai, Bi))


@pytest.mark.parametrize("m,k,n", [(777, 64, 64), (300, 40, 100), (515, 16, 68), (301, 32, 66), (129, 128, 128)])
def test_bf16_inputs_interleaved_columns(m, k, n):
    # bfloat16 fragments interleave columns in groups of four tiles when
    # n % 4 == 0 (binary32 C moves in 16-byte vectors); n = 66 keeps the
    # plain order.  Small integers: every result is exact.
    seed = 90 + m + k + n
    Ai = I.f32_to_bf16_bits(I.host_ints((m, k), seed, 1, -8, 8, dtype=np.float32))
    Bi = I.f32_to_bf16_bits(I.host_ints((k, n), seed, 2, -8, 8, dtype=np.float32))
    C0 = I.host_ints((m, n), seed, 3, -8, 8, dtype=np.float32)
    want = oracle.gemm_n(Ai, Bi, C0, 1.5, 0.5)
    announce("bf16 interleave", m, n, k)
    p = T.plan(m, n, k, "N", torch.bfloat16)
    p.set_tile(kernel=T.KERNEL_SPLITBF16)
    pk = T.pack(dev_bf16_bits(Bi))
    C = dev(C0, torch.float32)
    T.execute(p, dev_bf16_bits(Ai), pk, C, 1.5, 0.5)
    assert np.array_equal(host(C), want)
    # C at an address that is not 16-byte aligned (the kernel falls back)
    buf = torch.zeros(m * n + 1, dtype=torch.float32, device="cuda")
    Cu = buf[1:].view(m, n)
    Cu.copy_(dev(C0, torch.float32))
    T.execute(p, dev_bf16_bits(Ai), pk, Cu, 1.5, 0.5)
    assert np.array_equal(host(Cu), want)


def test_large_precision_sampled():
    # 2^20 rows of the precision workload (k = n = 256), sampled rows
    m, k, n = 1 << 20, 256, 256
    announce("precision sampled 2^20")
    A = I.device_col_scaled_uniform(m, k, I.BASE_SEED, 41, torch.float32)
    Bh = I.host_uniform((k, n), I.BASE_SEED, 42, dtype=np.float32)
    rows = torch.from_numpy(I.sample_rows(m, 2048, 9)).cuda()
    Ah = host(A[rows]).astype(np.float32)
    ref = oracle.gemm_n(Ah, Bh)
    for mode, tol in (("native", 1e-6), ("bf16x6", 1e-6), ("bf16x3", 2e-5)):
        p = T.plan(m, n, k, "N", torch.float32)
        if mode != "native":
            p.set_mode(mode)
        pk = T.pack(dev(Bh, torch.float32), "N", mode)
        C = torch.empty((m, n), dtype=torch.float32, device="cuda")
        T.execute(p, A, pk, C, 1.0, 0.0)
        assert_normwise(host(C[rows]), ref, tol, mode)


def colwise_rel_err(C_hat, C_ref):
    return np.linalg.norm(C_hat - C_ref, axis=0) / np.linalg.norm(C_ref, axis=0)


def test_tiny_and_huge_columns_of_B():
    # per-column scaling of B (a power of two per column, chosen at pack
    # time, undone exactly in the binary64 epilogue): a column of B scaled by
    # 2^-115 -- whose bfloat16 residual terms would underflow binary32 without
    # the scale -- and one scaled by 2^+100 keep the accuracy of the others
    m, k, n = 2048, 64, 32
    A, B = precision_inputs(m, k, n, 51)
    B = B.astype(np.float64)
    B[:, 3] *= 2.0 ** -115
    B[:, 7] *= 2.0 ** 100
    B = B.astype(np.float32)
    ref = oracle.gemm_n(A, B)
    for mode, tol in (("bf16x6", 1e-6), ("bf16x3", 2e-5)):
        C, pk = run_f32(A, B, None, 1.0, 0.0, mode)
        ec = colwise_rel_err(C, ref)
        print("[A12] B columns at 2^-115 / 2^100, %s: column errors %.2e / %.2e, worst %.2e"
              % (mode, ec[3], ec[7], ec.max()))
        assert ec.max() <= tol, (mode, ec)
        if mode == "bf16x6":  # three terms hold a binary32 value exactly
            assert torch.equal(T.unpack(pk).cpu(), torch.from_numpy(B))


def test_tiny_A_lo_term_underflow_is_bounded():
    # A is split in registers without a scale.  At |a| about 2^-115 the third
    # bfloat16 term (about 2^-16 of the second) falls below binary32's
    # normal range (2^-126), so the three-term product loses that term and
    # is only as good as the two-term one; at 2^-100 every term is normal
    # and the three-term accuracy holds.  Documented, not hidden: the bars
    # below are those of the two- and three-term splits.
    m, k, n = 2048, 64, 32
    A, B = precision_inputs(m, k, n, 52)
    # magnitudes in [1, 2) with random signs, so that the shifted values stay
    # normal binary32 numbers (at least 2^-115) and the shift is exact
    sign = np.where(I.host_uniform((m, k), 52, 8) < 0, -1.0, 1.0)
    A = (sign * I.host_uniform((m, k), 52, 9, 1.0, 2.0)).astype(np.float32)
    for shift, tol6 in ((-100, 1e-6), (-115, 2e-5)):
        As = np.ldexp(A.astype(np.float64), shift).astype(np.float32)
        assert np.array_equal(np.ldexp(As.astype(np.float64), -shift), A.astype(np.float64))  # exact shift
        ref = oracle.gemm_n(As, B)
        e6 = assert_normwise(run_f32(As, B, None, 1.0, 0.0, "bf16x6")[0], ref, tol6, "x6 A*2^%d" % shift)
        e3 = assert_normwise(run_f32(As, B, None, 1.0, 0.0, "bf16x3")[0], ref, 2e-5, "x3 A*2^%d" % shift)
        en = assert_normwise(run_f32(As, B, None, 1.0, 0.0, "native")[0], ref, 1e-6, "native A*2^%d" % shift)
        print("[A12] A scaled by 2^%d: x6 %.2e, x3 %.2e, native %.2e" % (shift, e6, e3, en))
