"""GPU parity of the wide kernels (op N, binary32 A and C, n = 128 or 256,
k <= 256): binary32 products and the two- / three-term bfloat16 splits,
each against the FP64 oracle on the same (widened) inputs.  Shapes cover
ragged row counts (partial 32-row tiles and partial workgroup tiles), k
below the packed class (zero-padded chunks), every row-tile depth (one
tile per wavefront runs eight wavefronts per workgroup, two per SIMD),
beta 0 and beta != 0, and exactly representable cases that must match bit
for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, dev, host, need_gpu

pytestmark = pytest.mark.gpu

TOL = {"native": 1e-6, "bf16x6": 1e-6, "bf16x3": 2e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def run_wide(A, B, C0, alpha, beta, mode, rt=0):
    m, k = A.shape
    n = B.shape[1]
    announce("wide", mode, m, n, k, "rt", rt, "beta", beta)
    p = T.plan(m, n, k, "N", torch.float32)
    if mode != "native":
        p.set_mode(mode)
    # one 32-row tile per wavefront: eight wavefronts per workgroup
    p.set_tile(kernel=T.KERNEL_WIDE, rows_per_wave=rt, waves_per_wg=8 if rt == 1 else 0)
    assert p.info()["kernel"] == "wide"
    pk = T.pack(dev(B, torch.float32), "N", mode)
    C = dev(C0, torch.float32) if C0 is not None else torch.full((m, n), np.nan, dtype=torch.float32, device="cuda")
    T.execute(p, dev(A, torch.float32), pk, C, alpha, beta)
    return host(C)


SHAPES = [(4096, 256, 256, 0), (1000, 256, 256, 0), (70001, 128, 128, 4), (70001, 128, 128, 2),
          (777, 64, 128, 0), (300, 200, 256, 0), (129, 8, 128, 0), (33, 96, 256, 0), (5000, 136, 128, 4),
          (4096, 256, 256, 1), (1000, 256, 256, 1), (70001, 128, 128, 1), (777, 64, 128, 1), (33, 96, 256, 1),
          (5000, 136, 128, 1), (300, 200, 256, 1)]


@pytest.mark.parametrize("mode", ["native", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("m,k,n,rt", SHAPES)
def test_wide_against_fp64(mode, m, k, n, rt):
    if rt == 4 and mode != "native":
        pytest.skip("four 32-row tiles per wavefront are built for binary32 products only")
    seed = 700 + m % 97 + k + n
    A = I.col_scaled_uniform(m, k, seed, 1)
    B = I.host_uniform((k, n), seed, 2, dtype=np.float32)
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32)
    C = run_wide(A, B, None, 1.0, 0.0, mode, rt)
    assert_normwise(C, oracle.gemm_n(A, B), TOL[mode], mode)
    C = run_wide(A, B, C0, 1.5, -0.5, mode, rt)
    assert_normwise(C, oracle.gemm_n(A, B, C0, 1.5, -0.5), TOL[mode], mode + " beta")


@pytest.mark.parametrize("mode", ["native", "bf16x6"])
def test_wide_column_scales(mode):
    # columns of B spread over 2^-20 .. 2^20: the per-column exponents of the
    # split modes land on the right (permuted) output columns
    m, k, n = 2000, 256, 256
    A = I.host_uniform((m, k), 710, 1, dtype=np.float32)
    B = (I.host_uniform((k, n), 710, 2, dtype=np.float32) *
         np.float32(2.0) ** I.host_ints((1, n), 710, 3, -20, 20, dtype=np.float32)).astype(np.float32)
    C = run_wide(A, B, None, 1.0, 0.0, mode)
    ref = oracle.gemm_n(A, B)
    # column by column (a column-relative check: one normwise figure would be
    # dominated by the largest columns)
    err = np.linalg.norm(C - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= TOL[mode], err.max()


@pytest.mark.parametrize("mode", ["native", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("n", [128, 256])
def test_wide_small_integers_exact(mode, n):
    # |entries| <= 4 are single bf16 terms and every partial sum is an
    # integer below 2^24: all three variants are exact
    m, k = 3000, 256
    A = I.host_ints((m, k), 720 + n, 1, -4, 4, dtype=np.float32)
    B = I.host_ints((k, n), 720 + n, 2, -4, 4, dtype=np.float32)
    C0 = I.host_ints((m, n), 720 + n, 3, -4, 4, dtype=np.float32)
    C = run_wide(A, B, C0, 1.0, 1.0, mode)
    assert np.array_equal(C, oracle.gemm_n(A, B, C0, 1.0, 1.0))


@pytest.mark.parametrize("mode", ["native", "bf16x6"])
@pytest.mark.parametrize("n", [128, 256])
def test_wide_closed_forms(mode, n):
    m = 1500
    A = I.host_uniform((m, n), 730 + n, 1, dtype=np.float32)
    C0 = I.host_uniform((m, n), 730 + n, 2, dtype=np.float32)
    # identity B: 1.5*A + 0.5*C0 rounded once to binary32
    C = run_wide(A, np.eye(n, dtype=np.float32), C0, 1.5, 0.5, mode)
    exp = (1.5 * A.astype(np.float64) + 0.5 * C0.astype(np.float64)).astype(np.float32).astype(np.float64)
    assert np.array_equal(C, exp)
    # all ones: k*alpha + beta*C0
    C = run_wide(np.ones((m, n), np.float32), np.ones((n, n), np.float32), C0, 1.5, 0.5, mode)
    assert np.array_equal(C, (n * 1.5 + 0.5 * C0.astype(np.float64)).astype(np.float32).astype(np.float64))


def test_wide_bf16x3_identity_keeps_16_bits():
    m, n = 700, 128
    A = I.host_uniform((m, n), 740, 1, dtype=np.float32)
    C = run_wide(A, np.eye(n, dtype=np.float32), None, 1.0, 0.0, "bf16x3")
    d = np.abs(C - A.astype(np.float64))
    assert np.all(d <= 2.0 ** -16 * np.abs(A)) and d.max() > 0


@pytest.mark.parametrize("mode", ["native", "bf16x6"])
def test_wide_matches_other_kernel(mode):
    # the wide kernel and the natural family agree to the tolerance; the
    # wide kernel is bitwise repeatable and gives the same bits with four or
    # eight wavefronts per workgroup
    m, k, n = 4000, 256, 256
    A = dev(I.col_scaled_uniform(m, k, 750, 1), torch.float32)
    B = dev(I.host_uniform((k, n), 750, 2, dtype=np.float32), torch.float32)
    pk = T.pack(B, "N", mode)
    outs = []
    for kern, rt, waves in ((T.KERNEL_WIDE, 0, 0), (T.KERNEL_WIDE, 0, 0), (T.KERNEL_WIDE, 1, 8),
                            (T.KERNEL_STREAM if mode == "native" else T.KERNEL_SPLITBF16, 0, 0)):
        p = T.plan(m, n, k, "N", torch.float32)
        if mode != "native":
            p.set_mode(mode)
        p.set_tile(kernel=kern, rows_per_wave=rt, waves_per_wg=waves)
        announce("wide vs", kern, rt, waves)
        C = torch.empty((m, n), dtype=torch.float32, device="cuda")
        T.execute(p, A, pk, C, 1.0, 0.0)
        outs.append(host(C))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])
    assert oracle.normwise_rel_err(outs[0], outs[3]) <= 2 * TOL[mode]


def test_wide_unaligned_operands():
    m, k, n = 256, 64, 128
    A = I.host_uniform((m, k), 760, 1, dtype=np.float32)
    B = I.host_uniform((k, n), 760, 2, dtype=np.float32)
    buf = torch.zeros(m * k + 1, dtype=torch.float32, device="cuda")
    buf[1:] = dev(A, torch.float32).reshape(-1)
    A_off = buf[1:].view(m, k)  # 4-byte aligned only
    announce("wide unaligned")
    p = T.plan(m, n, k, "N", torch.float32).set_tile(kernel=T.KERNEL_WIDE)
    C = torch.empty((m, n), dtype=torch.float32, device="cuda")
    T.execute(p, A_off, T.pack(dev(B, torch.float32)), C, 1.0, 0.0)  # native: the simple kernel takes over
    assert_normwise(host(C), oracle.gemm_n(A, B), 1e-6)
    q = T.plan(m, n, k, "N", torch.float32).set_mode("bf16x6").set_tile(kernel=T.KERNEL_WIDE)
    with pytest.raises(T.TsmmError):
        T.execute(q, A_off, T.pack(dev(B, torch.float32), "N", "bf16x6"), C, 1.0, 0.0)


@pytest.mark.parametrize("mode", ["bf16x6", "bf16x3"])
def test_wide_unit_scale_shortcut_is_the_general_epilogue(mode):
    # alpha = 1, beta = 0 scales the accumulators by the column exponents in
    # binary32 (one correctly rounded ldexp); the general binary64 epilogue
    # (alpha = 1, beta = 1 on a zero C) must give the same values, also for
    # columns whose results are subnormal (scaled by 2^-140) or near the top
    # of the binary32 range (2^+120)
    m, k, n = 3000, 64, 128
    A = I.host_uniform((m, k), 91, 1, dtype=np.float32)
    B = I.host_uniform((k, n), 91, 2, dtype=np.float64)
    B[:, 5] *= 2.0 ** -140
    B[:, 9] *= 2.0 ** -132
    B[:, 70] *= 2.0 ** 120
    B = B.astype(np.float32)
    Cs = run_wide(A, B, None, 1.0, 0.0, mode)
    Cg = run_wide(A, B, np.zeros((m, n), dtype=np.float32), 1.0, 1.0, mode)
    assert np.array_equal(Cs, Cg)
    assert np.count_nonzero(np.abs(Cs[:, 5]) < 2.0 ** -126) > m // 2  # the subnormal column is exercised
    ref = oracle.gemm_n(A, B)
    normal = [j for j in range(n) if j not in (5, 9)]
    assert_normwise(Cs[:, normal], ref[:, normal], TOL[mode], mode)
