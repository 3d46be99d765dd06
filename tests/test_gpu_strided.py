"""GPU parity of strided operands (tsmm_execute_ld): A and C as views into
wider buffers (leading dimensions larger than the natural ones), for each
kernel family and layout, against the FP64 oracle; the padding between
rows (columns) of C is never written."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def view_rows(x, pad, dtype):
    """x (r x c) as a row-major view with row stride c + pad."""
    r, c = x.shape
    buf = torch.full((r, c + pad), 777.0, dtype=dtype, device="cuda")
    buf[:, :c] = torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()
    return buf, buf[:, :c]


def view_cols(x, pad, dtype):
    """x (r x c) as a column-major view with column stride r + pad."""
    r, c = x.shape
    buf = torch.full((c, r + pad), 777.0, dtype=dtype, device="cuda")
    buf[:, :r] = torch.from_numpy(np.ascontiguousarray(x.T)).to(dtype).cuda()
    return buf, buf[:, :r].t()


# (layout, dtype, m, n, k, kernel to force or None, A pad, C pad)
CASES = [
    ("N", torch.float64, 5000, 32, 32, T.KERNEL_STREAM, 8, 6),       # vector mapping, interleaved columns
    ("N", torch.float64, 5000, 32, 32, T.KERNEL_STREAM, 3, 5),       # odd strides: any-shape fallback
    ("N", torch.float32, 3000, 64, 40, T.KERNEL_STREAM, 4, 12),
    ("N", torch.float64, 900, 64, 1000, T.KERNEL_SLAB, 24, 2),       # k-slab, split k
    ("N", torch.float32, 700, 128, 600, T.KERNEL_SLAB, 8, 4),
    ("N", torch.float32, 4000, 128, 64, T.KERNEL_WIDE, 8, 8),        # wide kernel: any-shape fallback
    ("N", torch.bfloat16, 2000, 64, 64, None, 8, 4),                 # bfloat16 inputs: fallback
    ("T", torch.float64, 64, 64, 5000, None, 16, 8),                 # op T split-k: fallback
    ("C", torch.float64, 4000, 32, 32, None, 6, 10),                 # column-major kernel
    ("C", torch.float32, 4000, 16, 16, None, 8, 4),
]


@pytest.mark.parametrize("layout,dtype,m,n,k,kernel,pa,pc", CASES)
def test_strided_against_oracle(layout, dtype, m, n, k, kernel, pa, pc):
    f = np.float32 if dtype != torch.float64 else np.float64
    seed = 9000 + m + n + k + pa
    if dtype == torch.bfloat16:
        A = I.bf16_bits_to_f32(I.host_bf16_uniform((m, k), seed, 1)).astype(np.float32)
        B = I.bf16_bits_to_f32(I.host_bf16_uniform((k, n), seed, 2)).astype(np.float32)
        out_dt = torch.float32
    else:
        A = I.host_uniform((k, m) if layout == "T" else (m, k), seed, 1, dtype=f)
        B = I.host_uniform((k, n), seed, 2, dtype=f)
        out_dt = dtype
    C0 = I.host_uniform((m, n), seed, 3, dtype=np.float32 if out_dt == torch.float32 else np.float64)
    if layout == "C":
        _, Av = view_cols(A, pa, dtype)
        cbuf, Cv = view_cols(C0, pc, out_dt)
        Bd = torch.from_numpy(np.ascontiguousarray(B.T)).to(dtype).cuda().t()
    else:
        _, Av = view_rows(A, pa, dtype)
        cbuf, Cv = view_rows(C0, pc, out_dt)
        Bd = torch.from_numpy(np.ascontiguousarray(B)).to(dtype).cuda()
    p = T.plan(m, n, k, layout, dtype)
    if kernel is not None:
        p.set_tile(kernel=kernel)
    pk = T.pack(Bd, layout)
    announce("strided", layout, dtype, m, n, k, pa, pc, p.describe())
    T.execute(p, Av, pk, Cv, 1.5, 0.5)
    want = oracle.gemm_t(A, B, C0, 1.5, 0.5) if layout == "T" else oracle.gemm_n(A, B, C0, 1.5, 0.5)
    tol = 1e-12 if dtype == torch.float64 else (1e-5 if dtype == torch.bfloat16 else 1e-6)
    assert_normwise(host(Cv), want, tol, p.describe())
    # the padding of C is untouched
    pad = cbuf[:, m:] if layout == "C" else cbuf[:, n:]
    assert bool((pad == 777.0).all())


def test_strides_below_natural_and_split_modes():
    m, k, n = 1000, 32, 32
    A = torch.zeros((m, k + 4), dtype=torch.float32, device="cuda")
    C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    pk = T.pack(torch.zeros((k, n), dtype=torch.float32, device="cuda"), "N", "bf16x6")
    p = T.plan(m, n, k, "N", torch.float32).set_mode("bf16x6")
    with pytest.raises(T.TsmmError) as e:
        T.execute(p, A[:, :k], pk, C)  # split modes need natural strides
    assert e.value.status == T.INVALID_VALUE
    lib = T._lib()
    q = T.plan(m, n, k, "N", torch.float32)
    pq = T.pack(torch.zeros((k, n), dtype=torch.float32, device="cuda"))
    st = lib.tsmm_execute_ld(q.handle, A.data_ptr(), k - 1, pq.handle, C.data_ptr(), n, 1.0, 0.0)
    assert st == T.INVALID_VALUE


def test_huge_strides_take_the_any_shape_kernel():
    # strides beyond 2^26 bytes: 16 rows of a tile would span more than the
    # out-of-range lane offset, so the plan runs the any-shape kernel; the
    # result matches the oracle and nothing between the rows is written
    m, n, k = 40, 8, 8
    ld = 1 << 24  # binary64 elements: 15 rows of C span 2^31 bytes
    A = I.host_uniform((m, k), 9100, 1)
    B = I.host_uniform((k, n), 9100, 2)
    C0 = I.host_uniform((m, n), 9100, 3)
    announce("huge strides", m, n, k, ld)
    abuf = torch.zeros((m, ld), dtype=torch.float64, device="cuda")
    abuf[:, :k] = torch.from_numpy(A).cuda()
    cbuf = torch.full((m, ld), 777.0, dtype=torch.float64, device="cuda")
    cbuf[:, :n] = torch.from_numpy(C0).cuda()
    p = T.plan(m, n, k, "N", torch.float64)
    T.execute(p, abuf[:, :k], T.pack(torch.from_numpy(B).cuda()), cbuf[:, :n], 1.5, 0.5)
    assert_normwise(host(cbuf[:, :n]), oracle.gemm_n(A, B, C0, 1.5, 0.5), 1e-12)
    assert int((cbuf[:, n:] != 777.0).sum().item()) == 0
    del abuf, cbuf
    torch.cuda.empty_cache()
