"""Pins of the FP64 oracle against facts fixed by the mathematics.

The oracle computes C = alpha*A*B + beta*C0 (AutoTSMM Sec. I, Eq. (1); the
output of Algorithm 1).  None of these checks re-types the oracle's loop:
they compare it with exact rational arithmetic, closed forms, exact integer
arithmetic, an independent library routine within the textbook error bound,
and special cases that reduce to simpler operations.  Non-square shapes with
alpha != 1 and beta not in {0, 1} make a dropped term, a wrong index, a
transposed operand or a misplaced scalar fail at least one check.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2208_08088_amd import inputs as I

U64 = 2.0 ** -53


def gamma(n, u=U64):
    return n * u / (1 - n * u)


def exact_gemm_n(A, B, C0, alpha, beta):
    m, k = A.shape
    n = B.shape[1]
    out = [[None] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = sum((Fraction(A[i, l]) * Fraction(B[l, j]) for l in range(k)), Fraction(0))
            out[i][j] = Fraction(alpha) * s + (Fraction(beta) * Fraction(C0[i, j]) if beta != 0 else 0)
    return out


@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (3, 5, 2), (7, 4, 6), (5, 9, 3), (2, 17, 5)])
def test_gemm_n_against_exact_rationals(m, k, n):
    seed = 100 + m * 31 + k * 7 + n
    A = I.host_uniform((m, k), seed, 1)
    B = I.host_uniform((k, n), seed, 2)
    C0 = I.host_uniform((m, n), seed, 3)
    alpha, beta = 1.3, -0.7
    C = oracle.gemm_n(A, B, C0, alpha, beta)
    ex = exact_gemm_n(A, B, C0, alpha, beta)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(m):
        for j in range(n):
            # sum: gamma_k; times alpha: 1 rounding; beta*c0: 1; final add: 1
            bound = gamma(k + 2) * abs(alpha) * absAB[i, j] + gamma(2) * abs(beta * C0[i, j])
            err = abs(Fraction(C[i, j]) - ex[i][j])
            assert err <= Fraction(bound) * (1 + 1e-12) + Fraction(2.0 ** -1070), (i, j)


@pytest.mark.parametrize("K,m,n", [(1, 1, 1), (6, 3, 2), (11, 4, 5), (33, 2, 3)])
def test_gemm_t_against_exact_rationals(K, m, n):
    seed = 200 + K + m + n
    A = I.host_uniform((K, m), seed, 1)
    B = I.host_uniform((K, n), seed, 2)
    C0 = I.host_uniform((m, n), seed, 3)
    alpha, beta = -0.9, 0.3
    C = oracle.gemm_t(A, B, C0, alpha, beta)
    ex = exact_gemm_n(np.ascontiguousarray(A.T), B, C0, alpha, beta)
    absAB = np.abs(A.T) @ np.abs(B)
    for i in range(m):
        for j in range(n):
            bound = gamma(K + 2) * abs(alpha) * absAB[i, j] + gamma(2) * abs(beta * C0[i, j])
            assert abs(Fraction(C[i, j]) - ex[i][j]) <= Fraction(bound) * (1 + 1e-12) + Fraction(2.0 ** -1070)


def test_small_integers_bit_exact():
    # |partial sums| stay far below 2^53, alpha and beta are dyadic: every
    # operation is exact, so the result equals exact integer arithmetic.
    m, k, n = 37, 13, 11
    A = I.host_ints((m, k), 7, 1, -8, 8)
    B = I.host_ints((k, n), 7, 2, -8, 8)
    C0 = I.host_ints((m, n), 7, 3, -8, 8)
    C = oracle.gemm_n(A, B, C0, 1.5, 0.5)
    Ai, Bi, Ci = A.astype(int).tolist(), B.astype(int).tolist(), C0.astype(int).tolist()
    for i in range(m):
        for j in range(n):
            s = sum(Ai[i][l] * Bi[l][j] for l in range(k))
            exp = Fraction(3, 2) * s + Fraction(1, 2) * Ci[i][j]
            assert Fraction(C[i, j]) == exp


def test_small_integers_bit_exact_op_t():
    K, m, n = 41, 6, 9
    A = I.host_ints((K, m), 8, 1, -8, 8)
    B = I.host_ints((K, n), 8, 2, -8, 8)
    C0 = I.host_ints((m, n), 8, 3, -8, 8)
    C = oracle.gemm_t(A, B, C0, -2.0, 0.25)
    Ai, Bi = A.astype(int), B.astype(int)
    exp = (-2 * (Ai.T.astype(object) @ Bi.astype(object))) + C0.astype(object) * Fraction(1, 4)
    assert all(Fraction(C[i, j]) == exp[i, j] for i in range(m) for j in range(n))


@pytest.mark.parametrize("k", [1, 16, 255])
def test_all_ones_closed_form(k):
    m, n = 9, 6
    A = np.ones((m, k))
    B = np.ones((k, n))
    C0 = I.host_uniform((m, n), 11, 3)
    alpha, beta = 1.5, 0.5
    C = oracle.gemm_n(A, B, C0, alpha, beta)
    # sum of k ones is exactly k; then RN(k*alpha) + RN(beta*c0)
    assert np.array_equal(C, (k * alpha) + beta * C0)
    Ct = oracle.gemm_t(np.ones((k, m)), np.ones((k, n)), C0, alpha, beta)
    assert np.array_equal(Ct, (k * alpha) + beta * C0)


def test_identity_B_closed_form():
    m, k = 23, 16
    A = I.host_uniform((m, k), 12, 1)
    C0 = I.host_uniform((m, k), 12, 3)
    C = oracle.gemm_n(A, np.eye(k), C0, 1.5, 0.5)
    # every dot product has one nonzero term: s == a exactly
    assert np.array_equal(C, 1.5 * A + 0.5 * C0)


def test_stacked_identity_op_t():
    reps, d = 8, 16
    A = np.tile(np.eye(d), (reps, 1))  # K x d with K = reps*d
    C = oracle.gemm_t(A, A, None, 1.5, 0.0)
    assert np.array_equal(C, reps * 1.5 * np.eye(d))


def test_against_library_matmul_within_bound():
    # numpy's matmul is an independent implementation; both must lie within
    # gamma_k |A||B| of the exact result, hence within 2*gamma_k of each other.
    m, k, n = 300, 64, 40
    A = I.host_normal((m, k), 13, 1)
    B = I.host_normal((k, n), 13, 2)
    C = oracle.gemm_n(A, B)
    bound = 2 * gamma(k) * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(C - A @ B) <= bound)
    K2 = 500
    At = I.host_normal((K2, 12), 13, 4)
    Bt = I.host_normal((K2, 7), 13, 5)
    Ct = oracle.gemm_t(At, Bt)
    assert np.all(np.abs(Ct - At.T @ Bt) <= 2 * gamma(K2) * (np.abs(At.T) @ np.abs(Bt)))


def test_op_t_is_op_n_of_the_transpose():
    K, m, n = 77, 10, 13
    A = I.host_uniform((K, m), 14, 1)
    B = I.host_uniform((K, n), 14, 2)
    C0 = I.host_uniform((m, n), 14, 3)
    # same products summed in the same (ascending) order: bitwise equal
    assert np.array_equal(oracle.gemm_t(A, B, C0, 0.75, -1.25),
                          oracle.gemm_n(np.ascontiguousarray(A.T), B, C0, 0.75, -1.25))


def test_blas_conventions():
    m, k, n = 5, 4, 3
    A = I.host_uniform((m, k), 15, 1)
    B = I.host_uniform((k, n), 15, 2)
    nanC = np.full((m, n), np.nan)
    # beta == 0: C0 is never read
    C = oracle.gemm_n(A, B, nanC, 2.0, 0.0)
    assert np.all(np.isfinite(C))
    # alpha == 0: A and B are never read, C = beta*C0
    C0 = I.host_uniform((m, n), 15, 3)
    C = oracle.gemm_n(np.full((m, k), np.nan), np.full((k, n), np.nan), C0, 0.0, 0.5)
    assert np.array_equal(C, 0.5 * C0)
    # k == 0: C = beta*C0
    C = oracle.gemm_n(np.zeros((m, 0)), np.zeros((0, n)), C0, 3.0, -2.0)
    assert np.array_equal(C, -2.0 * C0)
    # empty outputs
    assert oracle.gemm_n(np.zeros((0, k)), B).shape == (0, n)
    assert oracle.gemm_n(A, np.zeros((k, 0))).shape == (m, 0)


def test_thread_count_does_not_change_bits():
    m, k, n = 257, 33, 17
    A = I.host_normal((m, k), 16, 1)
    B = I.host_normal((k, n), 16, 2)
    C0 = I.host_normal((m, n), 16, 3)
    c1 = oracle.gemm_n(A, B, C0, 1.5, 0.5, threads=1)
    c8 = oracle.gemm_n(A, B, C0, 1.5, 0.5, threads=8)
    assert c1.tobytes() == c8.tobytes()
    t1 = oracle.gemm_t(A, A, None, 1.0, 0.0, threads=1)
    t8 = oracle.gemm_t(A, A, None, 1.0, 0.0, threads=5)
    assert t1.tobytes() == t8.tobytes()


def test_normwise_error_helper():
    C = np.array([[3.0, 4.0]])
    assert oracle.normwise_rel_err(C, C) == 0.0
    assert oracle.normwise_rel_err(np.array([[3.0, 4.0 + 5.0]]), C) == pytest.approx(1.0)
    assert oracle.normwise_rel_err(np.zeros((1, 2)), np.zeros((1, 2))) == 0.0
    assert oracle.normwise_rel_err(np.ones((1, 2)), np.zeros((1, 2))) == float("inf")


# ------------------------------------------------------------ bf16 split

def _golden_split_cases():
    path = os.path.join(os.path.dirname(__file__), "golden", "bf16_split_cases.txt")
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        rows.append(tuple(int(v, 16) for v in f[:4]))
    return rows


def test_split_bf16_hand_worked_cases():
    rows = _golden_split_cases()
    assert len(rows) >= 6
    x = np.array([r[0] for r in rows], dtype=np.uint32).view(np.float32)
    planes = oracle.split_bf16(x, 3)
    for idx, r in enumerate(rows):
        assert tuple(int(planes[t, idx]) for t in range(3)) == r[1:], hex(r[0])


def _bf16_to_f64(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_split_bf16_three_terms_are_exact():
    # hi + mid + lo == x for normal binary32 x across the exponent range
    # (24 significand bits fit in three 8-bit terms; residuals are exact)
    mant = I.host_uniform((4000,), 17, 1, 1.0, 2.0)
    ex = I.host_ints((4000,), 17, 2, -100, 100).astype(np.int64)
    sign = np.where(I.host_ints((4000,), 17, 3, 0, 1) > 0, 1.0, -1.0)
    x = (sign * np.ldexp(mant, ex)).astype(np.float32)
    p = oracle.split_bf16(x, 3)
    rec = _bf16_to_f64(p[0]) + _bf16_to_f64(p[1]) + _bf16_to_f64(p[2])
    assert np.array_equal(rec, x.astype(np.float64))
    # each term is at most half an ulp of the previous one
    for t in (1, 2):
        prev = np.abs(_bf16_to_f64(p[t - 1]))
        assert np.all(np.abs(_bf16_to_f64(p[t])) <= prev * 2.0 ** -8)
    # two terms keep 16 significand bits: relative error below 2^-16
    two = _bf16_to_f64(p[0]) + _bf16_to_f64(p[1])
    assert np.all(np.abs(two - x) <= np.abs(x.astype(np.float64)) * 2.0 ** -16)


def test_split_bf16_representable_values_need_one_term():
    bits = I.host_ints((1000,), 18, 1, 0x0080, 0x7F7F).astype(np.uint16)  # finite normal bf16
    x = (bits.astype(np.uint32) << 16).view(np.float32)
    p = oracle.split_bf16(x, 3)
    assert np.array_equal(p[0], bits)
    assert not p[1].any() and not p[2].any()


def test_split_bf16_agrees_with_generator_rounding():
    # the input generator's own bf16 rounding is a separate implementation of
    # the same rule
    x = I.host_uniform((5000,), 19, 1, -3.0, 3.0, dtype=np.float32)
    assert np.array_equal(oracle.split_bf16(x, 1)[0], I.f32_to_bf16_bits(x))


def test_column_scale_exponent():
    B = np.array([[0.5, 3.0, 0.0, 1.0, -2.0 ** -120],
                  [0.25, -5.0, 0.0, 1.999, 2.0 ** -121]], dtype=np.float32)
    assert oracle.column_scale_exp(B).tolist() == [-1, 2, 0, 0, -120]
    B2 = I.host_uniform((64, 32), 20, 1, dtype=np.float32) * np.float32(1000.0)
    e = oracle.column_scale_exp(B2)
    mx = np.max(np.abs(B2), axis=0).astype(np.float64)
    assert np.all((mx * 2.0 ** -e.astype(np.float64) >= 1.0) & (mx * 2.0 ** -e.astype(np.float64) < 2.0))


# --- PACKA (Algorithm 1: A scaled by alpha as it is packed) ---------------

def _rn(alpha, a, to32):
    # the product in exact rational arithmetic, rounded once to binary64
    # (float() of a Fraction rounds correctly), then to binary32
    x = float(Fraction(alpha) * Fraction(float(a)))
    return np.float32(x) if to32 else x


@pytest.mark.parametrize("alpha", [3.0, -0.7, 1e-3])
def test_pack_a_scaling_against_exact_rationals(alpha):
    A64 = I.host_uniform((7, 9), 21, 1, -4.0, 4.0)
    A32 = I.host_uniform((7, 9), 21, 2, -4.0, 4.0, dtype=np.float32)
    P64 = oracle.pack_a(A64, alpha)
    P32 = oracle.pack_a(A32, alpha)
    assert P64.dtype == np.float64 and P32.dtype == np.float32
    for i in range(7):
        for j in range(9):
            assert P64[i, j] == _rn(alpha, A64[i, j], False)
            assert P32[i, j] == _rn(alpha, A32[i, j], True)


def test_pack_a_unit_scale_is_the_plain_split():
    A = I.host_uniform((33, 40), 22, 1, -2.0, 2.0, dtype=np.float32)
    for terms in (2, 3):
        assert np.array_equal(oracle.pack_a(A, 1.0, terms), oracle.split_bf16(A, terms))
    assert np.array_equal(oracle.pack_a(A, 1.0), A)


def test_pack_a_power_of_two_shifts_exponents():
    # alpha = 2^-3 moves every nonzero term's exponent field down by 3 and
    # changes no significand bit (values stay far from the subnormal range)
    A = I.host_uniform((50, 24), 23, 1, -8.0, 8.0, dtype=np.float32)
    base = oracle.split_bf16(A, 3).astype(np.int32)
    got = oracle.pack_a(A, 2.0 ** -3, 3).astype(np.int32)
    nz = (base & 0x7FFF) != 0
    assert np.array_equal(got[~nz], base[~nz])
    assert np.array_equal(got[nz], base[nz] - (3 << 7))


def test_pack_a_split_reconstructs_the_scaled_value():
    A = I.host_uniform((64, 16), 24, 1, -1.0, 1.0, dtype=np.float32)
    alpha = 1.37
    p = oracle.pack_a(A, alpha, 3)
    rec = _bf16_to_f64(p[0]) + _bf16_to_f64(p[1]) + _bf16_to_f64(p[2])
    for i in range(0, 64, 7):
        for j in range(16):
            assert rec[i, j] == float(_rn(alpha, A[i, j], True))


def _two_product(a, b):
    """Error-free product (Dekker, with Veltkamp's split): a*b == p + e
    exactly for binary64 a, b far from overflow and underflow."""
    c = 134217729.0  # 2^27 + 1
    t = c * a
    ah = t - (t - a)
    al = a - ah
    t = c * b
    bh = t - (t - b)
    bl = b - bh
    p = a * b
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def test_two_product_is_exact():
    # checked against exact rationals on random pairs
    a = I.host_normal((64,), 5, 1)
    b = I.host_normal((64,), 5, 2) * 1e3
    p, e = _two_product(a, b)
    for x, y, pp, ee in zip(a, b, p, e):
        assert Fraction(x) * Fraction(y) == Fraction(pp) + Fraction(ee)


def test_op_t_oracle_error_at_the_full_reduction_length():
    # The reduction workload's shared dimension is K = 2^22 with normal(0, 1)
    # entries, where the GPU bar is a normwise relative error of 1e-12.  The
    # oracle sums in binary64 recursively (one rounding per step); here its
    # outputs are compared with the correctly rounded exact dot products
    # (every product split exactly into two binary64 values, the 2K terms
    # summed exactly by math.fsum).  Each output lies within the textbook
    # bound gamma_K * sum|a*b|, and the normwise error is far below 1e-12,
    # so the oracle can referee that bar.  (Each output depends only on its
    # own columns, so a 4-column slice gives the full problem's bits.)
    import math
    K = 1 << 22
    A = I.host_normal((K, 4), I.BASE_SEED, 21)
    B = I.host_normal((K, 4), I.BASE_SEED, 22)
    C = oracle.gemm_t(A, B)
    exact = np.empty((4, 4))
    absum = np.empty((4, 4))
    for i in range(4):
        for j in range(4):
            p, e = _two_product(A[:, i], B[:, j])
            exact[i, j] = math.fsum(np.concatenate([p, e]).tolist())
            absum[i, j] = math.fsum(np.abs(p).tolist())
    gam = K * 2.0 ** -53 / (1 - K * 2.0 ** -53)
    assert np.all(np.abs(C - exact) <= gam * absum * (1 + 1e-6))
    err = np.linalg.norm(C - exact) / np.linalg.norm(exact)
    print("oracle normwise error at K = 2^22 (normal inputs): %.2e" % err)
    assert 0.0 < err <= 2e-13
