"""GPU parity of every tile the install-time table hands out, at the size
of the class it was tuned for (AutoTSMM Sec. III: the install-time stage
picks the strategy; Eq. (1) / Algorithm 1's output line fix the result).

For each table entry the plan is built at the class's representative shape
(the autotuner's), its tile must be the table's, and the result is checked
against the FP64 oracle on sampled rows (rows are independent in op N, so
the sampled error is exact for those rows; op T is checked in full), with
alpha = 1.5 and beta in {0, 0.5}.  beta = 0 runs on a C full of NaN, which
must never be read.  Tolerances: binary64 1e-12 normwise; binary32
products max(1e-6, 2^-24 sqrt(k)); split-bf16 x6 1e-6; x3 2e-5 (its
two-term split is good to about 2^-16 per term)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2208_08088_amd import autotune as AT
from paper_2208_08088_amd import inputs as I
from paper_2208_08088_amd import tsmm as T
from tests._gpu_util import announce, assert_normwise, host, need_gpu

pytestmark = pytest.mark.gpu

_KERNEL_ID = {v: k for k, v in AT._KERNEL_NAME.items()}
TILE_FIELDS = ("rows_per_wave", "waves_per_wg", "wg_per_cu", "splitk", "nsplit")


def table_entries():
    """(class name, spec, expected tile) for every entry of the shipped table."""
    entries = AT.read_table(AT.DEFAULT_TABLE)
    out = []
    for name, spec in AT.CLASSES.items():
        key = "%s %s %s %d %d %d" % ((spec[0], AT._DT_NAME[spec[1]], spec[2]) + AT.table_key(*spec))
        if key not in entries:
            continue
        f = entries[key].split("#")[0].split(":")[1].split()
        tile = dict(kernel=_KERNEL_ID[f[0]], **dict(zip(TILE_FIELDS, map(int, f[1:6]))))
        if spec[0] == "B":
            tile["chunk_rows"] = int(f[6])
        out.append((name, spec, tile))
    return out


ENTRIES = table_entries()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_every_table_entry_is_collected():
    # the shipped table is not empty and every entry maps to a class
    assert len(ENTRIES) == len(AT.read_table(AT.DEFAULT_TABLE)) > 0


def tolerance(dt, mode, k):
    if dt == torch.float64:
        return 1e-12
    if mode == "bf16x6":
        return 1e-6
    if mode == "bf16x3":
        return 2e-5
    return max(1e-6, 2.0 ** -24 * math.sqrt(k))


def check_tile(p, tile):
    got = p.get_tile()
    assert p.info()["table"] == "1", p.describe()
    assert got["kernel"] == tile["kernel"], (p.describe(), tile)
    for f in TILE_FIELDS:
        if f == "splitk" and tile["kernel"] not in (T.KERNEL_SPLITK, T.KERNEL_SLAB):
            continue
        assert got[f] == tile[f], (f, p.describe(), tile)


def _sel(layouts):
    return pytest.mark.parametrize("name,spec,tile", [e for e in ENTRIES if e[1][0] in layouts],
                                   ids=[e[0] for e in ENTRIES if e[1][0] in layouts])


@_sel("NC")
def test_table_tile_op_n_and_colmajor(name, spec, tile):
    layout, dt, mode, m, n, k = spec
    colm = layout == "C"
    square = k > 256
    rows = I.sample_rows(m, 256 if square else 4096, 31)
    idx = torch.from_numpy(rows).cuda()
    seed = 7000 + k + n + (1 if colm else 0)
    if colm:  # column-major matrices are transposes of contiguous tensors
        A = I.device_uniform((k, m), I.BASE_SEED, seed, dt).t()
        Bd = I.device_uniform((n, k), I.BASE_SEED, seed + 1, dt).t()
        C = I.device_uniform((n, m), I.BASE_SEED, seed + 2, dt).t()
    elif mode != "native":
        A = I.device_col_scaled_uniform(m, k, I.BASE_SEED, seed, dt)
        Bd = I.device_uniform((k, n), I.BASE_SEED, seed + 1, dt)
        C = I.device_uniform((m, n), I.BASE_SEED, seed + 2, dt)
    else:
        A = I.device_uniform((m, k), I.BASE_SEED, seed, dt)
        Bd = I.device_uniform((k, n), I.BASE_SEED, seed + 1, dt)
        C = I.device_uniform((m, n), I.BASE_SEED, seed + 2, dt)
    p = T.plan(m, n, k, layout, dt)
    if mode != "native":
        p.set_mode(mode)
    check_tile(p, tile)
    pk = T.pack(Bd, layout, mode)
    As, Bh = host(A[idx]), host(Bd)
    tol = tolerance(dt, mode, k)
    for beta in (0.5, 0.0):
        announce("table entry", name, p.describe(), "beta", beta)
        if beta == 0.0:
            C.fill_(float("nan"))
            C0s = None
        else:
            C0s = host(C[idx])
        T.execute(p, A, pk, C, 1.5, beta)
        got = host(C[idx])
        assert np.all(np.isfinite(got)), (name, beta)
        ref = oracle.gemm_n(As, Bh, C0s, 1.5, beta)
        err = assert_normwise(got, ref, tol, "%s beta %g" % (name, beta))
        print("[table] %s beta %g: %s sampled normwise error %.3e (bar %.1e)" % (name, beta, p.describe(), err, tol))
    del A, Bd, C, pk
    torch.cuda.empty_cache()


def test_headline_k128_plan_is_the_table_tile():
    # the binary64 k = n = 128 plan behind the headline's largest sub-case
    entries = {e[0]: e[2] for e in ENTRIES}
    if "n_f64_k128" not in entries:
        pytest.skip("no table entry for binary64 k = n = 128")
    p = T.plan(1 << 23, 128, 128, "N", torch.float64)
    check_tile(p, entries["n_f64_k128"])
    assert p.info()["nsplit"] == str(entries["n_f64_k128"]["nsplit"])


@_sel("T")
def test_table_tile_op_t(name, spec, tile):
    layout, dt, mode, m, n, k = spec
    A = I.device_normal((k, m), I.BASE_SEED, 7100, dt)
    Bd = I.device_normal((k, n), I.BASE_SEED, 7101, dt)
    C = I.device_normal((m, n), I.BASE_SEED, 7102, dt)
    p = T.plan(m, n, k, "T", dt)
    check_tile(p, tile)
    pk = T.pack(Bd, "T")
    Ah, Bh = host(A), host(Bd)
    for beta in (0.5, 0.0):
        announce("table entry", name, p.describe(), "beta", beta)
        if beta == 0.0:
            C.fill_(float("nan"))
            C0 = None
        else:
            C0 = host(C)
        T.execute(p, A, pk, C, 1.5, beta)
        got = host(C)
        ref = oracle.gemm_t(Ah, Bh, C0, 1.5, beta)
        err = assert_normwise(got, ref, 1e-12, "%s beta %g" % (name, beta))
        print("[table] %s beta %g: %s normwise error %.3e" % (name, beta, p.describe(), err))


@_sel("B")
def test_table_tile_batched(name, spec, tile):
    # the 512-instance workload with the table's chunk size; every 16th
    # instance checked on its first and last rows
    _, dt, _, count, _, _ = spec
    ms, ns, ks = I.batched_shapes(count, I.BASE_SEED)
    As, Bs, packs, Cs = [], [], [], []
    for b in range(count):
        m, n, k = int(ms[b]), int(ns[b]), int(ks[b])
        As.append(I.device_uniform((m, k), I.BASE_SEED, 9000 + b, dt))
        Bs.append(I.device_uniform((k, n), I.BASE_SEED, 9600 + b, dt))
        packs.append(T.pack(Bs[-1]))
        Cs.append(torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda"))
    bp = T.plan_batched(ms, ns, ks, dt)
    got = bp.get_tile()
    assert got["chunk_rows"] == tile["chunk_rows"] and "table=1" in bp.describe(), bp.describe()
    announce("table entry", name, bp.describe())
    bp.execute(As, packs, Cs)
    worst = 0.0
    for b in range(0, count, 16):
        m = int(ms[b])
        sel = torch.tensor([0, 1, m // 2, m - 2, m - 1], device="cuda")
        A = host(As[b][sel])
        ref = oracle.gemm_n(A, host(Bs[b]))
        worst = max(worst, assert_normwise(host(Cs[b][sel]), ref, 1e-5 if dt == torch.bfloat16 else 1e-6,
                                           "instance %d" % b))
    print("[table] %s: worst sampled normwise error %.3e" % (name, worst))
