"""Install-time autotuner: measures candidate tiles per shape class on this
GPU and writes the tile table that tsmm_plan reads.

    python -m paper_2208_08088_amd.autotune [--out PATH] [--classes ...]

This is the paper's install-time stage together with its performance
evaluator (AutoTSMM Sec. III; Sec. IV-A.1): for every shape class the
candidates are generated the two ways the paper describes -- a sweep of
multiples of the register tile under the capacity bounds (rows per
wavefront, resident workgroups per compute unit, column groups) and the
largest power of two that fits -- each candidate is timed on inputs larger
than the last-level cache, and the fastest one is recorded.  Candidates the
library rejects (capacity, missing instantiation) are skipped.

Timings within TIE of the fastest count as a tie.  Where column groups
share A rows (nsplit > 1) the HBM traffic depends on how many workgroups
a compute unit holds, which the timing does not see, and a tie goes to
the count that reads A least (measured with the read counters at
m = 2^23, k = n = 128 binary64, beta 0 / beta 1):
  - row-major streaming kernel: the fewest (A read 1.00x / 1.27x at one
    workgroup per CU, 1.3-1.5x / 1.7x at 2 to 16), then the fewest row
    tiles per wavefront (two read A 1.05x / 1.8x at one workgroup per CU);
  - column-major kernel: the most (1.28x / 1.00x at 16 per CU, 1.06x /
    1.41x at one).
A tile with one column group reads A once and goes first; other ties go
to the fastest tile.

The table is plain text, one entry per class (see tsmm_api.cpp), written
atomically; classes already present are kept unless --retune is given, so
an interrupted run resumes where it stopped.
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys
import time

import numpy as np
import torch

from . import inputs as I
from . import tsmm as T

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tile_table.txt")

_DT_NAME = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}
_KERNEL_NAME = {T.KERNEL_SIMPLE: "simple", T.KERNEL_STREAM: "stream", T.KERNEL_SPLITK: "splitk",
                T.KERNEL_SPLITBF16: "splitbf16", T.KERNEL_VALU64: "valu64", T.KERNEL_WIDE: "wide",
                T.KERNEL_BATCHED: "batched", T.KERNEL_SLAB: "slab", T.KERNEL_COLMAJOR: "colmajor"}


def mclass_of(m):
    return 0 if m < (1 << 16) else (1 if m < (1 << 21) else 2)


# name: (layout, dtype, mode, m, n, k) -- representative shapes of the classes
CLASSES = {
    "n_f64_k8": ("N", torch.float64, "native", 1 << 23, 8, 8),
    "n_f64_k16": ("N", torch.float64, "native", 1 << 23, 16, 16),
    "n_f64_k32": ("N", torch.float64, "native", 1 << 23, 32, 32),
    "n_f64_k64": ("N", torch.float64, "native", 1 << 23, 64, 64),
    "n_f64_k128": ("N", torch.float64, "native", 1 << 23, 128, 128),
    "n_f64_k256": ("N", torch.float64, "native", 1 << 24, 256, 256),
    "n_f32_k8": ("N", torch.float32, "native", 1 << 23, 8, 8),
    "n_f32_k16": ("N", torch.float32, "native", 1 << 23, 16, 16),
    "n_f32_k32": ("N", torch.float32, "native", 1 << 23, 32, 32),
    "n_f32_k64": ("N", torch.float32, "native", 1 << 23, 64, 64),
    "n_f32_k128": ("N", torch.float32, "native", 1 << 23, 128, 128),
    "n_f32_k256": ("N", torch.float32, "native", 1 << 24, 256, 256),
    "n_f32x6_k256": ("N", torch.float32, "bf16x6", 1 << 24, 256, 256),
    "n_f32x3_k256": ("N", torch.float32, "bf16x3", 1 << 24, 256, 256),
    "t_f64_64x64": ("T", torch.float64, "native", 64, 64, 1 << 22),
    # the paper's own shape: square A (25600 x 25600) x B (25600 x 240)
    "n_f64_sq25600": ("N", torch.float64, "native", 25600, 240, 25600),
    # column-major operands (m = 2^23)
    "c_f64_k8": ("C", torch.float64, "native", 1 << 23, 8, 8),
    "c_f64_k32": ("C", torch.float64, "native", 1 << 23, 32, 32),
    "c_f64_k128": ("C", torch.float64, "native", 1 << 23, 128, 128),
    "n_f32_sq25600": ("N", torch.float32, "native", 25600, 240, 25600),
    # batched: the 512-instance workload (m uniform in [1024, 262144], k and
    # n from {4, ..., 128}); the tile is the chunk of rows a workgroup takes
    "b_f32_512": ("B", torch.float32, "native", 512, 0, 0),
    "b_bf16_512": ("B", torch.bfloat16, "native", 512, 0, 0),
}
BATCH_CHUNKS = (512, 1024, 2048, 4096, 8192, 16384, 32768)
BATCH_WPC = (1, 2, 4)
TIE = 0.02  # relative spread of repeated timings of one tile on this part


def tie_rank(t):
    """Order among tied tiles: lower is preferred (see the module notes).
    One column group (A read once by construction) comes first."""
    if t["nsplit"] > 1 and t["kernel"] == T.KERNEL_STREAM:
        return (1, t["wg_per_cu"], t["rows_per_wave"])
    if t["nsplit"] > 1 and t["kernel"] == T.KERNEL_COLMAJOR:
        return (1, -t["wg_per_cu"], 0)
    return (0, 0, 0)


def pick(timed):
    """The chosen (ms, tile) of [(ms, tile), ...]: among the tiles within
    TIE of the fastest, the one tie_rank prefers, then the faster."""
    fastest = min(ms for ms, _ in timed)
    near = [(tie_rank(t), ms, i) for i, (ms, t) in enumerate(timed) if ms <= fastest * (1.0 + TIE)]
    return timed[min(near)[2]]
HEADLINE = ["n_f64_k8", "n_f64_k32", "n_f64_k128", "t_f64_64x64"]


def _pow2_class(x, lo, hi):
    c = lo
    while c <= hi:
        if x <= c:
            return c
        c *= 2
    return 0


def table_key(layout, dt, mode, m, n, k):
    """(kc, nt, mclass) of the table entry tsmm_plan looks up for a shape."""
    if layout == "B":
        return 0, 0, 0
    if layout == "T":
        tiles = lambda d: 1 if (d + 15) // 16 <= 1 else (2 if (d + 15) // 16 <= 2 else 4)
        return tiles(m), tiles(n), mclass_of(k)
    bf16_family = dt == torch.bfloat16 or mode != "native"
    kc = _pow2_class(k, 32, 256) if bf16_family else _pow2_class(k, 4, 256)
    return kc, _pow2_class((n + 15) // 16, 1, 16), mclass_of(m)


def natural_kernel(p):
    if p.layout == T.COLMAJOR:
        return T.KERNEL_COLMAJOR
    if p.layout == T.OP_T:
        return T.KERNEL_SPLITK
    if p.dtype == T.BF16 or p.mode != T.MODE_NATIVE:
        return T.KERNEL_SPLITBF16
    return T.KERNEL_SLAB if p.k > 256 else T.KERNEL_STREAM


def candidates(p):
    """Candidate tiles for plan p (the plan's current tile first)."""
    base = p.get_tile()
    base.pop("chunk_rows", None)  # batched plans only
    out = [dict(base)]
    # the natural family's built-in default tile, whatever the plan picked
    # (the table's tile may be a neighbour of it; the sweep is centred on
    # the default, so that a retune does not drift with the table)
    try:
        p.set_tile(kernel=natural_kernel(p))
        nat = p.get_tile()
        nat.pop("chunk_rows", None)
        out.append(dict(nat))
    except T.TsmmError:
        nat = None
    p.set_tile(**base)
    kern = nat["kernel"] if nat else None
    if kern == T.KERNEL_STREAM:
        for ns in sorted({nat["nsplit"], nat["nsplit"] * 2}):
            for rt in (1, 2, 4, 8):
                for wpc in (1, 2, 4, 8, 16):
                    out.append(dict(kernel=kern, rows_per_wave=rt, waves_per_wg=4, wg_per_cu=wpc, splitk=1, nsplit=ns))
        if p.dtype == T.F64 and p.layout == T.OP_N and p.k % 8 == 0 and p.n % 16 == 0:
            # the binary64 vector-ALU kernel (rows_per_wave = columns per wavefront)
            for nb in (16, 32):
                for wpc in (1, 2, 3, 4, 8):
                    out.append(dict(kernel=T.KERNEL_VALU64, rows_per_wave=nb, waves_per_wg=4, wg_per_cu=wpc,
                                    splitk=1, nsplit=1))
    elif kern == T.KERNEL_SPLITBF16:
        for ns in sorted({nat["nsplit"], nat["nsplit"] * 2}):
            for rt in (1, 2):
                for wpc in (1, 2, 4, 8):
                    out.append(dict(kernel=kern, rows_per_wave=rt, waves_per_wg=4, wg_per_cu=wpc, splitk=1, nsplit=ns))
    elif kern == T.KERNEL_SLAB:
        # parts of the long k range; row tiles per wavefront where an
        # instantiation exists
        for rt in (1, 2, 4):
            for sk in sorted({nat["splitk"], 1, 2, 3, 4, 5, 6, 8, 12, 16}):
                out.append(dict(kernel=kern, rows_per_wave=rt, waves_per_wg=4, wg_per_cu=1, splitk=sk, nsplit=1))
    elif kern == T.KERNEL_COLMAJOR:
        # rows_per_wave: column groups inside the workgroup (1 or 2)
        total = nat["nsplit"] * nat["rows_per_wave"]
        for ng in (1, 2):
            for ns in sorted({max(1, total // ng), max(1, 2 * total // ng)}):
                for wpc in (1, 2, 4, 8, 16):
                    out.append(dict(kernel=kern, rows_per_wave=ng, waves_per_wg=4, wg_per_cu=wpc, splitk=1,
                                    nsplit=ns))
    elif kern == T.KERNEL_SPLITK:
        for rg in (1, 2, 4):
            for P in (256, 512, 1024, 2048):
                out.append(dict(kernel=kern, rows_per_wave=rg, waves_per_wg=4, wg_per_cu=1, splitk=P, nsplit=1))
    if p.dtype == T.F32 and p.layout == T.OP_N and p.n in (128, 256) and 0 < p.k <= 256 and p.k % 8 == 0:
        # the wide kernels (32-row tiles per wavefront; 4 only at n = 128),
        # four wavefronts per workgroup, or eight with one row tile each
        for rt in ((2, 4) if p.n == 128 and p.mode == T.MODE_NATIVE else (2,)):
            out.append(dict(kernel=T.KERNEL_WIDE, rows_per_wave=rt, waves_per_wg=4, wg_per_cu=1, splitk=1, nsplit=1))
        out.append(dict(kernel=T.KERNEL_WIDE, rows_per_wave=1, waves_per_wg=8, wg_per_cu=1, splitk=1, nsplit=1))
    seen, uniq = set(), []
    for c in out:
        key = tuple(sorted(c.items()))
        if key not in seen:
            seen.add(key)
            uniq.append(c)
    return uniq


def time_plan(p, As, pk, C, beta, reps):
    """Median milliseconds of one execute (HIP events on the current stream)."""
    T.execute(p, As[0], pk, C, 1.0, beta)  # warm-up
    times = []
    for r in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        T.execute(p, As[(r + 1) % len(As)], pk, C, 1.0, beta)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def tune_batched(name, spec, reps, log):
    """Chunk size and resident workgroups per CU of the persistent batched
    launch for one dtype."""
    _, dt, _, count, _, _ = spec
    ms, ns, ks = I.batched_shapes(count, I.BASE_SEED)
    As, packs, Cs = [], [], []
    for b in range(count):
        m, n, k = int(ms[b]), int(ns[b]), int(ks[b])
        As.append(I.device_uniform((m, k), I.BASE_SEED, 1000 + b, dt))
        packs.append(T.pack(I.device_uniform((k, n), I.BASE_SEED, 3000 + b, dt)))
        Cs.append(torch.empty((m, n), dtype=torch.float32, device="cuda"))
    bp = T.plan_batched(ms, ns, ks, dt)
    bp.bind(As, packs, Cs)
    best = None
    for chunk, wpc in itertools.product(BATCH_CHUNKS, BATCH_WPC):
        try:
            bp.set_chunk_rows(chunk, wpc)
        except T.TsmmError:
            continue  # that many copies of the largest packed B do not fit the LDS
        bp.execute()  # warm-up
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            bp.execute()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms_ = float(np.median(times))
        log("  %-14s chunk_rows=%d wg_per_cu=%d  %.3f ms" % (name, chunk, wpc, ms_))
        if best is None or ms_ < best[0]:
            best = (ms_, bp.get_tile())
    t = best[1]
    entry = "B %s native 0 0 0 : batched %d %d %d %d %d %d" % (
        _DT_NAME[dt], t["rows_per_wave"], t["waves_per_wg"], t["wg_per_cu"], t["splitk"], t["nsplit"],
        t["chunk_rows"])
    del As, packs, Cs, bp
    torch.cuda.empty_cache()
    return entry, best[0]


def tune_class(name, spec, reps, log):
    layout, dt, mode, m, n, k = spec
    if layout == "B":
        return tune_batched(name, spec, reps, log)
    if layout == "N":
        if mode == "native":
            As = [I.device_uniform((m, k), I.BASE_SEED, 900 + r, dt) for r in range(2)]
            B = I.device_uniform((k, n), I.BASE_SEED, 910, dt)
        else:
            As = [I.device_col_scaled_uniform(m, k, I.BASE_SEED, 900 + r, dt) for r in range(2)]
            B = I.device_uniform((k, n), I.BASE_SEED, 910, dt)
        pk = T.pack(B, "N", mode)
        C = torch.zeros((m, n), dtype=dt if dt != torch.bfloat16 else torch.float32, device="cuda")
    elif layout == "C":  # column-major operands: transposes of contiguous tensors
        As = [I.device_uniform((k, m), I.BASE_SEED, 900 + r, dt).t() for r in range(2)]
        B = I.device_uniform((n, k), I.BASE_SEED, 910, dt).t()
        pk = T.pack(B, "C")
        C = torch.zeros((n, m), dtype=dt, device="cuda").t()
    else:
        As = [I.device_normal((k, m), I.BASE_SEED, 920 + r, dt) for r in range(2)]
        B = I.device_normal((k, n), I.BASE_SEED, 930, dt)
        pk = T.pack(B, "T")
        C = torch.zeros((m, n), dtype=dt, device="cuda")
    p = T.plan(m, n, k, layout, dt)
    if mode != "native":
        p.set_mode(mode)
    timed = []
    for cand in candidates(p):
        try:
            p.set_tile(**cand)
        except T.TsmmError:
            continue
        # op N and column-major classes are timed with beta = 0 and beta = 1 (both are used)
        ms = time_plan(p, As, pk, C, 0.0, reps)
        if layout != "T":
            ms += time_plan(p, As, pk, C, 1.0, reps)
        log("  %-14s %s  %.3f ms" % (name, " ".join("%s=%d" % kv for kv in sorted(cand.items())), ms))
        timed.append((ms, p.get_tile()))
    best = pick(timed)
    key_kc, key_nt, mcl = table_key(layout, dt, mode, m, n, k)
    entry = "%s %s %s %d %d %d : %s %d %d %d %d %d" % (
        layout, _DT_NAME[dt], mode, key_kc, key_nt, mcl, _KERNEL_NAME[best[1]["kernel"]],
        best[1]["rows_per_wave"], best[1]["waves_per_wg"], best[1]["wg_per_cu"], best[1]["splitk"],
        best[1]["nsplit"])
    del As, B, C, pk
    torch.cuda.empty_cache()
    return entry, best[0]


def read_table(path):
    entries = {}
    if os.path.exists(path):
        for line in open(path):
            body = line.split("#")[0].strip()
            if body and not body.startswith("key "):
                key = " ".join(body.split(":")[0].split())
                entries[key] = line.rstrip("\n")
    return entries


def read_key(path):
    """The key lines of a table file ('' when it has none)."""
    if not os.path.exists(path):
        return ""
    return "".join(" ".join(l.split("#")[0].split()) + "\n" for l in open(path)
                   if l.split("#")[0].strip().startswith("key "))


def write_table(path, entries, header):
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        f.write(header)
        for key in sorted(entries):
            f.write(entries[key] + "\n")
    os.replace(tmp, path)


def main(argv=None):
    ap = argparse.ArgumentParser(description="tile-table autotuner")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--classes", nargs="*", default=None, help="class names (default: all)")
    ap.add_argument("--headline", action="store_true", help="only the headline classes")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--retune", action="store_true")
    a = ap.parse_args(argv)
    names = a.classes or (HEADLINE if a.headline else list(CLASSES))
    T._lib()
    props = torch.cuda.get_device_properties(0)
    key = T.table_key(0)  # the library only uses a table whose key lines match it
    header = ("# tile table written by paper_2208_08088_amd.autotune\n"
              "# device: %s (%s, %d CUs); torch hip %s; %s\n"
              "%s"
              "# layout dtype mode kc nt mclass : kernel rows_per_wave waves_per_wg wg_per_cu splitk nsplit\n"
              % (props.name, getattr(props, "gcnArchName", "?"), props.multi_processor_count,
                 torch.version.hip, time.strftime("%Y-%m-%d"), key))
    entries = read_table(a.out)
    if entries and read_key(a.out) != key:
        log = print
        log("[autotune] %s was tuned for %r; retuning every class for %r"
            % (a.out, read_key(a.out), key), flush=True)
        entries = {}
    log = lambda s: print(s, flush=True)
    for name in names:
        spec = CLASSES[name]
        key = "%s %s %s %d %d %d" % ((spec[0], _DT_NAME[spec[1]], spec[2]) + table_key(*spec))
        if key in entries and not a.retune:
            log("[autotune] %s already in the table; kept (use --retune)" % key)
            continue
        log("[autotune] class %s" % name)
        entry, ms = tune_class(name, spec, a.reps, log)
        assert " ".join(entry.split(":")[0].split()) == key, (entry, key)
        where = ("%d batched instances" % spec[3]) if spec[0] == "B" else "x".join(str(v) for v in spec[3:])
        entries[key] = entry + "  # %.3f ms at %s%s" % (ms, where, " (beta 0 + beta 1)" if spec[0] in "NC" else "")
        write_table(a.out, entries, header)
        log("[autotune] %s -> %s (%.3f ms)" % (name, entry, ms))
    return 0


if __name__ == "__main__":
    sys.exit(main())
