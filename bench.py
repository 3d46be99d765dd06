"""Benchmark of the pre-packed TSMM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-extras]

Workload (the headline): binary64 tall-A x small-B,
C = alpha*A*B + beta*C with m = 2^23 rows, k = n in {8, 32, 128} and
beta in {0, 1} -- six sub-cases.  B is packed once per k and reused by every
call.  A is fresh for every call: three A buffers per k, each larger than
the last-level cache, taken in turn so that no two consecutive calls of a k
(beta 0 and beta 1 of one step included) read the same A.  Every beta = 1
call computes the same contract: its C is restored from a pristine C0
(untimed device copies at the start of the step, followed by gigabytes of
other traffic before the call, so no C row is still in the last-level
cache).  One step = one execute of each of the six sub-cases.  Each execute
is timed with HIP events on the stream it runs on; the step time is the sum
of the six, so the untimed restores between steps are not counted.  The
value is the algorithmic HBM bytes of a step (A once, C once, plus C once
more when beta = 1; packing excluded, as the paper excludes it) over the
step time: GB/s, whole job.  The wall time of the bracketed steps, restores
included, is reported beside it.

Bandwidth ceilings (same run): hand-written read-only, write-only, copy
(1 read : 1 write) and 2-read : 1-write stream kernels (libtsmm_ceiling.so),
best launch shape of a small sweep, over buffers of each headline case's
own size (A and C of m = 2^23 rows of k = n = 8, 32, 128 doubles: 512 MiB,
2 GiB, 8 GiB; the rate of a plain stream falls with its buffer size, 13%
from 512 MiB to 8 GiB for a copy) and over 4 GiB for the op T extra's
reads; each headline case is also given as a fraction of the ceiling of
its own read : write mix at its own size (beta 0: copy; beta 1: 2 : 1).

Extras (same run, reported beside the headline): the 4096 x 16 latency
case, the op T split-k shape (C(64x64) = A^T B, A and B 2^22 x 64), the
binary32 precision comparison (m = 2^24, k = n = 256: binary32 products,
split-bf16 x3 / x6, binary64 on binary64 copies), the batched persistent
launch (512 uneven instances, replayed from a HIP graph), the paper's own
shape (square A 25600 x 25600 times B 25600 x N, N in {16, 64, 240}), the
runtime evaluator on a shape class the tile table does not hold, the
headline sizes with column-major operands, the reused packed A, and the
roofline kernel with all-zero A or B operands beside uniform ones (same
instructions and bytes; the difference is the operands' switching
activity, which the part's power limit turns into clock).

The `roofline` object is for the kernel that takes the most time in a step,
timed with HIP events on the stream it runs on; `cpu_baseline` times the
FP64 CPU oracle on a bounded row sample of the same workload on this host's
cores and reports the sampled error of the GPU results against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}
M_ROWS = 1 << 23
CPU_SAMPLE_ROWS = 7 << 20  # sampled rows of each sub-case: about 10 s of oracle time on 16 cores
CPU_ONE_THREAD_DIV = 32    # the one-thread leg runs 1/32 of that sample
KS = (8, 32, 128)
BETAS = (0.0, 1.0)


def opn_bytes(m, n, k, beta, sa=8, sc=8):
    return m * (k * sa + n * sc * (2 if beta != 0.0 else 1))


T_START = time.perf_counter()


def log(msg):
    """Progress line on stderr with the seconds since the start."""
    print("[bench] %s (%.1f s)" % (msg, time.perf_counter() - T_START), file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description="pre-packed TSMM benchmark")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default=None,
                    help="profile helper: run only these headline sub-cases (comma list, e.g. k128b1 or "
                         "k8b0,k128b1), after one calibration copy of known size and without the ceiling sweeps")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every launch of
    the binding goes to)."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, key, e0):
        e1 = self.torch.cuda.Event(enable_timing=True)
        e1.record()
        self.ev.append((key, e0, e1))

    def per_key_ms(self):
        self.torch.cuda.synchronize()
        out = {}
        for key, a, b in self.ev:
            out.setdefault(key, []).append(a.elapsed_time(b))
        return out


N_A_BUFFERS = 3  # A buffers per k: no two consecutive calls of a k share one


def headline(torch, T, I, args):
    """The binary64 streaming sweep: returns per-sub-case state."""
    cases = []
    for k in KS:
        n = k
        B = I.device_uniform((k, n), I.BASE_SEED, 100 + k, torch.float64)
        pk = T.pack(B)
        As = [I.device_uniform((M_ROWS, k), I.BASE_SEED, 200 + 10 * k + r, torch.float64)
              for r in range(N_A_BUFFERS)]
        for beta in BETAS:
            tag = "k%db%d" % (k, int(beta))
            if args.only and tag not in args.only.split(","):
                continue
            C = I.device_uniform((M_ROWS, n), I.BASE_SEED, 300 + 10 * k + int(beta), torch.float64)
            C0 = C.clone() if beta != 0.0 else None  # pristine copy, restored before every call
            p = T.plan(M_ROWS, n, k, "N", torch.float64)
            cases.append(dict(tag=tag, k=k, n=n, beta=beta, B=B, pk=pk, As=As, C=C, C0=C0, p=p,
                              bytes=opn_bytes(M_ROWS, n, k, beta), flops=2.0 * M_ROWS * n * k))
    return cases


def run_headline(torch, T, cases, steps, warmup):
    """Warm-up steps, then `steps` timed steps bracketed by synchronisations.
    Returns the bracketed wall time and the per-call event times."""
    timer = Timer(torch)
    step_no = [0]

    def step(record):
        # untimed: every beta != 0 case starts from its pristine C0
        for c in cases:
            if c["C0"] is not None:
                c["C"].copy_(c["C0"])
        for c in cases:
            # A index 2*step + beta (mod 3): beta 0 and beta 1 of a step, and
            # the last call of a step and the first of the next, differ
            A = c["As"][(2 * step_no[0] + int(c["beta"] != 0.0)) % N_A_BUFFERS]
            e0 = timer.start() if record else None
            T.execute(c["p"], A, c["pk"], c["C"], 1.0, c["beta"])
            if record:
                timer.stop(c["tag"], e0)
        step_no[0] += 1

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, timer.per_key_ms()


def kernel_source_hash():
    """First 16 hex digits of sha256 over the binary64 streaming kernel's sources."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_common.h", "k_stream.h", "k_stream_f64.hip"):
        with open(os.path.join(ROOT, "paper_2208_08088_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TILE_FIELDS = ("kernel", "kc", "nt", "vec", "rt", "waves", "wg_per_cu", "nsplit")


def plan_tile(describe):
    """The fields of a plan description that fix the launched kernel."""
    d = dict(f.split("=", 1) for f in describe.split() if "=" in f)
    return " ".join("%s=%s" % (f, d[f]) for f in TILE_FIELDS)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_stream_f64_headline_m2p23_pmc.txt")


def measured_traffic(case, describe):
    """HBM bytes per launch of headline sub-case `case` from the committed
    rocprofv3 counter summary, or None when it holds no figure for the
    case, or the kernel sources or the case's plan tile changed since."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(TRAFFIC_PROFILE)
              if "=" in line and not line.startswith("#"))
    if (kv.get("source_hash") != kernel_source_hash()
            or kv.get("%s.plan_tile" % case) != plan_tile(describe)):
        return None
    return float(kv["%s.traffic_bytes_per_launch" % case])


def bound_of(bytes_, flops, dt):
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_cmp = flops / (PEAK_TFLOPS[dt] * 1e12)
    return ("hbm", t_hbm) if t_hbm >= t_cmp else ("mfma", t_cmp)


CEIL_GRIDS = (256, 512, 1024, 2048, 4096)  # workgroups of 256 lanes (1 to 16 per compute unit)
CEIL_UNROLLS = (2, 4, 8)          # 16-byte vectors per lane per work item
CEIL_POLICIES = (0, 1)            # cache policy of loads / stores: default, non-temporal
CEIL_LAYOUTS = (0, 1)             # item layout: wavefronts interleaved at 1 KiB, or wave-contiguous


def ceilings(torch, nbytes=4 << 30, reps=5, detail=False):
    """Same-run bandwidth ceilings from the hand-written stream kernels of
    libtsmm_ceiling.so over `nbytes` buffers (at least twice the 256 MiB
    last-level cache): read-only, write-only, copy (1 : 1) and 2 reads :
    1 write.  For each mix the best median over the launch shapes, cache
    policies and item layouts; rates count every byte read and written."""
    import ctypes
    import itertools
    from paper_2208_08088_amd import build as B
    lib = ctypes.CDLL(B.CEIL_LIB)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.ceiling_read.argtypes = [vp, i64, vp, ci, ci, ci, ci, vp]
    lib.ceiling_write.argtypes = [vp, i64, ci, ci, ci, ci, vp]
    lib.ceiling_copy.argtypes = [vp, vp, i64, ci, ci, ci, ci, ci, vp]
    lib.ceiling_mix2.argtypes = [vp, vp, i64, ci, ci, ci, ci, ci, vp]
    n = nbytes // 8
    s0 = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    sink = torch.empty(max(CEIL_GRIDS) * 256 * 2, dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    kinds = {
        "read": (1, 0, lambda g, u, lp, sp, wl, st: lib.ceiling_read(P(s0), nbytes, P(sink), g, u, lp, wl, st)),
        "write": (0, 1, lambda g, u, lp, sp, wl, st: lib.ceiling_write(P(d), nbytes, g, u, sp, wl, st)),
        "copy": (1, 1, lambda g, u, lp, sp, wl, st: lib.ceiling_copy(P(s0), P(d), nbytes, g, u, lp, sp, wl, st)),
        "mix2": (2, 1, lambda g, u, lp, sp, wl, st: lib.ceiling_mix2(P(s0), P(d), nbytes, g, u, lp, sp, wl, st)),
    }
    out, rows = {}, []
    for name, (nr, nw, fn) in kinds.items():
        best = None
        for g, u, lp, sp, wl in itertools.product(CEIL_GRIDS, CEIL_UNROLLS, CEIL_POLICIES if nr else (0,),
                                                  CEIL_POLICIES if nw else (0,), CEIL_LAYOUTS):
            st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
            assert fn(g, u, lp, sp, wl, st) == 0, (name, g, u, lp, sp, wl)  # warm-up
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn(g, u, lp, sp, wl, st)
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            rows.append((name, g, u, lp, sp, wl, (nr + nw) * nbytes / ms / 1e6))
            if best is None or ms < best[0]:
                best = (ms, g, u, lp, sp, wl)
        ms, g, u, lp, sp, wl = best
        byt = (nr + nw) * nbytes
        out[name] = dict(reads=nr, writes=nw, bytes=byt, us=ms * 1e3, GB_s=byt / ms / 1e6,
                         hbm_frac=byt / ms / 1e6 / HBM_PEAK_GBS, grid=g, unroll=u, load_nt=lp, store_nt=sp,
                         wave_contiguous=wl)
    del s0, d, sink
    torch.cuda.empty_cache()
    out["kernel"] = ("libtsmm_ceiling.so stream kernels (two-stage register pipeline), %d MiB buffers, 16-byte "
                     "buffer loads/stores; best of %d launch shapes x cache policies x 2 item layouts"
                     % (nbytes >> 20, len(CEIL_GRIDS) * len(CEIL_UNROLLS)))
    if detail:
        out["sweep"] = rows
    return out


def calibration_copy(torch, nbytes=4 << 30):
    """One launch of the ceiling copy kernel over `nbytes` (read once,
    written once, default layout, non-temporal loads and stores): the
    kernel of known traffic that scales the HBM byte counters of a
    profiled run."""
    import ctypes
    from paper_2208_08088_amd import build as B
    lib = ctypes.CDLL(B.CEIL_LIB)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.ceiling_copy.argtypes = [vp, vp, i64, ci, ci, ci, ci, ci, vp]
    s0 = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    d = torch.empty_like(s0)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.ceiling_copy(ctypes.c_void_p(s0.data_ptr()), ctypes.c_void_p(d.data_ptr()), nbytes, 256, 4, 1, 1, 0,
                            st) == 0
    torch.cuda.synchronize()
    log("calibration copy: %d GiB read, %d GiB written" % (nbytes >> 30, nbytes >> 30))


def mfma_ceilings(torch, reps=5):
    """Same-run matrix-core ceilings (libtsmm_ceiling.so): back-to-back
    binary64 16x16x4 and bfloat16 32x32x16 products with no memory traffic,
    on operands drawn uniform in [-1, 1] and on zeros, one and two
    wavefronts per SIMD; the best median per product and operand kind.
    The part's clock falls with operand switching activity, so the
    random-operand rate is what a product kernel can sustain on such data."""
    import ctypes
    from paper_2208_08088_amd import build as B
    lib = ctypes.CDLL(B.CEIL_LIB)
    lib.ceiling_mfma.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p]
    g = torch.Generator(device="cuda")
    g.manual_seed(2208)
    operands = {
        0: {"random": torch.empty(4096, dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=g),
            "zeros": torch.zeros(4096, dtype=torch.float64, device="cuda")},
        1: {"random": torch.empty(16384, dtype=torch.float32, device="cuda").uniform_(-1, 1, generator=g)
            .to(torch.bfloat16), "zeros": torch.zeros(16384, dtype=torch.bfloat16, device="cuda")},
    }
    iters = {0: 4000, 1: 8000}
    flops_per = {0: 2048, 1: 32768}
    sink = torch.empty(512 * 256 * 2, dtype=torch.float64, device="cuda")
    out = {}
    for kind, name in ((0, "f64_16x16x4"), (1, "bf16_32x32x16")):
        row = {}
        for data, src in operands[kind].items():
            best = None
            for grid in (256, 512):
                st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
                assert lib.ceiling_mfma(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(sink.data_ptr()), kind, grid,
                                        iters[kind], st) == 0
                ts = []
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    lib.ceiling_mfma(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(sink.data_ptr()), kind, grid,
                                     iters[kind], st)
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1))
                ms = float(np.median(ts))
                tf = grid * 4 * iters[kind] * 32 * flops_per[kind] / ms / 1e9
                if best is None or tf > best[0]:
                    best = (tf, grid)
            peak = PEAK_TFLOPS["f64" if kind == 0 else "bf16"]
            row[data] = dict(TFLOP_s=best[0], peak_frac=best[0] / peak, waves_per_simd=best[1] // 256)
        out[name] = row
    del sink, operands
    torch.cuda.empty_cache()
    return out


OPT_READ_BYTES = (1 << 22) * (64 + 64) * 8  # the op T extra reads A and B, 2^22 x 64 doubles each


def extras_opt(torch, T, I, steps, warmup):
    K, m, n = 1 << 22, 64, 64
    A = I.device_normal((K, m), I.BASE_SEED, 21, torch.float64)
    B = I.device_normal((K, n), I.BASE_SEED, 22, torch.float64)
    p = T.plan(m, n, K, "T", torch.float64)
    pk = T.pack(B, "T")
    C = torch.empty((m, n), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        T.execute(p, A, pk, C, 1.0, 0.0)
    timer = Timer(torch)
    for _ in range(steps):
        e0 = timer.start()
        T.execute(p, A, pk, C, 1.0, 0.0)
        timer.stop("opt", e0)
    ms = float(np.median(timer.per_key_ms()["opt"]))
    byt = K * (m + n) * 8
    fl = 2.0 * K * m * n
    return dict(shape="A,B 2^22x64 f64, C=A^T B", plan=p.describe(), us=ms * 1e3, GB_s=byt / ms / 1e6,
                hbm_frac=byt / ms / 1e6 / HBM_PEAK_GBS, TFLOP_s=fl / ms / 1e9,
                roofline_frac=bound_of(byt, fl, "f64")[1] / (ms * 1e-3)), (A, B, C)


def extras_small(torch, T, I, calls=200):
    """The 4096 x 16 x 16 binary64 case (alpha 1.5, beta 0.5): a latency
    case, reported as microseconds per call over `calls` back-to-back calls."""
    m, k, n = 4096, 16, 16
    A = I.device_uniform((m, k), I.BASE_SEED, 11, torch.float64)
    B = I.device_uniform((k, n), I.BASE_SEED, 12, torch.float64)
    C0 = I.device_uniform((m, n), I.BASE_SEED, 13, torch.float64)
    p = T.plan(m, n, k, "N", torch.float64)
    pk = T.pack(B)
    C = C0.clone()
    T.execute(p, A, pk, C, 1.5, 0.5)
    first = C.clone()
    for _ in range(10):
        T.execute(p, A, pk, C, 1.5, 0.5)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        T.execute(p, A, pk, C, 1.5, 0.5)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / calls
    byt = opn_bytes(m, n, k, 0.5)
    # the same calls captured once in a graph (torch's CUDA-graph API on a
    # side stream; every execute is a plain kernel launch) and replayed
    per_graph = 20
    Cg = C0.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        T.execute(p, A, pk, Cg, 1.5, 0.5)  # warm the plan on the capture stream
        torch.cuda.synchronize()
        Cg.copy_(C0)
        with torch.cuda.graph(g, stream=side):
            for _ in range(per_graph):
                T.execute(p, A, pk, Cg, 1.5, 0.5)
    torch.cuda.current_stream().wait_stream(side)
    Ce = C0.clone()
    for _ in range(per_graph):
        T.execute(p, A, pk, Ce, 1.5, 0.5)
    Cg.copy_(C0)
    g.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(Cg, Ce))  # a replay gives the eager result
    replays = max(1, calls // per_graph)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    e1.synchronize()
    us_graph = e0.elapsed_time(e1) * 1e3 / (replays * per_graph)
    del g
    keep = dict(A=A.cpu().numpy(), B=B.cpu().numpy(), C0=C0.cpu().numpy(), C=first.cpu().numpy())
    return dict(shape="f64 4096x16 times 16x16, alpha 1.5, beta 0.5", plan=p.describe(), calls=calls,
                us_per_call=us, GB_s=byt / us / 1e3, graph_us_per_call=us_graph, graph_calls=replays * per_graph,
                graph_equals_eager=graph_ok, graph_GB_s=byt / us_graph / 1e3), keep


def extras_precision(torch, T, I, steps, warmup):
    m, k, n = 1 << 24, 256, 256
    A32 = I.device_col_scaled_uniform(m, k, I.BASE_SEED, 41, torch.float32)
    B32 = I.device_uniform((k, n), I.BASE_SEED, 42, torch.float32)
    out = {}
    rows = I.sample_rows(m, 4096, 17)
    idx = torch.from_numpy(rows).cuda()
    keep = {"A_rows": A32[idx].cpu().numpy(), "B": B32.cpu().numpy()}
    variants = [("f32_native", torch.float32, "native"), ("bf16x6", torch.float32, "bf16x6"),
                ("bf16x3", torch.float32, "bf16x3"), ("f64", torch.float64, "native")]
    for name, dt, mode in variants:
        if dt == torch.float64:
            A = A32.to(torch.float64)
            B = B32.to(torch.float64)
        else:
            A, B = A32, B32
        p = T.plan(m, n, k, "N", dt)
        if mode != "native":
            p.set_mode(mode)
        pk = T.pack(B, "N", mode)
        C = torch.empty((m, n), dtype=dt, device="cuda")
        for _ in range(warmup):
            T.execute(p, A, pk, C, 1.0, 0.0)
        timer = Timer(torch)
        for _ in range(max(3, steps // 4)):
            e0 = timer.start()
            T.execute(p, A, pk, C, 1.0, 0.0)
            timer.stop(name, e0)
        ms = float(np.median(timer.per_key_ms()[name]))
        s = 8 if dt == torch.float64 else 4
        byt = m * (k + n) * s
        fl = 2.0 * m * n * k
        bnd = bound_of(byt, fl, "f64" if dt == torch.float64 else ("bf16" if mode != "native" else "f32"))
        issued = {"bf16x6": 6, "bf16x3": 3}.get(name, 1) * fl
        out[name] = dict(plan=p.describe(), us=ms * 1e3, GB_s=byt / ms / 1e6, hbm_frac=byt / ms / 1e6 / HBM_PEAK_GBS,
                         TFLOP_s=fl / ms / 1e9, issued_TFLOP_s=issued / ms / 1e9,
                         roofline_frac=bnd[1] / (ms * 1e-3))
        keep[name] = C[idx].cpu().numpy()
        del A, B, C
        torch.cuda.empty_cache()
    return out, keep


def extras_square(torch, T, I, steps, warmup):
    """The paper's own workload shape: square A (25600 x 25600) times a
    tall-and-skinny B (25600 x N), binary64 and binary32, alpha 1, beta 0
    (the k-slab kernel).  GFLOP/s is the paper's figure of merit."""
    M = K = 25600
    out, keep = {}, {}
    rows = torch.from_numpy(I.sample_rows(M, 16, 23)).cuda()
    for dname, dt, peak in (("f64", torch.float64, PEAK_TFLOPS["f64"]), ("f32", torch.float32, PEAK_TFLOPS["f32"])):
        A = I.device_uniform((M, K), I.BASE_SEED, 61, dt)
        for N in (16, 64, 240):
            B = I.device_uniform((K, N), I.BASE_SEED, 62 + N, dt)
            C = torch.empty((M, N), dtype=dt, device="cuda")
            p = T.plan(M, N, K, "N", dt)
            pk = T.pack(B)
            for _ in range(warmup):
                T.execute(p, A, pk, C, 1.0, 0.0)
            timer = Timer(torch)
            for _ in range(steps):
                e0 = timer.start()
                T.execute(p, A, pk, C, 1.0, 0.0)
                timer.stop("sq", e0)
            ms = float(np.median(timer.per_key_ms()["sq"]))
            fl = 2.0 * M * N * K
            byt = (M * K + K * N + M * N) * A.element_size()
            name = "%s_n%d" % (dname, N)
            out[name] = dict(plan=p.describe(), us=ms * 1e3, TFLOP_s=fl / ms / 1e9, mfma_frac=fl / ms / 1e9 / peak,
                             GB_s=byt / ms / 1e6)
            keep[name] = (A[rows].cpu().numpy(), B.cpu().numpy(), C[rows].cpu().numpy())
            del B, C, pk
        del A
        torch.cuda.empty_cache()
    return out, keep


def extras_colmajor(torch, T, I, steps, warmup):
    """The headline sizes with column-major operands (the layout of the
    paper's analysis): binary64, m = 2^23, k = n in {8, 32, 128}, beta in
    {0, 1}; the bytes and the GB/s are counted as for the headline."""
    out = {}
    for k in KS:
        n = k
        A = I.device_uniform((k, M_ROWS), I.BASE_SEED, 400 + k, torch.float64).t()
        B = I.device_uniform((n, k), I.BASE_SEED, 410 + k, torch.float64).t()
        C = I.device_uniform((n, M_ROWS), I.BASE_SEED, 420 + k, torch.float64).t()
        pk = T.pack(B, "C")
        p = T.plan(M_ROWS, n, k, "C", torch.float64)
        for beta in BETAS:
            for _ in range(warmup):
                T.execute(p, A, pk, C, 1.0, beta)
            timer = Timer(torch)
            for _ in range(steps):
                e0 = timer.start()
                T.execute(p, A, pk, C, 1.0, beta)
                timer.stop("c", e0)
            ms = float(np.median(timer.per_key_ms()["c"]))
            byt = opn_bytes(M_ROWS, n, k, beta)
            out["k%db%d" % (k, int(beta))] = dict(plan=p.describe(), us=ms * 1e3, GB_s=byt / ms / 1e6,
                                                   hbm_frac=byt / ms / 1e6 / HBM_PEAK_GBS)
        del A, B, C, pk
        torch.cuda.empty_cache()
    return out


def extras_packed_a(torch, T, I, steps, warmup):
    """A packed once and reused (PACKA, alpha folded in): binary32 in the
    split-bf16 modes, beta = 0, fresh A (split in registers on every call,
    the plan's own kernel) against tsmm_pack_a's handle (the split-bf16
    kernel loading the pre-split terms, or the plan's wide kernel reading
    RN32(alpha*A)).  Bytes per call: 4*m*k (fresh, or the wide kernel) or
    2*terms*m*k (pre-split terms), plus 4*m*n."""
    out = {}
    for m, k, n in ((M_ROWS, 32, 32), (M_ROWS, 128, 128), (1 << 24, 256, 256)):
        A = I.device_uniform((m, k), I.BASE_SEED, 500 + k, torch.float32)
        B = I.device_uniform((k, n), I.BASE_SEED, 510 + k, torch.float32)
        C = torch.empty((m, n), dtype=torch.float32, device="cuda")
        for mode, terms in (("bf16x3", 2), ("bf16x6", 3)):
            p = T.plan(m, n, k, "N", torch.float32).set_mode(mode)
            pk = T.pack(B, "N", mode)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            pa = T.pack_a(A, mode, 1.0)
            torch.cuda.synchronize()
            pack_ms = (time.perf_counter() - w0) * 1e3
            row = dict(fresh_plan=p.describe(), pack_ms=pack_ms, packed_bytes=pa.nbytes())
            for key, fn in (("fresh", lambda: T.execute(p, A, pk, C, 1.0, 0.0)),
                            ("packed", lambda: T.execute_packed_a(p, pa, pk, C, 0.0))):
                for _ in range(warmup):
                    fn()
                timer = Timer(torch)
                for _ in range(steps):
                    e0 = timer.start()
                    fn()
                    timer.stop(key, e0)
                ms = float(np.median(timer.per_key_ms()[key]))
                # the packed call reads RN32(alpha*A) where the plan runs the
                # wide kernel, else the pre-split terms
                reads_a32 = key == "fresh" or p.info()["ran"] == "wide"
                row[key + "_ran"] = p.info()["ran"]
                byt = (4 if reads_a32 else 2 * terms) * m * k + 4 * m * n
                row[key + "_us"] = ms * 1e3
                row[key + "_GB_s"] = byt / ms / 1e6
                row[key + "_hbm_frac"] = byt / ms / 1e6 / HBM_PEAK_GBS
            row["speedup"] = row["fresh_us"] / row["packed_us"]
            out["%s_m2p%d_k%d" % (mode, m.bit_length() - 1, k)] = row
            del pa, pk
        del A, B, C
        torch.cuda.empty_cache()
    return out


def extras_tune(torch, T, I, steps, warmup):
    """The runtime evaluator on a shape class the tile table does not hold
    (binary64, m = 2^22, k = 24, n = 48): the built-in default tile against
    the tile tsmm_plan_tune keeps, and the wall time of the tuning call."""
    m, k, n = 1 << 22, 24, 48
    A = I.device_uniform((m, k), I.BASE_SEED, 71, torch.float64)
    pk = T.pack(I.device_uniform((k, n), I.BASE_SEED, 72, torch.float64))
    C = torch.empty((m, n), dtype=torch.float64, device="cuda")

    def time_plan(p):
        for _ in range(warmup):
            T.execute(p, A, pk, C, 1.0, 0.0)
        timer = Timer(torch)
        for _ in range(steps):
            e0 = timer.start()
            T.execute(p, A, pk, C, 1.0, 0.0)
            timer.stop("t", e0)
        return float(np.median(timer.per_key_ms()["t"]))

    T.tune_cache_clear()
    p = T.plan(m, n, k, "N", torch.float64)
    before = p.describe()
    t_default = time_plan(p)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    p.tune(A, pk, C, reps=3)
    tune_s = time.perf_counter() - w0
    t_tuned = time_plan(p)
    T.tune_cache_clear()
    byt = opn_bytes(m, n, k, 0.0)
    return dict(shape="f64 m=2^22 k=24 n=48 (no table entry)", default_plan=before, tuned_plan=p.describe(),
                default_us=t_default * 1e3, tuned_us=t_tuned * 1e3, default_GB_s=byt / t_default / 1e6,
                tuned_GB_s=byt / t_tuned / 1e6, tune_wall_s=tune_s)


def loop_ms(torch, T, plans, As, packs, Cs, steps, warmup):
    """Median milliseconds of one pass of single executes over every instance."""
    def one():
        for p, A, pk, C in zip(plans, As, packs, Cs):
            T.execute(p, A, pk, C, 1.0, 0.0)
    for _ in range(warmup):
        one()
    timer = Timer(torch)
    for _ in range(steps):
        e0 = timer.start()
        one()
        timer.stop("loop", e0)
    return float(np.median(timer.per_key_ms()["loop"]))


def extras_operand_activity(torch, T, I, steps, warmup):
    """The roofline kernel (binary64, m = 2^23, k = n = 128, beta 0, the
    table tile) on the same launch with uniform operands and with A or B
    all zeros: the instructions and the bytes moved are the same, only the
    switching activity of the operands changes.  A shorter time with zeros
    shows that the part's power limit, through its clock, bounds the kernel
    on real data."""
    m, k = M_ROWS, 128
    p = T.plan(m, k, k, "N", torch.float64)
    Br = I.device_uniform((k, k), I.BASE_SEED, 61, torch.float64)
    pk = {"uniform": T.pack(Br), "zero_B": T.pack(torch.zeros_like(Br))}
    pk["zero_A"] = pk["uniform"]
    Au = [I.device_uniform((m, k), I.BASE_SEED, 62 + r, torch.float64) for r in range(2)]
    Az = [torch.zeros((m, k), dtype=torch.float64, device="cuda") for _ in range(2)]
    C = torch.empty((m, k), dtype=torch.float64, device="cuda")
    timer = Timer(torch)
    for it in range(warmup + steps):
        for name in ("uniform", "zero_A", "zero_B"):
            A = (Az if name == "zero_A" else Au)[it % 2]
            e0 = timer.start()
            T.execute(p, A, pk[name], C, 1.0, 0.0)
            if it >= warmup:
                timer.stop(name, e0)
    per = {name: float(np.median(v)) * 1e3 for name, v in timer.per_key_ms().items()}
    out = dict(shape="f64 m=2^23 k=n=128, beta 0", plan=p.describe(),
               us={name: per[name] for name in ("uniform", "zero_A", "zero_B")})
    out["zero_A_speedup"] = per["uniform"] / per["zero_A"]
    out["zero_B_speedup"] = per["uniform"] / per["zero_B"]
    del Au, Az, C
    torch.cuda.empty_cache()
    return out


def extras_batched(torch, T, I, steps, warmup):
    """The 512-instance batched launch (graph replay), binary32 and bfloat16
    inputs; beside it, the same instances as 512 single executes in plain
    binary32 and in binary64 (on binary64 copies)."""
    count = 512
    ms_, ns_, ks_ = I.batched_shapes(count, I.BASE_SEED)
    sample = list(range(0, count, 64))  # instances whose first rows the CPU leg checks
    out = {}
    keep = {}
    for dname, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        As, packs, Cs = [], [], []
        byt = 0
        fl = 0.0
        t_roof = 0.0  # sum over instances of max(bytes / HBM peak, flops / matrix peak)
        for b in range(count):
            m, n, k = int(ms_[b]), int(ns_[b]), int(ks_[b])
            As.append(I.device_uniform((m, k), I.BASE_SEED, 1000 + b, dt))
            packs.append(T.pack(I.device_uniform((k, n), I.BASE_SEED, 3000 + b, dt)))
            Cs.append(torch.empty((m, n), dtype=torch.float32, device="cuda"))
            bi = m * (k * As[-1].element_size() + n * 4)
            byt += bi
            fl += 2.0 * m * n * k
            t_roof += bound_of(bi, 2.0 * m * n * k, "f32" if dt == torch.float32 else "bf16")[1]
        bp = T.plan_batched(ms_, ns_, ks_, dt)
        bp.bind(As, packs, Cs)
        g = bp.graph()
        for _ in range(warmup):
            g.launch()
        timer = Timer(torch)
        for _ in range(steps):
            e0 = timer.start()
            g.launch()
            timer.stop(dname, e0)
        ms = float(np.median(timer.per_key_ms()[dname]))
        row = dict(instances=count, plan=bp.describe(), us=ms * 1e3, GB_s=byt / ms / 1e6,
                   hbm_frac=byt / ms / 1e6 / HBM_PEAK_GBS, TFLOP_s=fl / ms / 1e9, bytes=byt,
                   roofline_us=t_roof * 1e6, roofline_frac=t_roof / (ms * 1e-3))
        torch.cuda.synchronize()
        keep[dname] = [(As[b][:1024].cpu().float().numpy(), T.unpack(packs[b]).cpu().float().numpy(),
                        Cs[b][:1024].cpu().numpy()) for b in sample]
        if dt == torch.float32:
            # the same instances one execute at a time: plain binary32 ...
            plans = [T.plan(int(ms_[b]), int(ns_[b]), int(ks_[b]), "N", dt) for b in range(count)]
            l32 = loop_ms(torch, T, plans, As, packs, Cs, steps, warmup)
            # ... and binary64 on binary64 copies of the same values
            del g, bp
            A64 = [a.double() for a in As]
            del As
            B64 = [T.pack(T.unpack(pk).double()) for pk in packs]
            del packs, Cs
            C64 = [torch.empty((int(ms_[b]), int(ns_[b])), dtype=torch.float64, device="cuda") for b in range(count)]
            plans64 = [T.plan(int(ms_[b]), int(ns_[b]), int(ks_[b]), "N", torch.float64) for b in range(count)]
            l64 = loop_ms(torch, T, plans64, A64, B64, C64, steps, warmup)
            del A64, B64, C64
            torch.cuda.empty_cache()
            row.update(loop_f32_us=l32 * 1e3, loop_f64_us=l64 * 1e3, speedup_vs_loop_f32=l32 / ms,
                       speedup_vs_loop_f64=l64 / ms)
            loops = (l32, l64)
        else:
            row.update(speedup_vs_loop_f32=loops[0] / ms, speedup_vs_loop_f64=loops[1] / ms)
            del g, bp, As, packs, Cs
            torch.cuda.empty_cache()
        out[dname] = row
    return out, keep


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(torch, I, cases, small=None):
    """The FP64 oracle on a row sample of the headline workload, on this
    host's cores (and on one core, on a smaller sample); also the sampled
    error of the GPU results, and the 4096 x 16 case checked in full."""
    import oracle
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    rows = I.sample_rows(M_ROWS, CPU_SAMPLE_ROWS, 3)
    idx = torch.from_numpy(rows).cuda()
    tot_bytes, tot_s, worst = 0, 0.0, 0.0
    per = []
    for c in cases:
        A = c["As"][0][idx].cpu().numpy()
        B = c["B"].cpu().numpy()
        C0 = c["C0s"] if "C0s" in c else None
        t0 = time.perf_counter()
        ref = oracle.gemm_n(A, B, C0, 1.0, c["beta"], threads=cores)
        dt = time.perf_counter() - t0
        tot_s += dt
        tot_bytes += opn_bytes(len(rows), c["n"], c["k"], c["beta"])
        if "Cs" in c:
            err = oracle.normwise_rel_err(c["Cs"], ref)
            worst = max(worst, err)
            per.append(dict(case=c["tag"], sample_err=err))
    # one thread, on the first rows of the same sample
    rows1 = rows[: len(rows) // CPU_ONE_THREAD_DIV]
    one_bytes, one_s = 0, 0.0
    for c in cases:
        A = c["As"][0][idx[: len(rows1)]].cpu().numpy()
        B = c["B"].cpu().numpy()
        C0 = c["C0s"][: len(rows1)] if "C0s" in c else None
        t0 = time.perf_counter()
        oracle.gemm_n(A, B, C0, 1.0, c["beta"], threads=1)
        one_s += time.perf_counter() - t0
        one_bytes += opn_bytes(len(rows1), c["n"], c["k"], c["beta"])
    out = dict(value=tot_bytes / tot_s / 1e9, unit="GB/s", cores=cores, kind="oracle",
               sample="%d sampled rows of each of the %d sub-cases (m=2^23 rows each), oracle time %.2f s"
                      % (len(rows), len(cases), tot_s),
               seconds=tot_s, cpu_model=cpu_model(), one_thread_GB_s=one_bytes / one_s / 1e9,
               one_thread_sample="%d rows of each sub-case, %.2f s" % (len(rows1), one_s),
               sample_err_max=worst, per_case=per)
    if small is not None:
        ref = oracle.gemm_n(small["A"], small["B"], small["C0"], 1.5, 0.5, threads=cores)
        out["small_4096x16_err"] = oracle.normwise_rel_err(small["C"], ref)
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2208_08088_amd import inputs as I
    from paper_2208_08088_amd import tsmm as T
    T._lib()  # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)

    if args.only:
        # profiling a single sub-case: one copy of known size for the
        # counters' calibration instead of the ceiling sweeps
        calibration_copy(torch)
        ceiling = mceil = None
    else:
        ceiling = {}
        for nb in sorted({M_ROWS * k * 8 for k in KS} | {OPT_READ_BYTES}):
            ceiling[nb] = ceilings(torch, nbytes=nb)
            log("ceilings over %d MiB: read %.0f, write %.0f, copy %.0f, 2:1 %.0f GB/s" % ((nb >> 20,) + tuple(
                ceiling[nb][kk]["GB_s"] for kk in ("read", "write", "copy", "mix2"))))
        mceil = mfma_ceilings(torch)
        log("matrix-core ceilings: f64 %.1f TF (random) / %.1f (zeros), bf16 %.0f / %.0f" % (
            mceil["f64_16x16x4"]["random"]["TFLOP_s"], mceil["f64_16x16x4"]["zeros"]["TFLOP_s"],
            mceil["bf16_32x32x16"]["random"]["TFLOP_s"], mceil["bf16_32x32x16"]["zeros"]["TFLOP_s"]))
    cases = headline(torch, T, I, args)
    log("headline cases ready: %s" % ", ".join(c["tag"] for c in cases))
    # snapshot sampled C0 rows and check one call of each case (for the CPU leg)
    rows = I.sample_rows(M_ROWS, CPU_SAMPLE_ROWS, 3)
    idx = torch.from_numpy(rows).cuda()
    for c in cases:
        c["C0s"] = c["C"][idx].cpu().numpy()
        T.execute(c["p"], c["As"][0], c["pk"], c["C"], 1.0, c["beta"])
        c["Cs"] = c["C"][idx].cpu().numpy()
    torch.cuda.synchronize()

    wall, per = run_headline(torch, T, cases, args.steps, args.warmup)
    step_bytes = sum(c["bytes"] for c in cases)
    step_ms = sum(float(np.mean(per[c["tag"]])) for c in cases)
    value = step_bytes / step_ms / 1e6
    breakdown = []
    dom = None
    for c in cases:
        msl = per[c["tag"]]
        ms = float(np.mean(msl))
        q = np.percentile(msl, [50, 90])
        bnd, t_ideal = bound_of(c["bytes"], c["flops"], "f64")
        row = dict(case=c["tag"], m=M_ROWS, k=c["k"], n=c["n"], beta=c["beta"], us=ms * 1e3,
                   GB_s=c["bytes"] / ms / 1e6, hbm_frac=c["bytes"] / ms / 1e6 / HBM_PEAK_GBS,
                   TFLOP_s=c["flops"] / ms / 1e9, bound=bnd, roofline_frac=t_ideal / (ms * 1e-3),
                   us_median=float(q[0]) * 1e3, us_min=float(np.min(msl)) * 1e3, us_p90=float(q[1]) * 1e3,
                   plan=c["p"].describe(), traffic_bytes=measured_traffic(c["tag"], c["p"].describe()))
        if ceiling is not None:
            mix = "mix2" if c["beta"] != 0.0 else "copy"
            cz = ceiling[M_ROWS * c["k"] * 8]  # A and C of this case are this size (k = n)
            row.update(mfma_ceiling_frac=c["flops"] / ms / 1e9 / mceil["f64_16x16x4"]["random"]["TFLOP_s"],
                       ceiling_mix=mix, ceiling_bytes=M_ROWS * c["k"] * 8,
                       ceiling_frac=c["bytes"] / ms / 1e6 / cz[mix]["GB_s"])
        breakdown.append(row)
        if dom is None or ms > dom[1]:
            dom = (c, ms, bnd)
    c, ms, bnd = dom
    if bnd == "hbm":
        ach, peak, unit = c["bytes"] / ms / 1e6, HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = c["flops"] / ms / 1e9, PEAK_TFLOPS["f64"], "TFLOP/s"
    pd = dict(f.split("=", 1) for f in c["p"].describe().split() if "=" in f)
    roofline = dict(kernel="%s f64 kc=%s nt=%s rt=%s nsplit=%s (%s)" % (pd["kernel"], pd["kc"], pd["nt"], pd["rt"],
                                                                   pd["nsplit"], c["tag"]), bound=bnd,
                    achieved=ach, peak=peak, unit=unit, frac=ach / peak, traffic=measured_traffic(c["tag"], c["p"].describe()),
                    per_launch_bytes=c["bytes"], per_launch_flops=c["flops"], avg_launch_us=ms * 1e3)
    log("headline done: %.1f GB/s" % value)

    result = dict(metric="TSMM GB/s (frac of HBM peak): FP64 plain vs split-BF16/FP32 at <=1e-6 rel err",
                  value=value, unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                  ms_per_step=step_ms, higher_is_better=True, scaling="weak", vs_baseline=None,
                  dtype="f64", data="synthetic",
                  config=dict(workload="binary64 tall-A x small-B, m=2^23, k=n in {8,32,128}, beta in {0,1}, "
                                       "packed B reused, fresh A per call", m=M_ROWS, k_n=list(KS),
                              betas=list(BETAS), step_bytes=step_bytes),
                  hbm_frac=value / HBM_PEAK_GBS, roofline=roofline, breakdown=breakdown,
                  timing="HIP events around each execute on its stream; step = sum of the six; beta = 1 C "
                         "restores between steps untimed",
                  wall_ms_per_step=wall / args.steps * 1e3,
                  ceilings=None if ceiling is None else {"%d_MiB" % (nb >> 20): v for nb, v in ceiling.items()},
                  mfma_ceilings=mceil)

    keep_s = None
    if not args.no_extras and not args.only:
        small, keep_s = extras_small(torch, T, I)
        log("small case done")
        opt, keep_t = extras_opt(torch, T, I, args.steps, args.warmup)
        opt["ceiling_frac"] = opt["GB_s"] / ceiling[OPT_READ_BYTES]["read"]["GB_s"]  # op T only reads
        log("op T done")
        prec, keep_p = extras_precision(torch, T, I, args.steps, args.warmup)
        for name, row in prec.items():  # issued products against the measured matrix-core rate
            key = "f64_16x16x4" if name == "f64" else ("bf16_32x32x16" if name.startswith("bf16") else None)
            if key:
                row["mfma_ceiling_frac"] = row["issued_TFLOP_s"] / mceil[key]["random"]["TFLOP_s"]
        log("precision done")
        torch.cuda.empty_cache()
        bat, keep_b = extras_batched(torch, T, I, args.steps, args.warmup)
        log("batched done")
        sq, keep_q = extras_square(torch, T, I, max(3, args.steps // 4), args.warmup)
        log("square done")
        tune = extras_tune(torch, T, I, args.steps, args.warmup)
        log("runtime evaluator done")
        colm = extras_colmajor(torch, T, I, args.steps, args.warmup)
        log("column-major done")
        pka = extras_packed_a(torch, T, I, args.steps, args.warmup)
        log("packed A done")
        act = extras_operand_activity(torch, T, I, max(3, args.steps // 4), 1)
        log("operand activity done")
        del keep_t
        result["extras"] = dict(small_4096x16=small, op_t_splitk=opt, precision_m2p24_k256=prec,
                                batched_512=bat, square_25600=sq, runtime_evaluator=tune,
                                colmajor_m2p23=colm, packed_a_reuse=pka, operand_activity_k128=act)

    if not args.no_cpu_baseline and not args.only:
        result["cpu_baseline"] = cpu_baseline(torch, I, cases, keep_s)
        if "extras" in result:
            # sampled errors of the precision variants against the oracle
            import oracle
            ref = oracle.gemm_n(keep_p["A_rows"], keep_p["B"], threads=len(os.sched_getaffinity(0)))
            for name, row in result["extras"]["precision_m2p24_k256"].items():
                row["sample_err"] = oracle.normwise_rel_err(keep_p[name], ref)
            # square A: 16 sampled rows of each case
            for name, row in result["extras"]["square_25600"].items():
                A, B, C = keep_q[name]
                row["sample_err"] = oracle.normwise_rel_err(C, oracle.gemm_n(A, B, threads=len(os.sched_getaffinity(0))))
            # batched: the first rows of every 64th instance
            for name, row in result["extras"]["batched_512"].items():
                row["sample_err"] = max(oracle.normwise_rel_err(C, oracle.gemm_n(A, B)) for A, B, C in keep_b[name])
        log("cpu baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
