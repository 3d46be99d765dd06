"""Seeded synthetic inputs for the TSMM tests and benchmark.

This module holds no arithmetic of the multiply itself: it only draws
matrices.  It is the one piece of code that both the oracle-side tests and
the GPU side use, so that both see bit-identical operands.

Host draws use a counter-based generator: the SplitMix64 finaliser
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) applied to (key, element index).  The key mixes the seed and a
stream id, so every tensor of a workload has its own independent stream and
any element can be regenerated on its own.  A uniform draw uses the top 53
bits: u = (h >> 11) * 2^-53, then lo + (hi - lo) * u; for [-1, 1] both
steps are exact in binary64.  Normal draws use the Box-Muller transform on
two uniforms (host libm; only ever computed on the host).

Large device-resident operands (hundreds of MiB and up) are drawn directly
on the GPU with torch's seeded Philox generator, because streaming them from
the host would dominate set-up time.  Their values are still a pure function
of (seed, stream, shape); whenever the oracle needs some of them they are
copied back to the host as inputs.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2208  # arbitrary fixed base seed of the workloads

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    """64-bit key of one tensor's stream."""
    with np.errstate(over="ignore"):
        s = np.array([(int(seed) & 0xFFFFFFFF) << 32 | (int(stream) & 0xFFFFFFFF)], dtype=np.uint64)
        return _mix(_mix(s + _GOLDEN) + _GOLDEN)[0]


def raw_u64(count: int, seed: int, stream: int, offset: int = 0) -> np.ndarray:
    """`count` 64-bit draws for element indices offset .. offset+count-1."""
    key = stream_key(seed, stream)
    idx = np.arange(offset, offset + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + (idx + np.uint64(1)) * _GOLDEN)


def host_uniform(shape, seed: int, stream: int, lo: float = -1.0, hi: float = 1.0,
                 dtype=np.float64, offset: int = 0) -> np.ndarray:
    """Uniform [lo, hi) draws of the given shape (row-major element order)."""
    n = int(np.prod(shape)) if len(shape) else 1
    u = (raw_u64(n, seed, stream, offset) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    x = lo + (hi - lo) * u
    return x.reshape(shape).astype(dtype)


def host_normal(shape, seed: int, stream: int, dtype=np.float64) -> np.ndarray:
    """Standard normal draws by Box-Muller over pairs of counter uniforms."""
    n = int(np.prod(shape)) if len(shape) else 1
    m = (n + 1) // 2
    h = raw_u64(2 * m, seed, stream)
    u1 = ((h[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53  # (0, 1]
    u2 = (h[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m, dtype=np.float64)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:n].reshape(shape).astype(dtype)


def host_ints(shape, seed: int, stream: int, lo: int, hi: int, dtype=np.float64) -> np.ndarray:
    """Integers uniform on [lo, hi] (inclusive), stored as floating point."""
    n = int(np.prod(shape)) if len(shape) else 1
    span = np.uint64(hi - lo + 1)
    v = (raw_u64(n, seed, stream) % span).astype(np.int64) + lo
    return v.reshape(shape).astype(dtype)


def f32_to_bf16_bits(x) -> np.ndarray:
    """Round binary32 values to bfloat16 (nearest, ties to even); uint16 bits.

    Used only to draw inputs that are exactly representable in bfloat16."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)
    return r


def bf16_bits_to_f32(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32)


def host_bf16_uniform(shape, seed: int, stream: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """bfloat16 bit patterns of uniform draws (uint16 array)."""
    return f32_to_bf16_bits(host_uniform(shape, seed, stream, lo, hi, dtype=np.float32))


def col_scaled_uniform(m: int, k: int, seed: int, stream: int, umin: float = -3.0,
                       umax: float = 3.0, dtype=np.float32) -> np.ndarray:
    """A[:, l] = U[-1, 1] * 10**u_l with u_l ~ U[umin, umax]: columns whose
    magnitudes span six decades (the precision workload)."""
    a = host_uniform((m, k), seed, stream, dtype=np.float64)
    u = host_uniform((k,), seed, stream + 1000, umin, umax)
    return (a * 10.0 ** u[None, :]).astype(dtype)


# ----------------------------------------------------------------- device

def device_uniform(shape, seed: int, stream: int, dtype, device="cuda", lo=-1.0, hi=1.0):
    """Uniform [lo, hi) tensor drawn on the device from a seeded generator."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) << 20) ^ int(stream))
    t = torch.empty(shape, dtype=dtype, device=device)
    t.uniform_(lo, hi, generator=g)
    return t


def device_normal(shape, seed: int, stream: int, dtype, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) << 20) ^ int(stream))
    t = torch.empty(shape, dtype=dtype, device=device)
    t.normal_(0.0, 1.0, generator=g)
    return t


def device_col_scaled_uniform(m: int, k: int, seed: int, stream: int, dtype, device="cuda",
                              umin: float = -3.0, umax: float = 3.0):
    """Device version of :func:`col_scaled_uniform` (column exponents drawn
    on the host, magnitudes on the device)."""
    import torch
    a = device_uniform((m, k), seed, stream, dtype, device)
    u = host_uniform((k,), seed, stream + 1000, umin, umax)
    scale = torch.tensor(10.0 ** u, dtype=dtype, device=device)
    a.mul_(scale[None, :])
    return a


def sample_rows(m: int, count: int, seed: int, stream: int = 999) -> np.ndarray:
    """Sorted distinct row indices in [0, m) for sampled checks; the first
    and the last row are always included."""
    count = max(2, min(count, m))
    h = (raw_u64(4 * count + 8, seed, stream) % np.uint64(m)).astype(np.int64)
    inner = np.unique(h[(h != 0) & (h != m - 1)])[: max(count - 2, 0)]
    return np.unique(np.concatenate([[0, m - 1], inner])).astype(np.int64)


# ------------------------------------------------------- workload recipes

def batched_shapes(count: int, seed: int, m_lo: int = 1024, m_hi: int = 262144,
                   kn_choices=(4, 8, 16, 32, 64, 128)):
    """Shapes of the batched workload: m uniform integer in [m_lo, m_hi],
    k and n drawn independently from kn_choices."""
    ms = host_ints((count,), seed, 501, m_lo, m_hi, dtype=np.int64)
    ch = np.asarray(kn_choices, dtype=np.int64)
    ks = ch[host_ints((count,), seed, 502, 0, len(ch) - 1, dtype=np.int64)]
    ns = ch[host_ints((count,), seed, 503, 0, len(ch) - 1, dtype=np.int64)]
    return ms, ns, ks
