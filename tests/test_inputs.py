"""The seeded input generators: deterministic, per-stream independent,
in range, and stable across versions (known-answer digest)."""
import hashlib

import numpy as np

from paper_2208_08088_amd import inputs as I


def test_deterministic_and_streams_differ():
    a = I.host_uniform((100, 7), 5, 1)
    assert np.array_equal(a, I.host_uniform((100, 7), 5, 1))
    assert not np.array_equal(a, I.host_uniform((100, 7), 5, 2))
    assert not np.array_equal(a, I.host_uniform((100, 7), 6, 1))


def test_offset_regenerates_any_slice():
    full = I.host_uniform((1000,), 9, 3)
    assert np.array_equal(full[400:450], I.host_uniform((50,), 9, 3, offset=400))


def test_ranges():
    u = I.host_uniform((20000,), 1, 1)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.03
    z = I.host_normal((20001,), 1, 2)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1.0) < 0.05
    n = I.host_ints((5000,), 1, 3, -8, 8)
    assert n.min() == -8 and n.max() == 8 and np.all(n == np.round(n))
    a = I.col_scaled_uniform(2000, 16, 1, 4)
    colmax = np.abs(a).max(axis=0)
    assert colmax.max() / colmax.min() > 10.0
    assert np.all(colmax < 1001.0) and np.all(colmax > 1e-3 * 0.5)


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.5], dtype=np.float32)
    assert I.f32_to_bf16_bits(x).tolist() == [0x3F80, 0x3F82, 0xBFC0]
    assert np.array_equal(I.bf16_bits_to_f32(np.array([0x3F80], np.uint16)), np.array([1.0], np.float32))


def test_known_answer_digest():
    h = hashlib.sha256(I.raw_u64(1000, 2208, 1).tobytes()).hexdigest()
    assert h == KNOWN_DIGEST


def test_sample_rows_and_batched_shapes():
    r = I.sample_rows(1 << 20, 64, 3)
    assert r[0] == 0 and r[-1] == (1 << 20) - 1 and np.all(np.diff(r) > 0) and len(r) == 64
    ms, ns, ks = I.batched_shapes(512, 2208)
    assert len(ms) == 512 and ms.min() >= 1024 and ms.max() <= 262144
    assert set(ns.tolist()) <= {4, 8, 16, 32, 64, 128} and set(ks.tolist()) <= {4, 8, 16, 32, 64, 128}


KNOWN_DIGEST = "33e375e4d2ca7aec34b1711036ee3f7fe0d94aeef661ec0915662b8e8dc717ac"
