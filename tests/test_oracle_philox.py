"""Pins for the oracle's Philox4x32-10 stream, uniform maps and Box-Muller.

CPU: structural and statistical properties, closed-form Box-Muller points.
GPU machine: the word stream against rocRAND's host Philox4x32-10 generator, an
independent implementation of the same published algorithm (the library
cannot initialise without a device, so that check is marked gpu).
"""

import ctypes
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox


def test_uniform_maps_are_exact_and_open():
    x = np.array([0, 1, 0x7FFFFFFF, 0xFFFFFFFF], dtype=np.uint32)
    u = philox.u32_to_unit(x)
    assert u[0] == 2.0 ** -33 and u[-1] == 1.0 - 2.0 ** -33
    assert np.all((u > 0) & (u < 1))
    v = philox.u52_to_unit(np.array([0, 0xFFFFFFFF], np.uint32), np.array([0, 0xFFFFFFFF], np.uint32))
    assert v[0] == 2.0 ** -53 and v[1] == 1.0 - 2.0 ** -53


def test_box_muller_closed_form_points():
    # r = 1 when u1 = exp(-1/2); angle 2 pi u2
    u1 = np.full(4, math.exp(-0.5))
    u2 = np.array([0.0, 0.25, 0.5, 0.125])
    a, b = philox.box_muller(u1, u2)
    assert np.allclose(a, [1.0, 0.0, -1.0, math.sqrt(0.5)], atol=1e-15)
    assert np.allclose(b, [0.0, 1.0, 0.0, math.sqrt(0.5)], atol=1e-15)


def words(n, key=(0, 0), lane=0):
    return philox.philox4x32_10(np.arange(n, dtype=np.uint64), lane, 0, 0, key)


def test_words_uniform_and_balanced():
    w = np.concatenate(words(1 << 18))
    # every bit position is balanced
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(w.size))
    # top byte histogram is uniform (chi-square)
    hist = np.bincount(w >> 24, minlength=256)
    assert stats.chisquare(hist).pvalue > 1e-4


def test_counter_and_key_avalanche():
    base = np.array(words(4096), dtype=np.uint64)
    for key, lane in [((1, 0), 0), ((0, 1), 0), ((0, 0), 1)]:
        other = np.array(words(4096, key=key, lane=lane), dtype=np.uint64)
        flips = np.unpackbits((base ^ other).astype(">u4").view(np.uint8)).mean()
        assert abs(flips - 0.5) < 0.01
    # deterministic
    assert np.array_equal(base, np.array(words(4096), dtype=np.uint64))


def test_normals_moments_and_ks():
    x0, x1, x2, x3 = words(1 << 18)
    a, b = philox.box_muller(philox.u32_to_unit(x0), philox.u32_to_unit(x1))
    z = np.concatenate([a, b])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 5 * math.sqrt(24 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


@pytest.mark.gpu
def test_words_match_rocrand_host_generator():
    """rocRAND's host Philox4x32-10, seed s, offset 0: first outputs are Philox(key(s), ctr=(i,0,0,0))."""
    try:
        lib = ctypes.CDLL("librocrand.so")
    except OSError:
        lib = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    for seed in (0, 0x0123456789ABCDEF):
        gen = ctypes.c_void_p()
        assert lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), 404) == 0
        assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        out = np.zeros(64, dtype=np.uint32)
        st = lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(out.size))
        lib.rocrand_destroy_generator(gen)
        assert st == 0
        ours = philox.philox4x32_10(np.arange(16, dtype=np.uint64), 0, 0, 0, philox.key_from_seed(seed))
        ours = np.stack(ours, axis=1).ravel()
        assert np.array_equal(out[:4], ours[:4]), (out[:8], ours[:8])
