"""The C-ABI library loads and exports every entry point declared in include/cefield.h;
host-only entry points (no device needed) agree with the oracle / definitions."""

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cefield.h")
LIB = os.path.join(ROOT, "paper_1406_6072_amd", "libcefield.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ce_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import ctypes
    assert os.path.exists(LIB), "libcefield.so not built"
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 15
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1406_6072_amd import binding
    assert sorted(binding.EXPORTED) == declared_symbols()
    assert "gfx950" in binding.version()


def test_status_strings():
    from paper_1406_6072_amd import binding
    for s in range(7):
        assert binding.status_string(s)


@pytest.mark.parametrize("L,prod", [(2048, 2048), (1024, 1024), (512, 512), (96, 96), (992, 992), (160, 160),
                                    (4096, 4096), (64, 64), (6, 6), (1184, 1184), (4064, 4064), (3998, 3998),
                                    (74, 74), (2 * 2039, 4078)])
def test_fft_factors_cover_length(L, prod):
    """Every even length up to 4096 factors: powers of two in radices 2..16, primes up to 31 in their own
    butterflies, larger primes (37 .. 2039) in the generic prime stage."""
    from paper_1406_6072_amd import binding
    r = binding.fft_factors(L)
    assert int(np.prod(r)) == prod
    for x in r:
        assert x in (2, 4, 8, 16) or all(x % p for p in range(2, int(x ** 0.5) + 1)), (L, r)


def test_every_even_side_is_a_supported_length():
    from paper_1406_6072_amd import binding
    for L in range(2, 4097, 2):
        r = binding.fft_factors(L)
        assert int(np.prod(r)) == L


def test_fft_factors_reject_out_of_range():
    from paper_1406_6072_amd import binding
    for L in (1, 4098, 8192):
        with pytest.raises(binding.CeError):
            binding.fft_factors(L)


@pytest.mark.parametrize("n,nb", [((64, 64), 32), ((16, 16, 16), 8), ((1024, 1024), 128), ((12, 12), 5),
                                  ((48, 80), 12), ((40, 24, 32), 6), ((64, 26), 10), ((18, 12), 9)])
def test_host_shell_table_matches_oracle(n, nb):
    from oracle import pk
    from paper_1406_6072_amd import binding
    d = len(n)
    nm, km = binding.shell_table(n, (0.5,) * d, nb)
    onm, okm = pk.shell_stats(n, 0.5, nb)
    assert np.array_equal(nm, onm)
    ok = onm > 0
    assert np.allclose(km[ok], okm[ok], rtol=1e-13)


@pytest.mark.parametrize("n,h,nb", [((16, 32), (2.0, 1.0), 10), ((24, 20), (0.5, 0.75), 12),
                                    ((12, 16, 10), (1.0, 0.5, 1.5), 7), ((30, 18), (1.0, 1.0 / 3.0), 9),
                                    ((64, 48), (0.25, 0.2), 16)])
def test_host_shell_table_rectangular_cells(n, h, nb):
    """Rectangular cells: the library's integer shell table equals the oracle's."""
    from oracle import pk
    from paper_1406_6072_amd import binding
    nm, km = binding.shell_table(n, h, nb)
    onm, okm = pk.shell_stats(n, h, nb)
    assert np.array_equal(nm, onm)
    ok = onm > 0
    assert np.allclose(km[ok], okm[ok], rtol=1e-13)


def test_host_shell_table_rejects_irrational_cell_ratio():
    from paper_1406_6072_amd import binding
    with pytest.raises(binding.CeError) as e:
        binding.shell_table((16, 16), (1.0, 0.5 ** 0.5), 4)
    assert e.value.status == binding.E_UNSUPPORTED


def test_shipped_schedule_file_is_well_formed():
    """The package's tuned launch schedules: one entry per shape and precision, values in the
    ranges the library accepts (the GPU tests load the file through ce_schedule_load)."""
    import json
    from paper_1406_6072_amd import binding
    rec = json.load(open(binding.DEFAULT_SCHEDULES))
    assert rec["format"] == "cefield-schedules" and rec["arch"] == "gfx950"
    keys = set()
    for e in rec["entries"]:
        key = (e["ndim"], tuple(e["n"]), e["precision"])
        assert key not in keys
        keys.add(key)
        assert e["ndim"] in (2, 3) and e["precision"] in ("f32", "f64")
        ln, li, ll, lb = e["lines"]
        assert ln == 0 or (ln % 2 == 0 and 2 <= ln <= 32)
        for v in (li, ll, lb):
            assert v == 0 or (v & (v - 1) == 0 and v <= 64)
        assert e["noise_order"] in (0, 1) and 1 <= e["noise_block"] <= 65536
        assert 0 <= e["noise_pairs"] <= 64 and 16384 <= e["bin_lds"] <= 163840
    assert (2, (1024, 1024, 1), "f32") in keys and (3, (256, 256, 256), "f32") in keys
