"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its host-side Toeplitz table matches the oracle, and argument errors are caught
before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import green, jm
from paper_1803_06237_amd import vie

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(vie_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = vie.lib()
    names = _declared()
    assert {"vie_plan", "vie_set_contrast", "vie_matvec", "vie_solve", "vie_destroy"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n


def test_version_string():
    assert b"gfx950" in vie.lib().vie_version()


@pytest.mark.parametrize("grid,kappa", [((8, 8, 32), 0.29266), ((3, 5, 7), 1.1), ((1, 1, 1), 0.0)])
def test_host_table_matches_oracle(grid, kappa):
    T = vie.green_table(grid, kappa)
    To = green.green_table(grid, kappa)
    assert np.max(np.abs(T - To)) < 2e-15


def test_host_table_sampled_at_long_grid():
    """Sampled entries of a 32 x 32 x 128 table (the long-guide cross-section) against
    the oracle evaluated one offset at a time."""
    kappa = 0.14633
    T = vie.green_table((32, 32, 128), kappa)
    rng = np.random.default_rng(5)
    ms = np.stack([rng.integers(0, 32, 30), rng.integers(0, 32, 30), rng.integers(0, 128, 30)], 1)
    ms = np.concatenate([ms, [[0, 0, 0], [1, 0, 0], [1, 1, 1], [31, 31, 127], [0, 2, 1]]])
    No = green.galerkin_N(ms, kappa)
    Nl = np.stack([T[:, m[0], m[1], m[2]] for m in ms], 1)
    assert np.max(np.abs(No - Nl)) < 2e-15


@pytest.mark.parametrize("grid,kappa", [((8, 8, 12), 0.29266), ((3, 5, 7), 1.1), ((2, 1, 3), 0.0)])
def test_host_curl_table_matches_oracle(grid, kappa):
    K = vie.curl_table(grid, kappa)
    Ko = jm.curl_table(grid, kappa)
    assert np.max(np.abs(K - Ko)) < 2e-15
    assert np.max(np.abs(Ko)) > 1e-3


def test_plan_rejects_bad_arguments_before_touching_the_device():
    L = vie.lib()
    h = ctypes.c_void_p()
    g = (ctypes.c_int * 3)(8, 8, 32)
    assert L.vie_plan(ctypes.byref(h), g, -1.0, 4.0, 2.085, 0, None) == vie.VIE_EINVAL
    assert L.vie_plan(ctypes.byref(h), g, 0.05, float("nan"), 2.085, 0, None) == vie.VIE_EINVAL
    big = (ctypes.c_int * 3)(64, 8, 32)
    assert L.vie_plan(ctypes.byref(h), big, 0.05, 4.0, 2.085, 0, None) == vie.VIE_EINVAL
    assert b"n1,n2 <= 32" in L.vie_last_error(None)
    zero = (ctypes.c_int * 3)(0, 8, 32)
    assert L.vie_plan(ctypes.byref(h), zero, 0.05, 4.0, 2.085, 0, None) == vie.VIE_EINVAL
    assert L.vie_green_table(zero, 0.1, None, 0) == vie.VIE_EINVAL
    # null plans are rejected by every call
    assert L.vie_matvec(None, None, None) == vie.VIE_EINVAL
    assert L.vie_set_contrast(None, None) == vie.VIE_EINVAL
    assert L.vie_circulant_build(None, 0, None) == vie.VIE_EINVAL
    assert L.vie_circulant_apply(None, None, None) == vie.VIE_EINVAL
    assert L.vie_get_tune(None, 0, None, None) == vie.VIE_EINVAL
    assert L.vie_set_tune(None, 0, 0, 0) == vie.VIE_EINVAL
    assert L.vie_curl_table(zero, 0.1, None, 0) == vie.VIE_EINVAL
    assert L.vie_jm_enable(None) == vie.VIE_EINVAL
    assert L.vie_jm_set_permeability(None, None) == vie.VIE_EINVAL
    assert L.vie_jm_set_route(None, 0, 1) == vie.VIE_EINVAL
    assert L.vie_jm_get_route(None, 0, None) == vie.VIE_EINVAL
    assert L.vie_jm_rhs(None, None, None, None) == vie.VIE_EINVAL
    assert L.vie_jm_matvec(None, None, None) == vie.VIE_EINVAL
    assert L.vie_jm_matvec_c64(None, None, None) == vie.VIE_EINVAL
    assert L.vie_jm_residual(None, None, None, None) == vie.VIE_EINVAL
    assert L.vie_jm_solve(None, None, None, 1e-8, None, None) == vie.VIE_EINVAL
    L.vie_destroy(None)


def test_block_maps_are_bijections_with_writes_in_bounds():
    """Every workgroup-to-work map of the product's pass kernels (z-pass pencil blocks
    with their XCD grouping, cross-section plane pairs) is a bijection onto its work
    items over all accepted shapes, and every write derived from an item fits its
    buffer; the checker itself refuses a planted non-injective map."""
    L = vie.lib()
    L.vie_check_block_maps.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int]
    buf = ctypes.create_string_buffer(512)
    rc = L.vie_check_block_maps(buf, 512, 0)
    assert rc == 0, buf.value.decode()
    assert buf.value.startswith(b"ok:")
    assert L.vie_check_block_maps(buf, 512, 1) != 0
    assert b"not injective" in buf.value
    assert L.vie_check_block_maps(buf, 512, 2) != 0
    assert b"bank conflict" in buf.value
