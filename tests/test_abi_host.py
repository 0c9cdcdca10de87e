"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every symbol the header declares; the header and the binding agree."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "galario_hip.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gal_[a-zA-Z0-9_]+)\s*\(", txt)))


def test_header_declares_what_the_binding_knows():
    from paper_1709_06999_amd import _native

    assert sorted(_native.exported_names()) == _header_functions()


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1709_06999_amd import _native

    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("HIP library not built")
    L = _native.lib()
    for name in _header_functions():
        assert hasattr(L, name), name
    assert b"gfx950" in L.gal_version()


def test_workspace_sizes_are_host_computable():
    from paper_1709_06999_amd import _native

    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("HIP library not built")
    L = _native.lib()
    # control block + partials + (N/2+1)(N+2) complex values
    for N, M in [(16, 0), (256, 10**4), (2048, 10**6), (8192, 5 * 10**6), (16384, 10**6)]:
        d = L.gal_workspace_bytes_d(N, M)
        f = L.gal_workspace_bytes_f(N, M)
        assert d >= (N // 2 + 1) * (N + 2) * 16 and f >= (N // 2 + 1) * (N + 2) * 8
        assert d > f
    assert L.gal_workspace_bytes_d(56, 10) == 0      # 7 is not a factor the FFTs take
    assert L.gal_workspace_bytes_d(47, 10) == 0      # odd
    # 48 = 2^4 3: the mixed-radix path, with a twiddle table and a sweep buffer
    assert L.gal_workspace_bytes_d(48, 10) >= 25 * 50 * 16 + 48 * 16 + 48 * 48 * 8
    assert L.gal_workspace_bytes_d(32768, 10) == 0   # above the supported range
    # 16384^2 in FP64: the four-step column pass writes the spectrum apart
    assert L.gal_workspace_bytes_d(16384, 10) >= 2 * 8193 * 16385 * 16
    # gradients stop at 8192
    assert L.gal_grad_workspace_bytes_d(16384, 10, 100) == 0
