"""The C-ABI library loads and exports every symbol the header declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "ibm_poisson.h")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_parses():
    names = declared_functions()
    for must in ["ibm_classify", "ibm_build_ghost_stencils", "poisson_setup", "poisson_solve", "poisson_submit",
                 "poisson_poll", "ibm_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2605_04335_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(P.EXPORTS) <= set(declared_functions())


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2605_04335_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(ImportError):
        P.lib()


def test_fdiv_magic_numbers():
    """The kernels divide by grid extents with a round-up multiplier
    (Granlund-Montgomery); check the host-side constants on a sweep."""
    import numpy as np

    def make(d):
        l = 0
        while (1 << l) < d:
            l += 1
        m = ((1 << 32) * ((1 << l) - d)) // d + 1
        return m & 0xFFFFFFFF, l

    rng = np.random.default_rng(0)
    for d in list(range(1, 70)) + [96, 127, 128, 129, 255, 256, 320, 384, 511, 512, 1024, 1536, 2048 * 1024 + 3]:
        m, s = make(d)
        ns = np.concatenate([np.arange(0, 3000), rng.integers(0, 2 ** 31, 3000)])
        for n in ns:
            n = int(n)
            q = (((n * m) >> 32) + n) >> s
            assert q == n // d
