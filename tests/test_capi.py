"""The C-ABI library loads and exports every declared symbol (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2509_10103_amd", "libnpo.so")
HDR = os.path.join(ROOT, "include", "npo.h")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:npo_status|const char\*)\s+(npo_\w+)\s*\(", src, re.M)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_library_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 19
    L = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_binding_covers_header():
    from paper_2509_10103_amd import npo
    assert set(declared()) == set(npo.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_host_checkpoint_schedule_matches_closed_form():
    from paper_2509_10103_amd import npo
    from oracle.checkpoint import closed_form
    for n in (1, 2, 3, 7, 20, 64, 100, 500):
        for s in (1, 2, 3, 5, 8, 40, 1000):
            rec = npo.npo_ckpt_count(n, s)
            assert rec + (n - 1) == closed_form(n, s)[0], (n, s)
    for n, s in ((4000, 8), (4000, 32), (4000, 128), (4000, 4000), (9817, 4000)):
        assert npo.npo_ckpt_count(n, s) + n - 1 == closed_form(n, s)[0]
