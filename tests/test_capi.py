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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
@pytest.mark.parametrize("grid,code", [
    ((7, 12, 24), -4),     # nr below the 7-point stencil
    ((65, 12, 24), -4),    # nr above one workgroup's column
    ((16, 7, 24), -4),     # ntheta not 2^a 3^b
    ((16, 12, 25), -4),    # nz not 2^a 3^b
    ((16, 12, 27), -4),    # nz odd (two axial columns share one azimuthal transform)
    ((16, 12, 4096), -4),  # nz above the supported range
])
def test_plan_create_rejects_unsupported_grids_before_any_device_call(grid, code):
    """Argument checks return their status synchronously, with a message, and
    touch no device (this runs without a GPU)."""
    from paper_2509_10103_amd import npo
    with pytest.raises(npo.NpoError) as e:
        npo.npo_plan_create(*grid, 10.0, 2000.0, 8.0, 1.0, 0.01, 0.0, 10)
    assert f"npo error {code}" in str(e.value)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
@pytest.mark.parametrize("args", [
    (16, 12, 24, -1.0, 2000.0, 8.0, 1.0, 0.01, 0.0, 10, 2),   # lz <= 0
    (16, 12, 24, 10.0, 0.0, 8.0, 1.0, 0.01, 0.0, 10, 2),      # Re <= 0
    (16, 12, 24, 10.0, 2000.0, 8.0, -1.0, 0.01, 0.0, 10, 2),  # A < 0
    (16, 12, 24, 10.0, 2000.0, 8.0, 1.0, 0.0, 0.0, 10, 2),    # dt <= 0
    (16, 12, 24, 10.0, 2000.0, 8.0, 1.0, 0.01, 0.0, 0, 2),    # nsteps < 1
    (16, 12, 24, 10.0, 2000.0, 8.0, 1.0, 0.01, 0.0, 10, 0),   # no corrector pass
    (16, 12, 24, 10.0, 2000.0, 8.0, 1.0, 0.01, 0.0, 10, 4),   # more passes than supported
])
def test_plan_create_rejects_bad_parameters(args):
    from paper_2509_10103_amd import npo
    with pytest.raises(npo.NpoError) as e:
        npo.npo_plan_create(*args)
    assert "npo error -1" in str(e.value)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_null_arguments_are_rejected():
    from paper_2509_10103_amd import npo
    L = npo.lib()
    assert L.npo_plan_create(None, None, None, 0, None) == -1
    assert L.npo_forward_step(None, None, None, None, 0, None) == -1
    assert L.npo_ckpt_count(0, 1, None) == -1
    assert b"null" in L.npo_last_error() or b"bad" in L.npo_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_hybrid_counts_match_the_recovery_model():
    """Sec. 2.4 two-level checkpoints: with n_file host checkpoints the adjoint
    sweep re-advances sum_i T(l_i) - (l_last - 1) steps, T(l) = S l - beta(N_G+1, S-1)
    the advances to recover an interval of l steps from N_G memory checkpoints
    (the oracle's closed form); no host checkpoints is the device-only count."""
    from paper_2509_10103_amd import npo
    from oracle.checkpoint import closed_form
    for n in (7, 40, 500, 9817):
        for s in (1, 3, 8, 40):
            assert npo.npo_hybrid_count(n, s, 0) == npo.npo_ckpt_count(n, s)
            for f in (1, 2, 5):
                if f >= n:
                    continue
                b = [n * i // (f + 1) for i in range(f + 2)]
                ls = [b[i + 1] - b[i] for i in range(f + 1)]
                model = sum(closed_form(l, s)[0] for l in ls) - (ls[-1] - 1)
                assert npo.npo_hybrid_count(n, s, f) == model, (n, s, f)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnpo.so not built")
def test_hybrid_plan_minimises_recovery_time():
    from paper_2509_10103_amd import npo
    for n, s, tio, tstep in ((9817, 8, 2e-3, 1.3e-3), (9817, 64, 5e-2, 1.3e-3), (4000, 4, 0.0, 1.0),
                             (4000, 4000, 1.0, 1.0)):
        f, t = npo.npo_hybrid_plan(n, s, tio, tstep, 64)
        costs = [k * tio + npo.npo_hybrid_count(n, s, k) * tstep for k in range(0, 65)]
        assert abs(t - min(costs)) <= 1e-12 * max(1.0, abs(t))
        assert costs[f] == min(costs)
