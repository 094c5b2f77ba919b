"""ctypes binding of libnpo.so (C ABI in include/npo.h).

Argument marshalling only: every numerical step runs in the HIP library.
Fields are torch complex128 tensors of shape (3, nr, M+1, 2K+1) on the GPU;
their data pointers and torch's current HIP stream are passed to the library.
Loading fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NPO_LIBRARY selects another build of the same library (the sanitizer build
# used by the host-side checks); the default is the in-tree libnpo.so.
_LIB_PATH = os.environ.get("NPO_LIBRARY") or os.path.join(_HERE, "libnpo.so")
_lib = None


class NpoError(RuntimeError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("nz", ctypes.c_int32), ("lz", ctypes.c_double)]


class Flow(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("wo", ctypes.c_double), ("amp", ctypes.c_double)]


class Time(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("t0", ctypes.c_double), ("nsteps", ctypes.c_int64), ("ncorr", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("nz", ctypes.c_int32), ("M", ctypes.c_int32),
                ("K", ctypes.c_int32), ("nk", ctypes.c_int32), ("field_elems", ctypes.c_int64),
                ("field_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("scalars_bytes", ctypes.c_int64), ("period", ctypes.c_double), ("k0", ctypes.c_double),
                ("dt", ctypes.c_double), ("t0", ctypes.c_double), ("nsteps", ctypes.c_int64)]


SCRATCH_BYTES = 64 << 20     # NPO_SCRATCH_BYTES of include/npo.h

_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "npo_last_error": (ctypes.c_char_p, []),
    "npo_plan_create": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(Flow), ctypes.POINTER(Time), ctypes.c_uint32,
                               ctypes.POINTER(_P)]),
    "npo_plan_destroy": (_I32, [_P]),
    "npo_plan_info": (_I32, [_P, ctypes.POINTER(Info)]),
    "npo_plan_tables": (_I32, [_P, _DP, _DP, _DP, _DP, ctypes.POINTER(_I32)]),
    "npo_base_flow": (_I32, [_P, _D, _P, _P, _P]),
    "npo_nonlinear": (_I32, [_P, _P, _P, _D, _P, _P]),
    "npo_nonlinear_adj": (_I32, [_P, _P, _P, _D, _P, _P, _P]),
    "npo_solve": (_I32, [_P, _P, _P, _P, _P]),
    "npo_solve_adj": (_I32, [_P, _P, _P, _P, _P]),
    "npo_forward_step": (_I32, [_P, _P, _P, _P, _I64, _P]),
    "npo_forward_step_noalloc": (_I32, [_P, _P, _P, _I64, _P]),
    "npo_adjoint_step": (_I32, [_P, _P, _P, _P, _P, _I64, _P]),
    "npo_forward_run": (_I32, [_P, _P, _P, _I32, _P, _P, _P]),
    "npo_adjoint_run": (_I32, [_P, _P, _P, _I32, _P, _P, ctypes.POINTER(_I64), _P]),
    "npo_forward_run_diag": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _I32, _P]),
    "npo_forward_run_hybrid": (_I32, [_P, _P, _P, _I32, _P, _I32, _P, _P, _P]),
    "npo_adjoint_run_hybrid": (_I32, [_P, _P, _P, _I32, _P, _I32, _P, _P, ctypes.POINTER(_I64), _P]),
    "npo_hybrid_count": (_I32, [_I64, _I32, _I32, ctypes.POINTER(_I64)]),
    "npo_hybrid_plan": (_I32, [_I64, _I32, _D, _D, _I32, ctypes.POINTER(_I32), _DP]),
    "npo_energy_diag": (_I32, [_P, _P, _P, _P, _P, _P]),
    "npo_ckpt_count": (_I32, [_I64, _I32, ctypes.POINTER(_I64)]),
    "npo_inner": (_I32, [_P, _P, _P, _P, _P, _P]),
    "npo_project": (_I32, [_P, _P, _P, _P, _P]),
    "npo_update": (_I32, [_P, _P, _P, _P, _D, _D, _P, _P, _P]),
    "npo_iterate": (_I32, [_P, _P, _P, _I32, _P, _P, _D, _D, _I32, _DP, _P]),
    "npo_normalize": (_I32, [_P, _P, _P, _D, _P]),
    "npo_euclid_grad": (_I32, [_P, _P, _D, _P, _P]),
    "npo_plan_set_tuning": (_I32, [_P, _I32, _I32, _I32]),
    "npo_plan_get_tuning": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "npo_plan_set_radial_block": (_I32, [_P, _I32]),
    "npo_plan_get_radial_block": (_I32, [_P, ctypes.POINTER(_I32)]),
    "npo_plan_set_graphs": (_I32, [_P, _I32]),
    "npo_plan_set_cfl_monitor": (_I32, [_P, _I32]),
    "npo_plan_set_adjoint": (_I32, [_P, _I32]),
    "npo_nonlinear_adj_cont": (_I32, [_P, _P, _P, _D, _P, _P, _P]),
    "npo_adjoint_step_cont": (_I32, [_P, _P, _P, _P, _P, _P, _I64, _P]),
    "npo_cfl_read": (_I32, [_P, _P, _P, _I32, _P]),
    "npo_plan_inject_fault": (_I32, [_P, _I32, _I64]),
    "npo_batch_create": (_I32, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_P)]),
    "npo_batch_destroy": (_I32, [_P]),
    "npo_batch_info": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "npo_batch_set_steps": (_I32, [_P, ctypes.POINTER(_P), _I64, _P]),
    "npo_batch_step": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I32, _P]),
    "npo_batch_forward_run": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I32, ctypes.POINTER(_P),
                                     ctypes.POINTER(_P), _P]),
    "npo_batch_adjoint_run": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I32, ctypes.POINTER(_P),
                                     ctypes.POINTER(_P), ctypes.POINTER(_I64), _P]),
    "npo_profile_begin": (_I32, [_P, _I32]),
    "npo_profile_read": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _DP]),
}

KERNEL_FAMILIES = ("curl", "zinv_fwd", "theta_fwd", "zfwd_fwd", "zinv_adj", "theta_adj", "zfwd_adj",
                   "solve_pred", "solve_corr", "solve_raw", "solve_adj", "adj_combine", "wdot", "project", "axpby",
                   "solve_adj2", "zinv_adjy")


def lib():
    """Load libnpo.so once; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise NpoError(f"{_LIB_PATH} not built; run paper_2509_10103_amd/build.py")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise NpoError(f"npo error {status}: {lib().npo_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# Argument checks before a call: a wrong dtype, a strided view or an undersized
# buffer would make the kernels read or write past an allocation, so they are
# refused here with NpoError instead.
_INFO = {}


def _plan_info(plan):
    key = plan.value if isinstance(plan, ctypes.c_void_p) else int(plan)
    inf = _INFO.get(key)
    if inf is None:
        inf = npo_plan_info(plan)
        _INFO[key] = inf
    return inf


def _dev(t, what):
    if t is None:
        raise NpoError(f"{what}: missing tensor")
    if not getattr(t, "is_cuda", False):
        raise NpoError(f"{what}: must be a device tensor")
    if not t.is_contiguous():
        raise NpoError(f"{what}: must be contiguous")
    return _ptr(t)


def _fld(plan, t, what, count=1):
    """A field (or `count` consecutive fields): complex128, contiguous, on the device."""
    import torch
    p = _dev(t, what)
    if t.dtype != torch.complex128:
        raise NpoError(f"{what}: dtype {t.dtype}, expected complex128")
    need = _plan_info(plan)["field_elems"] * count
    bad = t.numel() < need if count > 1 else t.numel() != need
    if bad:
        raise NpoError(f"{what}: {t.numel()} complex elements, expected {'at least ' if count > 1 else ''}{need}")
    return p


def _wsp(plan, ws):
    p = _dev(ws, "workspace")
    need = _plan_info(plan)["workspace_bytes"]
    if ws.numel() * ws.element_size() < need:
        raise NpoError(f"workspace: {ws.numel() * ws.element_size()} bytes, plan needs {need}")
    return p


def _scal(t, what, n=1):
    import torch
    p = _dev(t, what)
    if t.dtype != torch.float64 or t.numel() < n:
        raise NpoError(f"{what}: expected at least {n} float64 elements on the device")
    return p


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ plan
def npo_plan_create(nr, ntheta, nz, lz, re, wo, amp, dt, t0, nsteps, ncorr=2):
    g = Grid(nr, ntheta, nz, lz)
    f = Flow(re, wo, amp)
    t = Time(dt, t0, nsteps, ncorr)
    h = _P()
    _check(lib().npo_plan_create(ctypes.byref(g), ctypes.byref(f), ctypes.byref(t), 0, ctypes.byref(h)))
    return h


def npo_plan_destroy(plan):
    _INFO.pop(plan.value if isinstance(plan, ctypes.c_void_p) else int(plan), None)
    _check(lib().npo_plan_destroy(plan))


def npo_plan_info(plan):
    i = Info()
    _check(lib().npo_plan_info(plan, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in Info._fields_}


def npo_plan_tables(plan, nr):
    r, w = np.zeros(nr), np.zeros(nr)
    D1, D2 = np.zeros((2, nr, 7)), np.zeros((2, nr, 7))
    col0 = np.zeros(nr, dtype=np.int32)
    dp = lambda a: a.ctypes.data_as(_DP)
    _check(lib().npo_plan_tables(plan, dp(r), dp(w), dp(D1), dp(D2), col0.ctypes.data_as(ctypes.POINTER(_I32))))
    return r, w, D1, D2, col0


def npo_base_flow(plan, t, U_dev, dUdr_dev, stream=None):
    nr = _plan_info(plan)["nr"]
    _check(lib().npo_base_flow(plan, t, _scal(U_dev, "U_dev", nr), _scal(dUdr_dev, "dUdr_dev", nr),
                               _stream(stream)))


# --------------------------------------------------------- device calls
def npo_nonlinear(plan, ws, u, t, out, stream=None):
    _check(lib().npo_nonlinear(plan, _wsp(plan, ws), _fld(plan, u, "u"), t, _fld(plan, out, "out"), _stream(stream)))


def npo_nonlinear_adj(plan, ws, u, t, y, out, stream=None):
    _check(lib().npo_nonlinear_adj(plan, _wsp(plan, ws), _fld(plan, u, "u"), t, _fld(plan, y, "y"),
                                   _fld(plan, out, "out"), _stream(stream)))


def npo_solve(plan, ws, R, out, stream=None):
    _check(lib().npo_solve(plan, _ptr(ws), _fld(plan, R, "R"), _fld(plan, out, "out"), _stream(stream)))


def npo_solve_adj(plan, ws, y, out, stream=None):
    _check(lib().npo_solve_adj(plan, _ptr(ws), _fld(plan, y, "y"), _fld(plan, out, "out"), _stream(stream)))


def npo_forward_step(plan, ws, u_n, u_np1, n, stream=None):
    _check(lib().npo_forward_step(plan, _wsp(plan, ws), _fld(plan, u_n, "u_n"), _fld(plan, u_np1, "u_np1"), n,
                                  _stream(stream)))


def npo_forward_step_noalloc(plan, u_n, u_np1, n, stream=None):
    _check(lib().npo_forward_step_noalloc(plan, _fld(plan, u_n, "u_n"), _fld(plan, u_np1, "u_np1"), n,
                                          _stream(stream)))


def npo_adjoint_step(plan, ws, u_n, lam_np1, lam_n, n, stream=None):
    _check(lib().npo_adjoint_step(plan, _wsp(plan, ws), _fld(plan, u_n, "u_n"), _fld(plan, lam_np1, "lam_np1"),
                                  _fld(plan, lam_n, "lam_n"), n, _stream(stream)))


def npo_forward_run(plan, ws, ckpt, n_ckpt, u0, uN, stream=None):
    _check(lib().npo_forward_run(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                                 n_ckpt, _fld(plan, u0, "u0"), _fld(plan, uN, "uN"), _stream(stream)))


def _host_tier(plan, t, n_file):
    """Pinned host memory of n_file fields (torch pin_memory tensor)."""
    if n_file == 0:
        return None if t is None else ctypes.c_void_p(t.data_ptr())
    import torch
    if t is None or t.is_cuda or not t.is_pinned() or not t.is_contiguous():
        raise NpoError("host_tier: must be a contiguous pinned host tensor")
    need = _plan_info(plan)["field_bytes"] * n_file
    if t.numel() * t.element_size() < need:
        raise NpoError(f"host_tier: {t.numel() * t.element_size()} bytes, {n_file} fields need {need}")
    return ctypes.c_void_p(t.data_ptr())


def npo_forward_run_hybrid(plan, ws, ckpt, n_ckpt, host_tier, n_file, u0, uN, stream=None):
    _check(lib().npo_forward_run_hybrid(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                                        n_ckpt, _host_tier(plan, host_tier, n_file), n_file, _fld(plan, u0, "u0"),
                                        _fld(plan, uN, "uN"), _stream(stream)))


def npo_adjoint_run_hybrid(plan, ws, ckpt, n_ckpt, host_tier, n_file, lamN, lam0, stream=None):
    c = _I64()
    _check(lib().npo_adjoint_run_hybrid(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                                        n_ckpt, _host_tier(plan, host_tier, n_file), n_file, _fld(plan, lamN, "lamN"),
                                        _fld(plan, lam0, "lam0"), ctypes.byref(c), _stream(stream)))
    return c.value


def npo_hybrid_count(nsteps, n_ckpt, n_file):
    c = _I64()
    _check(lib().npo_hybrid_count(nsteps, n_ckpt, n_file, ctypes.byref(c)))
    return c.value


def npo_hybrid_plan(nsteps, n_ckpt, t_io, t_step, max_file):
    f = _I32()
    t = ctypes.c_double()
    _check(lib().npo_hybrid_plan(nsteps, n_ckpt, t_io, t_step, max_file, ctypes.byref(f), ctypes.byref(t)))
    return f.value, t.value


def diag_rows(nsteps, stride):
    """Rows of the history written by npo_forward_run_diag."""
    return (nsteps - 1) // stride + 2


def npo_forward_run_diag(plan, ws, ckpt, n_ckpt, u0, uN, hist_dev, stride, stream=None):
    rows = diag_rows(_plan_info(plan)["nsteps"], int(stride)) if stride >= 1 else 0
    _check(lib().npo_forward_run_diag(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                                      n_ckpt, _fld(plan, u0, "u0"), _fld(plan, uN, "uN"),
                                      _scal(hist_dev, "hist_dev", 5 * rows), stride, _stream(stream)))


def npo_energy_diag(plan, ws, u, out_dev, spec_dev=None, stream=None):
    inf = _plan_info(plan)
    spec = None if spec_dev is None else _scal(spec_dev, "spec_dev", (inf["M"] + 1) * inf["nk"])
    _check(lib().npo_energy_diag(plan, _wsp(plan, ws), _fld(plan, u, "u"), _scal(out_dev, "out_dev", 5), spec,
                                 _stream(stream)))


def npo_adjoint_run(plan, ws, ckpt, n_ckpt, lamN, lam0, stream=None):
    c = _I64()
    _check(lib().npo_adjoint_run(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                                 n_ckpt, _fld(plan, lamN, "lamN"), _fld(plan, lam0, "lam0"), ctypes.byref(c),
                                 _stream(stream)))
    return c.value


def npo_ckpt_count(nsteps, n_ckpt):
    c = _I64()
    _check(lib().npo_ckpt_count(nsteps, n_ckpt, ctypes.byref(c)))
    return c.value


def npo_inner(plan, ws, a, b, out_dev, stream=None):
    _check(lib().npo_inner(plan, _wsp(plan, ws), _fld(plan, a, "a"), _fld(plan, b, "b"), _scal(out_dev, "out_dev"),
                           _stream(stream)))


def npo_project(plan, ws, u, out, stream=None):
    _check(lib().npo_project(plan, _wsp(plan, ws), _fld(plan, u, "u"), _fld(plan, out, "out"), _stream(stream)))


def npo_update(plan, ws, u0, g, e0, alpha, u_new, info_dev, stream=None):
    _check(lib().npo_update(plan, _wsp(plan, ws), _fld(plan, u0, "u0"), _fld(plan, g, "g"), e0, alpha,
                            _fld(plan, u_new, "u_new"), _scal(info_dev, "info_dev", 5), _stream(stream)))


def npo_iterate(plan, ws, ckpt, n_ckpt, u0, uN, e0, tol=1e-8, max_halvings=30, stream=None):
    st = np.zeros(8)
    _check(lib().npo_iterate(plan, _wsp(plan, ws), _fld(plan, ckpt, "checkpoint arena", max(int(n_ckpt), 1)),
                             n_ckpt, _fld(plan, u0, "u0"), _fld(plan, uN, "uN"), e0, tol, max_halvings,
                             st.ctypes.data_as(_DP), _stream(stream)))
    keys = ("G_old", "G_new", "alpha", "alpha_max", "E0dag", "C0", "accepted", "forward_sweeps")
    return dict(zip(keys, st.tolist()))


def npo_normalize(plan, ws, u, e0, stream=None):
    _check(lib().npo_normalize(plan, _wsp(plan, ws), _fld(plan, u, "u"), e0, _stream(stream)))


def npo_plan_set_tuning(plan, zgroup, zb_fwd, zb_adj):
    _check(lib().npo_plan_set_tuning(plan, zgroup, zb_fwd, zb_adj))


def npo_plan_set_radial_block(plan, rg):
    _check(lib().npo_plan_set_radial_block(plan, rg))


def npo_plan_get_radial_block(plan):
    a = _I32()
    _check(lib().npo_plan_get_radial_block(plan, ctypes.byref(a)))
    return a.value


def npo_plan_set_graphs(plan, enable):
    _check(lib().npo_plan_set_graphs(plan, int(bool(enable))))


def npo_plan_set_adjoint(plan, kind):
    """0: exact discrete adjoint sweeps (default); 1: the continuous adjoint equations."""
    _check(lib().npo_plan_set_adjoint(plan, int(kind)))


def npo_nonlinear_adj_cont(plan, ws, u, t, y, out, stream=None):
    _check(lib().npo_nonlinear_adj_cont(plan, _wsp(plan, ws), _fld(plan, u, "u"), t, _fld(plan, y, "y"),
                                        _fld(plan, out, "out"), _stream(stream)))


def npo_adjoint_step_cont(plan, ws, u_n, u_np1, lam_np1, lam_n, n, stream=None):
    _check(lib().npo_adjoint_step_cont(plan, _wsp(plan, ws), _fld(plan, u_n, "u_n"), _fld(plan, u_np1, "u_np1"),
                                       _fld(plan, lam_np1, "lam_np1"), _fld(plan, lam_n, "lam_n"), n,
                                       _stream(stream)))


def npo_plan_set_cfl_monitor(plan, enable):
    _check(lib().npo_plan_set_cfl_monitor(plan, int(bool(enable))))


def npo_cfl_read(plan, ws, out_dev, reset=False, stream=None):
    _check(lib().npo_cfl_read(plan, _wsp(plan, ws), _scal(out_dev, "out_dev"), int(bool(reset)), _stream(stream)))


def npo_plan_inject_fault(plan, site, after):
    _check(lib().npo_plan_inject_fault(plan, site, after))


def npo_plan_get_tuning(plan):
    a, b_, c = _I32(), _I32(), _I32()
    _check(lib().npo_plan_get_tuning(plan, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c)))
    return a.value, b_.value, c.value


def npo_euclid_grad(plan, lam, scale, out, stream=None):
    _check(lib().npo_euclid_grad(plan, _fld(plan, lam, "lam"), scale, _fld(plan, out, "out"), _stream(stream)))


# ------------------------------------------------------------- batches
def _parr(ptrs):
    return (_P * len(ptrs))(*[p if isinstance(p, ctypes.c_void_p) else ctypes.c_void_p(p) for p in ptrs])


def npo_batch_create(plans):
    """plans: list of plan handles (they must outlive the batch)."""
    h = _P()
    _check(lib().npo_batch_create(_parr(plans), len(plans), ctypes.byref(h)))
    return h


def npo_batch_destroy(batch):
    _check(lib().npo_batch_destroy(batch))


def npo_batch_info(batch):
    a, b_, c = _I32(), _I32(), _I32()
    _check(lib().npo_batch_info(batch, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c)))
    return {"classes": a.value, "batched": b_.value, "launches": c.value}


def _batch_ws(plans, ws):
    return _parr([_wsp(p, w) for p, w in zip(plans, ws)])


def npo_batch_set_steps(batch, plans, ws, n, stream=None):
    _check(lib().npo_batch_set_steps(batch, _batch_ws(plans, ws), n, _stream(stream)))


def npo_batch_step(batch, plans, ws, states, phase, stream=None):
    """phase 0: states = [u_i]; phase 1: states = [u_i, lam_i, u_j, lam_j, ...]."""
    per = 2 if phase else 1
    ptrs = [_fld(plans[k // per], t, "state") for k, t in enumerate(states)]
    if len(ptrs) != per * len(plans):
        raise NpoError(f"{per * len(plans)} states expected")
    _check(lib().npo_batch_step(batch, _parr(ptrs), _batch_ws(plans, ws), phase, _stream(stream)))


def npo_batch_forward_run(batch, plans, ws, ckpts, n_ckpt, u0s, uNs, stream=None):
    _check(lib().npo_batch_forward_run(
        batch, _batch_ws(plans, ws), _parr([_fld(p, c, "checkpoint arena", max(int(n_ckpt), 1)) for p, c in zip(plans, ckpts)]),
        n_ckpt, _parr([_fld(p, u, "u0") for p, u in zip(plans, u0s)]),
        _parr([_fld(p, u, "uN") for p, u in zip(plans, uNs)]), _stream(stream)))


def npo_batch_adjoint_run(batch, plans, ws, ckpts, n_ckpt, lamNs, lam0s, stream=None):
    c = _I64()
    _check(lib().npo_batch_adjoint_run(
        batch, _batch_ws(plans, ws), _parr([_fld(p, a, "checkpoint arena", max(int(n_ckpt), 1)) for p, a in zip(plans, ckpts)]),
        n_ckpt, _parr([_fld(p, u, "lamN") for p, u in zip(plans, lamNs)]),
        _parr([_fld(p, u, "lam0") for p, u in zip(plans, lam0s)]), ctypes.byref(c), _stream(stream)))
    return c.value


def npo_profile_begin(plan, stride=1):
    _check(lib().npo_profile_begin(plan, stride))


def npo_profile_read(plan):
    n = len(KERNEL_FAMILIES)
    la = (_I64 * n)()
    sa = (_I64 * n)()
    av = np.zeros(n)
    _check(lib().npo_profile_read(plan, la, sa, av.ctypes.data_as(_DP)))
    return {k: dict(launches=la[i], sampled=sa[i], avg_ms=float(av[i])) for i, k in enumerate(KERNEL_FAMILIES)}


# ------------------------------------------------------- convenience
class Plan:
    """A plan plus its device workspace (torch allocations)."""

    def __init__(self, nr, ntheta, nz, lz, re, wo, amp, dt, t0=0.0, nsteps=1, ncorr=2, device="cuda"):
        import torch
        self.handle = npo_plan_create(nr, ntheta, nz, lz, re, wo, amp, dt, t0, nsteps, ncorr)
        self.info = npo_plan_info(self.handle)
        self.nr, self.M, self.K = nr, self.info["M"], self.info["K"]
        self.shape = (3, nr, self.M + 1, 2 * self.K + 1)
        self.device = device
        self.ws = torch.empty(self.info["workspace_bytes"], dtype=torch.uint8, device=device)
        self.scal = torch.zeros(8, dtype=torch.float64, device=device)

    def field(self):
        import torch
        return torch.zeros(self.shape, dtype=torch.complex128, device=self.device)

    def arena(self, n_ckpt):
        import torch
        return torch.empty((n_ckpt,) + self.shape, dtype=torch.complex128, device=self.device)

    def inner(self, a, b):
        npo_inner(self.handle, self.ws, a, b, self.scal)
        return float(self.scal[0].item())

    def energy(self, u):
        return 0.5 * self.inner(u, u)

    def close(self):
        if self.handle:
            npo_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
