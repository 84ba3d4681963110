"""ctypes binding of liblaglddmm (argument marshalling only).

Every function here forwards to the C-ABI entry point of the same name in
``include/laglddmm.h``; the work runs in the HIP kernels of the library.
Tensors must be float32, contiguous and on the current HIP device; the call
is enqueued on torch's current stream.  A missing library is an error: there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblaglddmm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "laglddmm.h")

LAG_OK, LAG_EINVAL, LAG_EUNSUPPORTED, LAG_EHIP, LAG_ENOMEM, LAG_EBREAKDOWN, LAG_ELINESEARCH, LAG_ETOOLARGE = range(8)
LAG_TRANSPORT, LAG_CONTINUITY = 0, 1
LAG_DIFFUSION, LAG_CURVATURE = 0, 1


class LagProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("img_m", ctypes.c_int32 * 3),
        ("vel_m", ctypes.c_int32 * 3),
        ("extent", ctypes.c_double * 3),
        ("nt_nodes", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("reg", ctypes.c_int32),
        ("nsteps", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("jac_blocks", ctypes.c_int32),
    ]


class LagPcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("relres", ctypes.c_double)]


class LagGnOptions(ctypes.Structure):
    _fields_ = [("gtol", ctypes.c_double), ("max_gn", ctypes.c_int32),
                ("pcg_tol", ctypes.c_double), ("pcg_maxit", ctypes.c_int32),
                ("armijo_c1", ctypes.c_double), ("max_halvings", ctypes.c_int32),
                ("graph_iters", ctypes.c_int32)]


class LagGnStepInfo(ctypes.Structure):
    _fields_ = [("assembled", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("halvings", ctypes.c_int32),
                ("stopped", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("J", ctypes.c_double), ("gnorm", ctypes.c_double),
                ("J_next", ctypes.c_double), ("mu", ctypes.c_double)]


class LagGnInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("J0", ctypes.c_double), ("J", ctypes.c_double),
                ("g0", ctypes.c_double), ("gnorm", ctypes.c_double)]


class LagCnnConfig(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("channels", ctypes.c_int32 * 4), ("in_scale", ctypes.c_float),
                ("out_scale", ctypes.c_float), ("seed", ctypes.c_uint64)]


class LagError(RuntimeError):
    def __init__(self, name, status, detail=""):
        self.status = status
        msg = f"{name} failed: {strerror(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "lag_problem_check": (_I, [ctypes.POINTER(LagProblem)]),
    "lag_problem_sizes": (_I, [ctypes.POINTER(LagProblem), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int64)]),
    "lag_strerror": (ctypes.c_char_p, [_I]),
    "lag_last_hip_error": (ctypes.c_char_p, []),
    "lag_plan_create": (_I, [ctypes.POINTER(LagProblem), ctypes.POINTER(_P)]),
    "lag_plan_create_tuned": (_I, [ctypes.POINTER(LagProblem), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_P)]),
    "lag_autotune_bricks": (_I, [ctypes.POINTER(LagProblem), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double), _P]),
    "lag_batch_solve": (_I, [ctypes.c_int32, ctypes.POINTER(LagProblem), ctypes.POINTER(_P), ctypes.POINTER(_P),
                             ctypes.POINTER(_P), ctypes.POINTER(LagGnOptions), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(LagGnInfo),
                             ctypes.POINTER(ctypes.c_int32)]),
    "lag_batch_solve_graph": (_I, [ctypes.c_int32, ctypes.POINTER(LagProblem), ctypes.POINTER(_P),
                                   ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(LagGnOptions),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(LagGnInfo),
                                   ctypes.POINTER(ctypes.c_int32)]),
    "lag_plan_destroy": (_I, [_P]),
    "lag_plan_problem": (_I, [_P, ctypes.POINTER(LagProblem)]),
    "lag_plan_flags": (_I, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _P]),
    "lag_adjoint_stats": (_I, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _P]),
    "lag_profile_enable": (_I, [_P, ctypes.c_int32]),
    "lag_profile_read": (_I, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "lag_trace": (_I, [_P, _P, ctypes.c_int32, _P, _P]),
    "lag_transport": (_I, [_P, _P, _P, _P, _P]),
    "lag_pushforward": (_I, [_P, _P, _P, _P, _P]),
    "lag_pushforward_noalloc": (_I, [ctypes.POINTER(LagProblem), _P, _P, _P, _P]),
    "lag_jvp": (_I, [_P, _P, _P, _P, _P, _P]),
    "lag_vjp": (_I, [_P, _P, _P, _P, _P, _P]),
    "gn_hessmat": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "spectral_precond_apply": (_I, [_P, _P, _P, _P]),
    "lag_reg_apply": (_I, [_P, _P, _P, _P]),
    "lag_objective": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "lag_gradient": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "lag_gradient_at_zero": (_I, [_P, _P, _P, _P, _P, _P]),
    "lag_dot": (_I, [_P, ctypes.c_int64, _P, _P, _P, _P]),
    "lag_pcg": (_I, [_P, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_int32,
                     ctypes.POINTER(LagPcgInfo), _P]),
    "lag_gn_default_options": (None, [ctypes.POINTER(LagGnOptions)]),
    "lag_restrict_image": (_I, [_P, _P, _P, _P]),
    "lag_prolong_velocity": (_I, [_P, _P, _P, _P]),
    "lag_resample_to_velocity_grid": (_I, [_P, _P, _P, _P]),
    "lag_multilevel_solve": (_I, [ctypes.POINTER(LagProblem), ctypes.c_int32, _P, _P, _P,
                                  ctypes.POINTER(LagGnOptions), ctypes.POINTER(LagGnInfo), _P]),
    "lag_jacobian_assemble": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_int32), _P]),
    "gn_hessmat_assembled": (_I, [_P, _P, _P, _P, _P]),
    "lag_jacobian_info": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)]),
    "lag_vjp_assembled": (_I, [_P, _P, _P, _P]),
    "lag_gradient_assembled": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "lag_pcg_assembled": (_I, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32,
                               ctypes.POINTER(LagPcgInfo), _P]),
    "lag_pcg_graph": (_I, [_P, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(LagPcgInfo), _P]),
    "lag_pcg_assembled_graph": (_I, [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(LagPcgInfo), _P]),
    "lag_gn_step": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(LagGnOptions), ctypes.c_double,
                         ctypes.POINTER(LagGnStepInfo), _P]),
    "lag_gn_solve": (_I, [_P, _P, _P, _P, ctypes.POINTER(LagGnOptions),
                          ctypes.POINTER(LagGnInfo), _P]),
    "lag_cnn_default_config": (None, [ctypes.POINTER(LagCnnConfig)]),
    "lag_cnn_create": (_I, [ctypes.POINTER(LagCnnConfig), ctypes.POINTER(_P)]),
    "lag_cnn_destroy": (_I, [_P]),
    "lag_cnn_param_count": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lag_cnn_get_params": (_I, [_P, _P]),
    "lag_cnn_set_params": (_I, [_P, _P]),
    "lag_cnn_get_grads": (_I, [_P, _P]),
    "lag_cnn_forward": (_I, [_P, _P, _P, _P, _P]),
    "lag_cnn_backward": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "lag_cnn_adam_step": (_I, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
}


def header_symbols(path=HEADER):
    """Names of the functions ``include/laglddmm.h`` declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def load(path=LIB_PATH):
    """Load the shared library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"liblaglddmm.so not built at {path}; run paper_1703_04446_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(status):
    return load().lag_strerror(int(status)).decode()


def _check(name, status):
    if status != LAG_OK:
        detail = ""
        if status == LAG_EHIP:
            detail = load().lag_last_hip_error().decode()
        raise LagError(name, status, detail)


def make_problem(dim, img_m, vel_m, nt_nodes=1, model="transport", reg="diffusion", nsteps=5,
                 alpha=1e-2, gamma=0.0, extent=(1.0, 1.0, 1.0), jac_blocks=0):
    """Fill a ``lag_problem`` (sizes x first; unused axes become 1).

    ``jac_blocks`` > 0 gives the plan storage for an assembled Jacobian
    (transport model with a stationary velocity only)."""
    p = LagProblem()
    p.dim = dim
    for a in range(3):
        p.img_m[a] = int(img_m[a]) if a < dim else 1
        p.vel_m[a] = int(vel_m[a]) if a < dim else 1
        p.extent[a] = float(extent[a]) if a < len(extent) else 1.0
    p.nt_nodes = nt_nodes
    p.model = {"transport": LAG_TRANSPORT, "continuity": LAG_CONTINUITY}[model] if isinstance(model, str) else model
    p.reg = {"diffusion": LAG_DIFFUSION, "curvature": LAG_CURVATURE}[reg] if isinstance(reg, str) else reg
    p.nsteps = nsteps
    p.alpha = alpha
    p.gamma = gamma
    p.jac_blocks = jac_blocks
    return p


def lag_problem_check(prob):
    return load().lag_problem_check(ctypes.byref(prob))


def lag_problem_sizes(prob):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check("lag_problem_sizes", load().lag_problem_sizes(ctypes.byref(prob), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


# ---------------------------------------------------------------------------
# device-side helpers (torch is used for memory and streams only)

def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, n=None, name="tensor", f64=False):
    """Device pointer of a contiguous GPU tensor: float32, or float64 where
    the C-ABI argument is a double* (f64=True)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    want = torch.float64 if f64 else torch.float32
    if t.dtype != want or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {want} tensor on the GPU, got {t.dtype} "
                         f"({'GPU' if t.is_cuda else 'CPU'}, {'contiguous' if t.is_contiguous() else 'strided'})")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owns a ``lag_plan``; sizes are read from the problem.  ``bricks``
    (image cells per brick per axis, e.g. from lag_autotune_bricks) selects
    lag_plan_create_tuned."""

    def __init__(self, prob: LagProblem, bricks=None):
        self.prob = prob
        self.n_points, self.n_unknowns = lag_problem_sizes(prob)
        h = ctypes.c_void_p()
        if bricks is None:
            _check("lag_plan_create", load().lag_plan_create(ctypes.byref(prob), ctypes.byref(h)))
        else:
            b = (ctypes.c_int32 * 3)(*[int(x) for x in (list(bricks) + [1, 1, 1])[:3]])
            _check("lag_plan_create_tuned", load().lag_plan_create_tuned(ctypes.byref(prob), b, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().lag_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def lag_plan_create(prob):
    return Plan(prob)


def lag_plan_destroy(plan):
    plan.close()


def lag_plan_flags(plan, clear=True):
    """Status bits of the plan's adjoint kernels (synchronises the stream)."""
    f = ctypes.c_int32()
    _check("lag_plan_flags", load().lag_plan_flags(plan.handle, ctypes.byref(f), int(bool(clear)), _stream()))
    return f.value


def lag_adjoint_stats(plan):
    """(deferred characteristics, bricks redone) of the last matrix-free
    adjoint product (synchronises the stream)."""
    d, r = ctypes.c_int32(), ctypes.c_int32()
    _check("lag_adjoint_stats", load().lag_adjoint_stats(plan.handle, ctypes.byref(d), ctypes.byref(r), _stream()))
    return d.value, r.value


def lag_profile_enable(plan, enable=True):
    _check("lag_profile_enable", load().lag_profile_enable(plan.handle, int(bool(enable))))


def lag_profile_read(plan):
    """(summed milliseconds, launches) of the timed matvec kernel launches."""
    ms, n = ctypes.c_double(), ctypes.c_int32()
    _check("lag_profile_read", load().lag_profile_read(plan.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def lag_trace(plan, v, direction, phi):
    _check("lag_trace", load().lag_trace(plan.handle, _ptr(v, plan.n_unknowns, "v"), int(direction),
                                         _ptr(phi, plan.prob.dim * plan.n_points, "phi"), _stream()))


def lag_transport(plan, T, phi, u):
    _check("lag_transport", load().lag_transport(plan.handle, _ptr(T, plan.n_points, "T"),
                                                 _ptr(phi, plan.prob.dim * plan.n_points, "phi"),
                                                 _ptr(u, plan.n_points, "u"), _stream()))


def lag_pushforward(plan, T, phi, u):
    _check("lag_pushforward", load().lag_pushforward(plan.handle, _ptr(T, plan.n_points, "T"),
                                                     _ptr(phi, plan.prob.dim * plan.n_points, "phi"),
                                                     _ptr(u, plan.n_points, "u"), _stream()))


def lag_pushforward_noalloc(prob, T, phi, u):
    """lag_pushforward without a plan; the library allocates nothing (its
    scratch is a fixed device array per GPU).  ``prob`` is a LagProblem."""
    n, _ = lag_problem_sizes(prob)
    _check("lag_pushforward_noalloc", load().lag_pushforward_noalloc(
        ctypes.byref(prob), _ptr(T, n, "T"), _ptr(phi, prob.dim * n, "phi"), _ptr(u, n, "u"), _stream()))


def lag_jvp(plan, v, T, dv, Jdv):
    _check("lag_jvp", load().lag_jvp(plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"),
                                     _ptr(dv, plan.n_unknowns, "dv"), _ptr(Jdv, plan.n_points, "Jdv"), _stream()))


def lag_vjp(plan, v, T, w, JTw):
    _check("lag_vjp", load().lag_vjp(plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"),
                                     _ptr(w, plan.n_points, "w"), _ptr(JTw, plan.n_unknowns, "JTw"), _stream()))


def gn_hessmat(plan, v, T, wvox, p, Hp):
    _check("gn_hessmat", load().gn_hessmat(plan.handle, _ptr(v, plan.n_unknowns, "v"),
                                           _ptr(T, plan.n_points, "T"), _ptr(wvox, plan.n_points, "wvox"),
                                           _ptr(p, plan.n_unknowns, "p"), _ptr(Hp, plan.n_unknowns, "Hp"),
                                           _stream()))


def spectral_precond_apply(plan, r, z):
    _check("spectral_precond_apply", load().spectral_precond_apply(
        plan.handle, _ptr(r, plan.n_unknowns, "r"), _ptr(z, plan.n_unknowns, "z"), _stream()))


def lag_reg_apply(plan, p, out):
    _check("lag_reg_apply", load().lag_reg_apply(plan.handle, _ptr(p, plan.n_unknowns, "p"),
                                                 _ptr(out, plan.n_unknowns, "out"), _stream()))


def lag_objective(plan, v, T, R, u, out3):
    _check("lag_objective", load().lag_objective(plan.handle, _ptr(v, plan.n_unknowns, "v"),
                                                 _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"),
                                                 _ptr(u, plan.n_points, "u"), _ptr(out3, 3, "out3", f64=True), _stream()))


def lag_gradient(plan, v, T, R, g, out3):
    _check("lag_gradient", load().lag_gradient(plan.handle, _ptr(v, plan.n_unknowns, "v"),
                                               _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"),
                                               _ptr(g, plan.n_unknowns, "g"), _ptr(out3, 3, "out3", f64=True), _stream()))


def lag_gradient_at_zero(plan, T, R, g, out3=None):
    _check("lag_gradient_at_zero", load().lag_gradient_at_zero(
        plan.handle, _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"), _ptr(g, plan.n_unknowns, "g"),
        _ptr(out3, 3, "out3", f64=True), _stream()))


def lag_dot(plan, x, y, out):
    n = x.numel()
    _check("lag_dot", load().lag_dot(plan.handle, n, _ptr(x, n, "x"), _ptr(y, n, "y"), _ptr(out, 1, "out", f64=True),
                                     _stream()))


def lag_pcg(plan, v, T, wvox, b, x, tol=0.1, maxit=50):
    info = LagPcgInfo()
    st = load().lag_pcg(plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"),
                        _ptr(wvox, plan.n_points, "wvox"), _ptr(b, plan.n_unknowns, "b"),
                        _ptr(x, plan.n_unknowns, "x"), float(tol), int(maxit), ctypes.byref(info), _stream())
    if st not in (LAG_OK, LAG_EBREAKDOWN):
        _check("lag_pcg", st)
    return {"iters": info.iters, "matvecs": info.matvecs, "breakdown": bool(info.breakdown),
            "relres": info.relres, "status": st}


def lag_jacobian_assemble(plan, v, T):
    """Assemble J(v); returns True if it fit the plan's capacity."""
    stored = ctypes.c_int32()
    _check("lag_jacobian_assemble", load().lag_jacobian_assemble(
        plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"), ctypes.byref(stored),
        _stream()))
    return bool(stored.value)


def lag_jacobian_info(plan):
    """(stored blocks, largest per-row block count, bytes per block)."""
    b, m, nb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check("lag_jacobian_info", load().lag_jacobian_info(plan.handle, ctypes.byref(b), ctypes.byref(m),
                                                         ctypes.byref(nb)))
    return b.value, m.value, nb.value


def gn_hessmat_assembled(plan, wvox, p, Hp):
    _check("gn_hessmat_assembled", load().gn_hessmat_assembled(
        plan.handle, _ptr(wvox, plan.n_points, "wvox"), _ptr(p, plan.n_unknowns, "p"),
        _ptr(Hp, plan.n_unknowns, "Hp"), _stream()))


def lag_vjp_assembled(plan, w, JTw):
    _check("lag_vjp_assembled", load().lag_vjp_assembled(
        plan.handle, _ptr(w, plan.n_points, "w"), _ptr(JTw, plan.n_unknowns, "JTw"), _stream()))


def lag_gradient_assembled(plan, v, T, R, g, out3):
    _check("lag_gradient_assembled", load().lag_gradient_assembled(
        plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"),
        _ptr(g, plan.n_unknowns, "g"), _ptr(out3, 3, "out3", f64=True), _stream()))


def lag_pcg_assembled(plan, wvox, b, x, tol=0.1, maxit=50):
    info = LagPcgInfo()
    st = load().lag_pcg_assembled(plan.handle, _ptr(wvox, plan.n_points, "wvox"), _ptr(b, plan.n_unknowns, "b"),
                                  _ptr(x, plan.n_unknowns, "x"), float(tol), int(maxit), ctypes.byref(info),
                                  _stream())
    if st not in (LAG_OK, LAG_EBREAKDOWN):
        _check("lag_pcg_assembled", st)
    return {"iters": info.iters, "matvecs": info.matvecs, "breakdown": bool(info.breakdown),
            "relres": info.relres, "status": st}


def lag_pcg_graph(plan, v, T, wvox, b, x, tol=0.1, maxit=50, iters_per_graph=4):
    info = LagPcgInfo()
    st = load().lag_pcg_graph(plan.handle, _ptr(v, plan.n_unknowns, "v"), _ptr(T, plan.n_points, "T"),
                              _ptr(wvox, plan.n_points, "wvox"), _ptr(b, plan.n_unknowns, "b"),
                              _ptr(x, plan.n_unknowns, "x"), float(tol), int(maxit), int(iters_per_graph),
                              ctypes.byref(info), _stream())
    if st not in (LAG_OK, LAG_EBREAKDOWN):
        _check("lag_pcg_graph", st)
    return {"iters": info.iters, "matvecs": info.matvecs, "breakdown": bool(info.breakdown),
            "relres": info.relres, "status": st}


def lag_pcg_assembled_graph(plan, wvox, b, x, tol=0.1, maxit=50, iters_per_graph=4):
    info = LagPcgInfo()
    st = load().lag_pcg_assembled_graph(plan.handle, _ptr(wvox, plan.n_points, "wvox"),
                                        _ptr(b, plan.n_unknowns, "b"), _ptr(x, plan.n_unknowns, "x"),
                                        float(tol), int(maxit), int(iters_per_graph), ctypes.byref(info),
                                        _stream())
    if st not in (LAG_OK, LAG_EBREAKDOWN):
        _check("lag_pcg_assembled_graph", st)
    return {"iters": info.iters, "matvecs": info.matvecs, "breakdown": bool(info.breakdown),
            "relres": info.relres, "status": st}


def lag_gn_step(plan, T, R, v, v_next, options=None, gstop=0.0):
    o = options if options is not None else lag_gn_default_options()
    info = LagGnStepInfo()
    st = load().lag_gn_step(plan.handle, _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"),
                            _ptr(v, plan.n_unknowns, "v"), _ptr(v_next, plan.n_unknowns, "v_next"),
                            ctypes.byref(o), float(gstop), ctypes.byref(info), _stream())
    if st not in (LAG_OK, LAG_ELINESEARCH):
        _check("lag_gn_step", st)
    d = {f: getattr(info, f) for f, _ in LagGnStepInfo._fields_}
    d["status"] = st
    return d


def lag_restrict_image(plan, f, coarse):
    n = plan.n_points
    _check("lag_restrict_image", load().lag_restrict_image(
        plan.handle, _ptr(f, n, "f"), _ptr(coarse, n >> plan.prob.dim, "coarse"), _stream()))


def lag_prolong_velocity(plan, v_coarse, v_fine):
    nu = plan.n_unknowns
    _check("lag_prolong_velocity", load().lag_prolong_velocity(
        plan.handle, _ptr(v_coarse, nu >> plan.prob.dim, "v_coarse"), _ptr(v_fine, nu, "v_fine"), _stream()))


def lag_resample_to_velocity_grid(plan, f, out):
    nvel = plan.n_unknowns // (plan.prob.nt_nodes * plan.prob.dim)
    _check("lag_resample_to_velocity_grid", load().lag_resample_to_velocity_grid(
        plan.handle, _ptr(f, plan.n_points, "f"), _ptr(out, nvel, "out"), _stream()))


def lag_multilevel_solve(prob, levels, T, R, v, options=None):
    """Coarse-to-fine solve; returns one info dict per level (coarsest first)."""
    o = options if options is not None else lag_gn_default_options()
    n_points, n_unknowns = lag_problem_sizes(prob)
    infos = (LagGnInfo * levels)()
    st = load().lag_multilevel_solve(ctypes.byref(prob), int(levels), _ptr(T, n_points, "T"),
                                     _ptr(R, n_points, "R"), _ptr(v, n_unknowns, "v"), ctypes.byref(o),
                                     infos, _stream())
    if st not in (LAG_OK, LAG_ELINESEARCH):
        _check("lag_multilevel_solve", st)
    out = []
    for i in range(levels):
        d = {f: getattr(infos[i], f) for f, _ in LagGnInfo._fields_}
        d["converged"] = bool(d["converged"])
        out.append(d)
    return out, st


def lag_gn_default_options():
    o = LagGnOptions()
    load().lag_gn_default_options(ctypes.byref(o))
    return o


def lag_gn_solve(plan, T, R, v, options=None):
    o = options if options is not None else lag_gn_default_options()
    info = LagGnInfo()
    st = load().lag_gn_solve(plan.handle, _ptr(T, plan.n_points, "T"), _ptr(R, plan.n_points, "R"),
                             _ptr(v, plan.n_unknowns, "v"), ctypes.byref(o), ctypes.byref(info), _stream())
    if st not in (LAG_OK, LAG_ELINESEARCH):
        _check("lag_gn_solve", st)
    return {"iters": info.iters, "pcg_iters": info.pcg_iters, "matvecs": info.matvecs,
            "converged": bool(info.converged), "J0": info.J0, "J": info.J, "g0": info.g0,
            "gnorm": info.gnorm, "status": st}


def problem_arrays_to_device(*arrays):
    """float32 contiguous device copies of NumPy arrays (test/bench helper)."""
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrays]


# ---- learned warm start ------------------------------------------------------

def lag_cnn_default_config():
    c = LagCnnConfig()
    load().lag_cnn_default_config(ctypes.byref(c))
    return c


class Cnn:
    """Owns a ``lag_cnn`` (the warm-start U-Net); parameters live on the GPU."""

    def __init__(self, config: LagCnnConfig | None = None):
        self.config = config if config is not None else lag_cnn_default_config()
        h = ctypes.c_void_p()
        _check("lag_cnn_create", load().lag_cnn_create(ctypes.byref(self.config), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        _check("lag_cnn_param_count", load().lag_cnn_param_count(h, ctypes.byref(n)))
        self.n_params = n.value
        self.size = self.config.size
        self.n_voxels = self.size ** 3

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().lag_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def lag_cnn_create(config=None):
    return Cnn(config)


def lag_cnn_destroy(net):
    net.close()


def lag_cnn_get_params(net):
    out = np.empty(net.n_params, dtype=np.float32)
    _check("lag_cnn_get_params", load().lag_cnn_get_params(net.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def lag_cnn_set_params(net, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != net.n_params:
        raise ValueError(f"expected {net.n_params} parameters, got {a.size}")
    _check("lag_cnn_set_params", load().lag_cnn_set_params(net.handle, a.ctypes.data_as(ctypes.c_void_p)))


def lag_cnn_get_grads(net):
    out = np.empty(net.n_params, dtype=np.float32)
    _check("lag_cnn_get_grads", load().lag_cnn_get_grads(net.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def lag_cnn_forward(net, T, R, v):
    n = net.n_voxels
    _check("lag_cnn_forward", load().lag_cnn_forward(net.handle, _ptr(T, n, "T"), _ptr(R, n, "R"),
                                                     _ptr(v, 3 * n, "v"), _stream()))


def lag_cnn_backward(net, T, R, target, v, loss):
    """Forward, loss (device float64 scalar tensor) and parameter gradients."""
    n = net.n_voxels
    _check("lag_cnn_backward", load().lag_cnn_backward(net.handle, _ptr(T, n, "T"), _ptr(R, n, "R"),
                                                       _ptr(target, 3 * n, "target"), _ptr(v, 3 * n, "v"),
                                                       _ptr(loss, 1, "loss", f64=True), _stream()))


def lag_cnn_adam_step(net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check("lag_cnn_adam_step", load().lag_cnn_adam_step(net.handle, float(lr), float(beta1), float(beta2),
                                                         float(eps), _stream()))


# ---- many problems at once -------------------------------------------------

def lag_autotune_bricks(prob):
    """(best brick target (3 ints), milliseconds per Gauss-Newton matvec)."""
    b = (ctypes.c_int32 * 3)()
    ms = ctypes.c_double()
    _check("lag_autotune_bricks", load().lag_autotune_bricks(ctypes.byref(prob), b, ctypes.byref(ms), _stream()))
    return [b[0], b[1], b[2]], ms.value


def lag_batch_solve(probs, Ts, Rs, vs, options=None, workers=4, autotune=True, bricks=None):
    """Solve len(probs) independent problems; returns (infos, statuses).
    ``bricks``: per pair a 3-list of brick targets (overrides autotune).
    ``workers=0`` calls lag_batch_solve_graph (lockstep, the PCG iterations of
    all pairs in one captured graph; autotune is then ignored)."""
    n = len(probs)
    if not (len(Ts) == len(Rs) == len(vs) == n):
        raise ValueError("probs, Ts, Rs and vs must have the same length")
    arr = (LagProblem * n)(*probs)
    ptrs = []
    for i in range(n):
        npnt, nu = lag_problem_sizes(probs[i])
        ptrs.append((_ptr(Ts[i], npnt, f"T[{i}]"), _ptr(Rs[i], npnt, f"R[{i}]"), _ptr(vs[i], nu, f"v[{i}]")))
    T = (ctypes.c_void_p * n)(*[p[0] for p in ptrs])
    R = (ctypes.c_void_p * n)(*[p[1] for p in ptrs])
    V = (ctypes.c_void_p * n)(*[p[2] for p in ptrs])
    o = options if options is not None else lag_gn_default_options()
    infos = (LagGnInfo * n)()
    st = (ctypes.c_int32 * n)()
    import torch
    torch.cuda.synchronize()       # inputs written on torch's stream are visible to the workers' streams
    bp = None
    if bricks is not None:
        flat = [int(x) for b in bricks for x in (list(b) + [1, 1, 1])[:3]]
        if len(flat) != 3 * n:
            raise ValueError("bricks: one 3-list per pair")
        bp = (ctypes.c_int32 * (3 * n))(*flat)
    if workers == 0:   # lockstep, PCG of all pairs in one captured graph
        rc = load().lag_batch_solve_graph(n, arr, T, R, V, ctypes.byref(o), bp, infos, st)
    else:
        rc = load().lag_batch_solve(n, arr, T, R, V, ctypes.byref(o), int(workers), bp, int(bool(autotune)),
                                    infos, st)
    if rc not in (LAG_OK, LAG_ELINESEARCH):
        _check("lag_batch_solve_graph" if workers == 0 else "lag_batch_solve", rc)
    out = []
    for i in range(n):
        d = {f: getattr(infos[i], f) for f, _ in LagGnInfo._fields_}
        d["converged"] = bool(d["converged"])
        out.append(d)
    return out, list(st)
