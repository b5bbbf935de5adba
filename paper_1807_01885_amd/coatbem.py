"""Thin ctypes binding of libcoatbem (argument marshalling only).

The names mirror the C-ABI in include/coatbem.h.  Arrays are torch tensors
on the GPU (device memory and streams come from PyTorch); every step of
the computation runs in the library's HIP kernels.  If the built library
is missing this module raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoatbem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_1807_01885_amd.build` "
        "(libcoatbem has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

CB_OK = 0
CB_E_INVALID = -1
CB_E_NOMEM = -2
CB_E_DEVICE = -3
CB_E_NOCONV = -4
CB_E_NONFINITE = -5
CB_E_STATE = -6
CB_E_UNSUPPORTED = -7
CB_FP64 = 0
CB_FP32 = 1
CB_DC_BZ = 0
CB_DC_ZERO = 1
CB_KERNEL_PADDED = 0
CB_KERNEL_PERIODIC = 1
CB_KERNEL_EXACT = 2
_KERNEL_MODES = {"padded": CB_KERNEL_PADDED, "periodic": CB_KERNEL_PERIODIC, "exact": CB_KERNEL_EXACT}


class cb_plan_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("dc_mode", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("autotune", ctypes.c_int),
                ("tune_cache", ctypes.c_char_p), ("fft_variant", ctypes.c_int),
                ("kernel_mode", ctypes.c_int)]


class cb_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("chunk", ctypes.c_int), ("init", ctypes.c_int),
                ("attach_tol", ctypes.c_double), ("max_rounds", ctypes.c_int),
                ("precond", ctypes.c_int), ("preload_d", ctypes.c_double)]


class cb_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("rounds", ctypes.c_int), ("resid", ctypes.c_double),
                ("F", ctypes.c_double), ("d", ctypes.c_double),
                ("area", ctypes.c_double), ("U_el", ctypes.c_double),
                ("U_ad", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cb_plan_info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("M", ctypes.c_int),
                ("precision", ctypes.c_int), ("dc_mode", ctypes.c_int),
                ("L", ctypes.c_double), ("dx", ctypes.c_double),
                ("h", ctypes.c_double), ("E1", ctypes.c_double),
                ("nu1", ctypes.c_double), ("E2", ctypes.c_double),
                ("nu2", ctypes.c_double), ("dgamma", ctypes.c_double),
                ("E1s", ctypes.c_double), ("E2s", ctypes.c_double),
                ("sigma_c", ctypes.c_double), ("k00", ctypes.c_double),
                ("dc", ctypes.c_double), ("validity_warning", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("fft_variant", ctypes.c_int),
                ("tune_us", ctypes.c_double), ("kernel_mode", ctypes.c_int),
                ("table_n", ctypes.c_int), ("nlayers", ctypes.c_int), ("H", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_d = ctypes.c_double
_i = ctypes.c_int
_SIGS = {
    "cb_plan_create": (_i, [ctypes.POINTER(_vp), _i, _d, _d, _d, _d, _d, _d, _d,
                            ctypes.POINTER(cb_plan_opts)]),
    "cb_plan_create_layered": (_i, [ctypes.POINTER(_vp), _i, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d),
                                    ctypes.POINTER(_d), _d, _d, _d, ctypes.POINTER(cb_plan_opts)]),
    "cb_transfer_table_layered": (_i, [_i, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                       _d, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "cb_plan_destroy": (_i, [_vp]),
    "cb_plan_get_info": (_i, [_vp, ctypes.POINTER(cb_plan_info)]),
    "cb_plan_get_table": (_i, [_vp, ctypes.POINTER(_d)]),
    "cb_plan_set_stream": (_i, [_vp, _vp]),
    "cb_transfer_table": (_i, [_i, _d, _d, _d, _d, _d, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "cb_transfer_table_exact": (_i, [_i, _d, _d, _d, _d, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "cb_transfer_table_exact_layered": (_i, [_i, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                             _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "cb_apply_K": (_i, [_vp, _vp, _vp]),
    "cb_apply_K_stages": (_i, [_vp, _vp, _vp, _i]),
    "cb_apply_K_batch": (_i, [_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "cb_apply_K_noalloc": (_i, [_i, _i, _vp, _vp, _vp, _vp]),
    "cb_apply_precond": (_i, [_vp, _i, _vp, _vp]),
    "cb_solve_indent": (_i, [_vp, _vp, _d, _vp, _vp, ctypes.POINTER(cb_solve_opts),
                             ctypes.POINTER(cb_result)]),
    "cb_solve_force": (_i, [_vp, _vp, _d, _vp, _vp, ctypes.POINTER(cb_solve_opts),
                            ctypes.POINTER(cb_result)]),
    "cb_sweep": (_i, [_vp, _vp, ctypes.POINTER(_d), _i, _vp, _vp,
                      ctypes.POINTER(cb_solve_opts), ctypes.POINTER(cb_result)]),
    "cb_solve_batch": (_i, [_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_d),
                            ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(cb_solve_opts), _i,
                            ctypes.POINTER(cb_result)]),
    "cb_sweep_batch": (_i, [_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i),
                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(cb_solve_opts), _i,
                            ctypes.POINTER(_vp)]),
    "cb_net_num_params": (_i, []),
    "cb_net_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _vp]),
    "cb_net_destroy": (_i, [_vp]),
    "cb_net_set_params": (_i, [_vp, _vp]),
    "cb_net_get_params": (_i, [_vp, _vp]),
    "cb_net_forward": (_i, [_vp, _i, _vp, _vp]),
    "cb_net_loss_grad": (_i, [_vp, _i, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "cb_net_adam_step": (_i, [_vp, ctypes.c_float]),
    "cb_net_features": (_i, [_vp, _vp, _i, _d, _d, _d, _d, _d, _d, _d, _vp]),
    "cb_net_warmstart": (_i, [_vp, _vp, _vp, _d, _d, _vp]),
    "cb_net_warmstart_batch": (_i, [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_d), _d,
                                    ctypes.POINTER(_vp)]),
    "cb_status_string": (ctypes.c_char_p, [_i]),
    "cb_last_error": (ctypes.c_char_p, []),
    "cb_version": (_i, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class CoatbemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libcoatbem status {status} ({_lib.cb_status_string(status).decode()}): {msg}")
        self.status = status


def _check(rc):
    if rc != CB_OK:
        raise CoatbemError(rc, _lib.cb_last_error().decode())
    return rc


def cb_version():
    return _lib.cb_version()


def cb_status_string(status):
    return _lib.cb_status_string(status).decode()


@dataclass
class Plan:
    handle: ctypes.c_void_p
    N: int
    dtype: torch.dtype
    device: torch.device

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cb_plan_destroy(self.handle)
            self.handle = None


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def cb_plan_create(N, L, h, E1, nu1, E2, nu2, dgamma=0.0, precision="fp64",
                   dc_mode="bz", stream=None, autotune=0, tune_cache=None, fft_variant=0,
                   kernel_mode="padded"):
    opts = cb_plan_opts(CB_FP64 if precision == "fp64" else CB_FP32,
                        CB_DC_BZ if dc_mode == "bz" else CB_DC_ZERO,
                        _stream_ptr(stream), int(autotune),
                        None if tune_cache is None else os.fsencode(tune_cache), int(fft_variant),
                        _KERNEL_MODES[kernel_mode])
    h_ = ctypes.c_void_p()
    _check(_lib.cb_plan_create(ctypes.byref(h_), int(N), float(L), float(h),
                               float(E1), float(nu1), float(E2), float(nu2),
                               float(dgamma), ctypes.byref(opts)))
    return Plan(h_, int(N), torch.float64 if precision == "fp64" else torch.float32,
                torch.device("cuda", torch.cuda.current_device()))


def cb_plan_create_layered(N, L, layers, Es, nus, dgamma=0.0, precision="fp64", dc_mode="bz", stream=None,
                           autotune=0, tune_cache=None, fft_variant=0, kernel_mode="padded"):
    """layers: sequence of (h, E, nu), top layer first, on a half-space (Es, nus)."""
    n = len(layers)
    arr = lambda k: (_d * max(n, 1))(*[float(l[k]) for l in layers])
    opts = cb_plan_opts(CB_FP64 if precision == "fp64" else CB_FP32,
                        CB_DC_BZ if dc_mode == "bz" else CB_DC_ZERO,
                        _stream_ptr(stream), int(autotune),
                        None if tune_cache is None else os.fsencode(tune_cache), int(fft_variant),
                        _KERNEL_MODES[kernel_mode])
    h_ = ctypes.c_void_p()
    _check(_lib.cb_plan_create_layered(ctypes.byref(h_), int(N), float(L), n, arr(0), arr(1), arr(2),
                                       float(Es), float(nus), float(dgamma), ctypes.byref(opts)))
    return Plan(h_, int(N), torch.float64 if precision == "fp64" else torch.float32,
                torch.device("cuda", torch.cuda.current_device()))


def cb_transfer_table_layered(N, L, layers, Es, nus, dc_mode="bz"):
    """Host-computed FP64 padded table ((N+1)^2) of a layered stack and k00."""
    import numpy as np
    n = len(layers)
    arr = lambda k: (_d * max(n, 1))(*[float(l[k]) for l in layers])
    out = np.empty((N + 1, N + 1), dtype=np.float64)
    k00 = ctypes.c_double()
    _check(_lib.cb_transfer_table_layered(int(N), float(L), n, arr(0), arr(1), arr(2), float(Es), float(nus),
                                          CB_DC_BZ if dc_mode == "bz" else CB_DC_ZERO,
                                          out.ctypes.data_as(ctypes.POINTER(_d)), ctypes.byref(k00)))
    return out, k00.value


def cb_plan_destroy(plan: Plan):
    if plan.handle:
        _check(_lib.cb_plan_destroy(plan.handle))
        plan.handle = None


def cb_plan_get_info(plan: Plan):
    info = cb_plan_info()
    _check(_lib.cb_plan_get_info(plan.handle, ctypes.byref(info)))
    return info.as_dict()


def cb_plan_get_table(plan: Plan):
    import numpy as np
    n = cb_plan_get_info(plan)["table_n"]
    out = np.empty((n, n), dtype=np.float64)
    _check(_lib.cb_plan_get_table(plan.handle, out.ctypes.data_as(ctypes.POINTER(_d))))
    return out


def cb_transfer_table(N, L, h, E1, nu1, E2, nu2, dc_mode="bz"):
    """Host-computed FP64 table ((N+1)^2) and the self-influence k00."""
    import numpy as np
    out = np.empty((N + 1, N + 1), dtype=np.float64)
    k00 = ctypes.c_double()
    _check(_lib.cb_transfer_table(int(N), float(L), float(h), float(E1), float(nu1), float(E2),
                                  float(nu2), CB_DC_BZ if dc_mode == "bz" else CB_DC_ZERO,
                                  out.ctypes.data_as(ctypes.POINTER(_d)), ctypes.byref(k00)))
    return out, k00.value


def cb_transfer_table_exact(N, L, h, E1, nu1, E2, nu2):
    """Host-computed exact cell coefficients and their table: (T, D), both (N+1)^2."""
    import numpy as np
    T = np.empty((N + 1, N + 1), dtype=np.float64)
    D = np.empty((N + 1, N + 1), dtype=np.float64)
    _check(_lib.cb_transfer_table_exact(int(N), float(L), float(h), float(E1), float(nu1), float(E2), float(nu2),
                                        T.ctypes.data_as(ctypes.POINTER(_d)), D.ctypes.data_as(ctypes.POINTER(_d))))
    return T, D


def cb_transfer_table_exact_layered(N, L, layers, Es, nus):
    """As cb_transfer_table_exact for a stack (h, E, nu), top layer first."""
    import numpy as np
    n = len(layers)
    arr = lambda k: (_d * max(n, 1))(*[float(l[k]) for l in layers])
    T = np.empty((N + 1, N + 1), dtype=np.float64)
    D = np.empty((N + 1, N + 1), dtype=np.float64)
    _check(_lib.cb_transfer_table_exact_layered(int(N), float(L), n, arr(0), arr(1), arr(2), float(Es), float(nus),
                                                T.ctypes.data_as(ctypes.POINTER(_d)),
                                                D.ctypes.data_as(ctypes.POINTER(_d))))
    return T, D


def cb_plan_set_stream(plan: Plan, stream=None):
    _check(_lib.cb_plan_set_stream(plan.handle, _stream_ptr(stream)))


def _arr(plan: Plan, x, name, dtype=None):
    dtype = dtype or plan.dtype
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if x.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {x.dtype}")
    if tuple(x.shape) != (plan.N, plan.N) or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {plan.N}x{plan.N} tensor")
    return ctypes.c_void_p(x.data_ptr())


def _opts(tol=0.0, max_iter=0, chunk=0, init=0, attach_tol=-1.0, max_rounds=0, precond=-1, preload_d=-1e300):
    return cb_solve_opts(float(tol), int(max_iter), int(chunk), int(init),
                         float(attach_tol), int(max_rounds), int(precond), float(preload_d))


def cb_apply_K(plan: Plan, p, u):
    _check(_lib.cb_apply_K(plan.handle, _arr(plan, p, "p"), _arr(plan, u, "u")))
    return u


def cb_apply_K_noalloc(N, precision, table, p, u, stream=None):
    """u = K p without a plan or any allocation; table: device (N+1)^2 of
    K^/M^2 in the precision ("fp64" or "fp32") of p and u."""
    dtype = torch.float64 if precision == "fp64" else torch.float32
    for name, x, shape in (("table", table, (N + 1, N + 1)), ("p", p, (N, N)), ("u", u, (N, N))):
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != dtype:
            raise ValueError(f"{name} must be a {dtype} GPU tensor")
        if tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor of shape {shape}")
    _check(_lib.cb_apply_K_noalloc(int(N), CB_FP64 if precision == "fp64" else CB_FP32,
                                   ctypes.c_void_p(table.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                   ctypes.c_void_p(u.data_ptr()), _stream_ptr(stream)))
    return u


def cb_apply_K_batch(plans, ps, us):
    """u_i = K_i p_i for several plans of one size and precision in one launch per stage."""
    n = len(plans)
    hp = (_vp * n)(*[pl.handle for pl in plans])
    hx = (_vp * n)(*[_arr(pl, p, "p").value for pl, p in zip(plans, ps)])
    hy = (_vp * n)(*[_arr(pl, u, "u").value for pl, u in zip(plans, us)])
    _check(_lib.cb_apply_K_batch(n, hp, hx, hy))
    return us


def cb_apply_precond(plan: Plan, which, x, y):
    _check(_lib.cb_apply_precond(plan.handle, int(which), _arr(plan, x, "x"), _arr(plan, y, "y")))
    return y


def cb_apply_K_stages(plan: Plan, p, u, stage_mask):
    pp = _arr(plan, p, "p") if p is not None else None
    uu = _arr(plan, u, "u") if u is not None else None
    _check(_lib.cb_apply_K_stages(plan.handle, pp, uu, int(stage_mask)))


def cb_solve_indent(plan: Plan, f, d, p, mask=None, raise_on_error=True, **opts):
    """f, p: float64 for every plan (the solution state is FP64)."""
    res = cb_result()
    m = _arr(plan, mask, "mask", torch.uint8) if mask is not None else None
    rc = _lib.cb_solve_indent(plan.handle, _arr(plan, f, "f", torch.float64), float(d),
                              _arr(plan, p, "p", torch.float64),
                              m, ctypes.byref(_opts(**opts)), ctypes.byref(res))
    if raise_on_error:
        _check(rc)
    return res.as_dict()


def cb_solve_force(plan: Plan, f, F, p, mask=None, raise_on_error=True, **opts):
    """f, p: float64 for every plan (the solution state is FP64)."""
    res = cb_result()
    m = _arr(plan, mask, "mask", torch.uint8) if mask is not None else None
    rc = _lib.cb_solve_force(plan.handle, _arr(plan, f, "f", torch.float64), float(F),
                             _arr(plan, p, "p", torch.float64),
                             m, ctypes.byref(_opts(**opts)), ctypes.byref(res))
    if raise_on_error:
        _check(rc)
    return res.as_dict()


def cb_sweep(plan: Plan, f, d_steps, p_state, mask_state, raise_on_error=True, **opts):
    n = len(d_steps)
    steps = (ctypes.c_double * n)(*[float(x) for x in d_steps])
    out = (cb_result * max(n, 1))()
    rc = _lib.cb_sweep(plan.handle, _arr(plan, f, "f", torch.float64), steps, n,
                       _arr(plan, p_state, "p_state", torch.float64),
                       _arr(plan, mask_state, "mask_state", torch.uint8),
                       ctypes.byref(_opts(**opts)), out)
    if raise_on_error:
        _check(rc)
    return [out[i].as_dict() for i in range(n)]


def cb_solve_batch(plans, fs, targets, modes, ps, workers=0, raise_on_error=True, **opts):
    """Solve len(plans) independent problems concurrently.  modes: 0 approach,
    1 force.  fs, ps: float64 GPU tensors of each plan's N x N."""
    n = len(plans)
    hp = (_vp * n)(*[pl.handle for pl in plans])
    hf = (_vp * n)(*[_arr(pl, f, "f", torch.float64).value for pl, f in zip(plans, fs)])
    hpp = (_vp * n)(*[_arr(pl, p, "p", torch.float64).value for pl, p in zip(plans, ps)])
    ht = (_d * n)(*[float(t) for t in targets])
    hm = (_i * n)(*[int(m) for m in modes])
    out = (cb_result * max(n, 1))()
    rc = _lib.cb_solve_batch(n, hp, hf, ht, hm, hpp, ctypes.byref(_opts(**opts)), int(workers), out)
    if raise_on_error:
        _check(rc)
    return [out[i].as_dict() for i in range(n)]


def cb_sweep_batch(plans, fs, d_steps, p_states, mask_states, workers=0, raise_on_error=True, **opts):
    """len(plans) independent sweeps concurrently; d_steps: one sequence of
    approaches per problem.  Returns one list of per-step results per problem."""
    n = len(plans)
    steps = [(ctypes.c_double * max(len(s), 1))(*[float(x) for x in s]) for s in d_steps]
    outs = [(cb_result * max(len(s), 1))() for s in d_steps]
    hp = (_vp * n)(*[pl.handle for pl in plans])
    hf = (_vp * n)(*[_arr(pl, f, "f", torch.float64).value for pl, f in zip(plans, fs)])
    hs = (_vp * n)(*[ctypes.cast(s, _vp).value for s in steps])
    hn = (_i * n)(*[len(s) for s in d_steps])
    hpp = (_vp * n)(*[_arr(pl, p, "p_state", torch.float64).value for pl, p in zip(plans, p_states)])
    hm = (_vp * n)(*[_arr(pl, m, "mask_state", torch.uint8).value for pl, m in zip(plans, mask_states)])
    ho = (_vp * n)(*[ctypes.cast(o, _vp).value for o in outs])
    rc = _lib.cb_sweep_batch(n, hp, hf, hs, hn, hpp, hm, ctypes.byref(_opts(**opts)), int(workers), ho)
    if raise_on_error:
        _check(rc)
    return [[outs[i][k].as_dict() for k in range(len(d_steps[i]))] for i in range(n)]


# ---------------------------------------------------------------------------
# Learned warm start
# ---------------------------------------------------------------------------
def cb_net_num_params():
    return _lib.cb_net_num_params()


@dataclass
class Net:
    handle: ctypes.c_void_p
    batch: int
    H: int
    W: int

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cb_net_destroy(self.handle)
            self.handle = None


def _dev(x, name, dtype, shape):
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if x.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {x.dtype}")
    if tuple(x.shape) != tuple(shape) or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous tensor of shape {tuple(shape)}")
    return ctypes.c_void_p(x.data_ptr())


def cb_net_create(batch, H, W=None, stream=None):
    W = H if W is None else W
    h_ = ctypes.c_void_p()
    _check(_lib.cb_net_create(ctypes.byref(h_), int(batch), int(H), int(W), _stream_ptr(stream)))
    return Net(h_, int(batch), int(H), int(W))


def cb_net_destroy(net: Net):
    if net.handle:
        _check(_lib.cb_net_destroy(net.handle))
        net.handle = None


def cb_net_set_params(net: Net, params):
    _check(_lib.cb_net_set_params(net.handle, _dev(params, "params", torch.float32, (cb_net_num_params(),))))


def cb_net_get_params(net: Net, out=None):
    if out is None:
        out = torch.empty(cb_net_num_params(), dtype=torch.float32, device="cuda")
    _check(_lib.cb_net_get_params(net.handle, _dev(out, "params", torch.float32, (cb_net_num_params(),))))
    return out


def cb_net_forward(net: Net, x, z16=None):
    n = x.shape[0]
    xx = _dev(x, "x", torch.float32, (n, net.H, net.W, 16))
    zz = _dev(z16, "z16", torch.float32, (n, net.H, net.W, 16)) if z16 is not None else None
    _check(_lib.cb_net_forward(net.handle, int(n), xx, zz))
    return z16


def cb_net_loss_grad(net: Net, x, t, grad=None):
    n = x.shape[0]
    loss = ctypes.c_double()
    gg = _dev(grad, "grad", torch.float32, (cb_net_num_params(),)) if grad is not None else None
    _check(_lib.cb_net_loss_grad(net.handle, int(n), _dev(x, "x", torch.float32, (n, net.H, net.W, 16)),
                                 _dev(t, "t", torch.float32, (n, net.H, net.W)), ctypes.byref(loss), gg))
    return loss.value


def cb_net_adam_step(net: Net, lr):
    _check(_lib.cb_net_adam_step(net.handle, ctypes.c_float(lr)))


def cb_net_features(net: Net, f, L, h, E1, nu1, E2, nu2, F, x):
    Nf = f.shape[0]
    _check(_lib.cb_net_features(net.handle, _dev(f, "f", torch.float64, (Nf, Nf)), int(Nf), float(L), float(h),
                                float(E1), float(nu1), float(E2), float(nu2), float(F),
                                _dev(x, "x", torch.float32, (net.H, net.W, 16))))
    return x


def cb_net_warmstart(net: Net, plan: Plan, f, F, p_out, cut=0.0):
    _check(_lib.cb_net_warmstart(net.handle, plan.handle, _arr(plan, f, "f", torch.float64), float(F), float(cut),
                                 _arr(plan, p_out, "p_out", torch.float64)))
    return p_out


def cb_net_warmstart_batch(net: Net, plans, fs, Fs, ps_out, cut=0.0):
    n = len(plans)
    hp = (_vp * n)(*[pl.handle for pl in plans])
    hf = (_vp * n)(*[_arr(pl, f, "f", torch.float64).value for pl, f in zip(plans, fs)])
    hpp = (_vp * n)(*[_arr(pl, p, "p_out", torch.float64).value for pl, p in zip(plans, ps_out)])
    hF = (_d * n)(*[float(F) for F in Fs])
    _check(_lib.cb_net_warmstart_batch(net.handle, n, hp, hf, hF, float(cut), hpp))
    return ps_out
