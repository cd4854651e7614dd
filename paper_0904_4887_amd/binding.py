"""ctypes binding of libdwp.so (argument marshalling only).

Every step of the solver runs in the HIP library; this module converts torch
tensors to device pointers, NumPy arrays to host pointers, and status codes to
exceptions.  PyTorch provides the device memory and the stream.  There is no
fallback: if the library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwp.so")

DWP_OK, DWP_EINVAL, DWP_ESTATE, DWP_ENOCONV, DWP_EHIP, DWP_ENOMEM, DWP_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "DWP_OK", -1: "DWP_EINVAL", -2: "DWP_ESTATE", -3: "DWP_ENOCONV", -4: "DWP_EHIP",
                -5: "DWP_ENOMEM", -6: "DWP_ENONFINITE"}
FP64, MIXED = 0, 1


class DWPError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("z_wet_lo", C.c_double), ("z_wet_hi", C.c_double),
                ("pre", C.c_int), ("post", C.c_int), ("coarse_sweeps", C.c_int), ("max_levels", C.c_int),
                ("cycles", C.c_int), ("scaled_dry", C.c_int), ("tol", C.c_double), ("max_outer", C.c_int),
                ("restart", C.c_int), ("warm_start", C.c_int), ("profile", C.c_int),
                ("smoother", C.c_int), ("fft_fp32", C.c_int), ("order", C.c_int), ("smooth6", C.c_int),
                ("krylov_fp32", C.c_int), ("krylov_fp16", C.c_int),
                ("semi_ratio", C.c_double)]


class Info(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("vcycles", C.c_int), ("restarts", C.c_int), ("k_w0", C.c_int),
                ("k_w1", C.c_int), ("n_levels", C.c_int), ("rel_res", C.c_double), ("energy", C.c_double),
                ("energy_eps_form", C.c_double), ("mean_rho_removed", C.c_double), ("t_total_ms", C.c_double),
                ("background", C.c_double), ("t_fft_ms", C.c_double), ("t_mg_ms", C.c_double),
                ("t_krylov_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EpsParams(C.Structure):
    _fields_ = [("eps_inf", C.c_double), ("delta", C.c_double), ("exclusion", C.c_int), ("z_lim", C.c_double),
                ("delta_z", C.c_double), ("model", C.c_int), ("beta", C.c_double), ("decay", C.c_double)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGNATURES = {
    "dwp_default_opts": (None, [C.POINTER(Opts)]),
    "dwp_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "dwp_destroy": (C.c_int, [_P]),
    "dwp_set_stream": (C.c_int, [_P, _P]),
    "dwp_set_grid": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                               C.POINTER(Opts)]),
    "dwp_set_opts": (C.c_int, [_P, C.POINTER(Opts)]),
    "dwp_set_epsilon": (C.c_int, [_P, _P]),
    "dwp_build_epsilon": (C.c_int, [_P, C.c_int, _D, _D, C.POINTER(EpsParams)]),
    "dwp_get_epsilon": (C.c_int, [_P, _P]),
    "dwp_build_epsilon_density": (C.c_int, [_P, _P, C.c_double, C.c_double, C.c_double]),
    "dwp_v_eps": (C.c_int, [_P, C.c_int, _P]),
    "dwp_build_rho": (C.c_int, [_P, C.c_int, _D, _D, _D, _P]),
    "dwp_solve": (C.c_int, [_P, _P, _P, _D, C.POINTER(Info)]),
    "dwp_backward": (C.c_int, [_P, _P, C.c_double, _P, _P, _P, C.POINTER(Info)]),
    "dwp_eps_gradient": (C.c_int, [_P, _P]),
    "dwp_eps_pair_gradient": (C.c_int, [_P, _P, _P, C.c_double, _P]),
    "dwp_forces": (C.c_int, [_P, C.c_int, _D, _D, _D, _D, C.POINTER(EpsParams), _D]),
    "dwp_forces_noalloc": (C.c_int, [_P, C.c_int, _D, _D, _D, _D, C.POINTER(EpsParams), _D]),
    "dwp_apply_operator": (C.c_int, [_P, _P, _P]),
    "dwp_vacuum_solve": (C.c_int, [_P, _P, _P]),
    "dwp_apply_split": (C.c_int, [_P, _P, _P]),
    "dwp_energy": (C.c_int, [_P, _P, _P, _D]),
    "dwp_plan": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.POINTER(Opts),
                           C.POINTER(C.c_int), C.c_int]),
    "dwp_last_error": (C.c_char_p, [_P]),
    "dwp_profile_count": (C.c_int, []),
    "dwp_profile_get": (C.c_int, [_P, C.c_int, C.POINTER(C.c_char_p), _D, C.POINTER(C.c_long), _D]),
    "dwp_profile_reset": (C.c_int, [_P]),
}

_lib_handle = None


def lib():
    """Load libdwp.so once; raise if it is absent (no fallback path exists)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0904_4887_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib_handle = h
    return _lib_handle


def default_opts(**kw):
    o = Opts()
    lib().dwp_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def plan(n, L, **kw):
    """Validate a grid and options on the host and return the wet-slab plan:
    dict(k_w0, k_w1, levels=[(nx, ny, nw), ...]).  Issues no device work."""
    o = default_opts(**kw)
    out = (C.c_int * (3 + 3 * 32))()
    st = lib().dwp_plan(int(n[0]), int(n[1]), int(n[2]), float(L[0]), float(L[1]), float(L[2]), C.byref(o),
                        out, len(out))
    if st != DWP_OK:
        raise DWPError(st, lib().dwp_last_error(None).decode())
    nl = out[2]
    return dict(k_w0=out[0], k_w1=out[1], levels=[tuple(out[3 + 3 * i:6 + 3 * i]) for i in range(nl)])


def _hostd(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a, a.ctypes.data_as(_D)


class Solver:
    """One libdwp context on one device, enqueueing on torch's current stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _P()
        st = lib().dwp_create(C.byref(h), int(device), _P(stream.cuda_stream))
        if st != DWP_OK:
            raise DWPError(st, lib().dwp_last_error(None).decode())
        self._h = h
        self.n = None
        self.L = None
        self.opts = None
        self.epoch = 0  # bumped by every call that changes the grid, the options or eps

    def close(self):
        if getattr(self, "_h", None):
            lib().dwp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != DWP_OK:
            raise DWPError(st, lib().dwp_last_error(self._h).decode())

    def _dev(self, t, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if self.n is not None and t.numel() != self.N:
            raise ValueError(f"{name} must hold {self.N} values")
        return _P(t.data_ptr())

    @property
    def N(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def h(self):
        return tuple(self.L[d] / self.n[d] for d in range(3))

    def empty(self):
        return self._torch.empty(self.shape, dtype=self._torch.float64, device=self.device)

    def set_grid(self, n, L, **opts):
        self.epoch += 1
        o = default_opts(**opts)
        self._check(lib().dwp_set_grid(self._h, int(n[0]), int(n[1]), int(n[2]), float(L[0]), float(L[1]),
                                       float(L[2]), C.byref(o)))
        self.n, self.L, self.opts = tuple(int(x) for x in n), tuple(float(x) for x in L), o

    def set_opts(self, **opts):
        self.epoch += 1
        o = Opts()
        C.memmove(C.byref(o), C.byref(self.opts), C.sizeof(Opts))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self._check(lib().dwp_set_opts(self._h, C.byref(o)))
        self.opts = o

    def set_epsilon(self, eps):
        self.epoch += 1
        self._check(lib().dwp_set_epsilon(self._h, self._dev(eps, "eps")))

    def build_epsilon(self, xyz, radius, params):
        self.epoch += 1
        x, xp = _hostd(xyz)
        r, rp = _hostd(radius)
        ep = eps_params(params)
        self._check(lib().dwp_build_epsilon(self._h, len(r), xp, rp, C.byref(ep)))

    def build_epsilon_density(self, rho, eps_inf, rho0, beta):
        """eps from an electron-density grid (Eq. 7); keeps d eps/d rho for v_eps."""
        self.epoch += 1
        self._check(lib().dwp_build_epsilon_density(self._h, self._dev(rho, "rho"), float(eps_inf), float(rho0),
                                                    float(beta)))

    def v_eps(self, add_phi=False, out=None):
        """V_eps (Eq. 6) of the last solution; add_phi: phi + V_eps (Eq. 5)."""
        out = self.empty() if out is None else out
        self._check(lib().dwp_v_eps(self._h, 1 if add_phi else 0, self._dev(out, "out")))
        return out

    def get_epsilon(self):
        out = self.empty()
        self._check(lib().dwp_get_epsilon(self._h, self._dev(out, "eps")))
        return out

    def build_rho(self, xyz, q, sigma, out=None):
        out = self.empty() if out is None else out
        x, xp = _hostd(xyz)
        qq, qp = _hostd(q)
        s, sp = _hostd(sigma)
        self._check(lib().dwp_build_rho(self._h, len(qq), xp, qp, sp, self._dev(out, "rho")))
        return out

    def solve(self, rho, phi=None, allow_noconv=False):
        """Returns (phi, E, info dict).  With opts.warm_start, phi is the guess
        (a new phi starts from zero)."""
        if phi is None:
            phi = self._torch.zeros(self.shape, dtype=self._torch.float64, device=self.device)
        e = C.c_double()
        info = Info()
        st = lib().dwp_solve(self._h, self._dev(rho, "rho"), self._dev(phi, "phi"), C.byref(e), C.byref(info))
        if not (allow_noconv and st == DWP_ENOCONV):
            self._check(st)
        return phi, e.value, info.as_dict()

    def backward(self, phi, g_E, g_phi=None, grad_rho=None, grad_eps=None, allow_noconv=False):
        """(grad_rho, grad_eps, info) of the map (rho, eps) -> (phi, E) at the
        solution phi of the current eps, for cotangents g_E (float) and g_phi
        (tensor or None); the adjoint solve runs in the library."""
        grad_rho = self.empty() if grad_rho is None else grad_rho
        grad_eps = self.empty() if grad_eps is None else grad_eps
        gp = None if g_phi is None else self._dev(g_phi, "g_phi")
        info = Info()
        st = lib().dwp_backward(self._h, self._dev(phi, "phi"), float(g_E), gp, self._dev(grad_rho, "grad_rho"),
                                self._dev(grad_eps, "grad_eps"), C.byref(info))
        if not (allow_noconv and st == DWP_ENOCONV):
            self._check(st)
        return grad_rho, grad_eps, info.as_dict()

    def eps_gradient(self, out=None):
        out = self.empty() if out is None else out
        self._check(lib().dwp_eps_gradient(self._h, self._dev(out, "dEdeps")))
        return out

    def eps_pair_gradient(self, a, b, scale, out=None):
        out = self.empty() if out is None else out
        self._check(lib().dwp_eps_pair_gradient(self._h, self._dev(a, "a"), self._dev(b, "b"), float(scale),
                                                self._dev(out, "out")))
        return out

    def forces(self, xyz, q, sigma, radius=None, params=None):
        """dE/dR, shape (n, 3).  params None: eps did not come from the atoms."""
        x, xp = _hostd(xyz)
        qq, qp = _hostd(q)
        s, sp = _hostd(sigma)
        n = len(qq)
        out = np.zeros((n, 3))
        if params is not None:
            r, rp = _hostd(radius)
            ep = eps_params(params)
            epp = C.byref(ep)
        else:
            rp, epp = None, None
        self._check(lib().dwp_forces(self._h, n, xp, rp, qp, sp, epp, out.ctypes.data_as(_D)))
        return out

    def forces_noalloc(self, xyz, q, sigma, radius=None, params=None):
        """forces() through dwp_forces_noalloc (no device allocation)."""
        x, xp = _hostd(xyz)
        qq, qp = _hostd(q)
        s, sp = _hostd(sigma)
        n = len(qq)
        out = np.zeros((n, 3))
        if params is not None:
            r, rp = _hostd(radius)
            ep = eps_params(params)
            epp = C.byref(ep)
        else:
            rp, epp = None, None
        self._check(lib().dwp_forces_noalloc(self._h, n, xp, rp, qp, sp, epp, out.ctypes.data_as(_D)))
        return out

    def apply_operator(self, phi, out=None):
        out = self.empty() if out is None else out
        self._check(lib().dwp_apply_operator(self._h, self._dev(phi, "phi"), self._dev(out, "out")))
        return out

    def vacuum_solve(self, r, out=None):
        out = self.empty() if out is None else out
        self._check(lib().dwp_vacuum_solve(self._h, self._dev(r, "r"), self._dev(out, "out")))
        return out

    def apply_split(self, r, out=None):
        out = self.empty() if out is None else out
        self._check(lib().dwp_apply_split(self._h, self._dev(r, "r"), self._dev(out, "out")))
        return out

    def profile_reset(self):
        self._check(lib().dwp_profile_reset(self._h))

    def profile(self):
        """{group: dict(name, ms, launches, bytes)} for groups with launches."""
        out = {}
        for g in range(lib().dwp_profile_count()):
            name, ms, n, by = C.c_char_p(), C.c_double(), C.c_long(), C.c_double()
            self._check(lib().dwp_profile_get(self._h, g, C.byref(name), C.byref(ms), C.byref(n), C.byref(by)))
            if n.value:
                nm = name.value.decode()
                out[nm] = dict(name=nm, ms=ms.value, launches=n.value, bytes=by.value)
        return out

    def energy(self, rho, phi):
        e = C.c_double()
        self._check(lib().dwp_energy(self._h, self._dev(rho, "rho"), self._dev(phi, "phi"), C.byref(e)))
        return e.value


def eps_params(p):
    if isinstance(p, EpsParams):
        return p
    model = int(p.get("model", 0))
    delta = float(p.get("delta", 0.0 if model else p["delta"]))
    return EpsParams(float(p["eps_inf"]), delta, int(p.get("exclusion", 0)),
                     float(p.get("z_lim", 0.0)), float(p.get("delta_z", delta)), model,
                     float(p.get("beta", 0.0)), float(p.get("decay", 0.0)))


def header_symbols(path=None):
    """Names of the functions declared in include/dwp.h."""
    import re
    path = path or os.path.join(os.path.dirname(HERE), "include", "dwp.h")
    text = open(path).read()
    return sorted(set(re.findall(r"\b(dwp_[a-z_]+)\s*\(", text)))


NAN = math.nan
