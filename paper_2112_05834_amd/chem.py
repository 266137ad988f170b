"""Python binding of libchem.so (the C ABI in include/chem.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the integration runs in the library's HIP kernels. The
library must be built (``paper_2112_05834_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchem.so")

PLAIN, PERSISTENT, PERSISTENT_BINNED = 0, 1, 2
RODAS3, ROS4 = 0, 1
JAC_ANALYTICAL, JAC_FD = 0, 1
STATE_FULL, STATE_NO_BATH = 0, 1
CELL_OK, CELL_MAX_STEPS, CELL_H_UNDERFLOW, CELL_NONFINITE, CELL_SINGULAR, CELL_T_RANGE = range(6)

_ERRORS = {-1: "CHEM_EINVAL", -2: "CHEM_EMECH", -3: "CHEM_EHIP", -4: "CHEM_ENOMEM", -5: "CHEM_ESTATE",
           -6: "CHEM_EUNSUPPORTED"}


class ChemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRORS.get(code, "?"), code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("cells_per_wave", ctypes.c_int32),
                ("queue_chunk", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("scheme", ctypes.c_int32), ("jacobian", ctypes.c_int32), ("state", ctypes.c_int32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


N_MODEL_PARAMS = 4545

_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libchem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libchem.so is not built: run paper_2112_05834_amd.build.build() "
                              "(hipcc, gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "chem_opts_default": (None, [ctypes.POINTER(Opts)]),
            "chem_mech_load": (i32, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
            "chem_mech_dims": (i32, [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "chem_mech_work": (i32, [_vp] + [ctypes.POINTER(dbl)] * 4),
            "chem_mech_free": (None, [_vp]),
            "chem_solver_create": (i32, [_vp, ctypes.POINTER(Opts), i32, ctypes.POINTER(_vp)]),
            "chem_solver_free": (None, [_vp]),
            "chem_solver_set_opts": (i32, [_vp, ctypes.POINTER(Opts)]),
            "chem_solver_get_opts": (i32, [_vp, ctypes.POINTER(Opts)]),
            "chem_integrate": (i32, [_vp, i64, dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "chem_integrate_steps": (i32, [_vp, i32, i64, dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "chem_integrate_noalloc": (i32, [_vp, i64, dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "chem_eval_rhs_jac": (i32, [_vp, i64, _vp, _vp, _vp, _vp]),
            "chem_lu_batch": (i32, [_vp, i64, _vp, _vp, _vp, _vp, _vp]),
            "chem_lu_batch_rocsolver": (i32, [i32, i64, _vp, _vp, _vp, _vp, _vp]),
            "chem_log_enable": (i32, [_vp, i64]),
            "chem_log_fetch": (i32, [_vp, _vp, _vp, ctypes.POINTER(i64), _vp]),
            "chem_features": (i32, [_vp, i64, dbl, _vp, _vp, _vp]),
            "chem_train_opts_default": (None, [ctypes.POINTER(TrainOpts)]),
            "chem_model_train": (i32, [_vp, i64, _vp, _vp, ctypes.POINTER(TrainOpts), _vp]),
            "chem_model_predict": (i32, [_vp, i64, _vp, _vp, _vp]),
            "chem_set_cost_override": (i32, [_vp, i64, _vp]),
            "chem_model_save": (i32, [_vp, ctypes.c_char_p]),
            "chem_model_load": (i32, [_vp, ctypes.c_char_p]),
            "chem_last_binning_used": (i32, [_vp, ctypes.POINTER(i32)]),
            "chem_model_get": (i32, [_vp, _vp, _vp, _vp]),
            "chem_model_set": (i32, [_vp, _vp, _vp, _vp]),
            "chem_model_grad": (i32, [_vp, i64, _vp, _vp, _vp, _vp, _vp]),
            "chem_bin_edges": (i32, [_vp, i64, _vp, _vp, _vp]),
            "chem_bin_order": (i32, [_vp, i64, _vp, _vp, _vp, _vp]),
            "chem_autotune": (i32, [_vp, i64, _vp, dbl, _vp]),
            "chem_autotune_cached": (i32, [_vp, ctypes.c_char_p, i64, _vp, dbl, _vp, ctypes.POINTER(i32)]),
            "chem_workspace_info": (i32, [_vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
            "chem_kernel_timing": (i32, [_vp, i32]),
            "chem_eval_counters": (i32, [_vp, _vp, _vp, i64]),
            "chem_kernel_times": (i32, [_vp, _vp, i32, ctypes.POINTER(i32)]),
            "chem_mech_elements": (i32, [_vp, ctypes.POINTER(i32), _vp]),
            "chem_zone_config": (i32, [_vp, _vp, _vp, _vp, dbl, dbl]),
            "chem_zone_bands": (i32, [_vp, dbl]),
            "chem_mixture_fraction": (i32, [_vp, i64, _vp, _vp, _vp]),
            "chem_integrate_zonal": (i32, [_vp, i64, dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "chem_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise ChemError(rc, lib().chem_last_error().decode())


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().chem_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_train_opts(**kw) -> TrainOpts:
    t = TrainOpts()
    lib().chem_train_opts_default(ctypes.byref(t))
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _ptr(t: Optional[torch.Tensor], dtype=None, device=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if device is not None and t.device != device:
        raise ValueError("%s must be on %s, got %s" % (name, device, t.device))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def lu_batch_rocsolver(A: torch.Tensor, b: Optional[torch.Tensor] = None):
    """chem_lu_batch_rocsolver: rocSOLVER's batched LU (and solve of b [batch,
    n]) in place on A [batch, n, n] holding column-major matrices (A[k, j, i] =
    element (i, j)). Returns (A, piv 1-based, info, b)."""
    batch, n = A.shape[0], A.shape[1]
    dev = A.device
    piv = torch.empty((batch, n), dtype=torch.int32, device=dev)
    info = torch.empty(batch, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib().chem_lu_batch_rocsolver(n, batch, _ptr(A, torch.float64, dev, batch * n * n, "A"), _ptr(piv),
                                             _ptr(info), _ptr(b, torch.float64, dev, batch * n, "b"), _stream(dev)))
    return A, piv, info, b


class Mechanism:
    """A parsed mechanism (host side)."""

    def __init__(self, path: str):
        h = _vp()
        _check(lib().chem_mech_load(path.encode(), ctypes.byref(h)))
        self._h = h
        ns, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().chem_mech_dims(h, ctypes.byref(ns), ctypes.byref(nr)))
        self.n_species, self.n_reactions = ns.value, nr.value
        self.n = self.n_species + 1

    def elements(self):
        """Atom counts [Ns, Ne] (numpy int32) of every species."""
        import numpy as np
        ne = ctypes.c_int32()
        _check(lib().chem_mech_elements(self._h, ctypes.byref(ne), None))
        counts = np.zeros((self.n_species, ne.value), dtype=np.int32)
        _check(lib().chem_mech_elements(self._h, ctypes.byref(ne), counts.ctypes.data_as(_vp)))
        return counts

    def work(self):
        v = [ctypes.c_double() for _ in range(4)]
        _check(lib().chem_mech_work(self._h, *[ctypes.byref(x) for x in v]))
        return {"flops_rhs": v[0].value, "flops_jac": v[1].value, "trans_rhs": v[2].value,
                "trans_jac": v[3].value}

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.chem_mech_free(self._h)
            self._h = None


@dataclasses.dataclass
class Result:
    phi: torch.Tensor
    h: Optional[torch.Tensor]
    n_acc: torch.Tensor
    n_rej: torch.Tensor
    status: torch.Tensor


class Solver:
    """Integrator bound to one HIP device."""

    def __init__(self, mech: Mechanism, opts: Optional[Opts] = None, device: int = 0):
        self.mech = mech
        self.device = torch.device("cuda", device)
        h = _vp()
        o = opts if opts is not None else default_opts()
        _check(lib().chem_solver_create(mech._h, ctypes.byref(o), int(device), ctypes.byref(h)))
        self._h = h
        self.ns = mech.n_species

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.chem_solver_free(self._h)
            self._h = None

    @property
    def opts(self) -> Opts:
        o = Opts()
        _check(lib().chem_solver_get_opts(self._h, ctypes.byref(o)))
        return o

    def set_opts(self, o: Opts = None, **kw):
        o = o if o is not None else self.opts
        for k, v in kw.items():
            setattr(o, k, v)
        _check(lib().chem_solver_set_opts(self._h, ctypes.byref(o)))

    def _outs(self, n, h_io, out):
        """h_io: a float64 tensor (in/out), None (start every cell at dt and
        return the proposals in a new tensor) or False (not kept: NULL)."""
        dev = self.device
        phi_out = out if out is not None else torch.empty((n, self.ns + 2), dtype=torch.float64, device=dev)
        if h_io is False:
            h = None
        else:
            h = h_io if h_io is not None else torch.zeros(n, dtype=torch.float64, device=dev)
        na = torch.empty(n, dtype=torch.int32, device=dev)
        nr = torch.empty(n, dtype=torch.int32, device=dev)
        st = torch.empty(n, dtype=torch.int8, device=dev)
        return phi_out, h, na, nr, st

    def integrate(self, phi: torch.Tensor, dt: float, h_io: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None) -> Result:
        """One chemistry step for every cell of phi ([n, 2+Ns] float64 on the
        solver's device). h_io (if given) is updated in place."""
        n = phi.shape[0]
        if phi.dim() != 2 or phi.shape[1] != self.ns + 2:
            raise ValueError("phi must be [n, %d]" % (self.ns + 2))
        phi_out, h, na, nr, st = self._outs(n, h_io, out)
        _check(lib().chem_integrate(self._h, n, float(dt),
                                    _ptr(phi, torch.float64, self.device, name="phi"),
                                    _ptr(phi_out, torch.float64, self.device, n * (self.ns + 2), "out"),
                                    _ptr(h, torch.float64, self.device, n, "h_io"),
                                    _ptr(na), _ptr(nr), _ptr(st), _stream(self.device)))
        return Result(phi_out, h, na, nr, st)

    def integrate_noalloc(self, phi: torch.Tensor, dt: float, h_io: Optional[torch.Tensor] = None,
                          out: Optional[torch.Tensor] = None) -> Result:
        """chem_integrate_noalloc: one chemistry step on the persistent queue
        whose device scratch is the library's static array (the library
        allocates nothing; the output tensors are allocated here unless
        given)."""
        n = phi.shape[0]
        if phi.dim() != 2 or phi.shape[1] != self.ns + 2:
            raise ValueError("phi must be [n, %d]" % (self.ns + 2))
        phi_out, h, na, nr, st = self._outs(n, h_io, out)
        _check(lib().chem_integrate_noalloc(self._h, n, float(dt),
                                            _ptr(phi, torch.float64, self.device, name="phi"),
                                            _ptr(phi_out, torch.float64, self.device, n * (self.ns + 2), "out"),
                                            _ptr(h, torch.float64, self.device, n, "h_io"),
                                            _ptr(na), _ptr(nr), _ptr(st), _stream(self.device)))
        return Result(phi_out, h, na, nr, st)

    # ---- zonal reference mapping ----
    def zone_config(self, coupling, y_fuel, y_ox, z_max: float, t_tol: float, dz: float = 0.0):
        """Mixture-fraction definition (host sequences: coupling per element,
        fuel and oxidiser compositions per species), mapping thresholds and
        the Z band width (0: one band)."""
        import numpy as np
        c = np.ascontiguousarray(coupling, dtype=np.float64)
        yf = np.ascontiguousarray(y_fuel, dtype=np.float64)
        yo = np.ascontiguousarray(y_ox, dtype=np.float64)
        if c.shape != (self.mech.elements().shape[1],) or yf.shape != (self.ns,) or yo.shape != (self.ns,):
            raise ValueError("coupling must be [n_elements], y_fuel and y_ox [n_species]")
        _check(lib().chem_zone_bands(self._h, 0.0))
        _check(lib().chem_zone_config(self._h, c.ctypes.data_as(_vp), yf.ctypes.data_as(_vp),
                                      yo.ctypes.data_as(_vp), float(z_max), float(t_tol)))
        _check(lib().chem_zone_bands(self._h, float(dz)))

    def mixture_fraction(self, phi: torch.Tensor) -> torch.Tensor:
        n = phi.shape[0]
        z = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().chem_mixture_fraction(self._h, n, _ptr(phi, torch.float64, self.device,
                                                            n * (self.ns + 2), "phi"),
                                           _ptr(z), _stream(self.device)))
        return z

    def integrate_zonal(self, phi: torch.Tensor, dt: float, h_io: Optional[torch.Tensor] = None,
                        out: Optional[torch.Tensor] = None):
        """One chemistry step with zonal reference mapping: (Result, mapped),
        mapped an int8 tensor (band + 1 of a cell that took its band
        reference's change of state, 0 for an integrated cell)."""
        n = phi.shape[0]
        if phi.dim() != 2 or phi.shape[1] != self.ns + 2:
            raise ValueError("phi must be [n, %d]" % (self.ns + 2))
        phi_out, h, na, nr, st = self._outs(n, h_io, out)
        mapped = torch.empty(n, dtype=torch.int8, device=self.device)
        _check(lib().chem_integrate_zonal(self._h, n, float(dt),
                                          _ptr(phi, torch.float64, self.device, n * (self.ns + 2), "phi"),
                                          _ptr(phi_out, torch.float64, self.device, n * (self.ns + 2), "out"),
                                          _ptr(h, torch.float64, self.device, n, "h_io"),
                                          _ptr(na), _ptr(nr), _ptr(st), _ptr(mapped), _stream(self.device)))
        return Result(phi_out, h, na, nr, st), mapped

    def integrate_steps(self, phi: torch.Tensor, dt: float, n_steps: int,
                        h_io: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> Result:
        n = phi.shape[0]
        if phi.dim() != 2 or phi.shape[1] != self.ns + 2:
            raise ValueError("phi must be [n, %d]" % (self.ns + 2))
        phi_out, h, na, nr, st = self._outs(n, h_io, out)
        _check(lib().chem_integrate_steps(self._h, int(n_steps), n, float(dt),
                                          _ptr(phi, torch.float64, self.device, name="phi"),
                                          _ptr(phi_out, torch.float64, self.device, n * (self.ns + 2), "out"),
                                          _ptr(h, torch.float64, self.device, n, "h_io"),
                                          _ptr(na), _ptr(nr), _ptr(st), _stream(self.device)))
        return Result(phi_out, h, na, nr, st)

    def eval_rhs_jac(self, phi: torch.Tensor, jac: bool = True):
        n = phi.shape[0]
        nn = self.ns + 1
        f = torch.empty((n, nn), dtype=torch.float64, device=self.device)
        J = torch.empty((n, nn, nn), dtype=torch.float64, device=self.device) if jac else None
        _check(lib().chem_eval_rhs_jac(self._h, n, _ptr(phi, torch.float64, self.device, name="phi"),
                                       _ptr(f), _ptr(J), _stream(self.device)))
        return f, J

    def lu_batch(self, A: torch.Tensor, b: Optional[torch.Tensor] = None):
        """In-place batched LU of A [batch, n, n] (and solve of b [batch, n])."""
        batch = A.shape[0]
        nn = self.ns + 1
        piv = torch.empty((batch, nn), dtype=torch.int32, device=self.device)
        info = torch.empty(batch, dtype=torch.int32, device=self.device)
        _check(lib().chem_lu_batch(self._h, batch, _ptr(A, torch.float64, self.device, batch * nn * nn, "A"),
                                   _ptr(piv), _ptr(info),
                                   _ptr(b, torch.float64, self.device, batch * nn, "b"), _stream(self.device)))
        return A, piv, info, b

    # ---- learned cost model ----
    def log_enable(self, capacity: int):
        _check(lib().chem_log_enable(self._h, int(capacity)))

    def log_fetch(self, capacity: int):
        f = torch.empty((capacity, 4), dtype=torch.float32, device=self.device)
        t = torch.empty(capacity, dtype=torch.float32, device=self.device)
        n = ctypes.c_int64()
        _check(lib().chem_log_fetch(self._h, _ptr(f), _ptr(t), ctypes.byref(n), _stream(self.device)))
        return f[:n.value], t[:n.value]

    def features(self, phi: torch.Tensor, dt: float) -> torch.Tensor:
        n = phi.shape[0]
        f = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        _check(lib().chem_features(self._h, n, float(dt), _ptr(phi, torch.float64, self.device, name="phi"),
                                   _ptr(f), _stream(self.device)))
        return f

    def model_train(self, feats: torch.Tensor, target: torch.Tensor, opts: Optional[TrainOpts] = None):
        n = feats.shape[0]
        t = opts if opts is not None else default_train_opts()
        _check(lib().chem_model_train(self._h, n, _ptr(feats, torch.float32, self.device, 4 * n, "feats"),
                                      _ptr(target, torch.float32, self.device, n, "target"), ctypes.byref(t),
                                      _stream(self.device)))

    def model_predict(self, feats: torch.Tensor) -> torch.Tensor:
        n = feats.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        _check(lib().chem_model_predict(self._h, n, _ptr(feats, torch.float32, self.device, 4 * n, "feats"),
                                        _ptr(out), _stream(self.device)))
        return out

    def set_cost_override(self, cost: Optional[torch.Tensor]):
        if cost is None:
            _check(lib().chem_set_cost_override(self._h, 0, None))
        else:
            _check(lib().chem_set_cost_override(self._h, cost.numel(),
                                                _ptr(cost, torch.float32, self.device, name="cost")))
        self._cost_ref = cost

    def model_save(self, path: str):
        _check(lib().chem_model_save(self._h, path.encode()))

    def model_load(self, path: str):
        _check(lib().chem_model_load(self._h, path.encode()))

    def last_binning_used(self) -> bool:
        u = ctypes.c_int32()
        _check(lib().chem_last_binning_used(self._h, ctypes.byref(u)))
        return bool(u.value)

    def model_get(self):
        """(params [4545], norm [8], edges [7] or None) as float32 numpy arrays."""
        import numpy as np
        p = np.empty(N_MODEL_PARAMS, dtype=np.float32)
        nv = np.empty(8, dtype=np.float32)
        _check(lib().chem_model_get(self._h, p.ctypes.data_as(_vp), nv.ctypes.data_as(_vp), None))
        e = np.empty(7, dtype=np.float32)
        rc = lib().chem_model_get(self._h, None, None, e.ctypes.data_as(_vp))
        return p, nv, (e if rc == 0 else None)

    def model_set(self, params, norm=None, edges=None):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_MODEL_PARAMS:
            raise ValueError("params must have %d elements" % N_MODEL_PARAMS)
        nv = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float32)
        if nv is not None and nv.size != 8:
            raise ValueError("norm must have 8 elements")
        if e is not None and e.size != 7:
            raise ValueError("edges must have 7 elements")
        _check(lib().chem_model_set(self._h, p.ctypes.data_as(_vp),
                                    None if nv is None else nv.ctypes.data_as(_vp),
                                    None if e is None else e.ctypes.data_as(_vp)))

    def model_grad(self, feats: torch.Tensor, target: torch.Tensor):
        """(loss, gradient [4545]) of the current weights over all samples as one batch."""
        n = feats.shape[0]
        g = torch.empty(N_MODEL_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().chem_model_grad(self._h, n, _ptr(feats, torch.float32, self.device, 4 * n, "feats"),
                                     _ptr(target, torch.float32, self.device, n, "target"), _ptr(g), _ptr(loss),
                                     _stream(self.device)))
        return loss, g

    def bin_edges(self, cost: torch.Tensor):
        import numpy as np
        e = np.empty(7, dtype=np.float32)
        _check(lib().chem_bin_edges(self._h, cost.numel(), _ptr(cost, torch.float32, self.device, name="cost"),
                                    e.ctypes.data_as(_vp), _stream(self.device)))
        return e

    def bin_order(self, cost: torch.Tensor, edges=None) -> torch.Tensor:
        import numpy as np
        n = cost.numel()
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float32)
        _check(lib().chem_bin_order(self._h, n, _ptr(cost, torch.float32, self.device, name="cost"),
                                    None if e is None else e.ctypes.data_as(_vp), _ptr(perm),
                                    _stream(self.device)))
        return perm

    def workspace_info(self):
        """(slots, bytes per slot) of the HBM workspace of large mechanisms."""
        a, b = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().chem_workspace_info(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def eval_counters(self, n_jac: Optional[torch.Tensor], n_fev: Optional[torch.Tensor]):
        """chem_eval_counters: int32 device tensors [n_cells] that every later
        integration call fills with the per-cell evaluations of J and of f
        (None for both to stop). The tensors must outlive their use."""
        self._counters = (n_jac, n_fev)     # keep them alive while the library holds their addresses
        cap = min([t.numel() for t in (n_jac, n_fev) if t is not None], default=0)
        _check(lib().chem_eval_counters(self._h, _ptr(n_jac, torch.int32, self.device, name="n_jac"),
                                       _ptr(n_fev, torch.int32, self.device, name="n_fev"), cap))

    def kernel_timing(self, enable: bool):
        _check(lib().chem_kernel_timing(self._h, 1 if enable else 0))

    def kernel_times(self, cap: int = 4096):
        """Durations (ms) of the integration-kernel launches recorded since
        kernel_timing(True); clears the record."""
        import numpy as np
        a = np.empty(max(cap, 1), dtype=np.float32)
        n = ctypes.c_int32()
        _check(lib().chem_kernel_times(self._h, a.ctypes.data_as(_vp), cap, ctypes.byref(n)))
        return a[:n.value].astype(np.float64)

    def autotune(self, phi_sample: torch.Tensor, dt: float, cache: Optional[str] = None) -> bool:
        """Pick the fastest launch shape on phi_sample; with a cache path, read
        it from / append it to that JSON-lines file. Returns True when the
        shape came from the cache."""
        p = _ptr(phi_sample, torch.float64, self.device, name="phi")
        if cache is None:
            _check(lib().chem_autotune(self._h, phi_sample.shape[0], p, float(dt), _stream(self.device)))
            return False
        hit = ctypes.c_int32()
        _check(lib().chem_autotune_cached(self._h, os.fsencode(cache), phi_sample.shape[0], p, float(dt),
                                          _stream(self.device), ctypes.byref(hit)))
        return bool(hit.value)
