"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU baseline leg of the
benchmark use this module. It builds ``liboracle.so`` from ``chem_oracle.c``
with gcc (see :func:`build`) and exposes the oracle's functions on numpy
arrays. Nothing in the GPU library imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "chem_oracle.c")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(verbose: bool = False) -> str:
    """Compile the oracle (C11, -O2, no FMA contraction) into liboracle.so."""
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-pthread", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_steps", ctypes.c_int),
                ("scheme", ctypes.c_int), ("jacobian", ctypes.c_int), ("state", ctypes.c_int)]


RODAS3, ROS4 = 0, 1
JAC_ANALYTICAL, JAC_FD = 0, 1
STATE_FULL, STATE_NO_BATH = 0, 1


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_mech_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_mech_free.argtypes = [ctypes.c_void_p]
        L.orc_mech_dims.argtypes = [ctypes.c_void_p, _ip, _ip]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_thermo.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_rates.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_omega.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_rhs.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp]
        L.orc_jac.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp]
        L.orc_jac_fd.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp, _dp]
        L.orc_state_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_state_jac.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_lu.argtypes = [ctypes.c_int, _dp, _ip]
        L.orc_lu_solve.argtypes = [ctypes.c_int, _dp, _ip, _dp]
        L.orc_rodas3_tableau.argtypes = [_dp, _dp, _dp, _dp, _dp]
        L.orc_rodas3_step.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, ctypes.c_double, _dp, _dp]
        L.orc_tableau.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double, _dp, _dp]
        L.orc_integrate.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_double,
                                    ctypes.POINTER(_Opts), _dp, _dp, _dp, _ip, _ip,
                                    ctypes.POINTER(ctypes.c_byte), ctypes.c_int]
        L.orc_integrate_counts.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_double,
                                           ctypes.POINTER(_Opts), _dp, _dp, _dp, _ip, _ip, _ip, _ip,
                                           ctypes.POINTER(ctypes.c_byte), ctypes.c_int]
        L.orc_mech_elements.argtypes = [ctypes.c_void_p, _ip, _ip]
        L.orc_mixture_fraction.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_long, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class Mech:
    """A mechanism parsed by the oracle."""

    def __init__(self, path: str):
        L = lib()
        h = ctypes.c_void_p()
        rc = L.orc_mech_load(path.encode(), ctypes.byref(h))
        if rc != 0:
            raise ValueError(L.orc_last_error().decode())
        self._h = h
        ns, nr = ctypes.c_int(), ctypes.c_int()
        L.orc_mech_dims(h, ctypes.byref(ns), ctypes.byref(nr))
        self.ns, self.nr = ns.value, nr.value
        self.n = self.ns + 1

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_mech_free(self._h)
            self._h = None

    def thermo(self, T: float):
        out = [np.zeros(self.ns) for _ in range(4)]
        lib().orc_thermo(self._h, float(T), *[_d(a) for a in out])
        return out  # cp/R, h/RT, s/R, d(cp/R)/dT

    def rates(self, T: float, p: float, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        kf, kr, q = np.zeros(self.nr), np.zeros(self.nr), np.zeros(self.nr)
        lib().orc_rates(self._h, float(T), float(p), _d(Y), _d(kf), _d(kr), _d(q))
        return kf, kr, q

    def omega(self, T: float, p: float, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        w = np.zeros(self.ns)
        lib().orc_omega(self._h, float(T), float(p), _d(Y), _d(w))
        return w

    def rhs(self, p: float, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.n)
        lib().orc_rhs(self._h, float(p), _d(y), _d(f))
        return f

    def jac(self, p: float, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros((self.n, self.n))
        lib().orc_jac(self._h, float(p), _d(y), _d(J))
        return J

    def jac_fd(self, p: float, y):
        """Forward-difference Jacobian (the integrator's FD mode)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        f0 = self.rhs(p, y)
        J = np.zeros((self.n, self.n))
        lib().orc_jac_fd(self._h, float(p), _d(y), _d(f0), _d(J))
        return J

    def state_rhs(self, p: float, y, state: int):
        """f of the integrated state (full, or without the bath gas)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(len(y))
        if lib().orc_state_rhs(self._h, int(state), float(p), _d(y), _d(f)) != 0:
            raise ValueError("bad state")
        return f

    def state_jac(self, p: float, y, state: int):
        """Analytical Jacobian of the integrated state."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros((len(y), len(y)))
        if lib().orc_state_jac(self._h, int(state), float(p), _d(y), _d(J)) != 0:
            raise ValueError("bad state")
        return J

    def rodas3_step(self, p: float, y, h: float):
        y = np.ascontiguousarray(y, dtype=np.float64)
        yn, e = np.zeros(self.n), np.zeros(self.n)
        info = lib().orc_rodas3_step(self._h, float(p), _d(y), float(h), _d(yn), _d(e))
        if info:
            raise FloatingPointError("singular matrix at column %d" % (info - 1))
        return yn, e

    def step(self, p: float, y, h: float, scheme: int = RODAS3):
        """One step of the given scheme from y with step h: (y_new, error vector)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        yn, e = np.zeros(self.n), np.zeros(self.n)
        info = lib().orc_step(self._h, int(scheme), float(p), _d(y), float(h), _d(yn), _d(e))
        if info < 0:
            raise ValueError("unknown scheme %d" % scheme)
        if info:
            raise FloatingPointError("singular matrix at column %d" % (info - 1))
        return yn, e

    def integrate(self, phi, dt: float, rtol=1e-6, atol=1e-10, max_steps=100000, h_io=None,
                  n_threads: int = 1, scheme: int = RODAS3, jacobian: int = JAC_ANALYTICAL,
                  state: int = STATE_FULL, counts: bool = False):
        """(phi_out, h, n_acc, n_rej, status); with counts also the per-cell
        evaluations of the Jacobian and of f (n_jac, n_fev), counted where
        they are made."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        n_cells = phi.shape[0]
        assert phi.shape[1] == self.ns + 2
        out = np.empty_like(phi)
        h = np.zeros(n_cells) if h_io is None else np.ascontiguousarray(h_io, dtype=np.float64).copy()
        na = np.zeros(n_cells, dtype=np.int32)
        nr = np.zeros(n_cells, dtype=np.int32)
        st = np.zeros(n_cells, dtype=np.int8)
        nj = np.zeros(n_cells, dtype=np.int32)
        nf = np.zeros(n_cells, dtype=np.int32)
        o = _Opts(rtol, atol, max_steps, scheme, jacobian, state)
        rc = lib().orc_integrate_counts(self._h, n_cells, float(dt), ctypes.byref(o), _d(phi), _d(out), _d(h),
                                        _i(na), _i(nr), _i(nj), _i(nf),
                                        st.ctypes.data_as(ctypes.POINTER(ctypes.c_byte)), int(n_threads))
        if rc != 0:
            raise ValueError(lib().orc_last_error().decode())
        return (out, h, na, nr, st, nj, nf) if counts else (out, h, na, nr, st)

    def elements(self):
        """Atom counts [Ns, Ne] of every species."""
        ne = ctypes.c_int()
        lib().orc_mech_elements(self._h, ctypes.byref(ne), None)
        counts = np.zeros((self.ns, ne.value), dtype=np.int32)
        lib().orc_mech_elements(self._h, ctypes.byref(ne), _i(counts))
        return counts

    def mixture_fraction(self, coupling, y_fuel, y_ox, phi):
        """Bilger mixture fraction of every cell (paper: Methodology, zonal
        reference mapping; the coupling function is Bilger's)."""
        c = np.ascontiguousarray(coupling, dtype=np.float64)
        yf = np.ascontiguousarray(y_fuel, dtype=np.float64)
        yo = np.ascontiguousarray(y_ox, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        assert c.shape == (self.elements().shape[1],) and yf.shape == yo.shape == (self.ns,)
        z = np.zeros(phi.shape[0])
        if lib().orc_mixture_fraction(self._h, _d(c), _d(yf), _d(yo), phi.shape[0], _d(phi), _d(z)) != 0:
            raise ValueError(lib().orc_last_error().decode())
        return z

    def integrate_zonal(self, phi, dt: float, coupling, y_fuel, y_ox, z_max: float, t_tol: float,
                        h_io=None, dz: float = 0.0, **kw):
        """Zonal reference mapping around the integrator (paper: Methodology,
        the DLBFoam paragraph: a cell is either solved or mapped from a
        reference solution of similar mixture fraction), read as:

        - the zone is every cell with Z <= z_max. With dz = 0 it is one band;
          with dz > 0 it is split into bands b = floor(max(Z, 0) / dz), so
          that a cell is mapped only from a reference of similar Z. Each
          band's reference is its cell of lowest index;
        - a zone cell other than its band's reference whose |T - T_ref| <=
          t_tol is mapped: it takes the reference's change of state over dt,
          T + (T_ref,out - T_ref,in) and Y_k + (Y_ref,out,k - Y_ref,in,k), with
          p, h unchanged, no steps counted and the reference's status;
        - every other cell is integrated as by :meth:`integrate`.

        Returns (phi_out, h, n_acc, n_rej, status, mapped), mapped holding
        the band + 1 of every mapped cell and 0 elsewhere."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        n = phi.shape[0]
        z = self.mixture_fraction(coupling, y_fuel, y_ox, phi)
        band = np.full(n, -1)
        for i in range(n):
            if z[i] <= z_max:
                band[i] = int(np.floor(max(z[i], 0.0) / dz)) if dz > 0 else 0
        mapped = np.zeros(n, dtype=np.int8)
        refs = {}
        for i in range(n):
            if band[i] < 0:
                continue
            if band[i] not in refs:
                refs[band[i]] = i
            elif abs(phi[i, 0] - phi[refs[band[i]], 0]) <= t_tol:
                mapped[i] = band[i] + 1
        solve = np.nonzero(mapped == 0)[0]
        out = phi.copy()
        h = np.zeros(n) if h_io is None else np.array(h_io, dtype=np.float64)
        na = np.zeros(n, dtype=np.int32)
        nr = np.zeros(n, dtype=np.int32)
        st = np.zeros(n, dtype=np.int8)
        if solve.size:
            o, hs, a, r, s = self.integrate(phi[solve], dt, h_io=h[solve], **kw)
            out[solve], h[solve], na[solve], nr[solve], st[solve] = o, hs, a, r, s
        for i in np.nonzero(mapped)[0]:
            ref = refs[mapped[i] - 1]
            out[i, 0] = phi[i, 0] + (out[ref, 0] - phi[ref, 0])
            out[i, 1] = phi[i, 1]
            for k in range(2, phi.shape[1]):
                out[i, k] = phi[i, k] + (out[ref, k] - phi[ref, k])
            st[i] = st[ref]
        return out, h, na, nr, st, mapped


def lu(A):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().orc_lu(n, _d(A), _i(piv))
    return A, piv, info


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=np.float64, copy=True)
    lib().orc_lu_solve(LU.shape[0], _d(np.ascontiguousarray(LU)), _i(np.ascontiguousarray(piv, dtype=np.int32)),
                       _d(b))
    return b


def tableau(scheme: int):
    """(stages, gamma, a [4,4], c [4,4], m [4], e [4]) of a scheme."""
    g = np.zeros(1)
    a, c = np.zeros(16), np.zeros(16)
    m, e = np.zeros(4), np.zeros(4)
    st = lib().orc_tableau(int(scheme), _d(g), _d(a), _d(c), _d(m), _d(e))
    if st < 0:
        raise ValueError("unknown scheme %d" % scheme)
    return st, g[0], a.reshape(4, 4), c.reshape(4, 4), m, e


def rodas3_tableau():
    g = np.zeros(1)
    a, c = np.zeros(16), np.zeros(16)
    m, e = np.zeros(4), np.zeros(4)
    lib().orc_rodas3_tableau(_d(g), _d(a), _d(c), _d(m), _d(e))
    return g[0], a.reshape(4, 4), c.reshape(4, 4), m, e
