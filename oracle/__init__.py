"""FP64 CPU oracle of the coupled LB freezing step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads ``oracle/liborc.so`` (built from ``orc.c`` by
``oracle/build.py``), which shares no code with the HIP library.

Layouts (all float64, C order):
  populations: (nlat*Q, nz, ny, nx), lattice 0 = f, 1..N = g_p, N+1 = h
  lagged fields: (N + dim + 3, nz, ny, nx) = phi_p^{n-1}, f_s^{n-1},
      u^{n-1} (dim), mdot^{n-1}, (rho C_p T mdot)^{n-1}
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

WALL, OPEN = 0, 1
# Readings of div u and of the volume source (see orc.c): DIV_MDOT takes
# div u := mdot, DIV_LAGGED the central difference of u^{n-1}; MDOT_FREEZE
# keeps the freezing term of eq. (fluid2) only, MDOT_PRINTED every printed term.
DIV_MDOT, DIV_LAGGED = 0, 1
MDOT_FREEZE, MDOT_PRINTED = 0, 1
DIRICHLET, ADIABATIC = 0, 1
_FLOW = {"wall": WALL, "open": OPEN}
_THERM = {"dirichlet": DIRICHLET, "adiabatic": ADIABATIC}

_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("nz", ctypes.c_int), ("nphase", ctypes.c_int),
        ("flow_bc", ctypes.c_int * 2), ("therm_bc", ctypes.c_int * 2),
        ("T_face", _D * 2),
        ("rho_l", _D * 4), ("rho_s", _D * 4), ("mu_l", _D * 4), ("mu_s", _D * 4),
        ("lam_l", _D * 4), ("lam_s", _D * 4), ("cp_l", _D * 4), ("cp_s", _D * 4),
        ("latent", _D * 4), ("freezes", ctypes.c_int * 4),
        ("sigma", (_D * 4) * 4), ("cos_theta", (_D * 4) * 4),
        ("eps", _D), ("tau_g", _D), ("T_melt", _D), ("E_ref", _D),
        ("gravity", _D * 3),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle/liborc.so is missing: run python oracle/build.py")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(OrcParams)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [P]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_ncell.restype = ctypes.c_long
        L.orc_ncell.argtypes = [ctypes.c_void_p]
        L.orc_q.argtypes = [ctypes.c_void_p]
        L.orc_naux.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_moments.argtypes = [ctypes.c_void_p, _PD]
        L.orc_diagnostics.argtypes = [ctypes.c_void_p, _PD]
        L.orc_get_state.argtypes = [ctypes.c_void_p, _PD, _PD]
        L.orc_set_state.argtypes = [ctypes.c_void_p, _PD, _PD]
        L.orc_set_readings.restype = ctypes.c_int
        L.orc_set_readings.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.orc_threads.restype = ctypes.c_int
        L.orc_lattice.restype = ctypes.c_int
        L.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _PD]
        L.orc_feq.argtypes = [ctypes.c_int, _D, _D, _PD, _PD]
        L.orc_geq.argtypes = [ctypes.c_int, _D, _PD, _PD]
        L.orc_heq.argtypes = [ctypes.c_int, _D, _D, _D, _D, _PD, _PD]
        L.orc_force.argtypes = [ctypes.c_int, _D, _PD, _PD, _PD, _D, _PD]
        L.orc_stencil.argtypes = [ctypes.c_int, _PD, _PD, _PD]
        L.orc_invert.argtypes = [P, _PD, _D, _PD, _PD]
        L.orc_enthalpy.restype = _D
        L.orc_enthalpy.argtypes = [P, _PD, _D, _D]
        L.orc_interface.argtypes = [P, _PD, _PD, _PD, _PD, _PD, _PD]
        L.orc_fd_field.argtypes = [P, _PD, _PD, _PD]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_PD)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(d: dict) -> OrcParams:
    """Marshal a parameter dict (see synth.make_params) into the oracle struct."""
    P = OrcParams()
    P.dim, P.nx, P.ny = d["dim"], d["nx"], d["ny"]
    P.nz = d.get("nz", 1) if d["dim"] == 3 else 1
    P.nphase = d["nphase"]
    for k in range(2):
        P.flow_bc[k] = _FLOW[d["flow_bc"][k]]
        P.therm_bc[k] = _THERM[d["therm_bc"][k]]
        P.T_face[k] = d["T_face"][k]
    for key in ("rho_l", "rho_s", "mu_l", "mu_s", "lam_l", "lam_s", "cp_l", "cp_s", "latent"):
        arr = getattr(P, key)
        for p, v in enumerate(d[key][:4]):
            arr[p] = float(v)
    for p, v in enumerate(d["freezes"][:4]):
        P.freezes[p] = int(v)
    for p in range(4):
        for q in range(4):
            P.sigma[p][q] = float(d["sigma"][p][q])
            P.cos_theta[p][q] = float(d["cos_theta"][p][q])
    P.eps, P.tau_g, P.T_melt, P.E_ref = d["eps"], d["tau_g"], d["T_melt"], d["E_ref"]
    for a in range(3):
        P.gravity[a] = d["gravity"][a]
    return P


class Oracle:
    """One simulation state advanced by the FP64 CPU oracle."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self._P = make_params(params)
        self._h = lib().orc_create(ctypes.byref(self._P))
        if not self._h:
            raise MemoryError("orc_create failed")
        self.dim = params["dim"]
        self.N = params["nphase"]
        self.Q = lib().orc_q(self._h)
        self.shape = (self._P.nz, self._P.ny, self._P.nx)
        self.ncell = int(np.prod(self.shape))
        self.nlat = self.N + 2
        self.naux = lib().orc_naux(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def set_readings(self, div=None, mdot=None):
        """Select the divergence and volume-source readings (DIV_*, MDOT_*)."""
        d = DIV_LAGGED if div is None else div
        m = MDOT_FREEZE if mdot is None else mdot
        if lib().orc_set_readings(self._h, int(d), int(m)) != 0:
            raise ValueError(f"unknown reading div={div} mdot={mdot}")

    def init(self, phi, T, u=None, p=None):
        phi = _f64(phi).reshape(self.N, self.ncell)
        T = _f64(T).reshape(self.ncell)
        u = None if u is None else _f64(u).reshape(self.dim, self.ncell)
        p = None if p is None else _f64(p).reshape(self.ncell)
        lib().orc_init(self._h, _ptr(phi), _ptr(T), _ptr(u), _ptr(p))

    def init_case(self, case):
        self.init(case["phi"], case["T"], case.get("u"), case.get("p"))

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def moments(self) -> dict:
        nf = self.N + 4 + self.dim + 2
        out = np.empty((nf,) + self.shape)
        lib().orc_moments(self._h, _ptr(out))
        N, d = self.N, self.dim
        return dict(phi=out[:N], rhoH=out[N], T=out[N + 1], fl=out[N + 2],
                    rho=out[N + 3], u=out[N + 4:N + 4 + d], p=out[N + 4 + d],
                    mdot=out[N + 5 + d])

    def diagnostics(self) -> dict:
        N = self.N
        out = np.empty(3 * N + 4)
        lib().orc_diagnostics(self._h, _ptr(out))
        return dict(mass=out[:N].copy(), vol_solid=out[N:2 * N].copy(),
                    vol=out[2 * N:3 * N].copy(), sum_rhoH=out[3 * N],
                    max_sum_phi_err=out[3 * N + 1], front=out[3 * N + 2],
                    nonfinite=bool(out[3 * N + 3]))

    def populations(self) -> np.ndarray:
        pop = np.empty((self.nlat * self.Q,) + self.shape)
        lib().orc_get_state(self._h, _ptr(pop), None)
        return pop

    def aux(self) -> np.ndarray:
        aux = np.empty((self.naux,) + self.shape)
        lib().orc_get_state(self._h, None, _ptr(aux))
        return aux

    def set_state(self, pop=None, aux=None):
        pop = None if pop is None else _f64(pop)
        aux = None if aux is None else _f64(aux)
        lib().orc_set_state(self._h, _ptr(pop), _ptr(aux))


def threads() -> int:
    return lib().orc_threads()


# ---- single-cell helpers for the pin tests -------------------------------
def lattice(dim):
    c = (ctypes.c_int * (19 * 3))()
    w = np.zeros(19)
    Q = lib().orc_lattice(dim, c, _ptr(w))
    cc = np.array(list(c), dtype=np.int64).reshape(19, 3)[:Q]
    return cc, w[:Q].copy()


def _q(dim):
    return 9 if dim == 2 else 19


def feq(dim, p, rho, u):
    out = np.zeros(_q(dim))
    lib().orc_feq(dim, p, rho, _ptr(_f64(np.resize(np.asarray(u, float), 3))), _ptr(out))
    return out


def geq(dim, phi, u):
    out = np.zeros(_q(dim))
    lib().orc_geq(dim, phi, _ptr(_f64(np.resize(np.asarray(u, float), 3))), _ptr(out))
    return out


def heq(dim, rhoH, T, rhocp, Eref, u):
    out = np.zeros(_q(dim))
    lib().orc_heq(dim, rhoH, T, rhocp, Eref, _ptr(_f64(np.resize(np.asarray(u, float), 3))),
                  _ptr(out))
    return out


def force(dim, S, F, rhoa, u, rho):
    out = np.zeros(_q(dim))
    v3 = lambda a: _f64(np.resize(np.asarray(a, float), 3))
    lib().orc_force(dim, S, _ptr(v3(F)), _ptr(v3(rhoa)), _ptr(v3(u)), rho, _ptr(out))
    return out


def stencil(dim, Xn):
    g = np.zeros(3)
    lap = np.zeros(1)
    lib().orc_stencil(dim, _ptr(_f64(Xn)), _ptr(g), _ptr(lap))
    return g[:dim].copy(), float(lap[0])


def invert(params, phi, rhoH):
    P = make_params(params)
    T = np.zeros(1)
    fl = np.zeros(1)
    ph = _f64(np.resize(np.asarray(phi, float), 4))
    lib().orc_invert(ctypes.byref(P), _ptr(ph), rhoH, _ptr(T), _ptr(fl))
    return float(T[0]), float(fl[0])


def enthalpy(params, phi, T, fl):
    P = make_params(params)
    ph = _f64(np.resize(np.asarray(phi, float), 4))
    return float(lib().orc_enthalpy(ctypes.byref(P), _ptr(ph), T, fl))


def interface(params, phi, grad, lap):
    """R_p (N,3), mu_p (N,), F_s (3,) for one cell."""
    P = make_params(params)
    N = params["nphase"]
    ph = np.zeros(4)
    ph[:N] = phi
    g = np.zeros((4, 3))
    g[:N, :np.shape(grad)[1]] = grad
    lp = np.zeros(4)
    lp[:N] = lap
    R = np.zeros((4, 3))
    mu = np.zeros(4)
    Fs = np.zeros(3)
    lib().orc_interface(ctypes.byref(P), _ptr(ph), _ptr(g), _ptr(lp), _ptr(R), _ptr(mu),
                        _ptr(Fs))
    return R[:N], mu[:N], Fs


def fd_field(params, X):
    """The step's finite differences of a scalar field X (nz, ny, nx) with copy
    ghosts at the wall-normal faces: grad (dim, nz, ny, nx), lap (nz, ny, nx)."""
    P = make_params(params)
    X = _f64(X)
    d = params["dim"]
    grad = np.zeros((d,) + X.shape)
    lap = np.zeros(X.shape)
    lib().orc_fd_field(ctypes.byref(P), _ptr(X), _ptr(grad), _ptr(lap))
    return grad, lap
