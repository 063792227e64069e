"""ctypes binding of the host emulator of the step kernel (liblbfreeze_emu.so).

The emulator runs the HIP kernel's own phase functions on the CPU; the CPU
tests compare it with the oracle to check the kernel's indexing and
physics before it runs on a GPU."""
import ctypes
import os

import numpy as np

from paper_2603_22902_amd import lbfreeze

EMU_PATH = os.path.join(os.path.dirname(lbfreeze.LIB_PATH), "liblbfreeze_emu.so")
SAN_PATH = os.path.join(os.path.dirname(lbfreeze.LIB_PATH), "lbf_emu_sanitize")
ADJ_SAN_PATH = os.path.join(os.path.dirname(lbfreeze.LIB_PATH), "lbf_emu_adj_sanitize")
_PD = ctypes.POINTER(ctypes.c_double)
_emu = None


def available():
    return os.path.exists(EMU_PATH)


def _lib():
    global _emu
    if _emu is None:
        _emu = ctypes.CDLL(EMU_PATH)
        _emu.lbf_emu_run.restype = ctypes.c_int
        _emu.lbf_emu_run.argtypes = [ctypes.POINTER(lbfreeze.lbf_params), _PD, _PD, _PD, _PD,
                                     ctypes.c_int, _PD, _PD, _PD]
        _emu.lbf_emu_adjoint.restype = ctypes.c_int
        _emu.lbf_emu_adjoint.argtypes = [ctypes.POINTER(lbfreeze.lbf_params), _PD, _PD, ctypes.c_int,
                                         ctypes.c_int, _PD, _PD]
    return _emu


def _p(a):
    return None if a is None else a.ctypes.data_as(_PD)


def run(case, nsteps):
    """Emulated run: returns (populations, aux, moments dict) like the oracle."""
    prm = case["params"]
    P = lbfreeze.make_params(prm)
    dim, N = prm["dim"], prm["nphase"]
    Q = 9 if dim == 2 else 19
    shape = case["T"].shape
    nc = int(np.prod(shape))
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    pop = np.empty(((N + 2) * Q,) + shape)
    aux = np.empty((N + dim + 3,) + shape)
    mom = np.empty((N + 6 + dim,) + shape)
    rc = _lib().lbf_emu_run(ctypes.byref(P), _p(f64(case["phi"])), _p(f64(case["T"])),
                            _p(f64(case.get("u"))), _p(f64(case.get("p"))), int(nsteps),
                            _p(pop), _p(aux), _p(mom))
    if rc != 0:
        raise RuntimeError("lbf_emu_run rejected the parameters")
    m = dict(phi=mom[:N], rhoH=mom[N], T=mom[N + 1], fl=mom[N + 2], rho=mom[N + 3],
             u=mom[N + 4:N + 4 + dim], p=mom[N + 4 + dim], mdot=mom[N + 5 + dim])
    return pop, aux, m


OBJECTIVES = {"frozen_fraction": 0, "front": 1}


def adjoint(params, phi, T, nsteps, objective="frozen_fraction"):
    """Emulated forward run from an equilibrium start (u = p = 0) and the
    reverse sweep: (J, grad[22]) with J the objective of the final state
    (the frozen fraction, or the front position sum f_s psi per wall-layer
    cell) and grad as lbf_adjoint_gradient."""
    P = lbfreeze.make_params(params)
    J = np.zeros(1)
    g = np.zeros(22)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    rc = _lib().lbf_emu_adjoint(ctypes.byref(P), _p(phi), _p(T), int(nsteps),
                                 OBJECTIVES[objective], _p(J), _p(g))
    if rc != 0:
        raise EmulatorError(rc, float(J[0]), g)
    return float(J[0]), g


class EmulatorError(RuntimeError):
    """A non-zero status of the emulated reverse sweep (LBF_ENAN = -5 for a
    non-finite objective or gradient); J and grad hold what was computed."""

    def __init__(self, rc, J, grad):
        super().__init__(f"lbf_emu_adjoint failed ({rc})")
        self.rc, self.J, self.grad = rc, J, grad
