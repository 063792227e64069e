"""ctypes binding of the lbfreeze C ABI (include/lbfreeze.h).

Argument marshalling only: every step of the solver runs in the HIP
library ``liblbfreeze.so`` built in this package directory.  PyTorch
provides the device buffer and the HIP stream.  Importing this module does
not need a GPU; creating a :class:`Solver` does, and raises if the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbfreeze.so")

LBF_OK, LBF_EINVAL, LBF_ENOMEM, LBF_EDEVICE, LBF_ENOTSUP, LBF_ENAN, LBF_ESTATE = 0, -1, -2, -3, -4, -5, -6
LBF_FP32, LBF_FP64, LBF_MIXED = 0, 1, 2
LBF_BC_WALL, LBF_BC_OPEN = 0, 1
LBF_TBC_DIRICHLET, LBF_TBC_ADIABATIC = 0, 1
LBF_M_PHI, LBF_M_RHOH, LBF_M_T, LBF_M_FL, LBF_M_RHO, LBF_M_U, LBF_M_P, LBF_M_MDOT = (1 << k for k in range(8))
LBF_M_ALL = 0xFF

_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)


class lbf_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("nphase", ctypes.c_int), ("precision", ctypes.c_int),
        ("flow_bc", ctypes.c_int * 2), ("therm_bc", ctypes.c_int * 2), ("T_face", _D * 2),
        ("rho_l", _D * 4), ("rho_s", _D * 4), ("mu_l", _D * 4), ("mu_s", _D * 4),
        ("lam_l", _D * 4), ("lam_s", _D * 4), ("cp_l", _D * 4), ("cp_s", _D * 4),
        ("latent", _D * 4), ("freezes", ctypes.c_int * 4),
        ("sigma", (_D * 4) * 4), ("cos_theta", (_D * 4) * 4),
        ("eps", _D), ("tau_g", _D), ("T_melt", _D), ("E_ref", _D), ("gravity", _D * 3),
    ]


class LbfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbfreeze error {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load liblbfreeze.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2603_22902_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbf_params)
        vp = ctypes.c_void_p
        L.lbf_check_params.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        L.lbf_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.lbf_init_fields.argtypes = [vp, _PD, _PD, _PD, _PD]
        L.lbf_step.argtypes = [vp, ctypes.c_int]
        L.lbf_step_timed.argtypes = [vp, ctypes.c_int, _PD]
        L.lbf_state_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_state_to_device.argtypes = [vp, vp]
        L.lbf_state_from_device.argtypes = [vp, vp, ctypes.c_longlong]
        L.lbf_step_states.argtypes = [vp, vp, vp]
        L.lbf_adjoint_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_adjoint_create.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.lbf_adjoint_seed.argtypes = [vp, _PD]
        L.lbf_adjoint_seed_objective.argtypes = [vp, ctypes.c_int, _PD]
        L.lbf_adjoint_step.argtypes = [vp, vp, vp]
        L.lbf_adjoint_finish.argtypes = [vp, vp]
        L.lbf_adjoint_gradient.argtypes = [vp, _PD]
        L.lbf_adjoint_state.argtypes = [vp, _PD, _PD]
        L.lbf_adjoint_destroy.argtypes = [vp]
        L.lbf_batch_bytes.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(vp)]
        L.lbf_batch_set_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.lbf_batch_tune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.lbf_batch_step.argtypes = [vp, ctypes.c_int]
        L.lbf_batch_set_launch.argtypes = [vp, ctypes.c_uint, ctypes.c_int]
        L.lbf_batch_capture.argtypes = [vp]
        L.lbf_batch_replay.argtypes = [vp, ctypes.c_int]
        L.lbf_batch_destroy.argtypes = [vp]
        L.lbf_batch_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_batch_state_to_device.argtypes = [vp, vp]
        L.lbf_batch_state_from_device.argtypes = [vp, vp, ctypes.c_longlong]
        L.lbf_batch_step_states.argtypes = [vp, vp, vp]
        L.lbf_batch_adjoint_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_batch_adjoint_create.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.lbf_batch_adjoint_seed.argtypes = [vp, ctypes.c_int, vp, _PD]
        L.lbf_batch_adjoint_step.argtypes = [vp, vp, vp]
        L.lbf_batch_adjoint_finish.argtypes = [vp, vp]
        L.lbf_batch_adjoint_gradient.argtypes = [vp, _PD]
        L.lbf_batch_adjoint_destroy.argtypes = [vp]
        L.lbf_bandwidth_probe.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.c_int, _PD, _PD]
        L.lbf_get_moments.argtypes = [vp, ctypes.c_uint, _PD]
        L.lbf_get_populations.argtypes = [vp, _PD]
        L.lbf_get_aux.argtypes = [vp, _PD]
        L.lbf_diagnostics.argtypes = [vp, _PD]
        L.lbf_diagnostics_noalloc.argtypes = [vp, _PD]
        L.lbf_snapshot_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbf_save_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbf_load_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbf_step_count.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
        L.lbf_destroy.argtypes = [vp]
        L.lbf_last_error.restype = ctypes.c_char_p
        L.lbf_last_error.argtypes = [vp]
        L.lbf_status_string.restype = ctypes.c_char_p
        L.lbf_status_string.argtypes = [ctypes.c_int]
        for name in ("lbf_check_params", "lbf_state_bytes", "lbf_create", "lbf_init_fields",
                     "lbf_step", "lbf_step_timed", "lbf_get_moments", "lbf_get_populations", "lbf_get_aux",
                     "lbf_diagnostics", "lbf_diagnostics_noalloc", "lbf_snapshot_bytes", "lbf_save_state", "lbf_load_state",
                     "lbf_step_count", "lbf_destroy", "lbf_state_device_bytes",
                     "lbf_state_to_device", "lbf_state_from_device", "lbf_step_states", "lbf_adjoint_bytes",
                     "lbf_adjoint_create", "lbf_adjoint_seed", "lbf_adjoint_seed_objective", "lbf_adjoint_step", "lbf_adjoint_finish",
                     "lbf_adjoint_gradient", "lbf_adjoint_state", "lbf_adjoint_destroy",
                     "lbf_batch_bytes", "lbf_batch_create", "lbf_batch_set_tiles", "lbf_batch_set_launch", "lbf_batch_tune",
                     "lbf_batch_step", "lbf_batch_capture", "lbf_batch_replay", "lbf_batch_destroy",
                     "lbf_batch_state_bytes", "lbf_batch_state_to_device", "lbf_batch_state_from_device", "lbf_batch_step_states",
                     "lbf_batch_adjoint_bytes", "lbf_batch_adjoint_create", "lbf_batch_adjoint_seed",
                     "lbf_batch_adjoint_step", "lbf_batch_adjoint_finish", "lbf_batch_adjoint_gradient",
                     "lbf_batch_adjoint_destroy", "lbf_bandwidth_probe"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


_FLOW = {"wall": LBF_BC_WALL, "open": LBF_BC_OPEN}
_THERM = {"dirichlet": LBF_TBC_DIRICHLET, "adiabatic": LBF_TBC_ADIABATIC}
_PREC = {"fp32": LBF_FP32, "fp64": LBF_FP64, "mixed": LBF_MIXED}


def make_params(d: dict) -> lbf_params:
    """Marshal a parameter dict (keys as in the C struct; flow_bc/therm_bc
    and precision may be given by name) into lbf_params."""
    P = lbf_params()
    P.dim, P.nx, P.ny = int(d["dim"]), int(d["nx"]), int(d["ny"])
    P.nz = int(d.get("nz", 1)) if P.dim == 3 else 1
    P.nphase = int(d["nphase"])
    prec = d.get("precision", "fp32")
    P.precision = _PREC[prec] if isinstance(prec, str) else int(prec)
    for k in range(2):
        fb, tb = d["flow_bc"][k], d["therm_bc"][k]
        P.flow_bc[k] = _FLOW[fb] if isinstance(fb, str) else int(fb)
        P.therm_bc[k] = _THERM[tb] if isinstance(tb, str) else int(tb)
        P.T_face[k] = float(d["T_face"][k])
    for key in ("rho_l", "rho_s", "mu_l", "mu_s", "lam_l", "lam_s", "cp_l", "cp_s", "latent"):
        arr = getattr(P, key)
        for p, v in enumerate(list(d[key])[:4]):
            arr[p] = float(v)
    for p, v in enumerate(list(d["freezes"])[:4]):
        P.freezes[p] = int(v)
    for p in range(4):
        for q in range(4):
            P.sigma[p][q] = float(d["sigma"][p][q])
            P.cos_theta[p][q] = float(d["cos_theta"][p][q])
    P.eps, P.tau_g, P.T_melt, P.E_ref = (float(d[k]) for k in ("eps", "tau_g", "T_melt", "E_ref"))
    for a in range(3):
        P.gravity[a] = float(d["gravity"][a])
    return P


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_PD)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def lbf_check_params(params: dict):
    """(status, message) of the host-side validation; needs no GPU."""
    P = make_params(params)
    buf = ctypes.create_string_buffer(256)
    s = lib().lbf_check_params(ctypes.byref(P), buf, 256)
    return s, buf.value.decode()


def lbf_state_bytes(params: dict) -> int:
    P = make_params(params)
    n = ctypes.c_size_t(0)
    s = lib().lbf_state_bytes(ctypes.byref(P), ctypes.byref(n))
    if s != LBF_OK:
        raise LbfError(s, lbf_check_params(params)[1])
    return int(n.value)


class Solver:
    """One simulation on one GPU: a context over a torch-allocated buffer.

    Methods mirror the C ABI: lbf_init_fields, lbf_step, lbf_get_moments,
    lbf_get_populations, lbf_get_aux, lbf_diagnostics, lbf_save_state,
    lbf_load_state.  Host arrays are float64 (N, nz, ny, nx) etc.
    """

    def __init__(self, params: dict, device: int = 0, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("lbfreeze needs a ROCm GPU; none is visible")
        self.params = dict(params)
        self._P = make_params(params)
        self.dim, self.N = self._P.dim, self._P.nphase
        self.Q = 9 if self.dim == 2 else 19
        self.shape = (self._P.nz if self.dim == 3 else 1, self._P.ny, self._P.nx)
        self.ncell = int(np.prod(self.shape))
        self.device = torch.device("cuda", device)
        nbytes = lbf_state_bytes(params)
        with torch.cuda.device(self.device):
            self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            base = self.buffer.data_ptr()
            aligned = (base + 255) & ~255
            h = ctypes.c_void_p(0)
            s = lib().lbf_create(ctypes.byref(self._P), ctypes.c_void_p(aligned), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if s != LBF_OK:
            raise LbfError(s, "lbf_create failed")
        self._h = h

    # -- helpers --------------------------------------------------------
    def _check(self, s):
        if s != LBF_OK:
            raise LbfError(s, lib().lbf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().lbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI ----------------------------------------------------------
    def lbf_init_fields(self, phi, T, u=None, p=None):
        nc = self.ncell
        phi, T = _f64(phi, self.N * nc), _f64(T, nc)
        u, p = _f64(u, self.dim * nc), _f64(p, nc)
        self._check(lib().lbf_init_fields(self._h, _ptr(phi), _ptr(T), _ptr(u), _ptr(p)))

    def lbf_step(self, n: int = 1):
        self._check(lib().lbf_step(self._h, int(n)))

    def lbf_step_timed(self, n: int) -> tuple:
        """n steps; returns the average (moments, collide) kernel durations
        per step in milliseconds, measured with HIP events on the stream."""
        ms = np.zeros(2)
        self._check(lib().lbf_step_timed(self._h, int(n), _ptr(ms)))
        return float(ms[0]), float(ms[1])

    def lbf_get_moments(self, mask: int = LBF_M_ALL) -> dict:
        N, d = self.N, self.dim
        layout = [(LBF_M_PHI, "phi", N), (LBF_M_RHOH, "rhoH", 1), (LBF_M_T, "T", 1),
                  (LBF_M_FL, "fl", 1), (LBF_M_RHO, "rho", 1), (LBF_M_U, "u", d),
                  (LBF_M_P, "p", 1), (LBF_M_MDOT, "mdot", 1)]
        nf = sum(k for m, _, k in layout if mask & m)
        out = np.empty((nf,) + self.shape)
        self._check(lib().lbf_get_moments(self._h, int(mask), _ptr(out)))
        res, k = {}, 0
        for m, name, cnt in layout:
            if mask & m:
                res[name] = out[k:k + cnt] if name in ("phi", "u") else out[k]
                k += cnt
        return res

    def lbf_get_populations(self) -> np.ndarray:
        out = np.empty(((self.N + 2) * self.Q,) + self.shape)
        self._check(lib().lbf_get_populations(self._h, _ptr(out)))
        return out

    def lbf_get_aux(self) -> np.ndarray:
        out = np.empty((self.N + self.dim + 3,) + self.shape)
        self._check(lib().lbf_get_aux(self._h, _ptr(out)))
        return out

    def lbf_diagnostics(self, check_nan: bool = True, noalloc: bool = False) -> dict:
        """lbf_diagnostics, or with noalloc=True lbf_diagnostics_noalloc (the
        same values from the library's static device scratch array)."""
        N = self.N
        out = np.empty(3 * N + 4)
        fn = lib().lbf_diagnostics_noalloc if noalloc else lib().lbf_diagnostics
        s = fn(self._h, _ptr(out))
        if s != LBF_ENAN or check_nan:
            self._check(s)
        return dict(mass=out[:N].copy(), vol_solid=out[N:2 * N].copy(), vol=out[2 * N:3 * N].copy(),
                    sum_rhoH=float(out[3 * N]), max_sum_phi_err=float(out[3 * N + 1]),
                    front=float(out[3 * N + 2]), nonfinite=bool(out[3 * N + 3]))

    def snapshot_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        self._check(lib().lbf_snapshot_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def lbf_save_state(self) -> bytearray:
        buf = bytearray(self.snapshot_bytes())
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        self._check(lib().lbf_save_state(self._h, cbuf, len(buf)))
        return buf

    def lbf_load_state(self, snap) -> None:
        snap = bytearray(snap)
        cbuf = (ctypes.c_char * len(snap)).from_buffer(snap)
        self._check(lib().lbf_load_state(self._h, cbuf, len(snap)))

    def step_count(self) -> int:
        n = ctypes.c_longlong(0)
        self._check(lib().lbf_step_count(self._h, ctypes.byref(n)))
        return int(n.value)

    def state_device_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        self._check(lib().lbf_state_device_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def lbf_state_to_device(self, dst) -> None:
        """Copy the current state into dst (a torch uint8 CUDA tensor of
        state_device_bytes(), contiguous), asynchronously on the stream."""
        self._check(lib().lbf_state_to_device(self._h, ctypes.c_void_p(dst.data_ptr())))

    def lbf_state_from_device(self, src, steps: int) -> None:
        self._check(lib().lbf_state_from_device(self._h, ctypes.c_void_p(src.data_ptr()), int(steps)))

    def lbf_step_states(self, src, dst) -> None:
        """One step from device state src to device state dst (torch uint8
        tensors of state_device_bytes()); the context's state is untouched."""
        self._check(lib().lbf_step_states(self._h, ctypes.c_void_p(src.data_ptr()),
                                          ctypes.c_void_p(dst.data_ptr())))

    # -- convenience ------------------------------------------------------
    def init_case(self, case: dict):
        self.lbf_init_fields(case["phi"], case["T"], case.get("u"), case.get("p"))


def bandwidth_probe(device: int = 0, mib: int = 2048, reps: int = 5) -> dict:
    """HBM rates of a float4 copy and a float4 read sweep on the device
    (lbf_bandwidth_probe), over two buffers of mib MiB: bytes per second."""
    import torch

    n = mib << 20
    a = torch.zeros(n, dtype=torch.uint8, device=device)
    b = torch.empty(n, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(device)
    torch.cuda.synchronize(device)
    c = np.zeros(1)
    r = np.zeros(1)
    s = lib().lbf_bandwidth_probe(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n,
                                  ctypes.c_void_p(stream.cuda_stream), int(reps), _ptr(c), _ptr(r))
    if s != LBF_OK:
        raise LbfError(s, "lbf_bandwidth_probe")
    return {"copy": float(c[0]), "read": float(r[0])}
