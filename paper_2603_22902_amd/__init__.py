"""MI355X-native coupled lattice-Boltzmann solver for N-phase flow with
liquid-solid phase change (arXiv:2603.22902), behind the C ABI of
include/lbfreeze.h.  The compute path is the HIP library liblbfreeze.so
built in this directory; :mod:`.lbfreeze` is its ctypes binding."""
from .lbfreeze import (LBF_M_ALL, LbfError, Solver, lbf_check_params, lbf_state_bytes,  # noqa: F401
                       make_params)
