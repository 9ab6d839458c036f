"""MI355X lattice-Boltzmann step with momentum-exchange force and torque
(Giovacchini & Ortiz, arXiv:1407.4524): HIP kernels behind the C ABI of
include/lbm.h, and a thin ctypes binding (:mod:`paper_1407_4524_amd.lbm`)."""
from .lbm import Batch, Domain, LbmError, lib  # noqa: F401
