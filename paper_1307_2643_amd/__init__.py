"""MI355X-native propagation of cosmic-ray nuclei through a periodic turbulent
magnetic-field grid (the 3D propagation hot path of CRPropa 3.0,
arXiv:1307.2643): hand-written HIP kernels behind a C-ABI (include/crp.h),
with this package as a thin ctypes binding."""
from . import crp  # noqa: F401
from .crp import Context, Params, CrpError, params_for  # noqa: F401
