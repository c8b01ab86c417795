"""MI355X-native single-relaxation-time Shan-Chen D3Q19 lattice Boltzmann.

The update (Section 2 of Chiappini, Xue, Falcucci & Sbragaglia, ligament
break-up with the pseudo-potential LBM) runs in hand-written HIP kernels in
``liblbm.so`` behind the C ABI of ``include/liblbm.h``; ``lbm`` is its ctypes
binding and ``analysis`` post-processes fields and diagnostics.
"""
from . import lbm  # noqa: F401  (raises if liblbm.so has not been built)
from .lbm import Batch, Lattice, LbmError, lbm_coexistence  # noqa: F401
