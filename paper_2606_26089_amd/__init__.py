"""fmdet: conditional flow-matching detector simulation on MI355X (gfx950).

The hot path (noise, truth encoding, velocity network, Euler/RK4 integration) runs in
the HIP kernels of libfmdet.so behind the C ABI of include/fmd.h; ``fmd`` is its
ctypes binding.
"""

from . import fmd  # noqa: F401
from .fmd import Model, linear_field, noise, pack_padded, param_count  # noqa: F401
