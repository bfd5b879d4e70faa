"""MI355X-native hot path of the laser-dielectric PIC method of arXiv 2502.13695.

The compute path is the HIP library ``libpic.so`` (C ABI in include/pic.h);
``paper_2502_13695_amd.pic`` is its ctypes binding.
"""

from . import pic  # noqa: F401
