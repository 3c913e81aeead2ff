"""MI355X-native MLFMM solver for the PMCHWT surface integral equation of
single- and multi-layer dielectric scatterers (arXiv:1704.06862).

The compute path is the HIP library ``libsfmm.so`` (C ABI in include/sfmm.h);
``paper_1704_06862_amd.sfmm`` is its ctypes binding.
"""

from .sfmm import Context, SfmmError, load  # noqa: F401
