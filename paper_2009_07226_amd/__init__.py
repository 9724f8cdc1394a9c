"""MI355X (gfx950) implementation of the projection / backprojection / CGLS
hot path of parallel-beam XCT reconstruction (Hidayetoglu et al., SC20).

The kernels live in libxct.so (C ABI: include/xct.h); this package is its
thin binding, the gradient solver of Eq. (1) built on it (``gradient``), and
seeded input generators.
"""
from .xct import (BF16, F16, F32, F64, Matrix, XctBackproject, XctError, XctProject, backproject,
                  backproject_streamed, cgls, count_nonfinite, device_memory, lib, library_loaded, profile_enable, profile_read, project,
                  project_streamed, projected_gradient, read_bandwidth)

__all__ = ["Matrix", "project", "backproject", "project_streamed", "backproject_streamed", "cgls", "count_nonfinite", "device_memory", "projected_gradient", "XctProject", "XctBackproject", "XctError", "lib",
           "library_loaded", "profile_enable", "profile_read", "read_bandwidth", "F32", "F16", "BF16", "F64"]
