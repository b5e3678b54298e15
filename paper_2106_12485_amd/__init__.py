"""MI355X-native hot path of the 2D EM-PIC timestep of arXiv 2106.12485.

The work runs in HIP kernels for gfx950 behind the C ABI of include/pic.h
(libpic.so, built in-tree); this package holds that source, the build step and
a ctypes binding that only marshals arguments.
"""
from .pic import (Simulation, Batch, batch_step_static, serve, PicError, make_cfg, mem_bytes,  # noqa: F401
                  lib,
                  KERNEL_NAMES,
                  PIC_OK, PIC_E_ARG, PIC_E_CFL, PIC_E_NOMEM, PIC_E_CAPACITY, PIC_E_HIP,
                  PIC_E_STATE, PIC_E_CANCELLED)
