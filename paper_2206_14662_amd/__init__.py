"""MI355X (gfx950) particle loop of an axisymmetric 2D3V (r,z) PIC code with
Monte-Carlo electron-neutral collisions (Le Bars et al., arXiv 2206.14662).

The compute lives in libpicmcc.so (HIP kernels behind the C ABI of
include/pic.h); `binding` marshals Python arguments to it.
"""
from .binding import (PIC_MODE_FP32_BATCHED, PIC_MODE_FP64_PLAIN, PicError, Sim, lib,  # noqa: F401
                      pic_auto_shift, pic_derive, pic_destroy, pic_diag, pic_get_charge,
                      pic_get_fields, pic_get_particles, pic_get_phi, pic_init, pic_last_error,
                      pic_set_fields, pic_set_particles, pic_set_step, pic_step, pic_sync,
                      pic_timing, pic_tuning)
