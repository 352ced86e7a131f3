"""Time-tiled acoustic-wave sweeps on MI355X (gfx950).

The product is the C-ABI library ``libwavett.so`` (declared in include/wave.h,
built by ``paper_1806_08299_amd.build``); ``paper_1806_08299_amd.wave`` is its
Python binding and autograd wrapper.
"""
from .wave import (DiffOp, ShotBatch, WaveError, WaveFn, WaveOp, lib, make_desc, wave_adjoint_grad, wave_ai_naive,  # noqa: F401
                   wave_ai_tight, wave_autotune, wave_bytes_per_point, wave_destroy, wave_flops_per_point,
                   wave_forward, wave_get_schedule, wave_init, wave_scratch_bytes, wave_set_model,
                   wave_set_schedule, wave_state_bytes, wave_tiled_max_depth)
