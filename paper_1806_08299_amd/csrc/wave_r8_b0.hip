// Batched sweep kernels (untiled, depth <= 2) of stencil radius 8 (space order 16), mode 0 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 8
#define WAVE_MODE 0
#define WAVE_BATCH 1
#include "wave_inst.inc"
