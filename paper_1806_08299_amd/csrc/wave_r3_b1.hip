// Batched sweep kernels (untiled, depth <= 2) of stencil radius 3 (space order 6), mode 1 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 3
#define WAVE_MODE 1
#define WAVE_BATCH 1
#include "wave_inst.inc"
