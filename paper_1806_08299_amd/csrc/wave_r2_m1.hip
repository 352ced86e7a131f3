// Sweep kernels of stencil radius 2 (space order 4), mode 1 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 2
#define WAVE_MODE 1
#define WAVE_BATCH 0
#include "wave_inst.inc"
