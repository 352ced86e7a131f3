// Sweep kernels of stencil radius 8 (space order 16), mode 2 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 8
#define WAVE_MODE 2
#define WAVE_BATCH 0
#include "wave_inst.inc"
