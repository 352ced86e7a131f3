// Sweep kernels of stencil radius 5 (space order 10), mode 0 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 5
#define WAVE_MODE 0
#define WAVE_BATCH 0
#include "wave_inst.inc"
