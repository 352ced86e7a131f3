// Sweep kernels of stencil radius 6 (space order 12), mode 1 (0 forward, 1 forward storing history, 2 adjoint with imaging).
#define WAVE_R 6
#define WAVE_MODE 1
#define WAVE_BATCH 0
#include "wave_inst.inc"
