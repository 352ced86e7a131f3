// Sweep kernels of stencil radius 2 (space order 4), mode 4 (the two-level Adams-Bashforth diffusion step; single-step kernel).
#define WAVE_R 2
#define WAVE_MODE 4
#define WAVE_BATCH 0
#include "wave_inst.inc"
