// Sweep kernels of stencil radius 7 (space order 14), mode 4 (the two-level Adams-Bashforth diffusion step; single-step kernel).
#define WAVE_R 7
#define WAVE_MODE 4
#define WAVE_BATCH 0
#include "wave_inst.inc"
