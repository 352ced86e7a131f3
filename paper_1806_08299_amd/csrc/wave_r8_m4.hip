// Sweep kernels of stencil radius 8 (space order 16), mode 4 (the two-level Adams-Bashforth diffusion step; single-step kernel).
#define WAVE_R 8
#define WAVE_MODE 4
#define WAVE_BATCH 0
#include "wave_inst.inc"
