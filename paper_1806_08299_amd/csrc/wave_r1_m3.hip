// Sweep kernels of stencil radius 1 (space order 2), mode 3 (explicit diffusion).
#define WAVE_R 1
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
