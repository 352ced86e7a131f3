// Sweep kernels of stencil radius 2 (space order 4), mode 3 (explicit diffusion).
#define WAVE_R 2
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
