// Sweep kernels of stencil radius 3 (space order 6), mode 3 (explicit diffusion).
#define WAVE_R 3
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
