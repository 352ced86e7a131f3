// Sweep kernels of stencil radius 4 (space order 8), mode 3 (explicit diffusion).
#define WAVE_R 4
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
