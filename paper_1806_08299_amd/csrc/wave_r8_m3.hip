// Sweep kernels of stencil radius 8 (space order 16), mode 3 (explicit diffusion).
#define WAVE_R 8
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
