// Sweep kernels of stencil radius 5 (space order 10), mode 3 (explicit diffusion).
#define WAVE_R 5
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
