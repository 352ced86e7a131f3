// Sweep kernels of stencil radius 7 (space order 14), mode 3 (explicit diffusion).
#define WAVE_R 7
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
