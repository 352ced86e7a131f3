// Sweep kernels of stencil radius 6 (space order 12), mode 3 (explicit diffusion).
#define WAVE_R 6
#define WAVE_MODE 3
#define WAVE_BATCH 0
#include "wave_inst.inc"
