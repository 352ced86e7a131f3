// Sweep kernels of stencil radius 3 (space order 6).
#define WAVE_R 3
#include "wave_inst.inc"
