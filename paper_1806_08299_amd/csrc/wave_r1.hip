// Sweep kernels of stencil radius 1 (space order 2).
#define WAVE_R 1
#include "wave_inst.inc"
