// Sweep kernels of stencil radius 2 (space order 4).
#define WAVE_R 2
#include "wave_inst.inc"
