// Sweep kernels of stencil radius 4 (space order 8).
#define WAVE_R 4
#include "wave_inst.inc"
