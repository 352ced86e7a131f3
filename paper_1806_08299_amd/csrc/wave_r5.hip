// Sweep kernels of stencil radius 5 (space order 10).
#define WAVE_R 5
#include "wave_inst.inc"
