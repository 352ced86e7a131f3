// Sweep kernels of stencil radius 7 (space order 14).
#define WAVE_R 7
#include "wave_inst.inc"
