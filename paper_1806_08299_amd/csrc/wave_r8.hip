// Sweep kernels of stencil radius 8 (space order 16).
#define WAVE_R 8
#include "wave_inst.inc"
