// Sweep kernels of stencil radius 6 (space order 12).
#define WAVE_R 6
#include "wave_inst.inc"
