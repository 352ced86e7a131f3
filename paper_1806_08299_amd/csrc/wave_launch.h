// wave_launch.h -- host-visible entry into the per-radius kernel instantiations.
#pragma once
#include <hip/hip_runtime.h>
#include "wave_device.h"

namespace wavett {

enum : int { KIND_UNTILED = 0, KIND_TILED = 1 };

// Thread-block shapes.  Untiled: core TY x TX.  Tiled: extended tile EY x EX.
//   3D untiled        4 waves x 4 rows       -> 16 x 64 core (256 threads)
//   3D tiled, shape 1 16 waves x 4 rows      -> 64 x 64 extended tile (1024 threads)
//   3D tiled, shape 2 16 waves x 2 rows      -> 32 x 64 extended tile (1024 threads)
//   3D tiled, shape 3 8 x 2 waves x 4 rows   -> 32 x 128 extended tile (1024 threads)
//   3D tiled, shape 4 4 x 2 waves x 4 rows   -> 16 x 128 extended tile (512 threads)
//   2D untiled        4 waves x 4 segments   -> 1 x 1024 (256 threads)
//   2D tiled          8 waves x 2 segments   -> 1 x 1024 (512 threads)
struct BlockShape { int nw, ry, ey, ex; };
constexpr int kNumShapes3D = 4;
// Untiled 3D block: waves x rows per thread (core 16 x 64 by default).
#ifndef WAVE_UNTILED_NW
#define WAVE_UNTILED_NW 4
#endif
#ifndef WAVE_UNTILED_RY
#define WAVE_UNTILED_RY 4
#endif
BlockShape block_shape(int kind, int dim, int shape);

// Largest fused depth T instantiated for (radius, dim, shape); 0 if none.
int tiled_tmax(int R, int dim, int shape);

// Launch one sweep of a single context (SweepArgs in the kernel-argument
// segment at static offsets).  `lds_bytes` is the dynamic LDS of the tiled kernel.
hipError_t launch_sweep(int R, int kind, int T, int dim, int mode, int shape, const SweepArgs& A,
                        dim3 grid, size_t lds_bytes, hipStream_t s);
// Launch one sweep over the shots of B (batched instantiations: untiled, or
// T <= kBatchTmax).
hipError_t launch_batch(int R, int kind, int T, int dim, int mode, int shape, const BatchArgs& B,
                        dim3 grid, size_t lds_bytes, hipStream_t s);

// Per-(radius, mode) entry points, one translation unit each.
#define WAVE_DECL1(RR, MM)                                                                          \
  hipError_t launch_sweep_r##RR##_m##MM(int kind, int T, int dim, int shape, const SweepArgs& A, \
                                        dim3 grid, size_t lds_bytes, hipStream_t s);              \
  hipError_t launch_batch_r##RR##_m##MM(int kind, int T, int dim, int shape, const BatchArgs& B, \
                                        dim3 grid, size_t lds_bytes, hipStream_t s);
#define WAVE_DECL(RR) WAVE_DECL1(RR, 0) WAVE_DECL1(RR, 1) WAVE_DECL1(RR, 2)
WAVE_DECL(1) WAVE_DECL(2) WAVE_DECL(3) WAVE_DECL(4) WAVE_DECL(5) WAVE_DECL(6) WAVE_DECL(7) WAVE_DECL(8)
#undef WAVE_DECL
#undef WAVE_DECL1
// Explicit diffusion (mode 3) and the two-level diffusion step (mode 4):
// single-context sweeps only.
#define WAVE_DECL(RR)                                                                            \
  hipError_t launch_sweep_r##RR##_m3(int kind, int T, int dim, int shape, const SweepArgs& A, \
                                     dim3 grid, size_t lds, hipStream_t s);                     \
  hipError_t launch_sweep_r##RR##_m4(int kind, int T, int dim, int shape, const SweepArgs& A, \
                                     dim3 grid, size_t lds, hipStream_t s);
WAVE_DECL(1) WAVE_DECL(2) WAVE_DECL(3) WAVE_DECL(4) WAVE_DECL(5) WAVE_DECL(6) WAVE_DECL(7) WAVE_DECL(8)
#undef WAVE_DECL

// Deepest time tile of the batched instantiations (bounds the build).
constexpr int kBatchTmax = 2;

// Depth limits per (radius, dim, shape), shared by host planning and the
// instantiation units.  Bounded by the register file: every fused level keeps
// a (2R+1)-plane window per column.
// 64 x 64 and 32 x 128: 16 waves of 4 rows (1024 threads) leave 128 registers
// per thread, half of what the 512-thread tiles may use, so the windows of
// fewer levels fit (deeper builds spill; at radius 1, with b carried from
// stage to stage, T = 3 fits both tiles and T = 4 on 64 x 64 spills 36 bytes).
// The 64 x 64 tile measured faster this way than as 8 waves of 8 rows (at
// radius 1, T = 3: 431.6 against 401.3 Gpts/s on 592^3): twice the waves per
// SIMD hide the latency that bounds it.
constexpr int kTmax3D_S1[9] = {0, 4, 2, 1, 1, 1, 1, 1, 1};
// 32 x 64: 16 waves of 2 rows (1024 threads), measured against 8 waves of 4
// rows (592^3 wave sweep at order 2: T = 3 422.7 against 390.5 Gpts/s; the
// Laplace operator, 500^3: order 2 T = 4 1434.8 against 1372.0, order 4 T = 3
// 686.4 against 578.5; order 4 T = 2 of the wave sweep 304.0 against 327.7,
// where 32 x 128 is faster than either).  Spill-free up to depth 6, 4, 3, 2,
// 2, 2, 1, 1 at radii 1..8; the deeper entries below spill and stay built for
// the depth sweeps.
constexpr int kTmax3D_S2[9] = {0, 6, 6, 4, 3, 2, 2, 2, 1};
constexpr int kTmax3D_S3[9] = {0, 3, 2, 1, 1, 1, 1, 1, 1};
// 16 x 128: bounded by the core, 16 - 2 r T >= 1 rows.
constexpr int kTmax3D_S4[9] = {0, 6, 3, 2, 1, 1, 1, 1, 0};
// 2D 1 x 1024: 8 waves of 2 slots (64 columns apart); measured against 4 waves
// of 4 slots (16384^2, 100 steps): order 2 801 against 783 Gpts/s (T = 6
// against 4), order 8 481 against 433 (T = 3), order 4 level.  Beyond these
// depths the windows of the fused levels leave too few waves per SIMD.
constexpr int kTmax2D[9] = {0, 8, 8, 6, 4, 2, 2, 2, 2};

}  // namespace wavett
