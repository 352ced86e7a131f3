// wave_device.h -- device-side building blocks shared by every sweep kernel.
//
// The paper's correctness criterion for time-tiling (evaluation chapter,
// "Functional correctness") is bitwise equality with the untiled sweep: every
// value must be reached through the same expression, only in another order of
// points.  Here that is guaranteed by construction: every kernel (untiled,
// time-tiled, forward, adjoint) evaluates a grid point through
// `wave_num<R, HAS_Y>()` and `wave_damp()` below, with explicit fused multiply-adds and
// contraction disabled for the whole library (-ffp-contract=off), so the
// arithmetic per point is one fixed sequence of IEEE operations no matter how
// the points are scheduled.
//
// The update is the leapfrog step for  m u_tt + m sigma u_t = lap u + q
// written with b = dt^2/m and st = sigma dt / 2:
//   u^{n+1} = [ b (L u^n + f) + 2 u^n - (1 - st) u^{n-1} ] / (1 + st)
// (f = sum_s w q for the forward sweep; sum_r w dd / dt^2 for the adjoint,
// which runs the same step backwards in time because the step's blocks are
// symmetric).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wavett {

constexpr int kMaxR = 8;

// Stencil weights in FP32: c0 = c_0 * sum_a h_a^-2, w[a][j-1] = c_j / h_a^2.
// Axis slots: 0 = streamed axis (z), 1 = middle axis (y, 3D only), 2 = unit
// stride axis (x).
struct Coefs {
  float c0;
  float w[3][kMaxR];
};

// One grid point, numerator of the update.  zm[j-1] = u(z-j), zp[j-1] = u(z+j),
// likewise y and x.  Operation order: centre, then axis z pairs j=1..R, axis
// y, axis x; then the forcing; then the time update.  Never reorder: the
// tiled/untiled bitwise equality rests on this sequence.  `damped` and
// `forced` are uniform over a launch or a plane and only skip operations that
// cannot change the result there (a forcing of +0, a damping factor of 1).
template <int R, bool HAS_Y>
__device__ __forceinline__ float wave_num(const Coefs& C, float uc,
                                          const float* zm, const float* zp,
                                          const float* ym, const float* yp,
                                          const float* xm, const float* xp,
                                          float uprev, float b, float st, float f,
                                          bool damped, bool forced) {
  float lap = C.c0 * uc;
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[0][j], zm[j] + zp[j], lap);
  if (HAS_Y) {
#pragma unroll
    for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[1][j], ym[j] + yp[j], lap);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[2][j], xm[j] + xp[j], lap);
  const float t = forced ? lap + f : lap;
  // with st == 0 the fused form equals 2u - u_prev exactly
  const float a = damped ? __builtin_fmaf(-(1.0f - st), uprev, 2.0f * uc) : 2.0f * uc - uprev;
  return __builtin_fmaf(b, t, a);
}

// One grid point of explicit diffusion (the Laplace-operator workload):
// u + (C.c0 u + sum of weighted pairs), the weights already scaled by
// dt a / h_axis^2.  Same operation order as wave_num's Laplacian (centre,
// then axis z, y, x pairs), then one addition.
template <int R, bool HAS_Y>
__device__ __forceinline__ float diff_next(const Coefs& C, float uc,
                                           const float* zm, const float* zp,
                                           const float* ym, const float* yp,
                                           const float* xm, const float* xp) {
  float lap = C.c0 * uc;
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[0][j], zm[j] + zp[j], lap);
  if (HAS_Y) {
#pragma unroll
    for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[1][j], ym[j] + yp[j], lap);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[2][j], xm[j] + xp[j], lap);
  return uc + lap;
}

// The two-level (Adams-Bashforth) diffusion step.  The rule
// u + dt a (3/2 L u^n - 1/2 L u^{n-1}) equals u + dt a L w with
// w = 3/2 u^n - 1/2 u^{n-1} (L is linear), so the sweeps stream w through
// the windows and planes the one-level step streams u through: ab2_input
// forms w once per loaded point (one rounding: -u^{n-1}/2 is exact), and
// ab2_next adds the scaled Laplacian of w to u^n.  Same operation order in
// every schedule.
__device__ __forceinline__ float ab2_input(float un, float unm1) { return __builtin_fmaf(1.5f, un, -0.5f * unm1); }

template <int R, bool HAS_Y>
__device__ __forceinline__ float ab2_next(const Coefs& C, float wc,
                                          const float* zm, const float* zp,
                                          const float* ym, const float* yp,
                                          const float* xm, const float* xp, float un) {
  float lap = C.c0 * wc;
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[0][j], zm[j] + zp[j], lap);
  if (HAS_Y) {
#pragma unroll
    for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[1][j], ym[j] + yp[j], lap);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) lap = __builtin_fmaf(C.w[2][j], xm[j] + xp[j], lap);
  return un + lap;
}

// Inside the absorbing layer divide by (1 + st) through the hardware
// reciprocal; elsewhere (st == 0) the numerator is the result.
__device__ __forceinline__ float wave_damp(float num, float st) {
  return (st != 0.0f) ? num * __builtin_amdgcn_rcpf(1.0f + st) : num;
}

// Gradient contribution of one adjoint step (imaging condition):
//   g <- g - u^j ((1+st) mu^{j-1} - 2 mu^j + (1-st) mu^{j+1})
// accumulated one time step at a time, in decreasing j, by every kernel.
__device__ __forceinline__ float image_step(float g, float u, float st,
                                            float mu_new, float mu_cur, float mu_old) {
  float t = (1.0f + st) * mu_new;
  t = __builtin_fmaf(-2.0f, mu_cur, t);
  t = __builtin_fmaf(1.0f - st, mu_old, t);
  return __builtin_fmaf(-u, t, g);
}

// Points where a forcing term enters (sources forward, receivers in the
// adjoint) or where values are sampled (receivers forward, sources in the
// adjoint).  Unique grid points sorted by (z, y, x); zptr is a CSR index over
// the streamed axis (n0 + 1 entries).  `table`/`samp` are [step][npts].
struct PointSet {
  const int32_t* zptr;
  const int32_t* y;
  const int32_t* x;
  int32_t npts;
};

// Tables of a call, in device memory: only the few planes holding points
// read them, so they are kept out of the kernel's live scalar state.
struct SweepAux {
  PointSet inj;                // forcing points
  const float* inj_table;      // [steps][inj.npts]
  PointSet smp;                // sampled points
  float* smp_out;              // [steps][smp.npts]
};

// Kernel modes: the wave sweep forward, forward storing the history, adjoint
// with imaging; explicit diffusion (one input level, no b, no damping); the
// two-level Adams-Bashforth diffusion step (single-step kernel only).
enum : int { MODE_FWD = 0, MODE_HIST = 1, MODE_ADJ = 2, MODE_DIFF = 3, MODE_AB2 = 4 };

// Everything a sweep launch needs (passed by value).
struct SweepArgs {
  Coefs C;
  int32_t n0, n1, n2;          // grid (2D: n1 == 1)
  int64_t s1, s0;              // strides of axis 1 and axis 0 (elements)
  const float* cur;            // level "n" (forward) or mu^{m} (adjoint)
  const float* prev;           // level n-1 / mu^{m+1}
  float* outA;                 // new top level (n+T)
  float* outB;                 // level n+T-1 (may be null for in-place T=1)
  const float* b;              // dt^2 / m
  // damping: st = (e(z) + e(y)) + e(x), e(i) = st_coef * d(i)^2 with d(i) the
  // depth of index i inside the absorbing layer of width nbl along that axis
  int32_t has_damp;            // 0: st == 0 everywhere
  int32_t nbl;
  float st_coef;               // sigma_max * dt / (2 nbl^2)
  const struct SweepAux* aux;  // forcing / sampling tables (device memory), read on the rare path only
  int32_t inj_zlo, inj_zhi;    // planes holding forcing points: [inj_zlo, inj_zhi)
  int32_t smp_zlo, smp_zhi;    // planes holding sampled points
  int32_t step0;               // step index produced by stage 1
  int32_t dir;                 // +1 forward, -1 adjoint: stage k produces step0 + dir (k-1)
  float* hist;                 // MODE_HIST: written; MODE_ADJ: read.  [slot][N]
  int32_t hist_base;           // slot = level - hist_base (level = step + 1)
  float* grad;                 // MODE_ADJ: gradient accumulator [N]
  // tiling
  int32_t skew;                // halo per fused step on the tiled axes
  int32_t core_y, core_x;      // core tile extents
  int32_t tiles_x;             // tiles along x; tile index = ty * tiles_x + tx
  int32_t ntiles;              // tiles per axis-0 segment
  int32_t nblocks;             // ntiles * number of axis-0 segments (1D grid)
  int32_t zchunk;              // streamed-axis segment length per block
  int32_t zlo, zhi;            // planes [zlo, zhi) this launch updates (the whole grid, or one
                               // slab of the skewed schedule); segments of zchunk planes from zlo
};

// LDS planes of the tiled kernel: each is (EX + 2R) x (EY + 2R_y) floats; one
// set of T planes, doubled (one barrier per plane instead of two) when both
// sets fit in the 160 KiB of LDS a gfx950 workgroup may use.
constexpr int tiled_plane_floats(int R, int EY, int EX, bool HY) { return (EX + 2 * R) * (EY + 2 * (HY ? R : 0)); }
constexpr int tiled_nbuf(int R, int T, int EY, int EX, bool HY) {
  return (2 * T * tiled_plane_floats(R, EY, EX, HY) * 4 <= 160 * 1024) ? 2 : 1;
}
constexpr size_t tiled_lds_bytes(int R, int T, int EY, int EX, bool HY) {
  return (size_t)tiled_nbuf(R, T, EY, EX, HY) * T * tiled_plane_floats(R, EY, EX, HY) * 4;
}

// Damping term of index i along an axis of n points (layer nbl wide).
__device__ __forceinline__ float damp_term(int i, int n, int nbl, float coef) {
  const int d = max(max(nbl - i, i - (n - 1 - nbl)), 0);
  return coef * (float)(d * d);
}

// Arguments of one launch: the windows of up to kMaxBatch independent shots
// (same radius, depth, tile shape and mode) whose workgroups share one grid.
// Shot s owns workgroups [off[s], off[s+1]).  Everything travels in the
// kernel-argument segment (under 4 KiB), so a launch needs no device table
// and every field is read with scalar loads from invariant memory.
constexpr int kMaxBatch = 12;
struct BatchArgs {
  int32_t n;                       // shots in this launch, 1..kMaxBatch
  int32_t off[kMaxBatch + 1];      // off[0] = 0, off[n] = grid size
  SweepArgs a[kMaxBatch];
};

// Kernel argument of a single-context launch (SweepArgs, fields at static
// offsets of the argument segment) or of a batched one (BatchArgs).
template <bool BATCH> struct LaunchArgs { using type = SweepArgs; };
template <> struct LaunchArgs<true> { using type = BatchArgs; };

// The arguments of this workgroup's shot and its workgroup index within the
// shot.  Batched: the shot is found by a fixed-trip scan over the prefix,
// fully unrolled so that its scalar loads are issued together (wave-uniform).
__device__ __forceinline__ const SweepArgs& shot_args(const SweepArgs& A, int& blk) {
  blk = (int)blockIdx.x;
  return A;
}
__device__ __forceinline__ const SweepArgs& shot_args(const BatchArgs& B, int& blk) {
  int s = 0;
#pragma unroll
  for (int i = 1; i < kMaxBatch; ++i) s += (i < B.n && (int)blockIdx.x >= B.off[i]) ? 1 : 0;
  blk = (int)blockIdx.x - B.off[s];
  return B.a[s];
}

// Work item `blk` of a shot: tiles vary fastest, then axis-0 segments, so
// the workgroups resident at any moment cover one compact front of the grid
// (neighbouring tiles re-read each other's halo columns from the shared
// last-level cache while they are still there).  Within a segment the tiles
// are taken in bands of kXcd tile rows, column by column.  Workgroups are
// dealt to the XCDs round-robin, so work item t + kXcd runs on the XCD of
// item t and, inside a band, is its neighbour along axis 2: the halo lines
// the two share come from that XCD's L2.  Rows past the last whole band keep
// the row-major order.
constexpr int kXcd = 8;   // XCDs of the chip
__device__ __forceinline__ void work_item(const SweepArgs& A, int blk, int& tile, int& chunk) {
  chunk = blk / A.ntiles;
  tile = blk % A.ntiles;
  const int band_tiles = kXcd * A.tiles_x;
  const int band = tile / band_tiles;
  if (band < A.ntiles / band_tiles) {
    const int l = tile - band * band_tiles;
    tile = (band * kXcd + l % kXcd) * A.tiles_x + l / kXcd;
  }
}

// Step of stage k (1-based) of a launch.
__device__ __forceinline__ int stage_step(const SweepArgs& A, int k) {
  return A.step0 + A.dir * (k - 1);
}

}  // namespace wavett
