// wave_kernels.h -- sweep kernels (templates), instantiated per stencil radius
// and mode in wave_r<R>_m<M>.hip (batched variants: wave_r<R>_b<M>.hip).
//
// Layout: one FP32 array per time level, row-major [n0][n1][n2] (2D: n1 == 1),
// axis 2 unit stride (the 64 lanes of a wavefront walk it, so every global
// access is a coalesced 256-byte row), axis 0 streamed through registers.
//
// k_untiled  -- one time step per launch ("spatial tiling" in the paper's
//               terms).  A workgroup owns a core tile of TY x TX columns and
//               streams one segment of axis 0 through a (2R+1)-plane register
//               window per column; the current plane plus an R-wide halo,
//               loaded from global memory, sits in LDS for the neighbours along
//               axes 1 and 2.  u^{n+1} overwrites u^{n-1} in place.
//
// k_tiled    -- T time steps per launch: the GPU form of the paper's
//               time-tiling (implementation chapter, "Time-tiling").  Along
//               axis 0 the T stages are pipelined with a lag of R planes each
//               (the minimum legal skew of the background chapter's skewing
//               section): a skewed parallelogram in (t, z) without redundant
//               work.  Across axes 1/2 every workgroup owns an extended tile of
//               EY x EX columns and recomputes a halo of `skew` points per fused
//               step (an overlapped trapezoid), so tiles never wait for each
//               other.  Stage k is valid on the tile shrunk by k*skew per side;
//               after T stages the core is exact.  Each stage's input plane is
//               staged in LDS; the z windows of every level live in registers.
//
// Modes.  MODE_FWD / MODE_HIST / MODE_ADJ sweep the wave equation (forward,
// forward storing every level, adjoint with the imaging condition fused).
// MODE_DIFF sweeps explicit diffusion, the paper's Laplace-operator workload:
// the same streaming and tiling with one input level -- no u^{n-1} or b
// stream, no damping or point terms -- writing to a different array.
//
// Register windows.  The (2R+1)-plane window of every level is a ring in
// registers.  In the tiled sweep the z loop is unrolled by the window length
// and the ring's rotation is a compile-time constant in each unrolled copy, so
// sliding the window costs no moves (for 2R+1 > kMaxUnrollW the window is
// shifted).  The untiled sweep shifts its single window (2R moves per row and
// plane): its loop body then fits the instruction cache, which measured 1-2 %
// faster than the unrolled ring, while the tiled sweep is faster unrolled.
// Neighbours along axis 1 that belong to the same thread come from those
// registers; only the others are read from LDS.
//
// Memory access discipline.  Global traffic goes through raw buffer
// instructions with one descriptor per array covering the segment of planes a
// workgroup may touch (at most kSegMax bytes).  The plane offset is the
// instruction's scalar offset and the column offset its vector offset; the
// hardware range check covers their sum.  Out-of-grid columns carry kOOB, and
// planes outside the grid (or, for stores, outside the planes a workgroup
// owns) get the segment length as scalar offset, so every such access lands
// past the descriptor without wrapping 32 bits: loads return 0 (the zero
// boundary values) and stores are dropped, with no branches and no 64-bit
// address arithmetic in the loop.  Every load is issued one plane ahead of its
// use (the tiled adjoint's history and gradient loads: at the start of the
// iteration that uses them).  Because b = dt^2/m also reads as 0 outside the grid, the update there
// evaluates to exactly +0 with no select.
#pragma once
#include <utility>

#include "wave_device.h"

namespace wavett {

// --------------------------------------------------------------- buffer access

typedef __amdgpu_buffer_rsrc_t rsrc_t;

constexpr uint32_t kSegMax = 0x40000000u;   // largest segment a descriptor covers (host-enforced)
constexpr uint32_t kOOB = 0x80000000u;      // column offset of an out-of-grid lane
#ifndef WAVE_MAX_UNROLL_W
#define WAVE_MAX_UNROLL_W 9
#endif
#ifndef WAVE_MAX_UNROLL_W_UNTILED
#define WAVE_MAX_UNROLL_W_UNTILED 0
#endif
#ifndef WAVE_FWD_PREFETCH
#define WAVE_FWD_PREFETCH 1   // planes of loads in flight in the plain forward single-step sweep
#endif
constexpr int kMaxUnrollW = WAVE_MAX_UNROLL_W;   // tiled: unroll the z loop by the window for 2R+1 <= this
constexpr int kMaxUnrollWUntiled = WAVE_MAX_UNROLL_W_UNTILED;   // untiled: likewise (0: always shift)

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// The b32 builtins move raw 32-bit words: reinterpret, never convert.
// voff: per-lane column offset; soff: wave-uniform plane offset.
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// A workgroup's segment of planes [lo, hi) of every array.
struct Seg {
  int lo, hi;
  uint32_t pb;    // bytes per plane
  uint32_t len;   // (hi - lo) * pb
  int64_t base;   // lo * plane elements
  // scalar offset of plane z: in range only for lo <= z < hi (and a <= z < b)
  __device__ __forceinline__ uint32_t off(int z) const {
    return (z >= lo && z < hi) ? (uint32_t)(z - lo) * pb : len;
  }
  __device__ __forceinline__ uint32_t off(int z, int a, int b) const {
    return (z >= a && z < b && z >= lo && z < hi) ? (uint32_t)(z - lo) * pb : len;
  }
  __device__ __forceinline__ rsrc_t rsrc(const float* p) const { return make_rsrc(p + base, len); }
};

// The point tables are read-only for the whole launch and indexed by uniform
// values, so they are read through the constant address space: scalar loads
// that do not join the vector-memory counter the plane prefetches wait on.
template <typename V>
__device__ __forceinline__ V cload(const V* p, int64_t i) {
  return ((const __attribute__((address_space(4))) V*)p)[i];
}

// A copy of a pointer the optimiser cannot see through, so that loads behind
// it stay on the rare path instead of being hoisted into live registers.
template <typename P>
__device__ __forceinline__ P opaque(P p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Points of plane z (CSR over the streamed axis).
__device__ __forceinline__ void plane_points(const PointSet& ps, int z, int& p0, int& p1) {
  p0 = cload(ps.zptr, z);
  p1 = cload(ps.zptr, z + 1);
}

// Points of plane z in the 64-column window [xw, xw + 64) of row y (all
// arguments wave-uniform): [a, b).  Within a plane the points are sorted by
// (y, x), so two binary searches (scalar loads) find the window and at most
// 64 points remain to compare per lane, however many points the plane holds.
// The window is clipped to the row, so that it never reaches into row y - 1
// or y + 1 (whose points would otherwise match a lane's x).
struct PtRange { int a, b; };
__device__ __forceinline__ PtRange window_points(const PointSet& ps, int z, int y, int xw, int n2) {
  int p0, p1;
  plane_points(ps, z, p0, p1);
  const int xlo = min(max(xw, 0), n2), xhi = max(min(max(xw + 64, 0), n2), xlo);
  const int64_t klo = (int64_t)y * n2 + xlo, khi = (int64_t)y * n2 + xhi;
  auto key = [&](int p) { return (int64_t)cload(ps.y, p) * n2 + cload(ps.x, p); };
  int lo = p0, hi = p1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (key(mid) < klo) lo = mid + 1; else hi = mid;
  }
  const int a = lo;
  hi = p1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (key(mid) < khi) lo = mid + 1; else hi = mid;
  }
  return PtRange{a, lo};
}

// Forcing value at (z, y, x) for `step` (0 where the point is not forced);
// x lies in the window [xw, xw + 64).
__device__ __forceinline__ float forcing_at(const SweepArgs& A, int z, int y, int xw, int x, int step) {
  const SweepAux* X = opaque(A.aux);
  const PointSet ps{cload(&X->inj.zptr, 0), cload(&X->inj.y, 0), cload(&X->inj.x, 0), cload(&X->inj.npts, 0)};
  const float* tab = cload(&X->inj_table, 0);
  const PtRange w = window_points(ps, z, y, xw, A.n2);
  float f = 0.0f;
  for (int p = w.a; p < w.b; ++p) {
    const float v = cload(tab, (int64_t)step * ps.npts + p);
    if (cload(ps.x, p) == x) f = v;
  }
  return f;
}

// Record v at (z, y, x) for `step` if that point is sampled; x lies in the
// window [xw, xw + 64).
__device__ __forceinline__ void sample_at(const SweepArgs& A, int z, int y, int xw, int x, int step, float v) {
  const SweepAux* X = opaque(A.aux);
  const PointSet ps{cload(&X->smp.zptr, 0), cload(&X->smp.y, 0), cload(&X->smp.x, 0), cload(&X->smp.npts, 0)};
  float* out = cload(&X->smp_out, 0);
  const PtRange w = window_points(ps, z, y, xw, A.n2);
  for (int p = w.a; p < w.b; ++p)
    if (cload(ps.x, p) == x) out[(int64_t)step * ps.npts + p] = v;
}

// The forcing values / samples of a thread's RY rows.  Row r lies at
// y = ybase + r, window xw = xbase (3D), or y = ybase, xw = xbase + 64 r (2D).
// The rows are visited in a loop that is not unrolled, each result reaching
// its row's register through uniform selects: one lookup is live at a time
// and its code exists once, whatever RY, T and the variant.
template <int RY, bool HY>
__device__ __forceinline__ void forcing_rows(const SweepArgs& A, int z, int ybase, int xbase, int lane, int step,
                                             float (&f)[RY]) {
#pragma unroll
  for (int i = 0; i < RY; ++i) f[i] = 0.0f;
#pragma unroll 1
  for (int r = 0; r < RY; ++r) {
    const int y = HY ? ybase + r : ybase, xw = HY ? xbase : xbase + 64 * r;
    const float v = forcing_at(A, z, y, xw, xw + lane, step);
#pragma unroll
    for (int i = 0; i < RY; ++i) f[i] = (i == r) ? v : f[i];
  }
}

template <int RY, bool HY, typename Keep>
__device__ __forceinline__ void sample_rows(const SweepArgs& A, int z, int ybase, int xbase, int lane, int step,
                                            const float (&v)[RY], Keep keep) {
#pragma unroll 1
  for (int r = 0; r < RY; ++r) {
    float vr = 0.0f;
    bool kr = false;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      vr = (i == r) ? v[i] : vr;
      kr = (i == r) ? keep(i) : kr;
    }
    if (kr) {
      const int y = HY ? ybase + r : ybase, xw = HY ? xbase : xbase + 64 * r;
      sample_at(A, z, y, xw, xw + lane, step, vr);
    }
  }
}

// Whole-wave "any lane" test (uniform result).
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }

template <typename F, int... Is>
__device__ __forceinline__ void unroll_rot(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}

// --------------------------------------------------------------- untiled sweep

// Thread slot i of (wave w, lane l):  3D: (ly, lx) = (w*RY + i, l);
// 2D: (0, (w*RY + i)*64 + l).
template <int R, int DIM, int MODE, int NW, int RY, bool BATCH>
__global__ __launch_bounds__(64 * NW) void k_untiled(typename LaunchArgs<BATCH>::type P) {
  int blk;
  const SweepArgs& A = shot_args(P, blk);
  constexpr bool HY = (DIM == 3);
  constexpr bool AB = (MODE == MODE_AB2);    // two-level diffusion: window of w = 3/2 u^n - 1/2 u^{n-1}
  constexpr bool DF = (MODE == MODE_DIFF) || AB;   // diffusion: no b, no damping, no points
  constexpr int W = 2 * R + 1;
  constexpr bool ROT = W <= kMaxUnrollWUntiled;
  constexpr int TY = HY ? NW * RY : 1;
  constexpr int TX = HY ? 64 : 64 * NW * RY;
  constexpr int RYH = HY ? R : 0;
  constexpr int LDW = TX + 2 * R;
  constexpr int LDH = TY + 2 * RYH;
  constexpr int PL = LDW * LDH;
  constexpr int NH = (HY ? 2 * R * TX : 0) + 2 * R * TY;
  constexpr int NT = 64 * NW;
  constexpr int HPT = (NH + NT - 1) / NT;
  constexpr int RSTEP = HY ? LDW : 64;   // LDS distance between a thread's rows
  constexpr int PLB = PL + 1;            // one plane plus a spare slot for unused halo writes
  __shared__ float lds[2 * PLB];

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  int tile, chunk;
  work_item(A, blk, tile, chunk);
  const int ty = tile / A.tiles_x, tx = tile % A.tiles_x;
  const int gy0 = ty * TY, gx0 = tx * TX;
  const int za = A.zlo + chunk * A.zchunk;
  const int zb = min(za + A.zchunk, A.zhi);
  const int n0 = A.n0;
  Seg sg;
  sg.lo = max(0, za - R);
  sg.hi = min(n0, zb + R);
  sg.pb = (uint32_t)A.s0 * 4u;
  sg.len = (uint32_t)(sg.hi - sg.lo) * sg.pb;
  sg.base = (int64_t)sg.lo * A.s0;
  const rsrc_t rc = sg.rsrc(A.cur), rp = sg.rsrc(A.prev), rb = sg.rsrc(A.b), ro = sg.rsrc(A.outA);

  // 3D: the rows of a thread are wave-uniform, so their damping terms are
  // scalars; the axis-2 term is per lane.  2D: slots differ along axis 2.
  uint32_t col[RY];
  float stx[HY ? 1 : RY];
  const int lid0 = (HY ? wv * RY + RYH : 0) * LDW + (HY ? lane : wv * RY * 64 + lane) + R;
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    const int ly = HY ? wv * RY + i : 0;
    const int lx = HY ? lane : (wv * RY + i) * 64 + lane;
    const int gy = gy0 + ly, gx = gx0 + lx;
    const bool in = gy < A.n1 && gx < A.n2;
    col[i] = in ? (uint32_t)(gy * (int)A.s1 + gx) * 4u : kOOB;
    if (!HY || i == 0) stx[HY ? 0 : i] = A.has_damp ? damp_term(gx, A.n2, A.nbl, A.st_coef) : 0.0f;
  }
  uint32_t hcol[HPT];
  int hlid[HPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int e = threadIdx.x + h * NT;
    int y = 0, x = 0;
    const bool valid = e < NH;
    if (valid) {
      if (HY && e < 2 * R * TX) {
        const int r = e / TX;
        x = e % TX;
        y = r < R ? r - R : TY + (r - R);
      } else {
        const int e2 = e - (HY ? 2 * R * TX : 0);
        y = e2 / (2 * R);
        const int c = e2 % (2 * R);
        x = c < R ? c - R : TX + (c - R);
      }
    }
    const int Y = gy0 + y, X = gx0 + x;
    const bool ok = valid && Y >= 0 && Y < A.n1 && X >= 0 && X < A.n2;
    hcol[h] = ok ? (uint32_t)(Y * (int)A.s1 + X) * 4u : kOOB;
    hlid[h] = valid ? (y + RYH) * LDW + x + R : PL;   // unused slots write the spare slot
  }

  // Window ring: logical plane j (0 oldest .. 2R newest) at rotation r lives
  // in slot (j + r) % W.
  float zw[RY][W];
  // NP sets of prefetch registers: plane z's loads are issued NP planes
  // ahead, into the set that iteration z consumes (no register moves).
  // Two planes in flight pay where a point reads few inputs for its
  // registers or many streams: diffusion +3-4 %, the recompute storing the
  // history and the adjoint with imaging -5 % time; the plain wave forward
  // measured equal and keeps one.
  constexpr int NP = (MODE == MODE_FWD) ? WAVE_FWD_PREFETCH : 2;
  static_assert(NP == 1 || !ROT, "a two-plane prefetch needs the shifted window");
  // AB: pc/pb hold u^n/u^{n-1} of the plane entering the window, pp u^n of
  // the plane being updated, ph/ph2 u^n/u^{n-1} of its halo.
  float pc[NP][RY], pp[NP][RY], pb[NP][RY], ph[NP][HPT], ph2[AB ? NP : 1][AB ? HPT : 1];
  // history / gradient: one time level per launch; the adjoint's u and g of
  // a plane are fetched with its other loads, NP planes ahead of their use
  const int step = A.step0;
  const int64_t N = (int64_t)n0 * A.s0;
  constexpr bool HIST = (MODE == MODE_HIST || MODE == MODE_ADJ);
  constexpr bool ADJ = (MODE == MODE_ADJ);
  const rsrc_t rh = HIST ? sg.rsrc(A.hist + (int64_t)(step + 1 - A.hist_base) * N) : ro;
  const rsrc_t rg = ADJ ? sg.rsrc(A.grad) : ro;
  float pu[ADJ ? NP : 1][ADJ ? RY : 1], pg[ADJ ? NP : 1][ADJ ? RY : 1];
  {
#pragma unroll
    for (int j = 1; j <= 2 * R; ++j) {   // planes za-R .. za+R-1: logical 0..2R-1 at rotation 1
      const uint32_t so = sg.off(za - R - 1 + j);
#pragma unroll
      for (int i = 0; i < RY; ++i)
        zw[i][j % W] = AB ? ab2_input(bload(rc, col[i], so), bload(rp, col[i], so)) : bload(rc, col[i], so);
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const uint32_t sc = sg.off(za + q + R), s1 = sg.off(za + q);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        pc[q][i] = bload(rc, col[i], sc);
        pp[q][i] = AB ? bload(rc, col[i], s1) : (DF ? 0.0f : bload(rp, col[i], s1));
        pb[q][i] = AB ? bload(rp, col[i], sc) : (DF ? 0.0f : bload(rb, col[i], s1));
      }
#pragma unroll
      for (int h = 0; h < HPT; ++h) {
        ph[q][h] = bload(rc, hcol[h], s1);
        if constexpr (AB) ph2[q][h] = bload(rp, hcol[h], s1);
      }
      if constexpr (ADJ) {
        const uint32_t sw = sg.off(za + q, za, zb);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          pu[q][i] = bload(rh, col[i], sw);
          pg[q][i] = bload(rg, col[i], sw);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RY; ++i) zw[i][0] = 0.0f;
  }

  const int nit = zb - za;
  // One plane; `rot` is the rotation after this iteration's push, `q` the
  // prefetch set holding this plane's loads.
  auto body = [&](int z, auto rotc, auto qc) {
    constexpr int rot = decltype(rotc)::value;
    constexpr int q = decltype(qc)::value;
    __builtin_amdgcn_sched_barrier(0);   // keep unrolled copies from overlapping (register pressure)
    float up[RY], bb[RY], hv[HPT], uu[ADJ ? RY : 1], gg[ADJ ? RY : 1];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      zw[i][(2 * R + rot) % W] = AB ? ab2_input(pc[q][i], pb[q][i]) : pc[q][i];
      up[i] = pp[q][i];
      bb[i] = pb[q][i];
      if constexpr (ADJ) {
        uu[i] = pu[q][i];
        gg[i] = pg[q][i];
      }
    }
#pragma unroll
    for (int h = 0; h < HPT; ++h) hv[h] = AB ? ab2_input(ph[q][h], ph2[AB ? q : 0][AB ? h : 0]) : ph[q][h];
    {  // issue the loads of plane z + NP before touching this plane's data
      const uint32_t sc = sg.off(z + NP + R), s1 = sg.off(z + NP);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        pc[q][i] = bload(rc, col[i], sc);
        if constexpr (AB) {
          pp[q][i] = bload(rc, col[i], s1);
          pb[q][i] = bload(rp, col[i], sc);
        } else if constexpr (!DF) {
          pp[q][i] = bload(rp, col[i], s1);
          pb[q][i] = bload(rb, col[i], s1);
        }
      }
#pragma unroll
      for (int h = 0; h < HPT; ++h) {
        ph[q][h] = bload(rc, hcol[h], s1);
        if constexpr (AB) ph2[q][h] = bload(rp, hcol[h], s1);
      }
      if constexpr (ADJ) {
        const uint32_t sw = sg.off(z + NP, za, zb);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          pu[q][i] = bload(rh, col[i], sw);
          pg[q][i] = bload(rg, col[i], sw);
        }
      }
    }
    float* buf = lds + (z & 1) * PLB;
#pragma unroll
    for (int i = 0; i < RY; ++i) buf[lid0 + i * RSTEP] = zw[i][(R + rot) % W];
#pragma unroll
    for (int h = 0; h < HPT; ++h) buf[hlid[h]] = hv[h];
    __syncthreads();

    const bool zown = z < zb;
    const float stz = A.has_damp ? damp_term(z, n0, A.nbl, A.st_coef) : 0.0f;
    const bool fz = zown && z >= A.inj_zlo && z < A.inj_zhi;
    const bool sz = zown && z >= A.smp_zlo && z < A.smp_zhi;
    const uint32_t so = sg.off(z, za, zb);   // stores: owned planes only
    // Wave-uniform variants keep every row of a plane in one straight-line
    // block: damping only where some lane of the wave is inside the layer,
    // forcing/sampling only on the planes that hold such points.
    bool dmp = false;
    if (A.has_damp) {
      bool rows_damped = false;
#pragma unroll
      for (int i = 0; i < RY; ++i)
        rows_damped |= HY && damp_term(gy0 + wv * RY + i, A.n1, A.nbl, A.st_coef) != 0.0f;
      bool lane_damped = stz != 0.0f || rows_damped;
#pragma unroll
      for (int i = 0; i < (HY ? 1 : RY); ++i) lane_damped |= stx[i] != 0.0f;
      dmp = wave_any(lane_damped);
    }
    auto rows = [&](auto dm, auto ev) {
      constexpr bool DM = decltype(dm)::value, EV = decltype(ev)::value;
      float v[RY], st[RY], fr[RY];
      const int ybase = gy0 + (HY ? wv * RY : 0), xbase = gx0 + (HY ? 0 : wv * RY * 64);
      if (EV && fz) forcing_rows<RY, HY>(A, z, ybase, xbase, lane, step, fr);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
        const float* row = buf + lid0 + i * RSTEP;
#pragma unroll
        for (int j = 1; j <= R; ++j) {
          zm[j - 1] = zw[i][(R - j + rot) % W];
          zp[j - 1] = zw[i][(R + j + rot) % W];
          xm[j - 1] = row[-j];
          xp[j - 1] = row[j];
          if (HY) {   // rows held by this thread come from registers
            ym[j - 1] = (i - j >= 0) ? zw[(i - j >= 0) ? i - j : 0][(R + rot) % W] : row[-j * LDW];
            yp[j - 1] = (i + j < RY) ? zw[(i + j < RY) ? i + j : 0][(R + rot) % W] : row[j * LDW];
          }
        }
        const float f = (EV && fz) ? fr[i] : 0.0f;
        st[i] = 0.0f;
        if (DM) {
          const float sty = HY ? damp_term(gy0 + wv * RY + i, A.n1, A.nbl, A.st_coef) : 0.0f;
          st[i] = (stz + sty) + stx[HY ? 0 : i];
        }
        if constexpr (AB) {
          v[i] = ab2_next<R, HY>(A.C, zw[i][(R + rot) % W], zm, zp, ym, yp, xm, xp, up[i]);
        } else if constexpr (DF) {
          v[i] = diff_next<R, HY>(A.C, zw[i][(R + rot) % W], zm, zp, ym, yp, xm, xp);
        } else {
          v[i] = wave_num<R, HY>(A.C, zw[i][(R + rot) % W], zm, zp, ym, yp, xm, xp, up[i], bb[i], st[i], f, DM,
                                 EV && fz);
          if (DM) v[i] = wave_damp(v[i], st[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        const uint32_t o = col[i];
        bstore(ro, o, so, v[i]);
        if (MODE == MODE_HIST) {
          bstore(rh, o, so, v[i]);
        } else if constexpr (ADJ) {
          bstore(rg, o, so, image_step(gg[i], uu[i], st[i], v[i], zw[i][(R + rot) % W], up[i]));
        }
      }
      if (EV && sz) sample_rows<RY, HY>(A, z, ybase, xbase, lane, step, v, [&](int i) { return col[i] != kOOB; });
    };
    using TT = std::true_type;
    using FF = std::false_type;
    if constexpr (DF) {
      rows(FF{}, FF{});
    } else if (fz || sz) {
      if (dmp) rows(TT{}, TT{}); else rows(FF{}, TT{});
    } else {
      if (dmp) rows(TT{}, FF{}); else rows(FF{}, FF{});
    }
  };
  // rotate the ring by one slot so that the fixed rotation 1 stays valid
  auto shift = [&]() {
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const float t0 = zw[i][0];
#pragma unroll
      for (int j = 0; j < W - 1; ++j) zw[i][j] = zw[i][j + 1];
      zw[i][W - 1] = t0;
    }
  };
  using Q0 = std::integral_constant<int, 0>;
  using Q1 = std::integral_constant<int, NP - 1>;
  // iterations past the segment end store nothing (empty plane descriptors)
  if constexpr (ROT) {
    for (int it = 0; it < nit; it += W)
      unroll_rot([&](auto r) { body(za + it + decltype(r)::value, std::integral_constant<int, decltype(r)::value + 1>{}, Q0{}); },
                 std::make_integer_sequence<int, W>{});
  } else if constexpr (NP == 1) {
    for (int it = 0; it < nit; ++it) {
      body(za + it, std::integral_constant<int, 1>{}, Q0{});
      shift();
    }
  } else {
    for (int it = 0; it < nit; it += 2) {
      body(za + it, std::integral_constant<int, 1>{}, Q0{});
      shift();
      body(za + it + 1, std::integral_constant<int, 1>{}, Q1{});
      shift();
    }
  }
}

// --------------------------------------------------------------- time-tiled sweep

// 3D: the NW waves form NW/NWX rows of NWX waves; wave (wy, wx) owns rows
// wy*RY .. wy*RY+RY-1 and columns wx*64 .. wx*64+63 of the extended tile.
template <int R, int T, int DIM, int MODE, int NW, int RY, int NWX, bool BATCH>
__global__ __launch_bounds__(64 * NW) void k_tiled(typename LaunchArgs<BATCH>::type P) {
  int blk;
  const SweepArgs& A = shot_args(P, blk);
  constexpr bool HY = (DIM == 3);
  constexpr bool DF = (MODE == MODE_DIFF);   // diffusion: one input level, no b
  constexpr int W = 2 * R + 1;
  constexpr bool ROT = W <= kMaxUnrollW;
  static_assert(HY || NWX == 1, "2D tiles are one row of waves");
  static_assert(NW % NWX == 0, "waves must fill whole rows");
  constexpr int NWY = NW / NWX;
  constexpr int EY = HY ? NWY * RY : 1;
  constexpr int EX = HY ? 64 * NWX : 64 * NW * RY;
  constexpr int RYH = HY ? R : 0;
  constexpr int LDW = EX + 2 * R;
  constexpr int PL = tiled_plane_floats(R, EY, EX, HY);
  constexpr int NBUF = tiled_nbuf(R, T, EY, EX, HY);
  constexpr int RSTEP = HY ? LDW : 64;
  extern __shared__ float lds[];   // NBUF * T planes

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int wy = wv / NWX, wx = wv % NWX;                              // 3D wave row / column
  const int H = A.skew * T;
  const int HYH = HY ? H : 0;
  const int CY = HY ? EY - 2 * H : 1;
  const int CX = EX - 2 * H;
  int tile, chunk;
  work_item(A, blk, tile, chunk);
  const int ty = tile / A.tiles_x, tx = tile % A.tiles_x;
  const int gy0 = ty * CY - HYH, gx0 = tx * CX - H;
  const int za = A.zlo + chunk * A.zchunk;
  const int zb = min(za + A.zchunk, A.zhi);
  const int n0 = A.n0;
  Seg sg;
  sg.lo = max(0, za - (T + 1) * R);
  sg.hi = min(n0, zb + (T + 1) * R);
  sg.pb = (uint32_t)A.s0 * 4u;
  sg.len = (uint32_t)(sg.hi - sg.lo) * sg.pb;
  sg.base = (int64_t)sg.lo * A.s0;
  const rsrc_t rc = sg.rsrc(A.cur), rp = sg.rsrc(A.prev), rb = sg.rsrc(A.b), ra = sg.rsrc(A.outA);
  const rsrc_t rB = A.outB ? sg.rsrc(A.outB) : make_rsrc(A.outA, 0u);

  for (int e = threadIdx.x; e < NBUF * T * PL; e += 64 * NW) lds[e] = 0.0f;

  // Column offsets (kOOB outside the grid).  3D: a thread's rows are
  // wave-uniform, so row validity, the core test along axis 1 and the damping
  // terms along axes 0/1 are scalars; along axis 2 they are per lane.
  uint32_t col[RY];
  bool xcore[HY ? 1 : RY];
  float stx[HY ? 1 : RY];
  const int lid0 = (HY ? wy * RY + RYH : 0) * LDW + (HY ? wx * 64 + lane : wv * RY * 64 + lane) + R;
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    const int ly = HY ? wy * RY + i : 0;
    const int lx = HY ? wx * 64 + lane : (wv * RY + i) * 64 + lane;
    const int gy = gy0 + ly, gx = gx0 + lx;
    const bool yin = gy >= 0 && gy < A.n1, xin = gx >= 0 && gx < A.n2;
    col[i] = (yin && xin) ? (uint32_t)(gy * (int)A.s1 + gx) * 4u : kOOB;
    if (!HY || i == 0) {
      xcore[HY ? 0 : i] = lx >= H && lx < H + CX;
      stx[HY ? 0 : i] = A.has_damp ? damp_term(gx, A.n2, A.nbl, A.st_coef) : 0.0f;
    }
  }
  const int wrow0 = HY ? wy * RY : 0;   // first row of this wave (3D)

  float win[T][RY][W];
#pragma unroll
  for (int k = 0; k < T; ++k)
#pragma unroll
    for (int i = 0; i < RY; ++i)
#pragma unroll
      for (int j = 0; j < W; ++j) win[k][i][j] = 0.0f;

  const int zs = za - T * R;   // first plane loaded
  const int nit = zb - za + 2 * T * R;
  const int64_t N = (int64_t)n0 * A.s0;
  // Adjoint imaging over the window: stage k's gradient term for a core
  // point is added to the running value that stage k-1 produced R
  // iterations earlier (the point's plane reaches stage k R planes later),
  // so grad is read once (by stage 1) and written once (by stage T) per
  // window, the terms summed in the per-step order of the single-step
  // sweep.  ocol: core columns (kOOB elsewhere); gq[k-1]: stage k's running
  // values of the last R iterations, oldest first.  An iteration issues its
  // history and gradient loads at its start and uses them after its
  // updates (a prefetch one iteration ahead measured slower: its second set
  // of registers spills at the deeper tiles).
  constexpr bool ADJ = (MODE == MODE_ADJ);
  constexpr int TQ = (ADJ && T > 1) ? T - 1 : 1;
  constexpr int RQ = (ADJ && T > 1) ? R : 1;
  uint32_t ocol[ADJ ? RY : 1];
  float gq[TQ][RQ][ADJ ? RY : 1];
  const rsrc_t rg = ADJ ? sg.rsrc(A.grad) : ra;
  auto hist_rsrc = [&](int k) { return sg.rsrc(A.hist + (int64_t)(stage_step(A, k) + 1 - A.hist_base) * N); };
  if constexpr (ADJ) {
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const int ly = HY ? wrow0 + i : 0;
      const bool rcore = !HY || (ly >= HYH && ly < HYH + CY);
      ocol[i] = (rcore && xcore[HY ? 0 : i]) ? col[i] : kOOB;
    }
#pragma unroll
    for (int k = 0; k < TQ; ++k)
#pragma unroll
      for (int j = 0; j < RQ; ++j)
#pragma unroll
        for (int i = 0; i < RY; ++i) gq[k][j][i] = 0.0f;
  }
  // b = dt^2/m: stage k + 1 needs at each iteration the value that stage k
  // used R iterations earlier (the same plane), so b is loaded once, for
  // stage 1, and carried to the later stages through R-entry register FIFOs
  // (bq[k-1]: stage k's values of the last R iterations, oldest first)
  // instead of T loads per plane.  Up to radius 2: there the FIFOs cost no
  // more registers than the loads they replace (592^3, order 2, T = 3 on
  // 64 x 64: 507.8 against 431.0 Gpts/s; order 4, T = 2 on 32 x 128: 419.2
  // against 375.9; 16384^2 2D orders 2 / 4: 935.5 / 717.2 against 801.8 /
  // 655.8).  Their (T-1) R entries per row outgrow the saving beyond that
  // (2D order 8, T = 3: 367.6 against 481.7).
  constexpr bool CB = !DF && T >= 2 && R <= 2;
  constexpr int NB = CB ? 1 : T;             // b planes loaded per iteration
  constexpr int TB = CB ? T - 1 : 1, RB = CB ? R : 1;
  float bq[TB][RB][RY];
  float pc[RY], pp[RY], pb[NB][RY];   // next iteration's loads
  {
    const uint32_t sc = sg.off(zs), sp = sg.off(zs - R);
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      pc[i] = bload(rc, col[i], sc);
      pp[i] = DF ? 0.0f : bload(rp, col[i], sp);
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const uint32_t sb = sg.off(zs - (k + 1) * R);
#pragma unroll
      for (int i = 0; i < RY; ++i) pb[k][i] = DF ? 0.0f : bload(rb, col[i], sb);
    }
    if constexpr (CB) {   // the FIFOs as if the pipeline had run before zs
#pragma unroll
      for (int k = 1; k < T; ++k)
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t sb = sg.off(zs - R + j - k * R);
#pragma unroll
          for (int i = 0; i < RY; ++i) bq[k - 1][j][i] = bload(rb, col[i], sb);
        }
    }
  }
  __syncthreads();

  // One iteration; `rot` is the rotation after this iteration's pushes.
  auto body = [&](int z0, auto rotc) {
    constexpr int rot = decltype(rotc)::value;
    __builtin_amdgcn_sched_barrier(0);   // keep unrolled copies from overlapping (register pressure)
    float cin[RY], pin[RY], bin[T][RY];
    float uin[ADJ ? T : 1][ADJ ? RY : 1], gin[ADJ ? T : 1][ADJ ? RY : 1];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      cin[i] = pc[i];
      pin[i] = pp[i];
      if constexpr (CB) {
        bin[0][i] = pb[0][i];
#pragma unroll
        for (int k = 1; k < T; ++k) bin[k][i] = bq[(k >= 1 && k < T) ? k - 1 : 0][0][i];
#pragma unroll
        for (int k = 1; k < T; ++k) {
#pragma unroll
          for (int j = 0; j + 1 < RB; ++j) bq[k - 1][j][i] = bq[k - 1][j + 1][i];
          bq[k - 1][RB - 1][i] = bin[k - 1][i];
        }
      } else {
#pragma unroll
        for (int k = 0; k < T; ++k) bin[k][i] = pb[(k < NB) ? k : 0][i];
      }
    }
    if constexpr (ADJ) {
      // stage 1 starts from grad; stage k > 1 from the oldest entry of its
      // FIFO, whose entries then age by one
#pragma unroll
      for (int k = 1; k <= T; ++k) {   // this iteration's history planes, used after the updates
        const rsrc_t rh = hist_rsrc(k);
        const uint32_t sw = sg.off(z0 - k * R, za, zb);
#pragma unroll
        for (int i = 0; i < RY; ++i) uin[k - 1][i] = bload(rh, ocol[i], sw);
      }
      const uint32_t sw = sg.off(z0 - R, za, zb);
#pragma unroll
      for (int i = 0; i < RY; ++i) gin[0][i] = bload(rg, ocol[i], sw);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
#pragma unroll
        for (int k = 1; k < T; ++k) {
          gin[k][i] = gq[k - 1][0][i];
#pragma unroll
          for (int j = 0; j + 1 < RQ; ++j) gq[k - 1][j][i] = gq[k - 1][j + 1][i];
        }
      }
    }
    {  // next iteration's loads first
      const int zn = z0 + 1;
      const uint32_t sc = sg.off(zn), sp = sg.off(zn - R);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        pc[i] = bload(rc, col[i], sc);
        if constexpr (!DF) pp[i] = bload(rp, col[i], sp);
      }
      if constexpr (!DF) {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const uint32_t sb = sg.off(zn - (k + 1) * R);
#pragma unroll
          for (int i = 0; i < RY; ++i) pb[k][i] = bload(rb, col[i], sb);
        }
      }
    }
    // Stage the input plane of every stage in LDS: for stage k+1 that is level
    // n+k at plane z0-(k+1)R, logical index R+1 of window k before this
    // iteration's pushes (rotation rot-1), i.e. slot (R + rot) % W.
    float* buf = lds + ((NBUF == 2) ? (z0 & 1) : 0) * (T * PL);
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
      for (int i = 0; i < RY; ++i) buf[k * PL + lid0 + i * RSTEP] = win[k][i][(R + rot) % W];
    __syncthreads();
    // push the freshly loaded plane z0 of level n into window 0
#pragma unroll
    for (int i = 0; i < RY; ++i) win[0][i][(2 * R + rot) % W] = cin[i];
    // Wave-uniform properties of every stage's plane, then one variant
    // (damping x forcing/sampling) for the whole iteration: all T stages form
    // one straight-line block, so the LDS reads of a stage can be issued
    // while the previous stage computes.  The damped form is exact where
    // st == 0, so it serves every stage once one stage needs it.
    bool any_dmp = false, any_ev = false;
#pragma unroll
    for (int k = 1; k <= T; ++k) {
      const int zk = z0 - k * R;
      const bool zown = zk >= za && zk < zb;
      any_ev |= (zk >= A.inj_zlo && zk < A.inj_zhi) || (zown && zk >= A.smp_zlo && zk < A.smp_zhi);
      if (A.has_damp) {
        const float stz = damp_term(zk, n0, A.nbl, A.st_coef);
        bool rows_damped = false;
#pragma unroll
        for (int i = 0; i < RY; ++i)
          rows_damped |= HY && damp_term(gy0 + wrow0 + i, A.n1, A.nbl, A.st_coef) != 0.0f;
        bool lane_damped = stz != 0.0f || rows_damped;
#pragma unroll
        for (int i = 0; i < (HY ? 1 : RY); ++i) lane_damped |= stx[i] != 0.0f;
        any_dmp |= wave_any(lane_damped);
      }
    }
    auto stages = [&](auto dm, auto ev) {
      constexpr bool DM = decltype(dm)::value, EV = decltype(ev)::value;
#pragma unroll
      for (int k = 1; k <= T; ++k) {
        const int zk = z0 - k * R;
        const bool zown = zk >= za && zk < zb;
        const int step = stage_step(A, k);
        const float* pl = buf + (k - 1) * PL;
        const float stz = (DM && A.has_damp) ? damp_term(zk, n0, A.nbl, A.st_coef) : 0.0f;
        const bool fz = EV && zk >= A.inj_zlo && zk < A.inj_zhi;
        const bool sz = EV && zown && zk >= A.smp_zlo && zk < A.smp_zhi;
        const uint32_t so = sg.off(zk, za, zb);   // stores: owned planes only
        const rsrc_t rh = (MODE == MODE_HIST) ? sg.rsrc(A.hist + (int64_t)(step + 1 - A.hist_base) * N) : ra;
        float v[RY], st[RY], upv[RY], fr[RY];
        const int ybase = gy0 + (HY ? wrow0 : 0), xbase = gx0 + (HY ? wx * 64 : wv * RY * 64);
        if (EV && fz) forcing_rows<RY, HY>(A, zk, ybase, xbase, lane, step, fr);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
          const float* row = pl + lid0 + i * RSTEP;
#pragma unroll
          for (int j = 1; j <= R; ++j) {
            zm[j - 1] = win[k - 1][i][(R - j + rot) % W];
            zp[j - 1] = win[k - 1][i][(R + j + rot) % W];
            xm[j - 1] = row[-j];
            xp[j - 1] = row[j];
            if (HY) {   // rows held by this thread come from registers
              ym[j - 1] = (i - j >= 0) ? win[k - 1][(i - j >= 0) ? i - j : 0][(R + rot) % W] : row[-j * LDW];
              yp[j - 1] = (i + j < RY) ? win[k - 1][(i + j < RY) ? i + j : 0][(R + rot) % W] : row[j * LDW];
            }
          }
          upv[i] = (k == 1) ? pin[i] : win[(k >= 2) ? k - 2 : 0][i][rot % W];
          const float f = (EV && fz) ? fr[i] : 0.0f;
          st[i] = 0.0f;
          if (DM) {
            const float sty = HY ? damp_term(gy0 + wrow0 + i, A.n1, A.nbl, A.st_coef) : 0.0f;
            st[i] = (stz + sty) + stx[HY ? 0 : i];
          }
          if constexpr (DF) {
            // Outside the grid the wave update is exactly 0 (b reads 0 there);
            // diffusion's u + lap is not, so zero it: the next stage must see
            // the zero ghosts the untiled sweep reads.
            const float d = diff_next<R, HY>(A.C, win[k - 1][i][(R + rot) % W], zm, zp, ym, yp, xm, xp);
            v[i] = (col[i] != kOOB && zk >= 0 && zk < n0) ? d : 0.0f;
          } else {
            v[i] = wave_num<R, HY>(A.C, win[k - 1][i][(R + rot) % W], zm, zp, ym, yp, xm, xp, upv[i],
                                   bin[k - 1][i], st[i], f, DM, EV && fz);
            if (DM) v[i] = wave_damp(v[i], st[i]);
          }
        }
        // in range only for core points of owned planes
        auto outoff = [&](int i) {
          const int ly = HY ? wrow0 + i : 0;
          const bool rcore = !HY || (ly >= HYH && ly < HYH + CY);
          return (rcore && xcore[HY ? 0 : i]) ? col[i] : kOOB;
        };
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          const uint32_t o = outoff(i);
          if (MODE == MODE_HIST) {
            bstore(rh, o, so, v[i]);
          } else if constexpr (ADJ) {
            const float g = image_step(gin[k - 1][i], uin[k - 1][i], st[i], v[i], win[k - 1][i][(R + rot) % W],
                                       upv[i]);
            if (k == T) bstore(rg, o, so, g);
            else gq[(k >= 1 && k < T) ? k - 1 : 0][RQ - 1][i] = g;
          }
          if (k == T) {
            bstore(ra, o, so, v[i]);
            if constexpr (!DF) bstore(rB, o, so, win[k - 1][i][(R + rot) % W]);
          }
        }
        if (EV && sz) sample_rows<RY, HY>(A, zk, ybase, xbase, lane, step, v, [&](int i) { return outoff(i) != kOOB; });
        if (k < T) {
#pragma unroll
          for (int i = 0; i < RY; ++i) win[k < T ? k : 0][i][(2 * R + rot) % W] = v[i];
        }
      }
    };
    using TT = std::true_type;
    using FF = std::false_type;
    if constexpr (DF) {
      stages(FF{}, FF{});
    } else if (any_ev) {
      if (any_dmp) stages(TT{}, TT{}); else stages(FF{}, TT{});
    } else {
      if (any_dmp) stages(TT{}, FF{}); else stages(FF{}, FF{});
    }
    if (NBUF == 1) __syncthreads();
  };
  if constexpr (ROT) {
    // iterations past the segment end store nothing (empty plane descriptors)
    for (int it = 0; it < nit; it += W)
      unroll_rot([&](auto r) { body(zs + it + decltype(r)::value, std::integral_constant<int, decltype(r)::value + 1>{}); },
                 std::make_integer_sequence<int, W>{});
  } else {
    for (int it = 0; it < nit; ++it) {
      body(zs + it, std::integral_constant<int, 1>{});
      // rotate every ring by one slot so that the fixed rotation 1 stays valid
#pragma unroll
      for (int k = 0; k < T; ++k)
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          const float t0 = win[k][i][0];
#pragma unroll
          for (int j = 0; j < W - 1; ++j) win[k][i][j] = win[k][i][j + 1];
          win[k][i][W - 1] = t0;
        }
    }
  }
}

}  // namespace wavett
