// wave_kernels.h -- sweep kernels (templates), instantiated per stencil radius
// in wave_r<R>.hip.
//
// Layout: one FP32 array per time level, row-major [n0][n1][n2] (2D: n1 == 1),
// axis 2 unit stride (the 64 lanes of a wavefront walk it, so every global
// access is a coalesced 256-byte row), axis 0 streamed through registers.
//
// k_untiled  -- one time step per launch ("spatial tiling" in the paper's
//               terms).  A workgroup owns a core tile of TY x TX columns and
//               streams one segment of axis 0 through a (2R+1)-plane register
//               window per column; the current plane plus an R-wide halo
//               loaded from global memory sits in LDS for the axis-1/axis-2
//               neighbours.  u^{n+1} overwrites u^{n-1} in place.
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
// Memory access discipline (both kernels): all global traffic goes through
// raw buffer instructions whose descriptor covers only the segment of planes
// a workgroup may touch.  Out-of-grid columns and planes use offsets beyond
// the descriptor's range, so the hardware returns 0 (the zero boundary
// values) or drops the store -- no branches and no address arithmetic in 64
// bits in the inner loop.  Every load is issued one plane ahead of its use.
#pragma once
#include "wave_device.h"

namespace wavett {

// --------------------------------------------------------------- buffer access

typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Offsets are bytes relative to a workgroup's segment base.  A segment is at
// most kSegMax bytes (host-enforced); any offset component >= kOOB makes the
// sum land outside every descriptor without wrapping 32 bits.
constexpr uint32_t kSegMax = 0x40000000u;
constexpr uint32_t kOOB = 0x40000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// The b32 builtins move raw 32-bit words: reinterpret, never convert.
__device__ __forceinline__ float bload(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}

// The point tables are read-only for the whole launch and indexed by uniform
// values, so they are read through the constant address space: scalar loads
// that do not join the vector-memory counter the plane prefetches wait on.
template <typename V>
__device__ __forceinline__ V cload(const V* p, int64_t i) {
  return ((const __attribute__((address_space(4))) V*)p)[i];
}

// Forcing value at column (y, x) among the points p0..p1 of the current plane.
__device__ __forceinline__ float forcing_in(const SweepArgs& A, int p0, int p1, int y, int x, int step) {
  float f = 0.0f;
  for (int p = p0; p < p1; ++p) {
    const float v = cload(A.inj_table, (int64_t)step * A.inj.npts + p);
    if (cload(A.inj.y, p) == y && cload(A.inj.x, p) == x) f = v;
  }
  return f;
}

__device__ __forceinline__ void sample_in(const SweepArgs& A, int p0, int p1, int y, int x, int step, float v) {
  for (int p = p0; p < p1; ++p)
    if (cload(A.smp.y, p) == y && cload(A.smp.x, p) == x) A.smp_out[(int64_t)step * A.smp.npts + p] = v;
}

// --------------------------------------------------------------- untiled sweep

// Thread slot i of (wave w, lane l):  3D: (ly, lx) = (w*RY + i, l);
// 2D: (0, (w*RY + i)*64 + l).
template <int R, int DIM, int MODE, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_untiled(SweepArgs A) {
  constexpr bool HY = (DIM == 3);
  constexpr int TY = HY ? NW * RY : 1;
  constexpr int TX = HY ? 64 : 64 * NW * RY;
  constexpr int RYH = HY ? R : 0;
  constexpr int LDW = TX + 2 * R;
  constexpr int LDH = TY + 2 * RYH;
  constexpr int PL = LDW * LDH;
  constexpr int NH = (HY ? 2 * R * TX : 0) + 2 * R * TY;
  constexpr int NT = 64 * NW;
  constexpr int HPT = (NH + NT - 1) / NT;
  __shared__ float lds[2 * PL];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ty = blockIdx.x / A.tiles_x, tx = blockIdx.x % A.tiles_x;
  const int gy0 = ty * TY, gx0 = tx * TX;
  const int za = blockIdx.y * A.zchunk;
  const int zb = min(za + A.zchunk, A.n0);
  const int zlo = max(0, za - R), zhi = min(A.n0, zb + R);
  const uint32_t PS = (uint32_t)A.s0 * 4u;
  const uint32_t seg = (uint32_t)(zhi - zlo) * PS;
  const int64_t base = (int64_t)zlo * A.s0;
  const rsrc_t rc = make_rsrc(A.cur + base, seg);
  const rsrc_t rp = make_rsrc(A.prev + base, seg);
  const rsrc_t rb = make_rsrc(A.b + base, seg);
  const rsrc_t ro = make_rsrc(A.outA + base, seg);
  auto zoff = [&](int z) -> uint32_t { return (z >= zlo && z < zhi) ? (uint32_t)(z - zlo) * PS : kOOB; };

  uint32_t col[RY];
  int lid[RY], gy[RY], gx[RY];
  float sty[RY], stx[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    const int ly = HY ? wv * RY + i : 0;
    const int lx = HY ? lane : (wv * RY + i) * 64 + lane;
    gy[i] = gy0 + ly;
    gx[i] = gx0 + lx;
    const bool in = gy[i] < A.n1 && gx[i] < A.n2;
    col[i] = in ? (uint32_t)(gy[i] * (int)A.s1 + gx[i]) * 4u : kOOB;
    lid[i] = (ly + RYH) * LDW + lx + R;
    sty[i] = (A.has_damp && HY && in) ? A.sty[gy[i]] : 0.0f;
    stx[i] = (A.has_damp && in) ? A.stx[gx[i]] : 0.0f;
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
    // unused slots write the (never read) corner of the padded plane
    hlid[h] = valid ? (y + RYH) * LDW + x + R : 0;
  }

  float zw[RY][2 * R + 1];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    zw[i][0] = 0.0f;
#pragma unroll
    for (int j = 1; j <= 2 * R; ++j) zw[i][j] = bload(rc, zoff(za - R - 1 + j) + col[i]);
  }
  // prefetch registers for the next plane
  float pc[RY], pp[RY], pb[RY], ph[HPT];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    pc[i] = bload(rc, zoff(za + R) + col[i]);
    pp[i] = bload(rp, zoff(za) + col[i]);
    pb[i] = bload(rb, zoff(za) + col[i]);
  }
#pragma unroll
  for (int h = 0; h < HPT; ++h) ph[h] = bload(rc, zoff(za) + hcol[h]);

  const int step = A.step0;
  const int64_t N = (int64_t)A.n0 * A.s0;
  for (int z = za; z < zb; ++z) {
    float up[RY], bb[RY], hv[HPT];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) zw[i][j] = zw[i][j + 1];
      zw[i][2 * R] = pc[i];
      up[i] = pp[i];
      bb[i] = pb[i];
    }
#pragma unroll
    for (int h = 0; h < HPT; ++h) hv[h] = ph[h];
    {  // issue the next plane's loads before touching this plane's data
      const uint32_t zc = zoff(z + 1 + R), z1 = zoff(z + 1);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        pc[i] = bload(rc, zc + col[i]);
        pp[i] = bload(rp, z1 + col[i]);
        pb[i] = bload(rb, z1 + col[i]);
      }
#pragma unroll
      for (int h = 0; h < HPT; ++h) ph[h] = bload(rc, z1 + hcol[h]);
    }
    float* buf = lds + (z & 1) * PL;
#pragma unroll
    for (int i = 0; i < RY; ++i) buf[lid[i]] = zw[i][R];
#pragma unroll
    for (int h = 0; h < HPT; ++h) buf[hlid[h]] = hv[h];
    __syncthreads();

    const float stz = A.has_damp ? cload(A.stz, z) : 0.0f;
    const int ip0 = A.inj.npts ? cload(A.inj.zptr, z) : 0, ip1 = A.inj.npts ? cload(A.inj.zptr, z + 1) : 0;
    const int sp0 = A.smp.npts ? cload(A.smp.zptr, z) : 0, sp1 = A.smp.npts ? cload(A.smp.zptr, z + 1) : 0;
    const uint32_t zo = zoff(z);
    rsrc_t rh = make_rsrc(A.b, 0u), rg = rh;
    if (MODE != MODE_FWD) {
      rh = make_rsrc(A.hist + (int64_t)(step + 1 - A.hist_base) * N + base, seg);
      if (MODE == MODE_ADJ) rg = make_rsrc(A.grad + base, seg);
    }
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
      const float* row = buf + lid[i];
#pragma unroll
      for (int j = 1; j <= R; ++j) {
        zm[j - 1] = zw[i][R - j];
        zp[j - 1] = zw[i][R + j];
        xm[j - 1] = row[-j];
        xp[j - 1] = row[j];
        if (HY) {
          ym[j - 1] = row[-j * LDW];
          yp[j - 1] = row[j * LDW];
        }
      }
      const float st = A.has_damp ? (stz + sty[i]) + stx[i] : 0.0f;
      const float f = (ip1 > ip0) ? forcing_in(A, ip0, ip1, gy[i], gx[i], step) : 0.0f;
      const float v = wave_point<R, HY>(A.C, zw[i][R], zm, zp, ym, yp, xm, xp, up[i], bb[i], st, f);
      const uint32_t o = zo + col[i];
      bstore(ro, o, v);
      if (sp1 > sp0 && col[i] < kOOB) sample_in(A, sp0, sp1, gy[i], gx[i], step, v);
      if (MODE == MODE_HIST) {
        bstore(rh, o, v);
      } else if (MODE == MODE_ADJ) {
        const float u = bload(rh, o);
        bstore(rg, o, image_step(bload(rg, o), u, st, v, zw[i][R], up[i]));
      }
    }
  }
}

// --------------------------------------------------------------- time-tiled sweep

template <int R, int T, int DIM, int MODE, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_tiled(SweepArgs A) {
  constexpr bool HY = (DIM == 3);
  constexpr int EY = HY ? NW * RY : 1;
  constexpr int EX = HY ? 64 : 64 * NW * RY;
  constexpr int RYH = HY ? R : 0;
  constexpr int LDW = EX + 2 * R;
  constexpr int LDH = EY + 2 * RYH;
  constexpr int PL = LDW * LDH;                                  // floats per LDS plane
  constexpr int NBUF = tiled_nbuf(R, T, EY, EX, HY);           // double-buffer when it fits
  extern __shared__ float lds[];                                 // NBUF * T planes

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int H = A.skew * T;
  const int HYH = HY ? H : 0;
  const int CY = HY ? EY - 2 * H : 1;
  const int CX = EX - 2 * H;
  const int ty = blockIdx.x / A.tiles_x, tx = blockIdx.x % A.tiles_x;
  const int gy0 = ty * CY - HYH, gx0 = tx * CX - H;
  const int za = blockIdx.y * A.zchunk;
  const int zb = min(za + A.zchunk, A.n0);
  const int zlo = max(0, za - T * R - R), zhi = min(A.n0, zb + T * R + R);
  const uint32_t PS = (uint32_t)A.s0 * 4u;
  const uint32_t seg = (uint32_t)(zhi - zlo) * PS;
  const int64_t base = (int64_t)zlo * A.s0;
  const rsrc_t rc = make_rsrc(A.cur + base, seg);
  const rsrc_t rp = make_rsrc(A.prev + base, seg);
  const rsrc_t rb = make_rsrc(A.b + base, seg);
  const rsrc_t ra = make_rsrc(A.outA + base, seg);
  const rsrc_t rB = make_rsrc(A.outB ? A.outB + base : A.outA + base, A.outB ? seg : 0u);
  auto zoff = [&](int z) -> uint32_t { return (z >= zlo && z < zhi) ? (uint32_t)(z - zlo) * PS : kOOB; };

  for (int e = threadIdx.x; e < NBUF * T * PL; e += 64 * NW) lds[e] = 0.0f;

  uint32_t col[RY], ccol[RY];   // column offset (OOB outside the grid); same, OOB outside the core
  int lid[RY], gy[RY], gx[RY];
  float sty[RY], stx[RY];
  bool inr[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    const int ly = HY ? wv * RY + i : 0;
    const int lx = HY ? lane : (wv * RY + i) * 64 + lane;
    gy[i] = gy0 + ly;
    gx[i] = gx0 + lx;
    inr[i] = gy[i] >= 0 && gy[i] < A.n1 && gx[i] >= 0 && gx[i] < A.n2;
    const bool core = inr[i] && lx >= H && lx < H + CX && (!HY || (ly >= HYH && ly < HYH + CY));
    col[i] = inr[i] ? (uint32_t)(gy[i] * (int)A.s1 + gx[i]) * 4u : kOOB;
    ccol[i] = core ? col[i] : kOOB;
    lid[i] = (ly + RYH) * LDW + lx + R;
    sty[i] = (A.has_damp && HY && inr[i]) ? A.sty[gy[i]] : 0.0f;
    stx[i] = (A.has_damp && inr[i]) ? A.stx[gx[i]] : 0.0f;
  }

  float win[T][RY][2 * R + 1];
#pragma unroll
  for (int k = 0; k < T; ++k)
#pragma unroll
    for (int i = 0; i < RY; ++i)
#pragma unroll
      for (int j = 0; j <= 2 * R; ++j) win[k][i][j] = 0.0f;

  const int zs = za - T * R;          // first plane loaded
  const int ze = zb + T * R;          // one past the last iteration
  float pc[RY], pp[RY], pb[T][RY];    // next iteration's loads
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    pc[i] = bload(rc, zoff(zs) + col[i]);
    pp[i] = bload(rp, zoff(zs - R) + col[i]);
#pragma unroll
    for (int k = 0; k < T; ++k) pb[k][i] = bload(rb, zoff(zs - (k + 1) * R) + col[i]);
  }
  __syncthreads();

  const int64_t N = (int64_t)A.n0 * A.s0;
  for (int z0 = zs; z0 < ze; ++z0) {
    float cin[RY], pin[RY], bin[T][RY];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      cin[i] = pc[i];
      pin[i] = pp[i];
#pragma unroll
      for (int k = 0; k < T; ++k) bin[k][i] = pb[k][i];
    }
    {  // next iteration's loads first
      const int zn = z0 + 1;
      const uint32_t oc = zoff(zn), op = zoff(zn - R);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        pc[i] = bload(rc, oc + col[i]);
        pp[i] = bload(rp, op + col[i]);
      }
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const uint32_t ob = zoff(zn - (k + 1) * R);
#pragma unroll
        for (int i = 0; i < RY; ++i) pb[k][i] = bload(rb, ob + col[i]);
      }
    }
    // Stage the input plane of every stage in LDS: for stage k+1 that is level
    // n+k at plane z0-(k+1)R, which sits at index R+1 of window k before this
    // iteration's pushes.
    float* buf = lds + ((NBUF == 2) ? (z0 & 1) : 0) * (T * PL);
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
      for (int i = 0; i < RY; ++i) buf[k * PL + lid[i]] = win[k][i][R + 1];
    __syncthreads();
    // push the freshly loaded plane z0 of level n into window 0
#pragma unroll
    for (int i = 0; i < RY; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) win[0][i][j] = win[0][i][j + 1];
      win[0][i][2 * R] = cin[i];
    }
#pragma unroll
    for (int k = 1; k <= T; ++k) {
      const int zk = z0 - k * R;
      const bool zin = zk >= 0 && zk < A.n0;
      const bool zown = zk >= za && zk < zb;
      const int step = stage_step(A, k);
      const float* pl = buf + (k - 1) * PL;
      const float stz = (A.has_damp && zin) ? cload(A.stz, zk) : 0.0f;
      const int ip0 = (A.inj.npts && zin) ? cload(A.inj.zptr, zk) : 0, ip1 = (A.inj.npts && zin) ? cload(A.inj.zptr, zk + 1) : 0;
      const int sp0 = (A.smp.npts && zown) ? cload(A.smp.zptr, zk) : 0, sp1 = (A.smp.npts && zown) ? cload(A.smp.zptr, zk + 1) : 0;
      const uint32_t zo = zoff(zk);
      const uint32_t zown_o = zown ? zo : kOOB;
      rsrc_t rh = make_rsrc(A.b, 0u), rg = rh;
      if (MODE != MODE_FWD) {
        rh = make_rsrc(A.hist + (int64_t)(step + 1 - A.hist_base) * N + base, seg);
        if (MODE == MODE_ADJ) rg = make_rsrc(A.grad + base, seg);
      }
      float res[RY];
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
        const float* row = pl + lid[i];
#pragma unroll
        for (int j = 1; j <= R; ++j) {
          zm[j - 1] = win[k - 1][i][R - j];
          zp[j - 1] = win[k - 1][i][R + j];
          xm[j - 1] = row[-j];
          xp[j - 1] = row[j];
          if (HY) {
            ym[j - 1] = row[-j * LDW];
            yp[j - 1] = row[j * LDW];
          }
        }
        const float up = (k == 1) ? pin[i] : win[(k >= 2) ? k - 2 : 0][i][0];
        const float st = A.has_damp ? (stz + sty[i]) + stx[i] : 0.0f;
        const float f = (ip1 > ip0) ? forcing_in(A, ip0, ip1, gy[i], gx[i], step) : 0.0f;
        float v = wave_point<R, HY>(A.C, win[k - 1][i][R], zm, zp, ym, yp, xm, xp, up, bin[k - 1][i], st, f);
        v = (inr[i] && zin) ? v : 0.0f;
        res[i] = v;
        const uint32_t o = zown_o + ccol[i];          // in range only for owned core points
        if (sp1 > sp0 && o < kOOB) sample_in(A, sp0, sp1, gy[i], gx[i], step, v);
        if (MODE == MODE_HIST) {
          bstore(rh, o, v);
        } else if (MODE == MODE_ADJ) {
          const float u = bload(rh, o);
          bstore(rg, o, image_step(bload(rg, o), u, st, v, win[k - 1][i][R], up));
        }
        if (k == T) {
          bstore(ra, o, v);
          bstore(rB, o, win[T - 1][i][R]);
        }
      }
      if (k < T) {
#pragma unroll
        for (int i = 0; i < RY; ++i) {
#pragma unroll
          for (int j = 0; j < 2 * R; ++j) win[k][i][j] = win[k][i][j + 1];
          win[k][i][2 * R] = res[i];
        }
      }
    }
    if (NBUF == 1) __syncthreads();
  }
}

}  // namespace wavett
