// wave_kernels.h -- sweep kernels (templates), instantiated per stencil radius
// in wave_r<R>.hip.
//
// Layout: one FP32 array per time level, row-major [n0][n1][n2] (2D: n1 == 1),
// axis 2 unit stride (lanes of a wavefront walk it, so every global access is
// coalesced), axis 0 streamed through registers.
//
// k_untiled  -- one time step per launch ("spatial tiling" in the paper's
//               terms).  A workgroup owns a core tile of TY x TX columns and
//               streams it along axis 0 with a (2R+1)-plane register window per
//               column; the current plane plus an R-wide halo, loaded from
//               global memory, sits in LDS for the axis-1/axis-2 neighbours.
//               u^{n+1} overwrites u^{n-1} in place.
//
// k_tiled    -- T time steps per launch: the GPU form of the paper's
//               time-tiling (implementation chapter, "Time-tiling").  Along
//               axis 0 the T stages are pipelined with a lag of R planes each
//               (the minimum legal skew of the background chapter's skewing
//               section), i.e. a skewed parallelogram in (t, z) with no
//               redundant work; across axes 1/2 every workgroup owns an
//               extended tile of EY x EX columns and recomputes a halo of
//               `skew` points per fused step (an overlapped trapezoid), so
//               tiles never wait for each other.  Stage k is valid on the tile
//               shrunk by k*skew on each side; after T stages the core is
//               exact.  Each stage's input plane is staged in LDS; the z
//               windows of every level live in registers.
#pragma once
#include "wave_device.h"

namespace wavett {

// --------------------------------------------------------------- small helpers

__device__ __forceinline__ float ld(const float* p, bool ok) { return ok ? *p : 0.0f; }

// st = (stz[z] + sty[y]) + stx[x] -- fixed order in every kernel.
__device__ __forceinline__ float damp_at(const SweepArgs& A, int z, int y, int x) {
  if (!A.has_damp) return 0.0f;
  const float a = A.stz[z];
  const float b = A.sty ? A.sty[y] : 0.0f;
  return (a + b) + A.stx[x];
}

// Forcing value at (z, y, x) for step `step` (0 if the point is not forced).
__device__ __forceinline__ float forcing(const SweepArgs& A, int z, int y, int x, int step) {
  float f = 0.0f;
  if (A.inj.npts == 0 || z < 0 || z >= A.n0) return f;
  const int p0 = A.inj.zptr[z], p1 = A.inj.zptr[z + 1];
  for (int p = p0; p < p1; ++p) {
    if (A.inj.y[p] == y && A.inj.x[p] == x) f = A.inj_table[(int64_t)step * A.inj.npts + p];
  }
  return f;
}

// Record `v` if (z, y, x) is a sampled point.
__device__ __forceinline__ void sample(const SweepArgs& A, int z, int y, int x, int step, float v) {
  if (A.smp.npts == 0 || A.smp_out == nullptr) return;
  const int p0 = A.smp.zptr[z], p1 = A.smp.zptr[z + 1];
  for (int p = p0; p < p1; ++p) {
    if (A.smp.y[p] == y && A.smp.x[p] == x) A.smp_out[(int64_t)step * A.smp.npts + p] = v;
  }
}

// --------------------------------------------------------------- untiled sweep

// Thread slot i of (wave w, lane l):  3D: (ly, lx) = (w*RY + i, l);
// 2D: (0, (w*RY + i)*64 + l).
template <int R, int DIM, int MODE, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_untiled(SweepArgs A) {
  constexpr bool HY = (DIM == 3);
  constexpr int TY = HY ? NW * RY : 1;
  constexpr int TX = HY ? 64 : 64 * NW * RY;
  constexpr int RYH = HY ? R : 0;           // LDS halo rows
  constexpr int LDW = TX + 2 * R;
  constexpr int LDH = TY + 2 * RYH;
  constexpr int NH = 2 * R * TX * (HY ? 1 : 0) + 2 * R * TY;   // halo elements per plane
  constexpr int NT = 64 * NW;
  constexpr int HPT = (NH + NT - 1) / NT;
  __shared__ float lds[LDH * LDW];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tiles_x = A.tiles_x;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x % tiles_x;
  const int gy0 = ty * TY, gx0 = tx * TX;
  const int za = blockIdx.y * A.zchunk;
  const int zb = min(za + A.zchunk, A.n0);

  int ly[RY], lx[RY], gy[RY], gx[RY];
  bool in[RY];
  int64_t off[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    ly[i] = HY ? wv * RY + i : 0;
    lx[i] = HY ? lane : (wv * RY + i) * 64 + lane;
    gy[i] = gy0 + ly[i];
    gx[i] = gx0 + lx[i];
    in[i] = (gy[i] < A.n1) && (gx[i] < A.n2);
    off[i] = (int64_t)gy[i] * A.s1 + gx[i];
  }
  // halo element coordinates (fixed per thread)
  int hly[HPT], hlx[HPT];
  bool hok[HPT];
  int64_t hoff[HPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int e = threadIdx.x + h * NT;
    int y = 0, x = 0;
    bool valid = e < NH;
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
    hly[h] = y;
    hlx[h] = x;
    const int Y = gy0 + y, X = gx0 + x;
    hok[h] = valid && Y >= 0 && Y < A.n1 && X >= 0 && X < A.n2;
    hoff[h] = hok[h] ? (int64_t)Y * A.s1 + X : 0;
  }

  float zw[RY][2 * R + 1];
  float nxt[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) {
      const int z = za - R - 1 + j;   // zw[i][j] holds plane za-R-1+j before the first shift
      zw[i][j] = ld(A.cur + (int64_t)z * A.s0 + off[i], in[i] && z >= 0 && z < A.n0 && j > 0);
    }
    const int z = za + R;
    nxt[i] = ld(A.cur + (int64_t)z * A.s0 + off[i], in[i] && z < A.n0);
  }

  const int step = A.step0;
  for (int z = za; z < zb; ++z) {
    // window now covers planes z-R .. z+R
#pragma unroll
    for (int i = 0; i < RY; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) zw[i][j] = zw[i][j + 1];
      zw[i][2 * R] = nxt[i];
      const int zn = z + 1 + R;
      nxt[i] = ld(A.cur + (int64_t)zn * A.s0 + off[i], in[i] && zn < A.n0 && z + 1 < zb);
    }
    float hv[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) hv[h] = ld(A.cur + (int64_t)z * A.s0 + hoff[h], hok[h]);
    float up[RY], bb[RY];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      up[i] = ld(A.prev + (int64_t)z * A.s0 + off[i], in[i]);
      bb[i] = ld(A.b + (int64_t)z * A.s0 + off[i], in[i]);
      lds[(ly[i] + RYH) * LDW + lx[i] + R] = zw[i][R];
    }
#pragma unroll
    for (int h = 0; h < HPT; ++h)
      if (threadIdx.x + h * NT < NH) lds[(hly[h] + RYH) * LDW + hlx[h] + R] = hv[h];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
      const float* row = lds + (ly[i] + RYH) * LDW + lx[i] + R;
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
      if (!in[i]) continue;
      const float st = damp_at(A, z, gy[i], gx[i]);
      const float f = forcing(A, z, gy[i], gx[i], step);
      const float v = wave_point<R, HY>(A.C, zw[i][R], zm, zp, ym, yp, xm, xp, up[i], bb[i], st, f);
      const int64_t idx = (int64_t)z * A.s0 + off[i];
      A.outA[idx] = v;
      sample(A, z, gy[i], gx[i], step, v);
      if (MODE == MODE_HIST) {
        A.hist[(int64_t)(step + 1 - A.hist_base) * ((int64_t)A.n0 * A.s0) + idx] = v;
      } else if (MODE == MODE_ADJ) {
        const float u = A.hist[(int64_t)(step + 1 - A.hist_base) * ((int64_t)A.n0 * A.s0) + idx];
        A.grad[idx] = image_step(A.grad[idx], u, st, v, zw[i][R], up[i]);
      }
    }
    __syncthreads();
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
  constexpr int PL = LDW * LDH;     // floats per LDS plane
  extern __shared__ float lds[];    // T planes

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int H = A.skew * T;
  const int HYH = HY ? H : 0;
  const int CY = HY ? EY - 2 * H : 1;
  const int CX = EX - 2 * H;
  const int ty = blockIdx.x / A.tiles_x, tx = blockIdx.x % A.tiles_x;
  const int gy0 = ty * CY - HYH, gx0 = tx * CX - H;
  const int za = blockIdx.y * A.zchunk;
  const int zb = min(za + A.zchunk, A.n0);

  for (int e = threadIdx.x; e < T * PL; e += 64 * NW) lds[e] = 0.0f;

  int ly[RY], lx[RY], gy[RY], gx[RY];
  bool in[RY], core[RY];
  int64_t off[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    ly[i] = HY ? wv * RY + i : 0;
    lx[i] = HY ? lane : (wv * RY + i) * 64 + lane;
    gy[i] = gy0 + ly[i];
    gx[i] = gx0 + lx[i];
    in[i] = gy[i] >= 0 && gy[i] < A.n1 && gx[i] >= 0 && gx[i] < A.n2;
    core[i] = in[i] && lx[i] >= H && lx[i] < H + CX && (!HY || (ly[i] >= HYH && ly[i] < HYH + CY));
    off[i] = in[i] ? (int64_t)gy[i] * A.s1 + gx[i] : 0;
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
  float nxt[RY], nprev[RY];
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    nxt[i] = ld(A.cur + (int64_t)zs * A.s0 + off[i], in[i] && zs >= 0 && zs < A.n0);
    const int z1 = zs - R;
    nprev[i] = ld(A.prev + (int64_t)z1 * A.s0 + off[i], in[i] && z1 >= 0 && z1 < A.n0);
  }
  __syncthreads();

  const int64_t N = (int64_t)A.n0 * A.s0;
  for (int z0 = zs; z0 < ze; ++z0) {
    // Stage the input plane of every stage in LDS: for stage k+1 that is level
    // n+k at plane z0-(k+1)R, which sits at index R+1 of window k before this
    // iteration's pushes.
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
      for (int i = 0; i < RY; ++i) lds[k * PL + (ly[i] + RYH) * LDW + lx[i] + R] = win[k][i][R + 1];
    float cur_in[RY], prev_in[RY];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      cur_in[i] = nxt[i];
      prev_in[i] = nprev[i];
      const int zn = z0 + 1;
      nxt[i] = ld(A.cur + (int64_t)zn * A.s0 + off[i], in[i] && zn >= 0 && zn < A.n0 && zn < ze);
      const int z1 = zn - R;
      nprev[i] = ld(A.prev + (int64_t)z1 * A.s0 + off[i], in[i] && z1 >= 0 && z1 < A.n0 && zn < ze);
    }
    __syncthreads();
    // push the freshly loaded plane z0 of level n into window 0
#pragma unroll
    for (int i = 0; i < RY; ++i) {
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) win[0][i][j] = win[0][i][j + 1];
      win[0][i][2 * R] = cur_in[i];
    }
#pragma unroll
    for (int k = 1; k <= T; ++k) {
      const int zk = z0 - k * R;
      const bool zin = zk >= 0 && zk < A.n0;
      const bool zown = zk >= za && zk < zb;
      const int step = stage_step(A, k);
      const float* pl = lds + (k - 1) * PL;
      float res[RY];
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        float zm[R], zp[R], ym[R], yp[R], xm[R], xp[R];
        const float* row = pl + (ly[i] + RYH) * LDW + lx[i] + R;
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
        const bool ok = in[i] && zin;
        const int64_t idx = (int64_t)zk * A.s0 + off[i];
        const float up = (k == 1) ? prev_in[i] : win[(k >= 2) ? k - 2 : 0][i][0];
        const float bb = ld(A.b + idx, ok);
        const float st = ok ? damp_at(A, zk, gy[i], gx[i]) : 0.0f;
        const float f = ok ? forcing(A, zk, gy[i], gx[i], step) : 0.0f;
        float v = wave_point<R, HY>(A.C, win[k - 1][i][R], zm, zp, ym, yp, xm, xp, up, bb, st, f);
        v = ok ? v : 0.0f;
        res[i] = v;
        if (ok && zown && core[i]) {
          sample(A, zk, gy[i], gx[i], step, v);
          if (MODE == MODE_HIST) {
            A.hist[(int64_t)(step + 1 - A.hist_base) * N + idx] = v;
          } else if (MODE == MODE_ADJ) {
            const float u = A.hist[(int64_t)(step + 1 - A.hist_base) * N + idx];
            A.grad[idx] = image_step(A.grad[idx], u, st, v, win[k - 1][i][R], up);
          }
          if (k == T) {
            A.outA[idx] = v;
            if (A.outB) A.outB[idx] = win[T - 1][i][R];
          }
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
    __syncthreads();
  }
}

}  // namespace wavett
