// wave_api.cpp -- host side of the C ABI declared in include/wave.h:
// validation, schedule planning, source/receiver tables, the forward and
// adjoint drivers (time windows, checkpoints, recompute), the autotuner and
// the arithmetic-intensity estimators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wave.h"
#include "wave_helpers.h"
#include "wave_kernels.h"
#include "wave_launch.h"

using namespace wavett;

// Device address of the static scratch array on the current device (resolved
// once per device); defined at the end of this file.
static hipError_t static_scratch_address(void** out);

// =========================================================== context

// One device operation of a driver, recorded instead of launched while the
// context belongs to a batch: a sweep launch (merged with the other shots'
// sweeps of the same instantiation) or any other kernel.
struct RecOp {
  bool sweep = false;
  int R = 0, kind = 0, T = 0, dim = 3, mode = 0, shape = 0;
  size_t lds = 0;
  SweepArgs A{};
  std::function<hipError_t(hipStream_t)> fn;
};
struct Recorder {
  std::vector<RecOp> ops;
};
// Captured batch, replayed while the call and every context are unchanged.
struct BatchGraph {
  std::vector<uint64_t> sig;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct wave_ctx {
  wave_desc d;
  int eq = 0;                    // 0: wave equation (wave_init); 1: explicit diffusion, 2: its
                                 // two-level Adams-Bashforth form (diff_init)
  int R = 0;
  int dim = 3;
  int64_t n0 = 1, n1 = 1, n2 = 1, N = 0;
  Coefs C{};
  // device state (carved from the caller's buffer)
  float* b = nullptr;
  float* w[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t stream = nullptr;
  // schedule: T == -1 untiled kernel, T >= 1 tiled kernel
  // shape: index into the table of extended tiles of the register-tiled
  // sweep (3D 1..kNumShapes3D; 2D 0); slab > 0: skewed schedule (T >= 1)
  int T = -1, skew = 0, shape = 1, zchunks = 0, slab = 0;
  int num_cu = 256;
  size_t max_lds = 65536;
  // checkpoints left by the last forward (for reuse by the adjoint)
  struct {
    bool valid = false;
    int nt = 0, K = 0, nsrc = 0, nrec = 0;
    int kept = 0;                // last segments whose history the forward kept
    const void* scratch = nullptr;
    const float* wavelet = nullptr;
    std::vector<double> src, rec;
  } ck;
  SweepAux aux_host[4];          // sources of the per-call table copies
  std::vector<char> stage[4];    // host images of the point tables (live sources of their copies)
  Recorder* rec = nullptr;       // non-null: device operations are recorded, not launched
  uint64_t id = 0;               // unique per context of the process
  uint64_t gen = 0;              // bumped by every call that rewrites the caller's scratch
  int last_kept = 0;             // segments the last wave_adjoint_grad kept the history of
  void* static_scratch = nullptr;   // device address of this GPU's static scratch array (wave_forward_static)
  BatchGraph* graph = nullptr;   // last batch led by this context
  hipStream_t cap = nullptr;     // stream the batch is captured on (the caller's may be the null stream)
  std::vector<hipStream_t> branch;   // streams of the batch graph's per-radius branches
  std::vector<hipEvent_t> join;      // their join events; fork event below
  hipEvent_t fork = nullptr;
  std::string err;
};

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

wave_status fail(wave_ctx* c, wave_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess)                                                           \
      return fail(ctx, WAVE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Launch a non-sweep kernel now, or record it when the context is recording.
template <class F>
wave_status enq(wave_ctx* c, F f) {
  if (c->rec) {
    RecOp op;
    op.fn = f;
    c->rec->ops.push_back(std::move(op));
    return WAVE_OK;
  }
  const hipError_t e = f(c->stream);
  if (e != hipSuccess) return fail(c, WAVE_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return WAVE_OK;
}

// Central second-derivative weights of order so, unit spacing (closed form).
void fd_weights(int so, double* c) {
  const int k = so / 2;
  double s = 0.0;
  for (int j = 1; j <= k; ++j) {
    double r = 1.0;
    for (int i = 1; i <= j; ++i) r *= double(k - i + 1) / double(k + i);
    double cj = 2.0 * r / (double(j) * double(j));
    if ((j & 1) == 0) cj = -cj;
    c[j] = cj;
    s += cj;
  }
  c[0] = -2.0 * s;
}

int64_t npts_of(const wave_desc* d) {
  int64_t n = 1;
  for (int a = 0; a < d->ndim; ++a) n *= d->shape[a];
  return n;
}

// Table index of the extended tile {ey, ex} of the register-tiled sweep:
// 3D 1..kNumShapes3D, 2D 0 (its one tile); {0, 0} = 0 (automatic); -1 if
// the tile is not built.
int tile_index(int ndim, int ey, int ex) {
  if (ey == 0 && ex == 0) return 0;
  if (ndim == 2) {
    const BlockShape bs = block_shape(KIND_TILED, 2, 0);
    return (ey == bs.ey && ex == bs.ex) ? 0 : -1;
  }
  for (int i = 1; i <= kNumShapes3D; ++i) {
    const BlockShape bs = block_shape(KIND_TILED, 3, i);
    if (ey == bs.ey && ex == bs.ex) return i;
  }
  return -1;
}

wave_status check_desc(const wave_desc* d, std::string& msg) {
  if (!d) { msg = "null descriptor"; return WAVE_EINVAL; }
  if (d->ndim != 2 && d->ndim != 3) { msg = "ndim must be 2 or 3"; return WAVE_EINVAL; }
  if (d->space_order < 2 || d->space_order > 16 || (d->space_order & 1)) {
    msg = "space_order must be even in 2..16";
    return WAVE_EINVAL;
  }
  for (int a = 0; a < d->ndim; ++a) {
    if (d->shape[a] < 1 || d->shape[a] > (1 << 20)) { msg = "bad shape"; return WAVE_EINVAL; }
    if (!(d->spacing[a] > 0.0) || !std::isfinite(d->spacing[a])) { msg = "bad spacing"; return WAVE_EINVAL; }
  }
  int64_t plane = d->ndim == 3 ? d->shape[1] * d->shape[2] : d->shape[1];
  if (plane >= (int64_t(1) << 31)) { msg = "plane too large"; return WAVE_EINVAL; }
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) { msg = "bad dt"; return WAVE_EINVAL; }
  if (d->nbl < 0) { msg = "nbl must be >= 0"; return WAVE_EINVAL; }
  if (d->nbl > 0) {
    for (int a = 0; a < d->ndim; ++a)
      if (2 * (int64_t)d->nbl >= d->shape[a]) { msg = "absorbing layer wider than half the grid"; return WAVE_EINVAL; }
    if (!(d->sigma_max >= 0.0) || !std::isfinite(d->sigma_max)) { msg = "bad sigma_max"; return WAVE_EINVAL; }
  }
  const int r = d->space_order / 2;
  if (d->skew != 0 && d->skew < r) { msg = "skew below the stencil radius"; return WAVE_ESKEW; }
  if (d->skew < 0) { msg = "bad skew"; return WAVE_EINVAL; }
  if (d->time_tile < -1 || d->time_tile > 8) { msg = "time_tile must be -1, 0 or 1..8"; return WAVE_EINVAL; }
  if (d->tile[0] < 0 || d->tile[1] < 0) { msg = "negative tile extent"; return WAVE_EINVAL; }
  if (tile_index(d->ndim, d->tile[0], d->tile[1]) < 0) {
    msg = "tile extent not in the table of built tiles";
    return WAVE_EUNSUPPORTED;
  }
  if (d->slab < 0) { msg = "slab must be >= 0"; return WAVE_EINVAL; }
  if (d->zchunks < 0) { msg = "zchunks must be >= 0"; return WAVE_EINVAL; }
  return WAVE_OK;
}

// Von Neumann limit: stable iff c_max dt sqrt(sum_a rho / h_a^2) <= 2 with
// rho = -(c_0 + 2 sum_j (-1)^j c_j), the symbol's magnitude at Nyquist.
double cfl_number(const wave_desc* d, double c_max) {
  double c[9];
  fd_weights(d->space_order, c);
  double rho = -c[0];
  for (int j = 1; j <= d->space_order / 2; ++j) rho -= 2.0 * c[j] * ((j & 1) ? -1.0 : 1.0);
  double s = 0.0;
  for (int a = 0; a < d->ndim; ++a) s += rho / (d->spacing[a] * d->spacing[a]);
  return c_max * d->dt * std::sqrt(s) / 2.0;
}

// ----------------------------------------------------------- point tables

// Unique grid points touched by a set of positions (multilinear corners),
// sorted by linear index = (z, y, x); plus the forward map position -> corners
// and the inverse map point -> (position, weight) in a fixed order.
struct PointTable {
  int npos = 0, npts = 0;
  std::vector<int32_t> zptr, y, x;          // per unique point; zptr over axis 0
  std::vector<int32_t> pos_ptr, corner_pt;  // position -> corners
  std::vector<float> corner_w;
  std::vector<int32_t> pt_ptr, pt_src;      // point -> contributions
  std::vector<float> pt_w;
};

void build_points(const wave_ctx* c, int npos, const double* xyz, PointTable& P) {
  const int nd = c->dim;
  const int64_t n[3] = {c->n0, nd == 3 ? c->n1 : c->n2, c->n2};
  struct Corner { int64_t lin; int pos; float w; };
  std::vector<Corner> corners;
  P.npos = npos;
  P.pos_ptr.assign(npos + 1, 0);
  std::vector<std::vector<std::pair<int64_t, float>>> per(npos);
  for (int p = 0; p < npos; ++p) {
    int64_t i0[3] = {0, 0, 0};
    double f[3] = {0, 0, 0};
    for (int a = 0; a < nd; ++a) {
      const double xi = xyz[(size_t)p * nd + a] / c->d.spacing[a];
      const double fl = std::floor(xi);
      i0[a] = (int64_t)fl;
      f[a] = xi - fl;
    }
    for (int bits = 0; bits < (1 << nd); ++bits) {
      double w = 1.0;
      int64_t lin = 0;
      bool inside = true;
      for (int a = 0; a < nd; ++a) {
        const int bit = (bits >> (nd - 1 - a)) & 1;
        const int64_t ia = i0[a] + bit;
        if (ia < 0 || ia >= n[a]) inside = false;
        w *= bit ? f[a] : 1.0 - f[a];
        lin = lin * n[a] + ia;
      }
      if (!inside || w == 0.0) continue;
      per[p].push_back({lin, (float)w});
    }
  }
  std::vector<int64_t> lins;
  for (auto& v : per)
    for (auto& e : v) lins.push_back(e.first);
  std::sort(lins.begin(), lins.end());
  lins.erase(std::unique(lins.begin(), lins.end()), lins.end());
  P.npts = (int)lins.size();
  const int64_t plane = (nd == 3) ? c->n1 * c->n2 : c->n2;
  P.zptr.assign(c->n0 + 1, 0);
  P.y.resize(P.npts);
  P.x.resize(P.npts);
  for (int u = 0; u < P.npts; ++u) {
    const int64_t z = lins[u] / plane, rem = lins[u] % plane;
    P.y[u] = (nd == 3) ? (int32_t)(rem / c->n2) : 0;
    P.x[u] = (int32_t)(rem % c->n2);
    P.zptr[z + 1]++;
  }
  for (int64_t z = 0; z < c->n0; ++z) P.zptr[z + 1] += P.zptr[z];
  auto find = [&](int64_t lin) { return (int32_t)(std::lower_bound(lins.begin(), lins.end(), lin) - lins.begin()); };
  P.corner_pt.clear();
  P.corner_w.clear();
  std::vector<std::vector<std::pair<int32_t, float>>> inv(P.npts);
  for (int p = 0; p < npos; ++p) {
    P.pos_ptr[p] = (int32_t)P.corner_pt.size();
    for (auto& e : per[p]) {
      const int32_t u = find(e.first);
      P.corner_pt.push_back(u);
      P.corner_w.push_back(e.second);
      inv[u].push_back({p, e.second});
    }
  }
  P.pos_ptr[npos] = (int32_t)P.corner_pt.size();
  P.pt_ptr.assign(P.npts + 1, 0);
  P.pt_src.clear();
  P.pt_w.clear();
  for (int u = 0; u < P.npts; ++u) {
    P.pt_ptr[u] = (int32_t)P.pt_src.size();
    for (auto& e : inv[u]) {
      P.pt_src.push_back(e.first);
      P.pt_w.push_back(e.second);
    }
  }
  P.pt_ptr[P.npts] = (int32_t)P.pt_src.size();
}

// Device image of a PointTable (int32/float arrays back to back).
struct DevPoints {
  PointSet set{};
  const int32_t* pos_ptr = nullptr;
  const int32_t* corner_pt = nullptr;
  const float* corner_w = nullptr;
  const int32_t* pt_ptr = nullptr;
  const int32_t* pt_src = nullptr;
  const float* pt_w = nullptr;
  int npos = 0;
  int zlo = 0, zhi = 0;   // planes holding points: [zlo, zhi)
};

size_t table_bytes_bound(int64_t n0, int npos, int nd) {
  const size_t maxc = (size_t)npos << nd;
  return align_up(sizeof(int32_t) * ((size_t)n0 + 1 + 2 * maxc + (npos + 1) + 2 * maxc + (maxc + 1) + 2 * maxc) + 64);
}

// Carves a scratch region and copies the tables into it (async on stream).
wave_status upload_points(wave_ctx* c, const PointTable& P, char*& cursor, DevPoints& D, std::vector<char>& host) {
  host.clear();
  auto put = [&](const void* p, size_t bytes) {
    size_t off = host.size();
    host.resize(off + bytes);
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  };
  const size_t o_z = put(P.zptr.data(), P.zptr.size() * 4);
  const size_t o_y = put(P.y.data(), P.y.size() * 4);
  const size_t o_x = put(P.x.data(), P.x.size() * 4);
  const size_t o_pp = put(P.pos_ptr.data(), P.pos_ptr.size() * 4);
  const size_t o_cp = put(P.corner_pt.data(), P.corner_pt.size() * 4);
  const size_t o_cw = put(P.corner_w.data(), P.corner_w.size() * 4);
  const size_t o_tp = put(P.pt_ptr.data(), P.pt_ptr.size() * 4);
  const size_t o_ts = put(P.pt_src.data(), P.pt_src.size() * 4);
  const size_t o_tw = put(P.pt_w.data(), P.pt_w.size() * 4);
  char* base = cursor;
  if (!host.empty()) HIP_TRY(c, hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, c->stream));
  cursor += align_up(host.size());
  D.set.zptr = (const int32_t*)(base + o_z);
  D.set.y = (const int32_t*)(base + o_y);
  D.set.x = (const int32_t*)(base + o_x);
  D.set.npts = P.npts;
  D.pos_ptr = (const int32_t*)(base + o_pp);
  D.corner_pt = (const int32_t*)(base + o_cp);
  D.corner_w = (const float*)(base + o_cw);
  D.pt_ptr = (const int32_t*)(base + o_tp);
  D.pt_src = (const int32_t*)(base + o_ts);
  D.pt_w = (const float*)(base + o_tw);
  D.npos = P.npos;
  D.zlo = D.zhi = 0;
  if (P.npts > 0) {
    int64_t z = 0;
    while (P.zptr[z + 1] == 0) ++z;
    D.zlo = (int)z;
    z = c->n0 - 1;
    while (P.zptr[z] == P.npts) --z;
    D.zhi = (int)z + 1;
  }
  return WAVE_OK;
}

// Device copy of the forcing/sampling tables of a window set (kept in ctx
// storage until the next call so the asynchronous copy has a live source).
wave_status upload_aux(wave_ctx* c, const DevPoints* inj, const float* inj_table, const DevPoints* smp,
                       float* smp_out, SweepAux* dev, SweepAux& host) {
  host = SweepAux{};
  if (inj) {
    host.inj = inj->set;
    host.inj_table = inj_table;
  }
  if (smp && smp_out) {
    host.smp = smp->set;
    host.smp_out = smp_out;
  }
  HIP_TRY(c, hipMemcpyAsync(dev, &host, sizeof(SweepAux), hipMemcpyHostToDevice, c->stream));
  return WAVE_OK;
}

dim3 grid1d(int64_t n) {
  int64_t b = (n + 255) / 256;
  return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536)));
}

wave_status fill(wave_ctx* c, float* p, int64_t n, float v) {
  if (n <= 0) return WAVE_OK;
  return enq(c, [=](hipStream_t st) {
    hipLaunchKernelGGL(k_fill, grid1d(n), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
  });
}

wave_status copy(wave_ctx* c, const float* s, float* d, int64_t n) {
  if (n <= 0) return WAVE_OK;
  return enq(c, [=](hipStream_t st) {
    hipLaunchKernelGGL(k_copy, grid1d(n), dim3(256), 0, st, s, d, n);
    return hipGetLastError();
  });
}

// ----------------------------------------------------------- schedule

struct Plan {
  int kind, T, shape;
  int tiles_x, tiles_y, zchunk, zc;
  int zlo, zhi;   // planes the launch updates
  size_t lds;
  int core_y, core_x;
};

// Axis-0 segments when the caller gives none.  The untiled 3D sweep runs
// best with segments of ~20-25 planes on MI355X (592^3: 24-32 segments
// 298-299 Gpts/s, 12 segments 285), i.e. about 32 workgroups per CU; the
// register-tiled wave sweeps with long segments, at most one workgroup per
// CU (592^3: 64 x 64 at depth 3 and 32 x 128 at depth 2 best with 2
// segments); wave_autotune refines.
int auto_zchunks(const wave_ctx* c, int64_t base_blocks, int kind, int T, int64_t nz) {
  // time-tiled diffusion (one level per stage, fewer registers): ~6 per CU
  // (500^3, order 2, depth 4: 8 segments 1481 Gpts/s, 3 segments 1111).
  // 2D (a row of 1 x 1024 tiles per plane): ~16 per CU (16384^2 wave,
  // order 4, depth 4: 256 segments 643 Gpts/s against 469 with 31).
  const int64_t tiled_per_cu = c->dim == 2 ? 16 : (c->eq == 1 ? 6 : 1);
  const int64_t target = (kind == KIND_UNTILED) ? (c->dim == 3 ? 32LL : 8LL) * c->num_cu : tiled_per_cu * c->num_cu;
  int64_t zc = (target + base_blocks - 1) / base_blocks;
  if (kind != KIND_UNTILED && c->dim == 3 && c->eq == 0) {
    // one resident workgroup per CU, each a long segment: the most segments
    // whose workgroups all run in the first wave (a second, partial wave of
    // such workgroups leaves most CUs idle: 592^3 at radius 1, 121 tiles,
    // 2 segments 400 Gpts/s against 329 with 3)
    zc = std::max<int64_t>(1, target / base_blocks);
  }
  // A segment re-reads 2R planes of window fill: keep it at least 4R long.
  const int64_t min_len = (kind == KIND_UNTILED) ? std::max<int64_t>(16, 4LL * c->R)
                                                 : std::max<int64_t>(16, 4LL * T * c->R);
  zc = std::min<int64_t>(zc, std::max<int64_t>(1, nz / min_len));
  return (int)std::max<int64_t>(1, zc);
}

// Plan of one launch over planes [zlo, zhi) (zhi < 0: the whole grid).
wave_status make_plan(wave_ctx* c, int kind, int T, Plan& p, int64_t zlo = 0, int64_t zhi = -1) {
  if (zhi < 0) zhi = c->n0;
  p.zlo = (int)zlo;
  p.zhi = (int)zhi;
  const int64_t nz = zhi - zlo;
  p.kind = kind;
  p.T = T;
  p.shape = (c->dim == 3) ? c->shape : 0;
  BlockShape bs = block_shape(kind, c->dim, p.shape);
  if (kind == KIND_UNTILED) {
    p.core_y = bs.ey;
    p.core_x = bs.ex;
    p.lds = 0;
  } else {
    if (T < 1 || T > tiled_tmax(c->R, c->dim, p.shape))
      return fail(c, WAVE_EUNSUPPORTED, "time-tile depth not built for this order and tile shape");
    const int H = c->skew * T;
    p.core_x = bs.ex - 2 * H;
    p.core_y = (c->dim == 3) ? bs.ey - 2 * H : 1;
    if (p.core_x < 1 || p.core_y < 1)
      return fail(c, WAVE_EUNSUPPORTED, "halo (skew * T) leaves no core in the extended tile");
    p.lds = tiled_lds_bytes(c->R, T, bs.ey, bs.ex, c->dim == 3);
    if (p.lds > c->max_lds) return fail(c, WAVE_EUNSUPPORTED, "tile needs more LDS than a workgroup can hold");
  }
  const int64_t ny = (c->dim == 3) ? c->n1 : 1;
  p.tiles_x = (int)((c->n2 + p.core_x - 1) / p.core_x);
  p.tiles_y = (int)((ny + p.core_y - 1) / p.core_y);
  const int64_t base = (int64_t)p.tiles_x * p.tiles_y;
  int zc = c->zchunks > 0 ? c->zchunks : auto_zchunks(c, base, kind, T, nz);
  zc = (int)std::min<int64_t>(zc, nz);
  p.zchunk = (int)((nz + zc - 1) / zc);
  // A workgroup addresses its segment of planes (chunk plus pipeline halo)
  // through one buffer descriptor per array, at most kSegMax bytes.
  const int64_t plane_bytes = c->n1 * c->n2 * (int64_t)sizeof(float);
  const int64_t halo = 2LL * ((kind == KIND_UNTILED ? 0 : T) + 1) * c->R;
  const int64_t max_chunk = (int64_t)kSegMax / plane_bytes - halo;
  if (max_chunk < 1) return fail(c, WAVE_EUNSUPPORTED, "grid plane too large for one buffer segment");
  if (p.zchunk > max_chunk) p.zchunk = (int)max_chunk;
  p.zc = (int)((nz + p.zchunk - 1) / p.zchunk);
  return WAVE_OK;
}

SweepArgs base_args(const wave_ctx* c) {
  SweepArgs A{};
  A.C = c->C;
  A.n0 = (int32_t)c->n0;
  A.n1 = (int32_t)((c->dim == 3) ? c->n1 : 1);
  A.n2 = (int32_t)c->n2;
  A.s1 = c->n2;
  A.s0 = (int64_t)A.n1 * c->n2;
  A.b = c->b;
  A.has_damp = (c->d.nbl > 0 && c->d.sigma_max > 0.0) ? 1 : 0;
  A.nbl = c->d.nbl;
  A.st_coef = A.has_damp ? (float)(c->d.sigma_max * c->d.dt / (2.0 * (double)c->d.nbl * (double)c->d.nbl)) : 0.0f;
  A.inj_zlo = A.inj_zhi = A.smp_zlo = A.smp_zhi = 0;
  A.skew = c->skew;
  A.dir = 1;
  return A;
}

// One launch advancing `T` steps (T = 1 for the untiled kernel).
wave_status launch_window(wave_ctx* c, const Plan& p, SweepArgs A) {
  A.core_y = p.core_y;
  A.core_x = p.core_x;
  A.tiles_x = p.tiles_x;
  A.ntiles = p.tiles_x * p.tiles_y;
  A.nblocks = A.ntiles * p.zc;
  A.zchunk = p.zchunk;
  A.zlo = p.zlo;
  A.zhi = p.zhi;
  dim3 grid((unsigned)A.nblocks);
  int mode = MODE_FWD;
  if (c->eq == 1) mode = MODE_DIFF;
  else if (c->eq == 2) mode = MODE_AB2;
  else if (A.grad) mode = MODE_ADJ;
  else if (A.hist) mode = MODE_HIST;
  if (c->rec) {
    RecOp op;
    op.sweep = true;
    op.R = c->R;
    op.kind = p.kind;
    op.T = p.T;
    op.dim = c->dim;
    op.mode = mode;
    op.shape = p.shape;
    op.lds = p.lds;
    op.A = A;
    c->rec->ops.push_back(std::move(op));
    return WAVE_OK;
  }
  hipError_t e = launch_sweep(c->R, p.kind, p.T, c->dim, mode, p.shape, A, grid, p.lds, c->stream);
  if (e != hipSuccess) return fail(c, WAVE_EHIP, std::string("sweep launch: ") + hipGetErrorString(e));
  return WAVE_OK;
}

// Rolling set of four wavefield buffers: (cur, prev) plus two free ones.
struct Waves {
  float* buf[4];
  int cur = 0, prev = 1;
  float* C() const { return buf[cur]; }
  float* P() const { return buf[prev]; }
};

// The tables and outputs a run of steps hands to every launch.
struct Window {
  const DevPoints* inj;
  const float* inj_table;
  const DevPoints* smp;
  float* smp_out;
  float* hist;
  int hist_base;
  float* grad;
  const SweepAux* aux;   // device copy of the forcing/sampling tables
};

// Launch arguments common to every launch of a run: forcing and sampling
// tables, history and gradient.
SweepArgs window_args(const wave_ctx* c, const Window& win) {
  SweepArgs A = base_args(c);
  A.aux = win.aux;
  if (win.inj && win.inj->set.npts > 0) {
    A.inj_zlo = win.inj->zlo;
    A.inj_zhi = win.inj->zhi;
  }
  if (win.smp && win.smp->set.npts > 0 && win.smp_out) {
    A.smp_zlo = win.smp->zlo;
    A.smp_zhi = win.smp->zhi;
  }
  A.hist = win.hist;
  A.hist_base = win.hist_base;
  A.grad = win.grad;
  return A;
}

// The skewed schedule (slab Z > 0, skew s >= r, depth T): the paper's time
// tile with the spatial loop along axis 0 skewed by the time index
// (implementation chapter, "Time-tiling"; background chapter, "Skewing"),
// executed tile after tile in their dependence order.  Step k of a time tile
// (0 <= k < T) updates, for slab j, the planes [jZ - ks, (j+1)Z - ks) clipped
// to the grid, and slab j runs all T steps before slab j+1.  Every plane of
// every step is computed exactly once, by the single-step kernel, so the
// result is bitwise that of the untiled sweep.  Legality with the two
// in-place levels (level n+1 overwrites n-1): the z-stencil of step k reads
// level n on [jZ-ks-r, (j+1)Z-ks+r); its right part lies in slab j's step k-1
// (s >= r), its left part in earlier slabs, and no later write has reached it
// yet, since step k+1 of slab j-1 stopped at jZ-(k+1)s <= jZ-ks-r.  Level n-1
// is read at the point only, which the in-place update reads before writing.
// Slab j's steps touch about Z + T s + 2r planes, which stay in the
// last-level cache between its launches.
// With `slots` (forward only), every level gets its own slot instead: level
// L > L0 at slot L - L0 - 1, levels L0 and L0 - 1 in W's (cur, prev), each
// step written out of place.  Nothing is overwritten then, and every plane a
// step reads comes from earlier slab-steps by the same argument.
wave_status run_steps_skewed(wave_ctx* c, Waves& W, int step0, int steps, int dir, const Window& win,
                             float* slots = nullptr, int L0 = 0) {
  const int64_t s = c->skew, Z = c->slab;
  auto level = [&](int L) -> float* {
    if (L == L0) return W.C();
    if (L == L0 - 1) return W.P();
    return slots + (size_t)(L - L0 - 1) * c->N;
  };
  int done = 0;
  while (done < steps) {
    const int Tw = std::min(c->T, steps - done);
    const int64_t J = (c->n0 + (int64_t)(Tw - 1) * s + Z - 1) / Z;
    for (int64_t j = 0; j < J; ++j) {
      for (int k = 0; k < Tw; ++k) {
        const int64_t lo = std::max<int64_t>(0, j * Z - k * s);
        const int64_t hi = std::min<int64_t>(c->n0, (j + 1) * Z - k * s);
        if (lo >= hi) continue;
        Plan p;
        wave_status st = make_plan(c, KIND_UNTILED, 1, p, lo, hi);
        if (st != WAVE_OK) return st;
        SweepArgs A = window_args(c, win);
        if (slots) {
          const int n = step0 + done + k;
          A.cur = level(n);
          A.prev = level(n - 1);
          A.outA = level(n + 1);
        } else {
          // level done+k sits in C() for even k, in P() for odd k
          float* cur = (k & 1) ? W.P() : W.C();
          float* old = (k & 1) ? W.C() : W.P();
          A.cur = cur;
          A.prev = old;
          A.outA = old;   // in place over the oldest level
        }
        A.outB = nullptr;
        A.step0 = step0 + dir * (done + k);
        A.dir = dir;
        if ((st = launch_window(c, p, A)) != WAVE_OK) return st;
      }
    }
    if ((Tw & 1) && !slots) std::swap(W.cur, W.prev);
    done += Tw;
  }
  return WAVE_OK;
}

// Advance `steps` steps starting at step index `step0` (direction dir), in
// windows of the context's depth.
wave_status run_steps(wave_ctx* c, Waves& W, int step0, int steps, int dir, const Window& win) {
  if (c->T >= 1 && c->slab > 0) return run_steps_skewed(c, W, step0, steps, dir, win);
  int done = 0;
  const bool untiled = (c->T < 0);
  while (done < steps) {
    int T = untiled ? 1 : std::min(c->T, steps - done);
    Plan p;
    wave_status s = make_plan(c, untiled ? KIND_UNTILED : KIND_TILED, T, p);
    if (s != WAVE_OK) return s;
    SweepArgs A = window_args(c, win);
    A.cur = W.C();
    A.prev = W.P();
    A.step0 = step0 + dir * done;
    A.dir = dir;
    int nc, np;
    if (untiled || T == 1) {
      A.outA = W.P();   // in place over the oldest level
      A.outB = nullptr;
      nc = W.prev;
      np = W.cur;
    } else {
      int f[2], k = 0;
      for (int i = 0; i < 4; ++i)
        if (i != W.cur && i != W.prev) f[k++] = i;
      A.outA = W.buf[f[0]];
      A.outB = W.buf[f[1]];
      nc = f[0];
      np = f[1];
    }
    s = launch_window(c, p, A);
    if (s != WAVE_OK) return s;
    W.cur = nc;
    W.prev = np;
    done += T;
  }
  return WAVE_OK;
}

// ----------------------------------------------------------- scratch layout

struct Layout {
  size_t aux = 0;                    // SweepAux blocks
  size_t tab_src = 0, tab_rec = 0;   // point tables
  size_t inj = 0;                    // forcing table [nt][npts_src]
  size_t smp = 0;                    // sample buffer [nt][npts_rec]
  size_t ckpt = 0;                   // [nseg][2][N]
  size_t adj_inj = 0, adj_smp = 0;   // adjoint forcing [nt][npts_rec], samples [nt][npts_src]
  size_t hist = 0;                   // [K][N]
  size_t adj_w = 0;                  // [4][N]
  size_t resid = 0;                  // batched gradient: residual [nt][nrec]
  size_t total = 0;
  int nseg = 0;
};

Layout layout(const wave_ctx* c, int nt, int nsrc, int nrec, int K, int adjoint) {
  Layout L;
  const int nd = c->dim;
  size_t o = 0;
  L.aux = o; o += align_up(4 * sizeof(SweepAux));
  L.tab_src = o; o += table_bytes_bound(c->n0, nsrc, nd);
  L.tab_rec = o; o += table_bytes_bound(c->n0, nrec, nd);
  L.inj = o; o += align_up(sizeof(float) * (size_t)nt * ((size_t)nsrc << nd));
  L.smp = o; o += align_up(sizeof(float) * (size_t)nt * ((size_t)nrec << nd));
  if (K > 0) {
    L.nseg = (nt + K - 1) / K;
    L.ckpt = o; o += align_up(sizeof(float) * (size_t)L.nseg * 2 * c->N);
  }
  if (adjoint) {
    const int Kh = std::min(std::max(K, 1), std::max(nt, 1));
    L.adj_inj = o; o += align_up(sizeof(float) * (size_t)nt * ((size_t)nrec << nd));
    L.adj_smp = o; o += align_up(sizeof(float) * (size_t)nt * ((size_t)nsrc << nd));
    L.hist = o; o += align_up(sizeof(float) * (size_t)Kh * c->N);
    L.adj_w = o; o += align_up(sizeof(float) * 4 * (size_t)c->N);
  }
  if (adjoint == 2) {
    L.resid = o; o += align_up(sizeof(float) * (size_t)nt * (size_t)nrec);
  }
  L.total = o;
  return L;
}

wave_status validate_coords(wave_ctx* c, int n, const double* xyz) {
  if (n < 0) return fail(c, WAVE_EINVAL, "negative point count");
  if (n > 0 && !xyz) return fail(c, WAVE_EINVAL, "null coordinates");
  for (int64_t i = 0; i < (int64_t)n * c->dim; ++i)
    if (!std::isfinite(xyz[i])) return fail(c, WAVE_EINVAL, "non-finite coordinate");
  return WAVE_OK;
}

// Steps [step0, step0 + steps) of the untiled sweep or the register tiles
// written straight into a contiguous run of history slots: level L > L0 lives
// at slot L - L0 - 1 of `hist`, levels L0 and L0 - 1 stay in W's (cur, prev).
// Every window reads its two levels where they lie and writes its last two
// into their own slots, out of place; a deeper window stores the levels in
// between as history (its last two land on the slots its outputs name, with
// the same values), so the history costs no store beyond the levels
// themselves.
wave_status run_steps_direct(wave_ctx* c, const Waves& W, int step0, int steps, const Window& win, float* hist,
                             int L0) {
  if (c->T >= 1 && c->slab > 0) {
    Waves V = W;
    return run_steps_skewed(c, V, step0, steps, 1, win, hist, L0);
  }
  auto level = [&](int L) -> float* {
    if (L == L0) return W.C();
    if (L == L0 - 1) return W.P();
    return hist + (size_t)(L - L0 - 1) * c->N;
  };
  const bool untiled = c->T < 0;
  int done = 0;
  while (done < steps) {
    const int T = untiled ? 1 : std::min(c->T, steps - done);
    Plan p;
    wave_status s = make_plan(c, untiled ? KIND_UNTILED : KIND_TILED, T, p);
    if (s != WAVE_OK) return s;
    const int n = step0 + done;
    SweepArgs A = window_args(c, win);
    A.cur = level(n);
    A.prev = level(n - 1);
    A.outA = level(n + T);
    A.outB = T >= 2 ? level(n + T - 1) : nullptr;
    if (T >= 2) {
      A.hist = hist;
      A.hist_base = L0 + 1;
    }
    A.step0 = n;
    A.dir = 1;
    if ((s = launch_window(c, p, A)) != WAVE_OK) return s;
    done += T;
  }
  return WAVE_OK;
}

// Forward core shared by wave_forward and the adjoint's own forward.  With
// keep_hist, the checkpoint segments from keep_from on store every level they
// produce (segment j's K levels at keep_hist + (j - keep_from) K N, level
// n + 1 of step n at slot n - jK) instead of a checkpoint.
wave_status forward_core(wave_ctx* c, int nt, int nsrc, const double* src, const float* wav, int nrec,
                         const double* rec, float* rec_out, const float* u_init, float* u_final, int K,
                         char* scratch, const Layout& L, float* keep_hist = nullptr, int keep_from = 0) {
  PointTable PS, PR;
  build_points(c, nsrc, src, PS);
  build_points(c, rec_out ? nrec : 0, rec, PR);
  DevPoints DS, DR;
  char* cur = scratch + L.tab_src;
  wave_status s = upload_points(c, PS, cur, DS, c->stage[0]);
  if (s) return s;
  cur = scratch + L.tab_rec;
  s = upload_points(c, PR, cur, DR, c->stage[1]);
  if (s) return s;
  float* table = (float*)(scratch + L.inj);
  float* samp = (float*)(scratch + L.smp);
  if (PS.npts > 0) {
    const int np = PS.npts;
    s = enq(c, [=](hipStream_t st) {
      hipLaunchKernelGGL(k_forcing_table, grid1d((int64_t)nt * np), dim3(256), 0, st, wav, nsrc, nt, DS.pt_ptr,
                         DS.pt_src, DS.pt_w, np, 1.0f, table);
      return hipGetLastError();
    });
    if (s) return s;
  }
  if (PR.npts > 0) {
    s = fill(c, samp, (int64_t)nt * PR.npts, 0.0f);
    if (s) return s;
  }
  Waves W;
  for (int i = 0; i < 4; ++i) W.buf[i] = c->w[i];
  if (u_init) {
    if ((s = copy(c, u_init, W.C(), c->N))) return s;
    if ((s = copy(c, u_init + c->N, W.P(), c->N))) return s;
  } else {
    if ((s = fill(c, W.C(), c->N, 0.0f))) return s;
    if ((s = fill(c, W.P(), c->N, 0.0f))) return s;
  }
  float* ck = K > 0 ? (float*)(scratch + L.ckpt) : nullptr;
  SweepAux* auxd = (SweepAux*)(scratch + L.aux);
  if ((s = upload_aux(c, &DS, table, PR.npts > 0 ? &DR : nullptr, samp, auxd, c->aux_host[0]))) return s;
  Window win{&DS, table, PR.npts > 0 ? &DR : nullptr, samp, nullptr, 0, nullptr, auxd};
  if (keep_hist && !ck) return fail(c, WAVE_EINVAL, "kept history needs checkpoints");
  // every schedule writes the kept levels straight into their slots
  const bool direct = keep_hist != nullptr;
  const int L0 = keep_from * K;
  bool ran_direct = false;
  int n = 0;
  while (n < nt) {
    const int seg = ck ? n / K : 0;
    const bool kept = keep_hist && seg >= keep_from;
    if (ck && n % K == 0 && !kept) {
      if ((s = copy(c, W.C(), ck + (size_t)seg * 2 * c->N, c->N))) return s;
      if ((s = copy(c, W.P(), ck + (size_t)seg * 2 * c->N + c->N, c->N))) return s;
    }
    const int upto = ck ? std::min(nt, (n / K + 1) * K) : nt;
    if (kept && direct) {
      if ((s = run_steps_direct(c, W, n, upto - n, win, keep_hist, L0))) return s;
      ran_direct = true;
    } else {
      Window w = win;
      if (kept) {
        w.hist = keep_hist + (size_t)(seg - keep_from) * K * c->N;
        w.hist_base = seg * K + 1;
      }
      if ((s = run_steps(c, W, n, upto - n, 1, w))) return s;
    }
    n = upto;
  }
  // where the last two levels lie
  const float* fin_c = W.C();
  const float* fin_p = W.P();
  if (ran_direct) {
    fin_c = nt > L0 ? keep_hist + (size_t)(nt - L0 - 1) * c->N : W.C();
    fin_p = nt - 1 > L0 ? keep_hist + (size_t)(nt - L0 - 2) * c->N : (nt - 1 == L0 ? W.C() : W.P());
  }
  if (rec_out && nrec > 0) {
    if (PR.npts > 0) {
      const int np = PR.npts;
      s = enq(c, [=](hipStream_t st) {
        hipLaunchKernelGGL(k_reduce_samples, grid1d((int64_t)nt * nrec), dim3(256), 0, st, samp, np, nt, DR.pos_ptr,
                           DR.corner_pt, DR.corner_w, nrec, 1.0f, rec_out);
        return hipGetLastError();
      });
      if (s) return s;
    } else {
      if ((s = fill(c, rec_out, (int64_t)nt * nrec, 0.0f))) return s;
    }
  }
  if (u_final) {
    if ((s = copy(c, fin_c, u_final, c->N))) return s;
    if ((s = copy(c, fin_p, u_final + c->N, c->N))) return s;
  }
  return WAVE_OK;
}

}  // namespace

// =========================================================== dispatch tables

namespace wavett {

BlockShape block_shape(int kind, int dim, int shape) {
  if (dim == 2) return {8, 2, 1, 1024};   // 8 waves x 2 slots of 64 columns
  if (kind == KIND_UNTILED) return {WAVE_UNTILED_NW, WAVE_UNTILED_RY, WAVE_UNTILED_NW * WAVE_UNTILED_RY, 64};
  if (shape == 2) return {16, 2, 32, 64};   // 16 waves x 2 rows (1024 threads)
  if (shape == 3) return {16, 4, 32, 128};
  if (shape == 4) return {8, 4, 16, 128};
  return {16, 4, 64, 64};   // 16 waves x 4 rows (1024 threads)
}

int tiled_tmax(int R, int dim, int shape) {
  if (R < 1 || R > 8) return 0;
  if (dim == 2) return kTmax2D[R];
  switch (shape) {
    case 2: return kTmax3D_S2[R];
    case 3: return kTmax3D_S3[R];
    case 4: return kTmax3D_S4[R];
    default: return kTmax3D_S1[R];
  }
}

hipError_t launch_sweep(int R, int kind, int T, int dim, int mode, int shape, const SweepArgs& A, dim3 grid,
                        size_t lds, hipStream_t s) {
  if (mode < 0 || mode > 4) return hipErrorInvalidValue;
#define WAVE_CASE(RR)                                                                  \
  case RR:                                                                             \
    return mode == 0 ? launch_sweep_r##RR##_m0(kind, T, dim, shape, A, grid, lds, s)  \
         : mode == 1 ? launch_sweep_r##RR##_m1(kind, T, dim, shape, A, grid, lds, s)  \
         : mode == 2 ? launch_sweep_r##RR##_m2(kind, T, dim, shape, A, grid, lds, s)  \
         : mode == 3 ? launch_sweep_r##RR##_m3(kind, T, dim, shape, A, grid, lds, s)  \
                     : launch_sweep_r##RR##_m4(kind, T, dim, shape, A, grid, lds, s);
  switch (R) {
    WAVE_CASE(1) WAVE_CASE(2) WAVE_CASE(3) WAVE_CASE(4) WAVE_CASE(5) WAVE_CASE(6) WAVE_CASE(7) WAVE_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef WAVE_CASE
}

hipError_t launch_batch(int R, int kind, int T, int dim, int mode, int shape, const BatchArgs& B, dim3 grid,
                        size_t lds, hipStream_t s) {
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
#define WAVE_CASE(RR)                                                                  \
  case RR:                                                                             \
    return mode == 0 ? launch_batch_r##RR##_m0(kind, T, dim, shape, B, grid, lds, s)  \
         : mode == 1 ? launch_batch_r##RR##_m1(kind, T, dim, shape, B, grid, lds, s)  \
                     : launch_batch_r##RR##_m2(kind, T, dim, shape, B, grid, lds, s);
  switch (R) {
    WAVE_CASE(1) WAVE_CASE(2) WAVE_CASE(3) WAVE_CASE(4) WAVE_CASE(5) WAVE_CASE(6) WAVE_CASE(7) WAVE_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef WAVE_CASE
}

}  // namespace wavett

// =========================================================== C ABI

extern "C" {

const char* wave_strerror(wave_status s) {
  switch (s) {
    case WAVE_OK: return "ok";
    case WAVE_EINVAL: return "invalid argument";
    case WAVE_ESKEW: return "skew below the stencil radius (illegal time tile)";
    case WAVE_ECFL: return "time step above the stability limit";
    case WAVE_ENOMEM: return "buffer too small";
    case WAVE_EHIP: return "HIP runtime error";
    case WAVE_ESTATE: return "invalid call sequence";
    case WAVE_EUNSUPPORTED: return "schedule not available for this order/shape";
  }
  return "unknown status";
}

const char* wave_last_error(const wave_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

size_t wave_state_bytes(const wave_desc* d) {
  std::string msg;
  wave_status s = check_desc(d, msg);
  if (s != WAVE_OK && s != WAVE_ESKEW) return 0;
  const int64_t N = npts_of(d);
  size_t o = align_up(sizeof(float) * N);          // b
  o += 4 * align_up(sizeof(float) * N);             // wavefields
  return o;
}

static wave_status apply_schedule(wave_ctx* c, int T, int skew, int shape, int slab, int zchunks) {
  if (skew != 0 && skew < c->R) return fail(c, WAVE_ESKEW, "skew below the stencil radius");
  if (skew < 0 || zchunks < 0 || slab < 0 || shape < 0 || shape > kNumShapes3D || T < -1 || T == 0)
    return fail(c, WAVE_EINVAL, "bad schedule");
  if (slab == 0 && T > 8) return fail(c, WAVE_EUNSUPPORTED, "register-tiled depth above 8");
  if (slab > 0 && T < 1) return fail(c, WAVE_EINVAL, "the skewed schedule needs a depth T >= 1");
  if (c->eq == 2 && T >= 1 && slab == 0)
    return fail(c, WAVE_EUNSUPPORTED, "the two-level step runs untiled or skewed (slab > 0) only");
  // tile {0, 0} (shape 0): the first entry of the table that builds depth T
  // at this order (3D)
  int auto_shape = 1;
  if (c->dim == 3 && shape == 0 && T >= 1 && slab == 0)
    for (int i = kNumShapes3D; i >= 1; --i)
      if (tiled_tmax(c->R, 3, i) >= T) auto_shape = i;
  c->T = T;
  c->skew = skew ? skew : c->R;
  c->shape = (c->dim == 3) ? (shape ? shape : auto_shape) : 0;
  c->slab = slab;
  c->zchunks = zchunks;
  if (T >= 1 && slab == 0) {
    Plan p;
    wave_status s = make_plan(c, KIND_TILED, T, p);
    if (s != WAVE_OK) return s;
  }
  return WAVE_OK;
}

wave_status wave_set_schedule(wave_ctx* c, int32_t T, int32_t skew, const int32_t* tile, int32_t slab,
                              int32_t zchunks) {
  if (!c) return WAVE_EINVAL;
  const int ey = tile ? tile[0] : 0, ex = tile ? tile[1] : 0;
  if (ey < 0 || ex < 0) return fail(c, WAVE_EINVAL, "negative tile extent");
  const int shape = tile_index(c->dim, ey, ex);
  if (shape < 0) return fail(c, WAVE_EUNSUPPORTED, "tile extent not in the table of built tiles");
  const int oT = c->T, os = c->skew, osh = c->shape, oz = c->zchunks, osl = c->slab;
  wave_status s = apply_schedule(c, T, skew, shape, slab, zchunks);
  if (s != WAVE_OK) {
    c->T = oT; c->skew = os; c->shape = osh; c->zchunks = oz; c->slab = osl;
  }
  return s;
}

wave_status wave_get_schedule(const wave_ctx* c, int32_t* T, int32_t* skew, int32_t* tile, int32_t* slab,
                              int32_t* zchunks) {
  if (!c) return WAVE_EINVAL;
  if (T) *T = c->T;
  if (skew) *skew = c->skew;
  if (tile) {
    tile[0] = tile[1] = 0;
    if (c->T >= 1 && c->slab == 0) {
      const BlockShape bs = block_shape(KIND_TILED, c->dim, c->shape);
      tile[0] = bs.ey;
      tile[1] = bs.ex;
    }
  }
  if (slab) *slab = c->slab;
  if (zchunks) *zchunks = c->zchunks;
  return WAVE_OK;
}

// Per block: the minimum of m and the number of entries that are not
// positive finite numbers (NaN included), as two floats out[2 blk], out[2 blk + 1].
__global__ void k_min_reduce(const float* m, int64_t n, float* out) {
  __shared__ float sh[256];
  __shared__ float bad[256];
  float v = 3.4e38f, nb = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = m[i];
    v = fminf(v, x);
    nb += (x > 0.0f && x <= 3.4028234e38f) ? 0.0f : 1.0f;   // false for NaN and +inf
  }
  sh[threadIdx.x] = v;
  bad[threadIdx.x] = nb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[threadIdx.x] = fminf(sh[threadIdx.x], sh[threadIdx.x + s]);
      bad[threadIdx.x] += bad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = sh[0];
    out[2 * blockIdx.x + 1] = bad[0];
  }
}

wave_status wave_set_model(wave_ctx* c, const float* m) {
  if (!c || !m) return fail(c, WAVE_EINVAL, "null model");
  if (c->eq != 0) return fail(c, WAVE_ESTATE, "not a wave-equation context");
  // min(m) and a count of invalid entries, through the wavefield buffer w[3]
  // as temporary space (overwritten by any sweep anyway).  One block per 256
  // points (at most 1024): the 2 nb floats written never pass the end of w[3]
  // (2 ceil(N/256) <= N for N > 64; at least 64 floats in the aligned region
  // otherwise).
  const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (c->N + 255) / 256));
  if (2 * (size_t)nb * sizeof(float) > align_up(sizeof(float) * (size_t)c->N))
    return fail(c, WAVE_EINVAL, "internal: model reduction larger than its buffer");
  hipLaunchKernelGGL(k_min_reduce, dim3(nb), dim3(256), 0, c->stream, m, c->N, c->w[3]);
  HIP_TRY(c, hipGetLastError());
  std::vector<float> part(2 * (size_t)nb);
  HIP_TRY(c, hipMemcpyAsync(part.data(), c->w[3], part.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float mn = 3.4e38f, nbad = 0.0f;
  for (int i = 0; i < nb; ++i) {
    mn = std::min(mn, part[2 * (size_t)i]);
    nbad += part[2 * (size_t)i + 1];
  }
  if (nbad != 0.0f || !(mn > 0.0f) || !std::isfinite(mn))
    return fail(c, WAVE_EINVAL, "model must be positive and finite everywhere");
  const double cmax = 1.0 / std::sqrt((double)mn);
  const double cfl = cfl_number(&c->d, cmax);
  if (cfl > 1.0 + 1e-12) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "dt exceeds the stability limit by a factor %.4f (c_max %.1f m/s)", cfl, cmax);
    return fail(c, WAVE_ECFL, buf);
  }
  hipLaunchKernelGGL(k_compute_b, grid1d(c->N), dim3(256), 0, c->stream, m, c->b, c->N, c->d.dt * c->d.dt);
  HIP_TRY(c, hipGetLastError());
  c->ck.valid = false;
  return WAVE_OK;
}

wave_status wave_init(const wave_desc* d, const float* m, void* state, size_t state_bytes, void* stream,
                      wave_ctx** out) {
  if (!out) return WAVE_EINVAL;
  *out = nullptr;
  std::string msg;
  wave_status s = check_desc(d, msg);
  if (s != WAVE_OK) return s;
  if (!m || !state) return WAVE_EINVAL;
  if (state_bytes < wave_state_bytes(d)) return WAVE_ENOMEM;
  static std::atomic<uint64_t> next_id{0};
  wave_ctx* c = new wave_ctx();
  c->id = ++next_id;
  c->d = *d;
  c->R = d->space_order / 2;
  c->dim = d->ndim;
  c->n0 = d->shape[0];
  c->n1 = d->ndim == 3 ? d->shape[1] : 1;
  c->n2 = d->ndim == 3 ? d->shape[2] : d->shape[1];
  c->N = npts_of(d);
  c->stream = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
      c->max_lds = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
    }
  }
  {
    const hipError_t e = static_scratch_address(&c->static_scratch);
    if (e != hipSuccess) {
      delete c;
      return WAVE_EHIP;
    }
  }
  // coefficients: FP64 then rounded once
  double cw[9];
  fd_weights(d->space_order, cw);
  double inv_h2[3] = {0, 0, 0};
  for (int a = 0; a < d->ndim; ++a) inv_h2[a] = 1.0 / (d->spacing[a] * d->spacing[a]);
  // axis slots: 0 = streamed (axis 0), 1 = y (3D axis 1), 2 = x (last axis)
  const double ih_z = inv_h2[0], ih_y = d->ndim == 3 ? inv_h2[1] : 0.0, ih_x = inv_h2[d->ndim - 1];
  c->C.c0 = (float)(cw[0] * (ih_z + ih_y + ih_x));
  for (int j = 1; j <= c->R; ++j) {
    c->C.w[0][j - 1] = (float)(cw[j] * ih_z);
    c->C.w[1][j - 1] = (float)(cw[j] * ih_y);
    c->C.w[2][j - 1] = (float)(cw[j] * ih_x);
  }
  // carve state
  char* p = (char*)state;
  c->b = (float*)p;
  p += align_up(sizeof(float) * c->N);
  for (int i = 0; i < 4; ++i) {
    c->w[i] = (float*)p;
    p += align_up(sizeof(float) * c->N);
  }
  const int T0 = d->time_tile == 0 ? -2 : d->time_tile;
  const int shape0 = tile_index(d->ndim, d->tile[0], d->tile[1]);
  s = apply_schedule(c, T0 == -2 ? -1 : T0, d->skew, shape0, T0 == -2 ? 0 : d->slab, d->zchunks);
  if (s != WAVE_OK) {
    delete c;
    return s;
  }
  s = wave_set_model(c, m);
  if (s != WAVE_OK) {
    delete c;
    return s;
  }
  if (T0 == -2) {
    // Default schedule from measurements on MI355X (592^3, layered model,
    // about one workgroup per CU of axis-0 segments): depth 3 on 32 x 128
    // tiles at radius 1 in 3D (1.92x the untiled sweep), depth 2 on 32 x 128
    // tiles at radius 2 (1.45x); from radius 3 on no time-tiled schedule
    // beats the untiled sweep, which is the default.  wave_autotune refines
    // by timing on the actual problem.
    // 2D (16384^2, 100 steps): depth 6 at radius 1 (2.8x), 4 at radius 2
    // (2.3x), 3 at radius 4 (1.7x; radius 3 takes the same depth), untiled
    // beyond.
    int best = -1;
    const int Td = c->dim == 3 ? (c->R <= 1 ? 3 : (c->R == 2 ? 2 : 0))
                               : (c->R <= 1 ? 6 : (c->R == 2 ? 4 : (c->R <= 4 ? 3 : 0)));
    if (Td > 0) {
      const int oshape = c->shape;
      if (c->dim == 3 && shape0 == 0) c->shape = 3;
      Plan pl;
      if (make_plan(c, KIND_TILED, Td, pl) == WAVE_OK) best = Td;
      else c->shape = oshape;
    }
    c->T = best;
    c->err.clear();
  }
  *out = c;
  return WAVE_OK;
}

void wave_destroy(wave_ctx* c) {
  if (!c) return;
  if (c->graph) {
    if (c->graph->exec) (void)hipGraphExecDestroy(c->graph->exec);
    if (c->graph->graph) (void)hipGraphDestroy(c->graph->graph);
    delete c->graph;
  }
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (hipStream_t b : c->branch) (void)hipStreamDestroy(b);
  for (hipEvent_t e : c->join) (void)hipEventDestroy(e);
  if (c->fork) (void)hipEventDestroy(c->fork);
  delete c;
}

// Segments (the last ones) whose history fits into scratch beyond the
// adjoint's layout.
static int kept_segments(const wave_ctx* c, int nt, int nsrc, int nrec, int K, size_t scratch_bytes) {
  const Layout L = layout(c, nt, nsrc, nrec, K, 1);
  if (K < 1 || L.nseg < 1 || scratch_bytes <= L.total) return 0;
  const size_t seg_bytes = align_up(sizeof(float) * (size_t)K * c->N);
  return (int)std::min<size_t>((size_t)L.nseg, (scratch_bytes - L.total) / seg_bytes);
}

size_t wave_scratch_bytes(const wave_ctx* c, int32_t nt, int32_t nsrc, int32_t nrec, int32_t K, int32_t adjoint) {
  if (!c || nt < 0 || nsrc < 0 || nrec < 0 || K < 0) return 0;
  if (c->eq != 0) return 2 * align_up(sizeof(float) * c->N);   // diffusion: wave_autotune's two levels
  return layout(c, nt, nsrc, nrec, K, adjoint).total;
}

wave_status wave_forward(wave_ctx* c, int32_t nt, int32_t nsrc, const double* src, const float* wav, int32_t nrec,
                         const double* rec, float* rec_out, const float* u_init, float* u_final, int32_t K,
                         void* scratch, size_t scratch_bytes) {
  if (!c) return WAVE_EINVAL;
  c->err.clear();
  if (c->eq != 0) return fail(c, WAVE_ESTATE, "not a wave-equation context (diffusion contexts use diff_forward)");
  c->ck.valid = false;
  if (nt < 0 || K < 0) return fail(c, WAVE_EINVAL, "negative nt or checkpoint interval");
  wave_status s;
  if ((s = validate_coords(c, nsrc, src)) || (s = validate_coords(c, nrec, rec))) return s;
  if (nt > 0 && nsrc > 0 && !wav) return fail(c, WAVE_EINVAL, "null wavelet");
  const Layout L = layout(c, nt, nsrc, nrec, K, 0);
  if (!scratch || scratch_bytes < L.total) return fail(c, WAVE_ENOMEM, "scratch buffer too small");
  c->gen++;
  // scratch beyond the adjoint's layout (of which this one is a prefix) keeps
  // the history of the last whole segments that fit for the adjoint
  float* keep_hist = nullptr;
  int nkeep = 0;
  if (K > 0 && !u_init) {
    nkeep = kept_segments(c, nt, nsrc, nrec, K, scratch_bytes);
    if (nkeep > 0) keep_hist = (float*)((char*)scratch + layout(c, nt, nsrc, nrec, K, 1).total);
  }
  s = forward_core(c, nt, nsrc, src, wav, nrec, rec, rec_out, u_init, u_final, K, (char*)scratch, L, keep_hist,
                   L.nseg - nkeep);
  if (s != WAVE_OK) return s;
  if (K > 0 && !u_init) {
    c->ck.kept = nkeep;
    c->ck.valid = true;
    c->ck.nt = nt;
    c->ck.K = K;
    c->ck.nsrc = nsrc;
    c->ck.nrec = nrec;
    c->ck.scratch = scratch;
    c->ck.wavelet = wav;
    c->ck.src.assign(src, src + (size_t)nsrc * c->dim);
  }
  return WAVE_OK;
}

// Recompute + adjoint + imaging over every checkpoint segment, given the
// checkpoints of a forward with interval K in the scratch of layout L.  Point
// tables are rebuilt into the same scratch regions: for the same coordinates
// their bytes equal those of the forward (so a recorded forward still reads
// what it wrote).  Segments from keep_from on read the history the forward
// kept in keep_hist and are not recomputed.
static wave_status adjoint_core(wave_ctx* c, int nt, int nsrc, const double* src, const float* wav, int nrec,
                                const double* rec, const float* resid, float* grad_m, float* grad_q, int K, char* sc,
                                const Layout& L, float* keep_hist = nullptr, int keep_from = 0) {
  wave_status s;
  PointTable PS, PR;
  build_points(c, nsrc, src, PS);
  build_points(c, nrec, rec, PR);
  DevPoints DS, DR;
  char* cur = sc + L.tab_src;
  if ((s = upload_points(c, PS, cur, DS, c->stage[2]))) return s;
  cur = sc + L.tab_rec;
  if ((s = upload_points(c, PR, cur, DR, c->stage[3]))) return s;
  float* table = (float*)(sc + L.inj);
  if (PS.npts > 0) {
    const int np = PS.npts;
    s = enq(c, [=](hipStream_t st) {
      hipLaunchKernelGGL(k_forcing_table, grid1d((int64_t)nt * np), dim3(256), 0, st, wav, nsrc, nt, DS.pt_ptr,
                         DS.pt_src, DS.pt_w, np, 1.0f, table);
      return hipGetLastError();
    });
    if (s) return s;
  }
  float* atab = (float*)(sc + L.adj_inj);
  if (PR.npts > 0) {
    const float inv_dt2 = (float)(1.0 / (c->d.dt * c->d.dt));
    const int np = PR.npts;
    s = enq(c, [=](hipStream_t st) {
      hipLaunchKernelGGL(k_forcing_table, grid1d((int64_t)nt * np), dim3(256), 0, st, resid, nrec, nt, DR.pt_ptr,
                         DR.pt_src, DR.pt_w, np, inv_dt2, atab);
      return hipGetLastError();
    });
    if (s) return s;
  }
  float* asmp = (float*)(sc + L.adj_smp);
  if (grad_q && PS.npts > 0) {
    if ((s = fill(c, asmp, (int64_t)nt * PS.npts, 0.0f))) return s;
  }
  float* ck = (float*)(sc + L.ckpt);
  float* hist = (float*)(sc + L.hist);
  float* aw = (float*)(sc + L.adj_w);
  Waves M;
  for (int i = 0; i < 4; ++i) M.buf[i] = aw + (size_t)i * c->N;
  if ((s = fill(c, M.C(), c->N, 0.0f))) return s;
  if ((s = fill(c, M.P(), c->N, 0.0f))) return s;
  if ((s = fill(c, grad_m, c->N, 0.0f))) return s;
  SweepAux* auxd = (SweepAux*)(sc + L.aux);
  const DevPoints* bw_inj = PR.npts > 0 ? &DR : nullptr;
  const DevPoints* bw_smp = (grad_q && PS.npts > 0) ? &DS : nullptr;
  if ((s = upload_aux(c, &DS, table, nullptr, nullptr, auxd + 1, c->aux_host[1]))) return s;
  if ((s = upload_aux(c, bw_inj, atab, bw_smp, asmp, auxd + 2, c->aux_host[2]))) return s;
  Window fw{&DS, table, nullptr, nullptr, nullptr, 0, nullptr, auxd + 1};   // history slots come per window
  Window bw{bw_inj, atab, bw_smp, asmp, hist, 0, grad_m, auxd + 2};
  for (int seg = L.nseg - 1; seg >= 0; --seg) {
    const int c0 = seg * K, c1 = std::min(nt, c0 + K);
    if (keep_hist && seg >= keep_from) {
      bw.hist = keep_hist + (size_t)(seg - keep_from) * K * c->N;
    } else {
      // the recompute reads its first two levels from the checkpoint and
      // writes every level straight into its history slot
      Waves Ck;
      Ck.buf[0] = ck + (size_t)seg * 2 * c->N;
      Ck.buf[1] = Ck.buf[0] + c->N;
      Ck.buf[2] = Ck.buf[3] = nullptr;
      if ((s = run_steps_direct(c, Ck, c0, c1 - c0, fw, hist, c0))) return s;
      bw.hist = hist;
    }
    bw.hist_base = c0 + 1;
    if ((s = run_steps(c, M, c1 - 1, c1 - c0, -1, bw))) return s;
  }
  if (grad_q && nsrc > 0) {
    if (PS.npts > 0) {
      const int np = PS.npts;
      const float dt2 = (float)(c->d.dt * c->d.dt);
      s = enq(c, [=](hipStream_t st) {
        hipLaunchKernelGGL(k_reduce_samples, grid1d((int64_t)nt * nsrc), dim3(256), 0, st, asmp, np, nt, DS.pos_ptr,
                           DS.corner_pt, DS.corner_w, nsrc, dt2, grad_q);
        return hipGetLastError();
      });
      if (s) return s;
    } else if ((s = fill(c, grad_q, (int64_t)nt * nsrc, 0.0f))) {
      return s;
    }
  }
  return WAVE_OK;
}

wave_status wave_adjoint_grad(wave_ctx* c, int32_t nt, int32_t nsrc, const double* src, const float* wav,
                              int32_t nrec, const double* rec, const float* resid, float* grad_m, float* grad_q,
                              int32_t K, int32_t reuse, void* scratch, size_t scratch_bytes) {
  if (!c) return WAVE_EINVAL;
  c->err.clear();
  if (c->eq != 0) return fail(c, WAVE_ESTATE, "not a wave-equation context");
  if (nt < 0 || K < 1) return fail(c, WAVE_EINVAL, "need nt >= 0 and a checkpoint interval >= 1");
  if (!grad_m) return fail(c, WAVE_EINVAL, "null grad_m");
  if (nt > 0 && nrec > 0 && !resid) return fail(c, WAVE_EINVAL, "null residual");
  wave_status s;
  if ((s = validate_coords(c, nsrc, src)) || (s = validate_coords(c, nrec, rec))) return s;
  if (nt > 0 && nsrc > 0 && !wav) return fail(c, WAVE_EINVAL, "null wavelet");
  const Layout L = layout(c, nt, nsrc, nrec, K, 1);
  if (!scratch || scratch_bytes < L.total) return fail(c, WAVE_ENOMEM, "scratch buffer too small");
  char* sc = (char*)scratch;
  if (reuse) {
    const bool ok = c->ck.valid && c->ck.nt == nt && c->ck.K == K && c->ck.nsrc == nsrc && c->ck.nrec == nrec &&
                    c->ck.scratch == scratch &&
                    c->ck.wavelet == wav &&
                    std::equal(c->ck.src.begin(), c->ck.src.end(), src);
    if (!ok) return fail(c, WAVE_ESTATE, "no matching checkpoints from a preceding forward");
  }
  c->gen++;
  // scratch beyond the layout keeps the history of the last whole segments
  // that fit, straight from the forward: those are not recomputed (with
  // reuse, the segments the preceding wave_forward kept)
  const int nkeep = reuse ? c->ck.kept : kept_segments(c, nt, nsrc, nrec, K, scratch_bytes);
  if (reuse && nkeep > kept_segments(c, nt, nsrc, nrec, K, scratch_bytes))
    return fail(c, WAVE_ESTATE, "scratch smaller than the preceding forward's");
  float* keep_hist = nkeep > 0 ? (float*)(sc + L.total) : nullptr;
  const int keep_from = L.nseg - nkeep;
  c->last_kept = nkeep;
  if (!reuse) {
    s = forward_core(c, nt, nsrc, src, wav, 0, nullptr, nullptr, nullptr, nullptr, K, sc, L, keep_hist, keep_from);
    if (s != WAVE_OK) return s;
  }
  c->ck.valid = false;
  return adjoint_core(c, nt, nsrc, src, wav, nrec, rec, resid, grad_m, grad_q, K, sc, L, keep_hist, keep_from);
}

size_t wave_history_segment_bytes(const wave_ctx* c, int32_t K) {
  if (!c || c->eq != 0 || K < 1) return 0;
  return align_up(sizeof(float) * (size_t)K * c->N);
}

int32_t wave_last_kept_segments(const wave_ctx* c) { return c ? c->last_kept : -1; }

// Replays the recorded operations of every shot on `st` in one interleaved
// sequence: each shot's non-sweep operations run in its own order; the
// pending sweeps of all shots are merged, one launch per group of equal
// (radius, kind, depth, dim, mode, shape), at most kMaxBatch shots each.  A
// group of one uses the single-context kernel.
// Forward-only batches merge shots in lockstep within groups of at most this
// many bytes of per-step working set (16 B per point), run one group after
// another: the 256 MiB last-level cache then keeps a group's levels between
// steps.  On the 32-shot workload that is 0.998x the shots run one by one
// against 0.977x for one lockstep group.  Gradient batches keep one group:
// merging all shots' many small launches wins there (1.08x against 1.02x).
constexpr size_t kBatchGroupBytes = size_t(96) << 20;

static wave_status replay_merged(wave_ctx* lead, std::vector<Recorder>& recs, hipStream_t st) {
  const size_t n = recs.size();
  std::vector<size_t> pos(n, 0);
  auto same = [](const RecOp& x, const RecOp& y) {
    return x.R == y.R && x.kind == y.kind && x.T == y.T && x.dim == y.dim && x.mode == y.mode && x.shape == y.shape;
  };
  for (;;) {
    for (size_t i = 0; i < n; ++i) {
      auto& ops = recs[i].ops;
      while (pos[i] < ops.size() && !ops[pos[i]].sweep) {
        const hipError_t e = ops[pos[i]].fn(st);
        if (e != hipSuccess) return fail(lead, WAVE_EHIP, std::string("batched kernel: ") + hipGetErrorString(e));
        ++pos[i];
      }
    }
    std::vector<size_t> pend;
    for (size_t i = 0; i < n; ++i)
      if (pos[i] < recs[i].ops.size()) pend.push_back(i);
    if (pend.empty()) return WAVE_OK;
    std::vector<bool> done(pend.size(), false);
    for (size_t g = 0; g < pend.size(); ++g) {
      if (done[g]) continue;
      const RecOp& key = recs[pend[g]].ops[pos[pend[g]]];
      std::vector<size_t> grp;
      for (size_t h = g; h < pend.size() && grp.size() < (size_t)kMaxBatch; ++h)
        if (!done[h] && same(recs[pend[h]].ops[pos[pend[h]]], key)) {
          grp.push_back(pend[h]);
          done[h] = true;
        }
      hipError_t e;
      if (grp.size() == 1) {
        const RecOp& op = recs[grp[0]].ops[pos[grp[0]]];
        e = launch_sweep(op.R, op.kind, op.T, op.dim, op.mode, op.shape, op.A, dim3((unsigned)op.A.nblocks), op.lds, st);
      } else {
        BatchArgs B{};
        B.n = (int32_t)grp.size();
        int64_t total = 0;
        for (size_t k = 0; k < grp.size(); ++k) {
          const RecOp& op = recs[grp[k]].ops[pos[grp[k]]];
          B.off[k] = (int32_t)total;
          B.a[k] = op.A;
          total += op.A.nblocks;
        }
        if (total >= (int64_t(1) << 31)) return fail(lead, WAVE_EUNSUPPORTED, "batched grid too large");
        B.off[grp.size()] = (int32_t)total;
        e = launch_batch(key.R, key.kind, key.T, key.dim, key.mode, key.shape, B, dim3((unsigned)total), key.lds, st);
      }
      if (e != hipSuccess) return fail(lead, WAVE_EHIP, std::string("batched sweep: ") + hipGetErrorString(e));
      for (size_t k : grp) ++pos[k];
    }
  }
}

wave_status wave_batch(wave_ctx* const* ctxs, int32_t nshots, int32_t nt, const int32_t* nsrc,
                       const double* const* src_xyz, const float* const* wavelet_dev, const int32_t* nrec,
                       const double* const* rec_xyz, float* const* rec_dev, const float* const* dobs_dev,
                       float* const* grad_m_dev, int32_t K, void* const* scratch_dev, const size_t* scratch_bytes) {
  if (!ctxs || nshots < 1 || !ctxs[0]) return WAVE_EINVAL;
  wave_ctx* lead = ctxs[0];
  lead->err.clear();
  for (int i = 0; i < nshots; ++i)
    if (ctxs[i] && ctxs[i]->eq != 0) return fail(lead, WAVE_ESTATE, "a shot context is not a wave-equation context");
  if (nt < 0) return fail(lead, WAVE_EINVAL, "negative nt");
  if (!nsrc || !src_xyz || !wavelet_dev || !nrec || !rec_xyz || !rec_dev || !scratch_dev || !scratch_bytes)
    return fail(lead, WAVE_EINVAL, "null per-shot array");
  const bool grad = grad_m_dev != nullptr;
  if (grad && (!dobs_dev || K < 1)) return fail(lead, WAVE_EINVAL, "gradient needs observed data and K >= 1");
  const int Kf = grad ? K : 0;
  const hipStream_t st = lead->stream;
  std::vector<Layout> lay(nshots);
  for (int i = 0; i < nshots; ++i) {
    wave_ctx* c = ctxs[i];
    if (!c) return fail(lead, WAVE_EINVAL, "null context");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(lead, WAVE_EINVAL, "a context appears twice in the batch");
    if (c->stream != st) return fail(lead, WAVE_EINVAL, "all contexts of a batch must share one stream");
    if (c->T >= 1 && c->slab == 0 && (c->T > kBatchTmax || (c->dim == 3 && c->shape > 2)))
      return fail(lead, WAVE_EUNSUPPORTED,
                  "batched shots need the untiled sweep, the skewed schedule or a register-tiled depth <= 2 "
                  "on a 64x64 or 32x64 tile");
    wave_status s;
    if ((s = validate_coords(c, nsrc[i], src_xyz[i])) || (s = validate_coords(c, nrec[i], rec_xyz[i])))
      return fail(lead, s, "shot " + std::to_string(i) + ": " + c->err);
    if (nt > 0 && nsrc[i] > 0 && !wavelet_dev[i]) return fail(lead, WAVE_EINVAL, "null wavelet");
    if (nt > 0 && nrec[i] > 0 && !rec_dev[i]) return fail(lead, WAVE_EINVAL, "null receiver output");
    if (grad && (!grad_m_dev[i] || (nt > 0 && nrec[i] > 0 && !dobs_dev[i])))
      return fail(lead, WAVE_EINVAL, "null gradient or observed data");
    lay[i] = layout(c, nt, nsrc[i], nrec[i], Kf, grad ? 2 : 0);
    if (!scratch_dev[i] || scratch_bytes[i] < lay[i].total)
      return fail(lead, WAVE_ENOMEM, "scratch buffer of shot " + std::to_string(i) + " too small");
  }
  // Everything the captured sequence depends on, including each context's
  // generation (bumped by every call that rewrites its scratch).
  // One graph branch per radius for a forward-only batch (32 shots of orders
  // 4 and 8: 1.02x against 0.995x the shots one by one on a single branch);
  // one branch for a gradient batch, where merging all shots in lockstep
  // paid more before the adjoint fetched its history and gradient ahead
  // (71.7 against 70.4 Gpts/s) and measures level since (3.850 against
  // 3.853 s).  WAVE_BATCH_BRANCHES=0 / =1 forces one branch / one per radius.
  const char* env_b = std::getenv("WAVE_BATCH_BRANCHES");
  const bool use_branches = env_b && env_b[0] ? env_b[0] != '0' : !grad;
  auto signature = [&]() {
    std::vector<uint64_t> sig = {(uint64_t)nshots, (uint64_t)nt, (uint64_t)Kf, (uint64_t)grad, (uint64_t)use_branches};
    for (int i = 0; i < nshots; ++i) {
      const wave_ctx* c = ctxs[i];
      const uint64_t v[] = {c->id, c->gen, (uint64_t)c->T, (uint64_t)c->skew, (uint64_t)c->shape, (uint64_t)c->slab,
                          (uint64_t)c->zchunks, (uint64_t)nsrc[i], (uint64_t)nrec[i],
                          (uint64_t)(uintptr_t)wavelet_dev[i], (uint64_t)(uintptr_t)rec_dev[i],
                          (uint64_t)(uintptr_t)(grad ? dobs_dev[i] : nullptr),
                          (uint64_t)(uintptr_t)(grad ? grad_m_dev[i] : nullptr),
                          (uint64_t)(uintptr_t)scratch_dev[i], (uint64_t)scratch_bytes[i]};
      sig.insert(sig.end(), std::begin(v), std::end(v));
      for (int k = 0; k < nsrc[i] * c->dim; ++k) {
        uint64_t b;
        std::memcpy(&b, &src_xyz[i][k], 8);
        sig.push_back(b);
      }
      for (int k = 0; k < nrec[i] * c->dim; ++k) {
        uint64_t b;
        std::memcpy(&b, &rec_xyz[i][k], 8);
        sig.push_back(b);
      }
    }
    return sig;
  };
  // Same call on unchanged contexts: replay the captured graph.
  if (lead->graph && lead->graph->exec && lead->graph->sig == signature()) {
    HIP_TRY(lead, hipGraphLaunch(lead->graph->exec, st));
    return WAVE_OK;
  }
  // Record every shot's operations (table uploads happen now, on the stream).
  std::vector<Recorder> recs(nshots);
  wave_status s = WAVE_OK;
  for (int i = 0; i < nshots && s == WAVE_OK; ++i) {
    wave_ctx* c = ctxs[i];
    char* sc = (char*)scratch_dev[i];
    c->err.clear();
    c->ck.valid = false;
    c->gen++;
    c->rec = &recs[i];
    s = forward_core(c, nt, nsrc[i], src_xyz[i], wavelet_dev[i], nrec[i], rec_xyz[i], rec_dev[i], nullptr, nullptr,
                     Kf, sc, lay[i]);
    if (s == WAVE_OK && grad) {
      float* resid = (float*)(sc + lay[i].resid);
      const float* rec = rec_dev[i];
      const float* obs = dobs_dev[i];
      const int64_t nn = (int64_t)nt * nrec[i];
      if (nn > 0)
        s = enq(c, [=](hipStream_t q) {
          hipLaunchKernelGGL(k_sub, grid1d(nn), dim3(256), 0, q, rec, obs, resid, nn);
          return hipGetLastError();
        });
      if (s == WAVE_OK)
        s = adjoint_core(c, nt, nsrc[i], src_xyz[i], wavelet_dev[i], nrec[i], rec_xyz[i], resid, grad_m_dev[i],
                         nullptr, Kf, sc, lay[i]);
    }
    c->rec = nullptr;
    if (s != WAVE_OK && c != lead) s = fail(lead, s, "shot " + std::to_string(i) + ": " + c->err);
  }
  if (s != WAVE_OK) return s;
  // Capture the merged sequence once and launch it.
  if (lead->graph) {
    if (lead->graph->exec) (void)hipGraphExecDestroy(lead->graph->exec);
    if (lead->graph->graph) (void)hipGraphDestroy(lead->graph->graph);
    delete lead->graph;
    lead->graph = nullptr;
  }
  // Capture on a stream of our own (default priority): nothing runs while
  // capturing; the graph is then launched on the caller's stream, after the
  // table uploads made there during recording.
  // Shots of different stencil radii never share a launch (their kernels
  // differ).  With branches, the shots of each radius are captured on a stream of their own,
  // forked from the capture stream and joined back, so the graph holds one
  // independent branch per radius and the launches of different orders run
  // side by side on the GPU.
  std::vector<int> radii;
  for (int i = 0; i < nshots; ++i)
    if (std::find(radii.begin(), radii.end(), ctxs[i]->R) == radii.end()) radii.push_back(ctxs[i]->R);
  const bool branches = use_branches && radii.size() > 1;
  if (!lead->cap) HIP_TRY(lead, hipStreamCreateWithFlags(&lead->cap, hipStreamNonBlocking));
  if (branches) {
    while (lead->branch.size() < radii.size()) {
      hipStream_t b = nullptr;
      hipEvent_t e = nullptr;
      HIP_TRY(lead, hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
      lead->branch.push_back(b);
      HIP_TRY(lead, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      lead->join.push_back(e);
    }
    if (!lead->fork) HIP_TRY(lead, hipEventCreateWithFlags(&lead->fork, hipEventDisableTiming));
  }
  HIP_TRY(lead, hipStreamBeginCapture(lead->cap, hipStreamCaptureModeRelaxed));
  {
    // one branch per radius (or one for all), each replaying its shots in
    // groups (forward-only: consecutive shots up to kBatchGroupBytes)
    const size_t nb = branches ? radii.size() : 1;
    hipError_t ef = hipSuccess;
    if (branches) ef = hipEventRecord(lead->fork, lead->cap);
    for (size_t b = 0; b < nb && s == WAVE_OK && ef == hipSuccess; ++b) {
      hipStream_t bs = branches ? lead->branch[b] : lead->cap;
      if (branches && (ef = hipStreamWaitEvent(bs, lead->fork, 0)) != hipSuccess) break;
      std::vector<std::vector<Recorder>> groups;
      size_t acc = 0;
      for (int i = 0; i < nshots; ++i) {
        if (branches && ctxs[i]->R != radii[b]) continue;
        const size_t ws = 16u * (size_t)ctxs[i]->N;
        if (groups.empty() || (!grad && acc + ws > kBatchGroupBytes)) {
          groups.emplace_back();
          acc = 0;
        }
        groups.back().push_back(std::move(recs[i]));
        acc += ws;
      }
      for (auto& g : groups) {
        s = replay_merged(lead, g, bs);
        if (s != WAVE_OK) break;
      }
      if (branches && s == WAVE_OK) {
        if ((ef = hipEventRecord(lead->join[b], bs)) != hipSuccess) break;
        if ((ef = hipStreamWaitEvent(lead->cap, lead->join[b], 0)) != hipSuccess) break;
      }
    }
    if (s == WAVE_OK && ef != hipSuccess) s = fail(lead, WAVE_EHIP, std::string("batch branches: ") + hipGetErrorString(ef));
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(lead->cap, &g);
  if (s != WAVE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ec != hipSuccess) return fail(lead, WAVE_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(lead, WAVE_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  lead->graph = new BatchGraph{signature(), g, x};
  HIP_TRY(lead, hipGraphLaunch(x, st));
  return WAVE_OK;
}

}  // extern "C"

namespace {

struct Cand { int T, skew, shape, slab, zc; };

// Model of one candidate's cost per point-update, from the schedule's
// geometry alone: compulsory bytes x the workgroup's halo re-load x the
// tight bound's correction (memory side), and the redundant work of a
// register tile (compute side).  The guided autotuner calibrates the two
// sides' rates on the GPU from three timed anchors.
struct CandModel {
  double mem;     // bytes per point-update the schedule is expected to move
  double work;    // computed points per useful point-update
  int kind;       // 0: single-step kernel over the whole grid, 1: register-tiled, 2: skewed
};

CandModel cand_model(wave_ctx* c, const Cand& k) {
  CandModel M{};
  const int R = c->R;
  const int mode = c->eq == 0 ? 0 : (c->eq == 1 ? 3 : 4);
  const double bc = wave_bytes_per_point(k.T, mode);
  const int shape = (c->dim == 3) ? k.shape : 0;
  double h = 1.0, rho = 1.0, t0 = (double)c->n0;
  int ey = 1, ex = 1;
  if (k.T >= 1 && k.slab == 0) {
    M.kind = 1;
    const BlockShape bs = block_shape(KIND_TILED, c->dim, shape);
    ey = bs.ey;
    ex = bs.ex;
    const int H = k.skew * k.T;
    const double cy = c->dim == 3 ? (double)(bs.ey - 2 * H) : 1.0, cx = (double)(bs.ex - 2 * H);
    rho = (c->dim == 3 ? (double)bs.ey : 1.0) * (double)bs.ex / std::max(1.0, cy * cx);
    h = rho;   // every level the tile loads is loaded over the extended tile
    Plan p;
    const int ok = c->shape, oT = c->T, os = c->skew, osl = c->slab, oz = c->zchunks;
    c->shape = shape ? shape : 1;
    c->T = k.T;
    c->skew = k.skew;
    c->slab = 0;
    c->zchunks = k.zc;
    if (make_plan(c, KIND_TILED, k.T, p) == WAVE_OK) {
      t0 = p.zchunk;
      h *= (p.zchunk + 2.0 * (k.T + 1) * R) / p.zchunk;   // pipeline fill of each segment
    }
    c->shape = ok; c->T = oT; c->skew = os; c->slab = osl; c->zchunks = oz;
  } else {
    M.kind = k.slab > 0 ? 2 : 0;
    const BlockShape bs = block_shape(KIND_UNTILED, c->dim, 0);
    ey = bs.ey;
    ex = bs.ex;
    // one of the streams (the input level) is read with its halo
    const double ext = (c->dim == 3 ? (bs.ey + 2.0 * R) / bs.ey : 1.0) * (bs.ex + 2.0 * R) / bs.ex;
    h = 1.0 + (ext - 1.0) / (mode == 0 ? 4.0 : 2.0);
    const int64_t len = k.slab > 0 ? std::min<int64_t>(k.slab, c->n0) : c->n0;
    const int64_t base = (int64_t)((c->n2 + bs.ex - 1) / bs.ex) * ((c->n1 + bs.ey - 1) / bs.ey);
    int zc = k.zc > 0 ? k.zc : auto_zchunks(c, base, KIND_UNTILED, 1, len);
    zc = (int)std::max<int64_t>(1, std::min<int64_t>(zc, len));
    const double seg = (double)((len + zc - 1) / zc);
    t0 = k.slab > 0 ? (double)k.slab : seg;
    h *= 1.0 + (2.0 * R / seg) / (mode == 0 ? 4.0 : 2.0);   // window fill of each segment
  }
  // the paper's tight bound: faces of the tiles that do not fit one L2 are
  // re-loaded; its ratio to the naive bound scales the compulsory bytes
  const double D[3] = {(double)c->n0, (double)c->n1, (double)c->n2};
  const double del[3] = {(double)R, (double)R, (double)R};
  const double tl[3] = {t0, (double)ey, (double)ex};
  const int nd = c->dim;
  const double Dn[3] = {D[0], nd == 3 ? D[1] : D[2], D[2]};
  const double tn[3] = {tl[0], nd == 3 ? tl[1] : tl[2], tl[2]};
  const int Tt = std::max(1, k.T);
  const double naive = wave_ai_naive(1.0, Tt);
  const double tight = wave_ai_tight(1.0, Tt, nd, Dn, del, tn, 4.0 * 1024 * 1024 / 4.0);
  const double corr = (std::isfinite(tight) && tight > 0.0) ? naive / tight : 1.0;
  M.mem = bc * h * corr;
  M.work = rho;
  return M;
}

// Scratch of the autotuner's trials: wave_forward's layout for trial_steps
// steps with the given point sets, then a wavelet of zeros [steps][nsrc] and
// the receiver samples [steps][nrec]; diffusion: two levels.
size_t autotune_bytes(const wave_ctx* c, int trial_steps, int nsrc, int nrec) {
  if (c->eq != 0) return 2 * align_up(sizeof(float) * c->N);
  return layout(c, trial_steps, nsrc, nrec, 0, 0).total + align_up(sizeof(float) * (size_t)trial_steps * nsrc) +
         align_up(sizeof(float) * (size_t)trial_steps * nrec);
}

wave_status autotune_impl(wave_ctx* c, int trial_steps, int repeats, int max_T, int keep, int nsrc, const double* src,
                          int nrec, const double* rec, void* scratch, size_t scratch_bytes, double* best,
                          int* timed_count) {
  if (!c || trial_steps < 1 || repeats < 1 || keep < 0) return WAVE_EINVAL;
  // Wave equation: trial forwards with the scratch layout of wave_forward,
  // carrying the operator's sources (a zero wavelet) and receivers, whose
  // lookups cost the schedules differently.  Diffusion: trial diff_forward
  // calls from a zero field in the first half of the scratch into its
  // second half.
  const bool diff = c->eq != 0;
  if (diff && (nsrc > 0 || nrec > 0)) return fail(c, WAVE_EINVAL, "a diffusion context has no sources or receivers");
  wave_status vs;
  if ((vs = validate_coords(c, nsrc, src)) || (vs = validate_coords(c, nrec, rec))) return vs;
  const Layout L = diff ? Layout{} : layout(c, trial_steps, nsrc, nrec, 0, 0);
  const size_t level = align_up(sizeof(float) * c->N);
  if (!scratch || scratch_bytes < autotune_bytes(c, trial_steps, nsrc, nrec))
    return fail(c, WAVE_ENOMEM, "scratch buffer too small");
  float* twav = diff ? nullptr : (float*)((char*)scratch + L.total);
  float* trec = diff ? nullptr : (float*)((char*)scratch + L.total + align_up(sizeof(float) * (size_t)trial_steps * nsrc));
  c->gen++;
  c->ck.valid = false;   // the trial sweeps overwrite the state (and perhaps the scratch)
  if (diff) {
    wave_status fs = fill(c, (float*)scratch, c->N, 0.0f);
    if (fs != WAVE_OK) return fs;
  } else if (nsrc > 0) {
    wave_status fs = fill(c, twav, (int64_t)trial_steps * nsrc, 0.0f);
    if (fs != WAVE_OK) return fs;
  }
  std::vector<Cand> cands;
  cands.push_back({-1, c->R, c->shape ? c->shape : 1, 0, 0});
  // register-tiled: every built tile and depth at the minimum skew
  const int nshapes = c->dim == 3 ? kNumShapes3D : 1;
  if (c->eq != 2) {
    for (int si = 1; si <= nshapes; ++si) {
      const int sh = c->dim == 3 ? si : 0;
      const int tm = std::min<int>(max_T > 0 ? max_T : 8, tiled_tmax(c->R, c->dim, sh));
      for (int T = 1; T <= tm; ++T) cands.push_back({T, c->R, sh, 0, 0});
    }
  }
  // skewed: depths 2..16 (up to max_T) on slabs of 32 and 64 planes
  const int tskew = max_T > 0 ? max_T : 16;
  for (int T = 2; T <= tskew && T <= trial_steps; T *= 2)
    for (int Z : {32, 64})
      if (Z < c->n0) cands.push_back({T, c->R, c->shape ? c->shape : 1, Z, 0});
  const int oT = c->T, os = c->skew, osh = c->shape, oz = c->zchunks, osl = c->slab;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  auto time_one = [&](const Cand& k) -> double {
    if (apply_schedule(c, k.T, k.skew, k.shape ? k.shape : 1, k.slab, k.zc) != WAVE_OK) return 1e300;
    double tmin = 1e300;
    for (int r = 0; r < repeats + 1; ++r) {
      hipEventRecord(e0, c->stream);
      const wave_status st =
          diff ? diff_forward(c, trial_steps, (const float*)scratch, (float*)((char*)scratch + level))
               : forward_core(c, trial_steps, nsrc, src, twav, nrec, rec, nrec > 0 ? trec : nullptr, nullptr,
                              nullptr, 0, (char*)scratch, L);
      if (st != WAVE_OK) return 1e300;
      hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) return 1e300;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) tmin = std::min(tmin, (double)ms * 1e-3);   // first run is a warm-up
    }
    return tmin;
  };
  auto better = [](const std::pair<double, Cand>& x, const std::pair<double, Cand>& y) { return x.first < y.first; };
  int ntimed = 0;
  auto timed_one = [&](const Cand& k) {
    ++ntimed;
    return time_one(k);
  };
  // Phase 1: kind, depth and tile at the default number of axis-0 segments:
  // every candidate, or (keep > 0) the ones an intensity model calibrated on
  // three timed anchors ranks fastest.
  std::vector<std::pair<double, Cand>> timed;
  if (keep == 0) {
    for (const Cand& k : cands) timed.push_back({timed_one(k), k});
  } else {
    // anchors: the untiled sweep (memory-bound on MI355X at every order:
    // gives the rate of the memory side), the shallowest register tile
    // (compute-bound: the register kernels' cost per computed point) and a
    // skewed schedule (the single-step kernel's cost when its data is cached)
    // (the register kernels' cost per computed point changes with the depth:
    // two register anchors on the 32 x 64 tile, T = 1 and the deepest built,
    // and a linear interpolation in T between them)
    std::vector<Cand> anchors = {cands[0]};
    int r_lo = -1, r_hi = -1, r_sk = -1;
    for (const Cand& k : cands)
      if (k.slab == 0 && k.T >= 1 && (c->dim == 2 || k.shape == 2)) {
        if (r_lo < 0) { r_lo = (int)anchors.size(); anchors.push_back(k); }
        else if (k.T > anchors[r_lo].T) { if (r_hi < 0) { r_hi = (int)anchors.size(); anchors.push_back(k); } else anchors[r_hi] = k; }
      }
    for (const Cand& k : cands)
      if (k.slab > 0) { r_sk = (int)anchors.size(); anchors.push_back(k); break; }
    std::vector<double> t_a(anchors.size());
    std::vector<CandModel> m_a(anchors.size());
    for (size_t i = 0; i < anchors.size(); ++i) {
      t_a[i] = timed_one(anchors[i]);
      m_a[i] = cand_model(c, anchors[i]);
      timed.push_back({t_a[i], anchors[i]});
    }
    const double bw = m_a[0].mem / t_a[0];                  // the untiled sweep: memory-bound
    // compute time per unit of work: the single-step kernel (the faster of
    // the untiled and skewed anchors bounds it), the register kernels by depth
    double phi_single = t_a[0];
    if (r_sk >= 0 && t_a[r_sk] < 1e300) phi_single = std::min(phi_single, t_a[r_sk]);
    auto phi_reg = [&](int T) {
      if (r_lo < 0) return 1e300;
      const double lo = t_a[r_lo] / m_a[r_lo].work;
      if (r_hi < 0 || t_a[r_hi] >= 1e300) return lo;
      const double hi = t_a[r_hi] / m_a[r_hi].work;
      const double f = (double)(T - anchors[r_lo].T) / (double)(anchors[r_hi].T - anchors[r_lo].T);
      return lo + std::min(1.0, std::max(0.0, f)) * (hi - lo);
    };
    std::vector<std::pair<double, Cand>> pred;
    for (const Cand& k : cands) {
      bool is_anchor = false;
      for (const Cand& a : anchors)
        is_anchor |= (a.T == k.T && a.shape == k.shape && a.slab == k.slab && a.skew == k.skew);
      if (is_anchor) continue;
      const CandModel m = cand_model(c, k);
      const double cmp = m.kind == 1 ? m.work * phi_reg(k.T) : phi_single;
      pred.push_back({std::max(m.mem / bw, cmp), k});
    }
    std::stable_sort(pred.begin(), pred.end(), better);
    for (size_t i = 0; i < pred.size() && (int)i < keep; ++i) timed.push_back({timed_one(pred[i].second), pred[i].second});
  }
  std::stable_sort(timed.begin(), timed.end(), better);
  double best_t = timed.empty() ? 1e300 : timed[0].first;
  Cand bc = timed.empty() ? Cand{oT, os, osh, osl, oz} : timed[0].second;
  // the fastest untiled timing, for the final choice below, and every
  // untiled timing (for the segment-count preference)
  double best_untiled = 1e300;
  Cand bu = cands[0];
  std::vector<std::pair<double, Cand>> untiled_t;
  for (const auto& tk : timed)
    if (tk.second.T < 0) {
      untiled_t.push_back(tk);
      if (tk.first < best_untiled) { best_untiled = tk.first; bu = tk.second; }
    }
  auto consider = [&](const Cand& k) {
    const double t = timed_one(k);
    if (k.T < 0) untiled_t.push_back({t, k});
    if (k.T < 0 && t < best_untiled) { best_untiled = t; bu = k; }
    if (t < best_t) {
      best_t = t;
      bc = k;
    }
  };
  // Phase 2: the number of axis-0 segments (grid size against per-workgroup
  // pipeline fill) for the five fastest schedules: at low orders a time-tiled
  // schedule that phase 1 ranks behind the untiled sweep can overtake it
  // with more segments.  The untiled sweep is always among them: it is the
  // reference of the final choice below.
  const int zcs[8] = {1, 2, 4, 8, 12, 16, 24, 32};
  std::vector<Cand> seg;
  for (size_t t = 0; t < std::min<size_t>(keep == 0 ? 5 : 2, timed.size()); ++t) {
    if (timed[t].first >= 1e300) break;
    seg.push_back(timed[t].second);
  }
  bool has_untiled = false;
  for (const Cand& k : seg) has_untiled |= k.T < 0;
  if (!has_untiled && best_untiled < 1e300) seg.push_back(bu);
  for (const Cand& b : seg)
    for (int z : zcs) {
      if (z > c->n0) break;
      Cand k = b;
      k.zc = z;
      consider(k);
    }
  // Phase 3: the skewing factor of the best register-tiled schedule (the
  // minimum legal skew r, a multiple of four, twice r), or the slab
  // thickness and depth of the best skewed schedule.
  if (bc.T >= 1 && bc.slab == 0) {
    const Cand b0 = bc;
    for (int sk : {(c->R + 3) / 4 * 4, 2 * c->R}) {
      if (sk == b0.skew) continue;
      Cand k = b0;
      k.skew = sk;
      consider(k);
    }
  } else if (bc.slab > 0) {
    const Cand b0 = bc;
    for (int Z : {16, 24, 48, 96, 128}) {
      if (Z >= c->n0) continue;
      Cand k = b0;
      k.slab = Z;
      consider(k);
    }
    const Cand b1 = bc;
    for (int T : {b1.T / 2, b1.T * 2}) {
      if (T < 2 || T > trial_steps || T > tskew) continue;
      Cand k = b1;
      k.T = T;
      consider(k);
    }
  }
  // Among untiled segment counts within the trials' spread (1 %) of the
  // fastest, the largest: the forward trials often cannot tell them apart,
  // while the gradient's history and adjoint sweeps of the same schedule run
  // faster with more workgroups (336^3, order 8: 231 against 242 us per
  // adjoint launch with 32 segments against 12, the forward level).
  if (best_untiled < 1e300) {
    const BlockShape ubs = block_shape(KIND_UNTILED, c->dim, 0);
    const int64_t ubase = (int64_t)((c->n2 + ubs.ex - 1) / ubs.ex) * ((c->n1 + ubs.ey - 1) / ubs.ey);
    auto segs = [&](const Cand& k) { return k.zc > 0 ? k.zc : auto_zchunks(c, ubase, KIND_UNTILED, 1, c->n0); };
    for (const auto& tk : untiled_t)
      if (tk.first <= 1.01 * best_untiled && segs(tk.second) > segs(bu)) bu = tk.second;
    if (bc.T < 0) {
      best_t = std::min(best_t, best_untiled);
      bc = bu;
    }
  }
  // A time-tiled schedule replaces the untiled sweep only when it is faster
  // by more than the trials' run-to-run spread (1 %): at a tie the reference
  // schedule is kept.
  if (bc.T >= 1 && best_untiled < 1e300 && best_t > 0.99 * best_untiled) {
    bc = bu;
    best_t = best_untiled;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->err.clear();
  wave_status s = apply_schedule(c, bc.T, bc.skew, bc.shape ? bc.shape : 1, bc.slab, bc.zc);
  if (s != WAVE_OK) {
    c->T = oT; c->skew = os; c->shape = osh; c->zchunks = oz; c->slab = osl;
    return s;
  }
  if (best) *best = best_t / trial_steps;
  if (timed_count) *timed_count = ntimed;
  return WAVE_OK;
}

}  // namespace

extern "C" {

wave_status wave_autotune(wave_ctx* c, int32_t trial_steps, int32_t repeats, int32_t max_T, void* scratch,
                          size_t scratch_bytes, double* best) {
  return autotune_impl(c, trial_steps, repeats, max_T, 0, 0, nullptr, 0, nullptr, scratch, scratch_bytes, best,
                       nullptr);
}

wave_status wave_autotune_guided(wave_ctx* c, int32_t trial_steps, int32_t repeats, int32_t max_T, int32_t keep,
                                 void* scratch, size_t scratch_bytes, double* best, int32_t* timed) {
  if (keep < 1) return c ? fail(c, WAVE_EINVAL, "keep must be >= 1") : WAVE_EINVAL;
  int n = 0;
  const wave_status s =
      autotune_impl(c, trial_steps, repeats, max_T, keep, 0, nullptr, 0, nullptr, scratch, scratch_bytes, best, &n);
  if (timed) *timed = n;
  return s;
}

size_t wave_autotune_scratch_bytes(const wave_ctx* c, int32_t trial_steps, int32_t nsrc, int32_t nrec) {
  if (!c || trial_steps < 1 || nsrc < 0 || nrec < 0) return 0;
  return autotune_bytes(c, trial_steps, nsrc, nrec);
}

wave_status wave_autotune_points(wave_ctx* c, int32_t trial_steps, int32_t repeats, int32_t max_T, int32_t keep,
                                 int32_t nsrc, const double* src_xyz, int32_t nrec, const double* rec_xyz,
                                 void* scratch, size_t scratch_bytes, double* best, int32_t* timed) {
  if (c && (nsrc < 0 || nrec < 0)) return fail(c, WAVE_EINVAL, "negative point count");
  int n = 0;
  const wave_status s = autotune_impl(c, trial_steps, repeats, max_T, keep, nsrc, src_xyz, nrec, rec_xyz, scratch,
                                      scratch_bytes, best, &n);
  if (timed) *timed = n;
  return s;
}

// Scratch of wave_autotune_gradient: the forward trials' (autotune_bytes),
// or a gradient's layout for trial_steps steps with checkpoints every K
// followed by grad_m [N], grad_q [steps][nsrc], a zero wavelet
// [steps][nsrc] and a zero residual [steps][nrec], whichever is larger.
static size_t grad_tune_bytes(const wave_ctx* c, int trial_steps, int nsrc, int nrec, int K) {
  const size_t g = layout(c, trial_steps, nsrc, nrec, K, 1).total + align_up(sizeof(float) * c->N) +
                   2 * align_up(sizeof(float) * (size_t)trial_steps * nsrc) +
                   align_up(sizeof(float) * (size_t)trial_steps * nrec);
  return std::max(autotune_bytes(c, trial_steps, nsrc, nrec), g);
}

size_t wave_autotune_gradient_scratch_bytes(const wave_ctx* c, int32_t trial_steps, int32_t nsrc, int32_t nrec,
                                            int32_t K) {
  if (!c || c->eq != 0 || trial_steps < 1 || nsrc < 0 || nrec < 0 || K < 1) return 0;
  return grad_tune_bytes(c, trial_steps, nsrc, nrec, K);
}

wave_status wave_autotune_gradient(wave_ctx* c, int32_t trial_steps, int32_t repeats, int32_t max_T, int32_t K,
                                   int32_t nsrc, const double* src_xyz, int32_t nrec, const double* rec_xyz,
                                   void* scratch, size_t scratch_bytes, double* best, int32_t* timed) {
  if (!c) return WAVE_EINVAL;
  if (c->eq != 0) return fail(c, WAVE_ESTATE, "not a wave-equation context");
  if (trial_steps < 1 || repeats < 1 || K < 1 || nsrc < 0 || nrec < 0)
    return fail(c, WAVE_EINVAL, "need trial_steps, repeats, K >= 1 and point counts >= 0");
  wave_status s;
  if ((s = validate_coords(c, nsrc, src_xyz)) || (s = validate_coords(c, nrec, rec_xyz))) return s;
  if (!scratch || scratch_bytes < grad_tune_bytes(c, trial_steps, nsrc, nrec, K))
    return fail(c, WAVE_ENOMEM, "scratch buffer too small");
  // 1. the forward autotuner with the operator's points
  int n = 0;
  double fbest = 0;
  s = autotune_impl(c, trial_steps, repeats, max_T, 0, nsrc, src_xyz, nrec, rec_xyz, scratch, scratch_bytes, &fbest,
                    &n);
  if (s != WAVE_OK) return s;
  // 2. trial gradients of the forward's winner, the untiled sweep and the
  //    register tiles of depth 2..4 on 32 x 64 and 32 x 128 (2D: 1 x 1024):
  //    the adjoint's kernels hold more registers than the forward's, so the
  //    forward's ranking does not carry over
  struct GC { int T, skew, shape, slab, zc; };
  std::vector<GC> cands;
  cands.push_back({c->T, c->skew, c->shape, c->slab, c->zchunks});
  cands.push_back({-1, c->R, c->dim == 3 ? 1 : 0, 0, c->T < 0 ? c->zchunks : 0});
  const int tcap = std::min(4, max_T > 0 ? max_T : 8);
  for (int sh : (c->dim == 3 ? std::vector<int>{2, 3} : std::vector<int>{0}))
    for (int T = 2; T <= std::min(tcap, tiled_tmax(c->R, c->dim, sh)); ++T) cands.push_back({T, c->R, sh, 0, 0});
  const Layout L = layout(c, trial_steps, nsrc, nrec, K, 1);
  char* base = (char*)scratch + L.total;
  float* gm = (float*)base;
  base += align_up(sizeof(float) * c->N);
  float* gq = (float*)base;
  base += align_up(sizeof(float) * (size_t)trial_steps * nsrc);
  float* wav = (float*)base;
  base += align_up(sizeof(float) * (size_t)trial_steps * nsrc);
  float* res = (float*)base;
  if (nsrc > 0 && (s = fill(c, wav, (int64_t)trial_steps * nsrc, 0.0f))) return s;
  if (nrec > 0 && (s = fill(c, res, (int64_t)trial_steps * nrec, 0.0f))) return s;
  const GC first = cands[0];
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  auto time_grad = [&](const GC& k) -> double {
    if (apply_schedule(c, k.T, k.skew, k.shape, k.slab, k.zc) != WAVE_OK) return 1e300;
    double tmin = 1e300;
    for (int r = 0; r < repeats + 1; ++r) {
      hipEventRecord(e0, c->stream);
      const wave_status st = wave_adjoint_grad(c, trial_steps, nsrc, src_xyz, wav, nrec, rec_xyz, res, gm,
                                               nsrc > 0 ? gq : nullptr, K, 0, scratch, L.total);
      if (st != WAVE_OK) return 1e300;
      hipEventRecord(e1, c->stream);
      if (hipEventSynchronize(e1) != hipSuccess) return 1e300;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) tmin = std::min(tmin, (double)ms * 1e-3);
    }
    return tmin;
  };
  double bt = 1e300, ut = 1e300;
  GC bk = first, uk = cands[1];
  for (size_t i = 0; i < cands.size(); ++i) {
    bool dup = false;
    for (size_t j = 0; j < i; ++j)
      dup |= cands[j].T == cands[i].T && cands[j].shape == cands[i].shape && cands[j].slab == cands[i].slab &&
             cands[j].zc == cands[i].zc && cands[j].skew == cands[i].skew;
    if (dup) continue;
    const double t = time_grad(cands[i]);
    ++n;
    if (cands[i].T < 0 && t < ut) { ut = t; uk = cands[i]; }
    if (t < bt) { bt = t; bk = cands[i]; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->err.clear();
  // a time-tiled schedule replaces the untiled sweep only beyond the trials'
  // spread (1 %)
  if (bk.T >= 1 && ut < 1e300 && bt > 0.99 * ut) { bk = uk; bt = ut; }
  if (bt >= 1e300) bk = first;
  s = apply_schedule(c, bk.T, bk.skew, bk.shape, bk.slab, bk.zc);
  if (s != WAVE_OK) return s;
  c->ck.valid = false;
  if (best) *best = bt < 1e300 ? bt / trial_steps : fbest;
  if (timed) *timed = n;
  return WAVE_OK;
}



// ----------------------------------------------------------- estimators

int32_t wave_tiled_max_depth(int32_t space_order, int32_t ndim, int32_t ey, int32_t ex) {
  if (space_order < 2 || space_order > 16 || (space_order & 1) || (ndim != 2 && ndim != 3)) return 0;
  const int shape = tile_index(ndim, ey, ex);
  if (shape < 0 || (ndim == 3 && shape == 0)) return 0;
  return tiled_tmax(space_order / 2, ndim, shape);
}

double wave_ai_naive(double ai_space, int32_t t_t) { return ai_space * (double)t_t; }

double wave_ai_tight(double ai_space, int32_t t_t, int32_t n, const double* D, const double* delta, const double* tile,
                     double omega) {
  if (n < 1 || n > 8 || t_t < 1 || !D || !delta || !tile) return NAN;
  double F[8], bfrac[8];
  double vol = 1.0;
  for (int i = 0; i < n; ++i) vol *= D[i];
  for (int i = 0; i < n; ++i) {
    double f = 2.0 * delta[i];
    for (int j = 0; j < i; ++j) f *= tile[j];
    for (int k = i + 1; k < n; ++k) f *= D[k];
    F[i] = f * (double)t_t;                                   // time-tiling: faces grow t_t-fold
    bfrac[i] = 2.0 * (delta[i] / D[i]) * std::floor(D[i] / tile[i]);
  }
  // deepest face that still does not fit: i* = max{i : F_i >= omega}
  int istar = -1;
  for (int i = 0; i < n; ++i)
    if (F[i] >= omega) istar = i;
  double frac = 0.0;
  if (istar >= 1) {
    for (int j = 0; j < istar; ++j) frac = frac + bfrac[j] - frac * bfrac[j];   // union of B_1..B_{i*-1}
  } else if (istar == 0) {
    frac = (F[0] - omega) * std::floor(D[0] / tile[0]) / vol;
  }
  return wave_ai_naive(ai_space, t_t) / (1.0 + frac);
}

wave_status wave_tile_extent(int32_t ndim, int32_t index, int32_t* ey, int32_t* ex) {
  if ((ndim != 2 && ndim != 3) || !ey || !ex) return WAVE_EINVAL;
  if (index < 1 || index > (ndim == 3 ? kNumShapes3D : 1)) return WAVE_EINVAL;
  const BlockShape bs = block_shape(KIND_TILED, ndim, ndim == 3 ? index : 0);
  *ey = bs.ey;
  *ex = bs.ex;
  return WAVE_OK;
}

double wave_flops_per_point(int32_t ndim, int32_t so, int32_t damped) {
  // centre product, per axis per pair one add + one FMA, forcing add, (1 - st),
  // 2u, two FMAs; inside the layer one add, the reciprocal and one multiply.
  const double r = so / 2;
  return 1.0 + 3.0 * ndim * r + 7.0 + (damped ? 3.0 : 0.0);
}

double wave_bytes_per_point(int32_t T, int32_t mode) {
  // compulsory traffic per point-update: read u^n, u^{n-1}, b once per launch,
  // write one level (in place, T <= 1) or two levels (ping-pong, T >= 2);
  // history +4 B (write or read, one level per step); imaging gradient read
  // and written once per window, +8/T B.
  const double Tt = T < 1 ? 1.0 : (double)T;
  if (mode == 3) return 8.0 / Tt;   // diffusion: read u^n, write u^{n+T}
  if (mode == 4) return T <= 1 ? 12.0 : 16.0 / Tt;   // two-level: read 2 levels, write 1 (2 per time tile)
  double base = (T <= 1) ? 16.0 : 20.0 / Tt;
  if (mode == 1) base += 4.0;
  if (mode == 2) base += 4.0 + 8.0 / Tt;
  return base;
}

double diff_flops_per_point(int32_t ndim, int32_t so, int32_t scheme) {
  // centre product, per axis per pair one add + one FMA, the final add; the
  // two-level step also forms 3/2 u^n - 1/2 u^{n-1} (a multiply and an FMA)
  const double r = so / 2;
  return 2.0 + 3.0 * ndim * r + (scheme == 1 ? 3.0 : 0.0);
}

// ====================================================== explicit diffusion

// The Laplace-operator workload of the paper's evaluation chapter, read as
// explicit diffusion u^{n+1} = u^n + dt a (L u^n) with zero ghosts.  It runs
// on the wave context's schedule, plans and sweep kernels in MODE_DIFF.

static wave_desc diff_as_wave(const diff_desc* d) {
  wave_desc w{};
  w.ndim = d->ndim;
  w.space_order = d->space_order;
  for (int a = 0; a < 3; ++a) {
    w.shape[a] = d->shape[a];
    w.spacing[a] = d->spacing[a];
  }
  w.dt = d->dt;
  w.nbl = 0;
  w.sigma_max = 0.0;
  w.time_tile = d->time_tile;
  w.skew = d->skew;
  w.tile[0] = d->tile[0];
  w.tile[1] = d->tile[1];
  w.slab = d->slab;
  w.zchunks = d->zchunks;
  return w;
}

// Stability limit of explicit diffusion: dt a sum_a rho / h_a^2 <= 2 for the
// forward-Euler step, <= 1 for the two-step Adams-Bashforth rule (its region
// on the negative real axis is [-1, 0]), with rho the magnitude of the
// weights' symbol at the Nyquist wavenumber.  Returns the ratio to the limit.
static double diff_stability(const diff_desc* d) {
  double c[9];
  fd_weights(d->space_order, c);
  double rho = -c[0];
  for (int j = 1; j <= d->space_order / 2; ++j) rho -= 2.0 * c[j] * ((j & 1) ? -1.0 : 1.0);
  double s = 0.0;
  for (int a = 0; a < d->ndim; ++a) s += rho / (d->spacing[a] * d->spacing[a]);
  return d->dt * d->alpha * s / (d->scheme == 1 ? 1.0 : 2.0);
}

// Levels of state: the one-level step ping-pongs two, the two-level step
// rotates three (the new level overwrites the one two steps back).
static int diff_levels(const diff_desc* d) { return d->scheme == 1 ? 3 : 2; }

// Default skewed schedule of the two-level step (0: untiled), from
// measurements on MI355X (500^3, 32 steps: T = 16 on 64-plane slabs 1.32x
// the untiled sweep at order 2, 1.24x at order 4; 0.95x at order 8).
static int ab2_default_depth(const wave_ctx* c) { return (c->dim == 3 && c->R <= 2) ? 16 : 0; }
static int ab2_default_slab(const wave_ctx* c) { (void)c; return 64; }


size_t diff_state_bytes(const diff_desc* d) {
  if (!d || d->scheme < 0 || d->scheme > 1) return 0;
  const wave_desc w = diff_as_wave(d);
  std::string msg;
  wave_status s = check_desc(&w, msg);
  if (s != WAVE_OK && s != WAVE_ESKEW) return 0;
  return diff_levels(d) * align_up(sizeof(float) * npts_of(&w));
}

wave_status diff_init(const diff_desc* d, void* state, size_t state_bytes, void* stream, wave_ctx** out) {
  if (!out) return WAVE_EINVAL;
  *out = nullptr;
  if (!d) return WAVE_EINVAL;
  const wave_desc w = diff_as_wave(d);
  std::string msg;
  wave_status s = check_desc(&w, msg);
  if (s != WAVE_OK) return s;
  if (!(d->alpha > 0.0) || !std::isfinite(d->alpha)) return WAVE_EINVAL;
  if (d->scheme < 0 || d->scheme > 1) return WAVE_EINVAL;
  if (diff_stability(d) > 1.0 + 1e-12) return WAVE_ECFL;
  if (!state) return WAVE_EINVAL;
  if (state_bytes < diff_state_bytes(d)) return WAVE_ENOMEM;
  static std::atomic<uint64_t> next_id{1u << 30};
  wave_ctx* c = new wave_ctx();
  c->id = ++next_id;
  c->eq = d->scheme == 1 ? 2 : 1;
  c->d = w;
  c->R = d->space_order / 2;
  c->dim = d->ndim;
  c->n0 = d->shape[0];
  c->n1 = d->ndim == 3 ? d->shape[1] : 1;
  c->n2 = d->ndim == 3 ? d->shape[2] : d->shape[1];
  c->N = npts_of(&w);
  c->stream = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
      c->max_lds = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
    }
  }
  // weights times dt a / h_axis^2, FP64 then rounded once
  double cw[9];
  fd_weights(d->space_order, cw);
  double k[3] = {0, 0, 0};
  for (int a = 0; a < d->ndim; ++a) k[a] = d->dt * d->alpha / (d->spacing[a] * d->spacing[a]);
  const double kz = k[0], ky = d->ndim == 3 ? k[1] : 0.0, kx = k[d->ndim - 1];
  c->C.c0 = (float)(cw[0] * (kz + ky + kx));
  for (int j = 1; j <= c->R; ++j) {
    c->C.w[0][j - 1] = (float)(cw[j] * kz);
    c->C.w[1][j - 1] = (float)(cw[j] * ky);
    c->C.w[2][j - 1] = (float)(cw[j] * kx);
  }
  char* p = (char*)state;
  for (int i = 0; i < diff_levels(d); ++i) c->w[i] = (float*)(p + i * align_up(sizeof(float) * c->N));
  const int shape0 = tile_index(d->ndim, d->tile[0], d->tile[1]);
  s = apply_schedule(c, d->time_tile == 0 ? -1 : d->time_tile, d->skew, shape0,
                     d->time_tile == 0 ? 0 : d->slab, d->zchunks);
  if (s == WAVE_OK && c->eq == 2 && d->time_tile == 0) {
    // two-level step: the skewed schedule by default where it measured
    // faster than the untiled sweep on MI355X (see diff_desc)
    const int Ta = ab2_default_depth(c), Za = ab2_default_slab(c);
    if (Ta > 0) s = apply_schedule(c, Ta, 0, 0, Za, 0);
  }
  if (s != WAVE_OK) {
    delete c;
    return s;
  }
  // Default from measurements on MI355X (32 steps): 3D (500^3) depth 4 on
  // 32 x 64 tiles at radius 1 (3.2x the untiled sweep), depth 2 at radius 2
  // (1.9x); at radii 3 and 4 the skewed schedule, depth 8 on 64-plane slabs
  // in 2 segments (500^3: 1.20x and 1.10x; 600^3: 1.05x and 0.98x -- no
  // register-tiled depth held up on both grids); untiled beyond.  2D
  // (16384^2, measured with the earlier 4-wave layout of the 2D tile) depth
  // 4 up to radius 2 (3.3x, 2.7x), depth 2 up to radius 4 (1.7x), untiled
  // beyond.
  int Td = 0;
  if (c->dim == 3) Td = c->R == 1 ? 4 : (c->R == 2 ? 2 : 0);
  else Td = c->R <= 2 ? 4 : (c->R <= 4 ? 2 : 0);
  if (d->time_tile == 0 && Td > 0 && c->eq == 1) {
    const int oshape = c->shape;
    if (c->dim == 3 && shape0 == 0) c->shape = 2;
    Plan pl;
    if (make_plan(c, KIND_TILED, Td, pl) == WAVE_OK) c->T = Td;
    else c->shape = oshape;
  } else if (d->time_tile == 0 && c->eq == 1 && c->dim == 3 && (c->R == 3 || c->R == 4) && c->n0 > 64) {
    c->T = 8;
    c->slab = 64;
    c->zchunks = d->zchunks ? d->zchunks : 2;
  }
  c->err.clear();
  *out = c;
  return WAVE_OK;
}

// The two-level step, nt >= 1 steps.  Level l lives in u0 (l = 0, and
// l = -1: u^{-1} = u^0), u_out (l = nt) or state level (l - 1) % 3; the
// launch producing level l + 1 reads levels l and l - 1 (both through the
// stencil) and overwrites level l - 2.  Skewed (slab > 0): level l - 2's last
// readers are step l - 1 (as its t - 1 level) and step l (as its t - 2
// level) of later slabs, from planes (j+1)Z - (k-1)s - r on, beyond what
// slab j's step k writes ((j+1)Z - ks) since s >= r.
static wave_status ab2_forward(wave_ctx* c, int nt, const float* u0, float* u_out) {
  auto buf = [&](int l) -> float* { return l <= 0 ? (float*)u0 : (l == nt ? u_out : c->w[(l - 1) % 3]); };
  auto launch = [&](int l, int64_t lo, int64_t hi) -> wave_status {
    Plan p;
    wave_status s = make_plan(c, KIND_UNTILED, 1, p, lo, hi);
    if (s != WAVE_OK) return s;
    SweepArgs A = base_args(c);
    A.cur = buf(l);
    A.prev = buf(l - 1);
    A.b = A.cur;   // not read in this mode
    A.outA = buf(l + 1);
    A.outB = nullptr;
    A.step0 = l;
    A.dir = 1;
    return launch_window(c, p, A);
  };
  if (!(c->T >= 1 && c->slab > 0)) {
    for (int l = 0; l < nt; ++l) {
      wave_status s = launch(l, 0, c->n0);
      if (s != WAVE_OK) return s;
    }
    return WAVE_OK;
  }
  const int64_t sk = c->skew, Z = c->slab;
  int done = 0;
  while (done < nt) {
    const int Tw = std::min(c->T, nt - done);
    const int64_t J = (c->n0 + (int64_t)(Tw - 1) * sk + Z - 1) / Z;
    for (int64_t j = 0; j < J; ++j) {
      for (int k = 0; k < Tw; ++k) {
        const int64_t lo = std::max<int64_t>(0, j * Z - k * sk);
        const int64_t hi = std::min<int64_t>(c->n0, (j + 1) * Z - k * sk);
        if (lo >= hi) continue;
        wave_status s = launch(done + k, lo, hi);
        if (s != WAVE_OK) return s;
      }
    }
    done += Tw;
  }
  return WAVE_OK;
}

wave_status diff_forward(wave_ctx* c, int32_t nt, const float* u0, float* u_out) {
  if (!c) return WAVE_EINVAL;
  c->err.clear();
  if (c->eq != 1 && c->eq != 2) return fail(c, WAVE_ESTATE, "not a diffusion context");
  if (nt < 0) return fail(c, WAVE_EINVAL, "negative nt");
  if (!u0 || !u_out) return fail(c, WAVE_EINVAL, "null field");
  // One launch reads its input while other workgroups write its output, so
  // no two of u0, u_out and the two state levels may share a byte.
  auto overlap = [&](const void* p, const void* q) {
    const char* a = (const char*)p;
    const char* b = (const char*)q;
    const size_t n = sizeof(float) * (size_t)c->N;
    return a < b + n && b < a + n;
  };
  if (overlap(u0, u_out)) return fail(c, WAVE_EINVAL, "u_out must not overlap u0");
  for (int i = 0; i < (c->eq == 2 ? 3 : 2); ++i)
    if (overlap(u0, c->w[i]) || overlap(u_out, c->w[i]))
      return fail(c, WAVE_EINVAL, "u0 and u_out must not overlap the context's state");
  if (nt == 0) return copy(c, u0, u_out, c->N);
  if (c->eq == 2) return ab2_forward(c, nt, u0, u_out);
  if (c->T >= 1 && c->slab > 0) {
    // The skewed schedule (see run_steps_skewed).  Level l lives in u0
    // (l = 0), u_out (l = nt) or state level (l - 1) % 2: level l + 1
    // overwrites level l - 1, whose last reader (step l - 1 of a later slab,
    // planes from (j+1)Z - (k-1)s - r on) lies beyond what the write reaches
    // ((j+1)Z - ks) since s >= r.
    auto buf = [&](int l) -> float* { return l == 0 ? (float*)u0 : (l == nt ? u_out : c->w[(l - 1) & 1]); };
    const int64_t sk = c->skew, Z = c->slab;
    int done = 0;
    while (done < nt) {
      const int Tw = std::min(c->T, nt - done);
      const int64_t J = (c->n0 + (int64_t)(Tw - 1) * sk + Z - 1) / Z;
      for (int64_t j = 0; j < J; ++j) {
        for (int k = 0; k < Tw; ++k) {
          const int64_t lo = std::max<int64_t>(0, j * Z - k * sk);
          const int64_t hi = std::min<int64_t>(c->n0, (j + 1) * Z - k * sk);
          if (lo >= hi) continue;
          Plan p;
          wave_status s = make_plan(c, KIND_UNTILED, 1, p, lo, hi);
          if (s != WAVE_OK) return s;
          SweepArgs A = base_args(c);
          A.cur = buf(done + k);
          A.prev = A.cur;   // not read in this mode
          A.b = A.cur;      // not read in this mode
          A.outA = buf(done + k + 1);
          A.outB = nullptr;
          A.step0 = done + k;
          A.dir = 1;
          if ((s = launch_window(c, p, A))) return s;
        }
      }
      done += Tw;
    }
    return WAVE_OK;
  }
  const bool untiled = c->T < 0;
  const float* src = u0;
  int k = 0, done = 0;
  while (done < nt) {
    const int T = untiled ? 1 : std::min(c->T, nt - done);
    Plan p;
    wave_status s = make_plan(c, untiled ? KIND_UNTILED : KIND_TILED, T, p);
    if (s != WAVE_OK) return s;
    SweepArgs A = base_args(c);
    A.cur = src;
    A.prev = src;   // not read in this mode
    A.b = src;      // not read in this mode
    float* dst = (done + T == nt) ? u_out : c->w[k];
    A.outA = dst;
    A.outB = nullptr;
    A.step0 = done;
    A.dir = 1;
    if ((s = launch_window(c, p, A))) return s;
    src = dst;
    k ^= 1;
    done += T;
  }
  return WAVE_OK;
}

}  // extern "C"

// ====================================================== static scratch

// Scratch of wave_forward_static: one array per GPU, in the code object's
// device data, so that a call needs no allocation.  Host code never uses the
// array's name as an address (it is a host-side stand-in there); the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept per device.
static __device__ __align__(256) unsigned char scratch[WAVE_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_addr[kMaxDevices] = {};
}  // namespace

static hipError_t static_scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_static_addr[dev] = p;
  }
  *out = g_static_addr[dev];
  return hipSuccess;
}

extern "C" {

wave_status wave_forward_static(wave_ctx* c, int32_t nt, int32_t nsrc, const double* src, const float* wav,
                                int32_t nrec, const double* rec, float* rec_out, const float* u_init,
                                float* u_final) {
  if (!c) return WAVE_EINVAL;
  c->err.clear();
  if (c->eq != 0) return fail(c, WAVE_ESTATE, "not a wave-equation context");
  if (!c->static_scratch) return fail(c, WAVE_EHIP, "static scratch address not resolved");
  if (nt < 0 || nsrc < 0 || nrec < 0) return fail(c, WAVE_EINVAL, "negative nt or point count");
  const size_t need = layout(c, nt, nsrc, nrec, 0, 0).total;
  if (need > (size_t)WAVE_STATIC_SCRATCH_BYTES) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "call needs %zu bytes of scratch, above the static maximum of %zu",
                  need, (size_t)WAVE_STATIC_SCRATCH_BYTES);
    return fail(c, WAVE_ENOMEM, buf);
  }
  return wave_forward(c, nt, nsrc, src, wav, nrec, rec, rec_out, u_init, u_final, 0, c->static_scratch,
                      (size_t)WAVE_STATIC_SCRATCH_BYTES);
}

}  // extern "C"
