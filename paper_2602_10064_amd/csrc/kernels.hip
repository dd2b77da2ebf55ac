// HIP kernels of the TACAW hot path for gfx950 (MI355X).
//
//   k_splat      projected potential of every slice of a batch of frames
//                (Gaussian form factors point-sampled in real space, separable
//                per-atom profiles staged in LDS)
//   k_row<N,M>   row pass over a batch of waves: [iFFT_x] -> * exp(i sigma V)
//                -> FFT_x, one row per thread group, LDS-staged Stockham
//   k_col<N,M>   column pass: FFT_y -> * P(k) -> [iFFT_y]; the last slice
//                stops after P and leaves the exit wave psi(k) in place
//   k_time       per (probe, k): FP64 frame mean, FP64 subtraction, time FFT,
//                |.|^2 / F^2 for the kept frequency bins
//   setup        twiddles, propagator factors, probe aperture fill
#include <hip/hip_runtime.h>

#include "fft_engine.h"
#include "tacaw_internal.h"

namespace tacaw {

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8).
// Remap so that each XCD works on a contiguous range of logical tiles: tiles
// that share 128-byte lines then share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int x = bid % 8, j = bid / 8;
  const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return start + j;
}

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------
__global__ void k_twiddles(float2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
  }
}

// numpy fftfreq: index i -> i (i < (n+1)/2) or i - n, times 1/(n d)
__device__ __forceinline__ double fftfreq(int i, int n, double d) {
  const int is = (i < (n + 1) / 2) ? i : i - n;
  return (double)is * (1.0 / ((double)n * d));
}

__global__ void k_prop_factor(float2* out, int n, double d, double lam, double dz, double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double k = fftfreq(i, n, d);
    double s, c;
    sincos(-M_PI * lam * dz * k * k, &s, &c);
    out[i] = make_float2((float)(c * scale), (float)(s * scale));
  }
}

__device__ __forceinline__ bool in_aperture(int ix, int iy, int nx, int ny, double dx, double dy,
                                            double lam, double alpha) {
  const double kx = fftfreq(ix, nx, dx);
  const double ky = fftfreq(iy, ny, dy);
  const double kk = sqrt(ky * ky + kx * kx);
  return lam * kk <= alpha;
}

__global__ void k_aperture_count(int* count, int nx, int ny, double dx, double dy, double lam,
                                 double alpha) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nx * ny && in_aperture(i % nx, i / nx, nx, ny, dx, dy, lam, alpha)) atomicAdd(count, 1);
}

// Reciprocal-space incident probe A(k) exp(-2 pi i k.r) / sqrt(count * nx * ny);
// an unnormalised inverse 2D FFT of it is the unit-norm real-space probe.
__global__ void k_probe_fill(float2* out, const double* rloc, const int* count, int n_probes, int nx,
                             int ny, double dx, double dy, double lam, double alpha) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)nx * ny;
  if (i >= per * n_probes) return;
  const int p = (int)(i / per);
  const int e = (int)(i % per);
  const int ix = e % nx, iy = e / nx;
  float2 v = make_float2(0.f, 0.f);
  if (in_aperture(ix, iy, nx, ny, dx, dy, lam, alpha)) {
    const double kx = fftfreq(ix, nx, dx), ky = fftfreq(iy, ny, dy);
    const double amp = 1.0 / sqrt((double)(*count) * (double)nx * (double)ny);
    double s, c;
    sincospi(-2.0 * (kx * rloc[2 * p] + ky * rloc[2 * p + 1]), &s, &c);
    v = make_float2((float)(amp * c), (float)(amp * s));
  }
  out[i] = v;
}

// ---------------------------------------------------------------------------
// Lane tables: one launch advances up to MAX_LANES (job, frame batch) lanes of
// the same grid size by one pass; each lane has its own slice and mode.  The
// table is a by-value kernel argument (read with scalar loads).
// ---------------------------------------------------------------------------
template <typename Table>
__device__ __forceinline__ int find_lane(const Table& t, int b) {
  int L = 0;
  for (int i = 1; i < t.n; ++i)
    if (b >= t.l[i].block_start) L = i;
  return L;
}

// ---------------------------------------------------------------------------
// Projected potential
// ---------------------------------------------------------------------------
// sum over periodic images of exp2(-e2 d^2) for |d| <= rc, where d is the
// pixel distance from grid node `node` to an atom at pixel ipos + fpos.
__device__ __forceinline__ float profile(int node, int ipos, float fpos, int n, float e2, float rc,
                                         int img) {
  int di = (node - ipos) % n;
  if (di < 0) di += n;
  if (di >= n - n / 2) di -= n;  // di in [-(n/2), n - n/2)
  const float d0 = (float)di - fpos;
  float g = 0.f;
  for (int k = -img; k <= img; ++k) {
    const float d = d0 + (float)(k * n);
    if (fabsf(d) <= rc) g += exp2f(-e2 * d * d);
  }
  return g;
}

// Periodic distance in pixels from position u to the node interval [lo, hi].
__device__ __forceinline__ float interval_distance(float u, int lo, int hi, int n) {
  const float c = 0.5f * (float)(lo + hi), h = 0.5f * (float)(hi - lo);
  float d = u - c;
  d -= (float)n * rintf(d / (float)n);
  return fmaxf(0.f, fabsf(d) - h);
}

// One workgroup computes a 32 x 64 tile of V for one (frame, slice).  Each
// candidate atom contributes, per Gaussian term, an outer product of a column
// profile and a row profile (the 2D Gaussian and its periodic images factor
// into x and y parts); the profiles of up to SPLAT_MC atoms are staged in LDS
// and every thread accumulates a 2 x 4 block of pixels.  Terms whose own
// cutoff box misses the tile are skipped by a per-atom bit mask.  The
// summation order is fixed, so the result is deterministic.
__global__ void __launch_bounds__(256) k_splat(SplatTable tab) {
  __shared__ float gx[SPLAT_MC][N_GAUSS][SPLAT_TX];
  __shared__ float gy[SPLAT_MC][N_GAUSS][SPLAT_TY];
  __shared__ AtomPos sp_pos[SPLAT_MC];
  __shared__ int sp_spc[SPLAT_MC];
  __shared__ int sp_mask[SPLAT_MC];

  const int L = find_lane(tab, blockIdx.x);
  const SplatArgs& a = tab.l[L].a;
  const int nsl = tab.l[L].n_slices_launch;
  const int lb = blockIdx.x - tab.l[L].block_start;
  const int tid = threadIdx.x;
  const int n_tiles = a.tiles_x * a.tiles_y;
  const int tile = lb % n_tiles;
  const int sl = (lb / n_tiles) % nsl;
  const int fl = lb / (n_tiles * nsl);
  const int s = a.slice0 + sl;
  const int f = a.f0 + fl;
  const int tx0 = (tile % a.tiles_x) * SPLAT_TX;
  const int ty0 = (tile / a.tiles_x) * SPLAT_TY;
  const int cs = a.tile_start[s * n_tiles + tile];
  const int ce = a.tile_start[s * n_tiles + tile + 1];

  const int ry = (tid / (SPLAT_TX / 4)) * 2;  // 0, 2, .., 30
  const int cx = (tid % (SPLAT_TX / 4)) * 4;  // 0, 4, .., 60
  float acc0[4] = {0.f, 0.f, 0.f, 0.f};
  float acc1[4] = {0.f, 0.f, 0.f, 0.f};

  for (int c0 = cs; c0 < ce; c0 += SPLAT_MC) {
    const int mc = min(SPLAT_MC, ce - c0);
    __syncthreads();
    if (tid < mc) {
      const int atom = a.tile_atoms[c0 + tid];
      const AtomPos p = a.pos[(size_t)f * a.n_atoms + atom];
      const int spc = a.species[atom];
      sp_pos[tid] = p;
      sp_spc[tid] = spc;
      const float dxs = interval_distance((float)p.ix + p.fx, tx0, tx0 + SPLAT_TX - 1, a.pnx);
      const float dys = interval_distance((float)p.iy + p.fy, ty0, ty0 + SPLAT_TY - 1, a.pny);
      int mask = 0;
      for (int i = 0; i < N_GAUSS; ++i) {
        const float* c = a.coef + (spc * N_GAUSS + i) * COEF_STRIDE;
        if (dxs <= c[3] && dys <= c[4]) mask |= 1 << i;
      }
      sp_mask[tid] = mask;
    }
    __syncthreads();
    for (int e = tid; e < mc * N_GAUSS * SPLAT_TX; e += 256) {
      const int m = e / (N_GAUSS * SPLAT_TX);
      const int i = (e / SPLAT_TX) % N_GAUSS;
      const int x = e % SPLAT_TX;
      const float* c = a.coef + (sp_spc[m] * N_GAUSS + i) * COEF_STRIDE;
      gx[m][i][x] = profile(tx0 + x, sp_pos[m].ix, sp_pos[m].fx, a.pnx, c[1], c[3], a.img_x);
    }
    for (int e = tid; e < mc * N_GAUSS * SPLAT_TY; e += 256) {
      const int m = e / (N_GAUSS * SPLAT_TY);
      const int i = (e / SPLAT_TY) % N_GAUSS;
      const int y = e % SPLAT_TY;
      const float* c = a.coef + (sp_spc[m] * N_GAUSS + i) * COEF_STRIDE;
      gy[m][i][y] = c[0] * profile(ty0 + y, sp_pos[m].iy, sp_pos[m].fy, a.pny, c[2], c[4], a.img_y);
    }
    __syncthreads();
    for (int m = 0; m < mc; ++m) {
      const int mask = sp_mask[m];
#pragma unroll
      for (int i = 0; i < N_GAUSS; ++i) {
        if (!(mask & (1 << i))) continue;
        const float2 g = *reinterpret_cast<const float2*>(&gy[m][i][ry]);
        const float4 h = *reinterpret_cast<const float4*>(&gx[m][i][cx]);
        acc0[0] += g.x * h.x;
        acc0[1] += g.x * h.y;
        acc0[2] += g.x * h.z;
        acc0[3] += g.x * h.w;
        acc1[0] += g.y * h.x;
        acc1[1] += g.y * h.y;
        acc1[2] += g.y * h.z;
        acc1[3] += g.y * h.w;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int y = ty0 + ry + r;
    if (y < a.pny) {
      float* out = a.V + (((size_t)fl * nsl + sl) * a.pny + y) * a.pnx;
      const float* acc = r == 0 ? acc0 : acc1;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (tx0 + cx + j < a.pnx) out[tx0 + cx + j] = acc[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass: [iFFT_x] -> * exp(i sigma V) -> FFT_x for RPI rows per block
// ---------------------------------------------------------------------------
template <int N, int VAR>
struct RowCfg {
  static constexpr int G = Plan<N>::G;
  static constexpr int cap_thr = 256 / G;
  static constexpr int cap_lds = 4096 / N > 0 ? 4096 / N : 1;
  static constexpr int RPI0 = cap_thr < cap_lds ? cap_thr : cap_lds;
  // largest power of two not above RPI0
  static constexpr int RPIB = RPI0 >= 64 ? 64 : RPI0 >= 32 ? 32 : RPI0 >= 16 ? 16 : RPI0 >= 8 ? 8
                            : RPI0 >= 4 ? 4 : RPI0 >= 2 ? 2 : 1;
  // variant 1 doubles the rows per block where threads and LDS allow
  static constexpr int RPI = (VAR == 1 && 2 * RPIB * G <= 1024 && 2 * RPIB * N <= 8192) ? 2 * RPIB : RPIB;
  static constexpr int THREADS = RPI * G;
};

template <int N, int VAR>
__global__ void __launch_bounds__((RowCfg<N, VAR>::THREADS)) k_row(PassTable tab) {
  using PL = Plan<N>;
  constexpr int G = PL::G;
  constexpr int RPI = RowCfg<N, VAR>::RPI;
  __shared__ float2 tw[N];
  __shared__ float2 rows[RPI][N];

  const int L = find_lane(tab, blockIdx.x);
  const PassArgs& a = tab.l[L].a;
  const int mode = tab.l[L].mode;
  const int lb = blockIdx.x - tab.l[L].block_start;

  for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = a.tw_x[i];
  const int g = threadIdx.x / G;
  const int t = threadIdx.x % G;
  float2* buf = rows[g];

  const long total = (long)a.n_probes * a.fb * a.ny;
  const long rid = (long)lb * RPI + g;
  const bool active = rid < total;
  int p = 0, fl = 0, y = 0;
  float2* row = nullptr;
  if (active) {
    const long w = rid / a.ny;
    y = (int)(rid % a.ny);
    p = (int)(w / a.fb);
    fl = (int)(w % a.fb);
    row = a.exit + (((size_t)p * a.n_frames + a.f0 + fl) * a.ny + y) * (size_t)N;
  }

  if (active) {
    if (mode == ROW_FIRST) {
      if (a.plane) {
        for (int x = t; x < N; x += G) buf[x] = make_float2(a.plane_amp, 0.f);
      } else {
        const float2* src = a.probe0 + ((size_t)p * a.ny + y) * (size_t)N;
        for (int x = t; x < N; x += G) buf[x] = src[x];
      }
    } else {
      for (int x = t; x < N; x += G) buf[x] = row[x];
    }
  }
  __syncthreads();
  if (mode != ROW_FIRST) StagesIP<N, G, true, 1, typename PL::R>::run(buf, tw, t);
  if (mode == ROW_INVERSE_ONLY) {
    if (active)
      for (int x = t; x < N; x += G) row[x] = buf[x];
    return;
  }
  if (active) {
    const int ox = a.plane ? 0 : a.origin[2 * p];
    const int oy = a.plane ? 0 : a.origin[2 * p + 1];
    int yy = oy + y;
    if (yy >= a.pny) yy -= a.pny;
    const float* vrow =
        a.V + (((size_t)fl * a.v_slices + (a.slice - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
    for (int x = t; x < N; x += G) {
      int xx = ox + x;
      if (xx >= a.pnx) xx -= a.pnx;
      float sn, cs;
      sincosf(a.sigma * vrow[xx], &sn, &cs);
      buf[x] = cmul(buf[x], make_float2(cs, sn));
    }
  }
  __syncthreads();
  StagesIP<N, G, false, 1, typename PL::R>::run(buf, tw, t);
  if (active)
    for (int x = t; x < N; x += G) row[x] = buf[x];
}

// ---------------------------------------------------------------------------
// Column pass: FFT_y -> * P -> [iFFT_y] on CT adjacent columns per block
// ---------------------------------------------------------------------------
template <int N, int VAR>
struct ColCfg {
  static constexpr int G = Plan<N>::G;
  static constexpr int CTB = N <= 512 ? COL_CT : COL_CT / 2;
  static constexpr int CT = VAR == 1 ? CTB : CTB / 2;
  static constexpr int LD = N + 1;  // padded column stride in LDS
  static constexpr int THREADS = G * CT;
};

template <int N, int VAR>
__global__ void __launch_bounds__((ColCfg<N, VAR>::THREADS)) k_col(PassTable tab) {
  using PL = Plan<N>;
  constexpr int G = PL::G;
  constexpr int CT = ColCfg<N, VAR>::CT;
  constexpr int LD = ColCfg<N, VAR>::LD;
  __shared__ float2 tw[N];
  __shared__ float2 cols[CT * LD];

  const int tile_g = xcd_remap(blockIdx.x, gridDim.x);
  const int L = find_lane(tab, tile_g);
  const PassArgs& a = tab.l[L].a;
  const int mode = tab.l[L].mode;
  const int tile = tile_g - tab.l[L].block_start;

  for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = a.tw_y[i];
  const int tiles_per_wave = a.nx / CT;
  const int w = tile / tiles_per_wave;
  const int x0 = (tile % tiles_per_wave) * CT;
  const int p = w / a.fb;
  const int fl = w % a.fb;
  float2* wave = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;

  for (int e = threadIdx.x; e < CT * N; e += blockDim.x) {
    const int c = e % CT, yy = e / CT;
    cols[c * LD + yy] = wave[(size_t)yy * a.nx + x0 + c];
  }
  __syncthreads();
  const int c = threadIdx.x / G;
  const int t = threadIdx.x % G;
  float2* buf = cols + c * LD;
  if (mode == COL_INVERSE_ONLY) {
    StagesIP<N, G, true, 1, typename PL::R>::run(buf, tw, t);
  } else {
    StagesIP<N, G, false, 1, typename PL::R>::run(buf, tw, t);
    const float2 pxv = a.px[x0 + c];
    for (int yy = t; yy < N; yy += G) buf[yy] = cmul(buf[yy], cmul(pxv, a.py[yy]));
    __syncthreads();
    if (mode == COL_REGULAR) StagesIP<N, G, true, 1, typename PL::R>::run(buf, tw, t);
  }
  for (int e = threadIdx.x; e < CT * N; e += blockDim.x) {
    const int cc = e % CT, yy = e / CT;
    wave[(size_t)yy * a.nx + x0 + cc] = cols[cc * LD + yy];
  }
}

// ---------------------------------------------------------------------------
// Time stage: FP64 frame mean + subtraction, time FFT, |.|^2 / F^2
// ---------------------------------------------------------------------------
constexpr int TIME_G = 64;        // threads per k column (one wavefront)
constexpr int TIME_LDS_C = 2048;  // complex values per ping-pong buffer

__global__ void __launch_bounds__(256) k_time(TimeArgs a) {
  extern __shared__ float2 sm[];
  const int F = a.n_frames;
  const int KT = a.kt;
  float2* tw = sm;
  float2* bufA = sm + F;
  float2* bufB = bufA + KT * F;
  __shared__ double red[2][4][TIME_G];

  for (int i = threadIdx.x; i < F; i += blockDim.x) tw[i] = a.tw[i];
  const int tiles_per_probe = a.n_k / KT;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int p = tile / tiles_per_probe;
  const int k0 = (tile % tiles_per_probe) * KT;
  const float2* src = a.exit + (size_t)p * F * a.n_k + k0;
  for (int e = threadIdx.x; e < KT * F; e += blockDim.x) {
    const int c = e % KT, f = e / KT;
    bufA[c * F + f] = src[(size_t)f * a.n_k + c];
  }
  __syncthreads();
  const int c = threadIdx.x / TIME_G;
  const int t = threadIdx.x % TIME_G;
  float2* col = bufA + c * F;
  // FP64 mean over frames (fixed summation order: strided partial sums, tree)
  double sr = 0.0, si = 0.0;
  for (int f = t; f < F; f += TIME_G) {
    sr += (double)col[f].x;
    si += (double)col[f].y;
  }
  red[0][c][t] = sr;
  red[1][c][t] = si;
  __syncthreads();
  for (int h = TIME_G / 2; h > 0; h >>= 1) {
    if (t < h) {
      red[0][c][t] += red[0][c][t + h];
      red[1][c][t] += red[1][c][t + h];
    }
    __syncthreads();
  }
  const double mr = red[0][c][0] / (double)F;
  const double mi = red[1][c][0] / (double)F;
  for (int f = t; f < F; f += TIME_G) {
    const float2 v = col[f];
    col[f] = make_float2((float)((double)v.x - mr), (float)((double)v.y - mi));
  }
  __syncthreads();
  float2* res = stockham_rt<false>(F, bufA + c * F, bufB + c * F, tw, t, TIME_G);
  // res is bufA- or bufB-based for every column alike (same stage count)
  const bool inA = (res == bufA + c * F);
  float2* resbase = inA ? bufA : bufB;
  float* dst = a.spec + (size_t)p * a.n_bins * a.n_k + k0;
  for (int e = threadIdx.x; e < KT * a.n_bins; e += blockDim.x) {
    const int cc = e % KT, m = e / KT;
    const float2 v = resbase[cc * F + m];
    dst[(size_t)m * a.n_k + cc] = (v.x * v.x + v.y * v.y) * a.inv_f2;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define TACAW_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) \
  X(640) X(768) X(1024)

bool grid_supported(int n) {
  switch (n) {
#define CASE(NN) case NN:
    TACAW_SIZES(CASE)
#undef CASE
    return true;
    default:
      return false;
  }
}

template <int N, int VAR>
static hipError_t row_launch(PassTable& t, hipStream_t s) {
  constexpr int RPI = RowCfg<N, VAR>::RPI;
  int blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    const long total = (long)a.n_probes * a.fb * a.ny;
    t.l[i].block_start = blocks;
    blocks += (int)((total + RPI - 1) / RPI);
  }
  hipLaunchKernelGGL((k_row<N, VAR>), dim3(blocks), dim3(RowCfg<N, VAR>::THREADS), 0, s, t);
  return hipGetLastError();
}

template <int N, int VAR>
static hipError_t col_launch(PassTable& t, hipStream_t s) {
  constexpr int CT = ColCfg<N, VAR>::CT;
  int blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.nx % CT != 0) return hipErrorInvalidValue;
    t.l[i].block_start = blocks;
    blocks += a.n_probes * a.fb * (a.nx / CT);
  }
  hipLaunchKernelGGL((k_col<N, VAR>), dim3(blocks), dim3(ColCfg<N, VAR>::THREADS), 0, s, t);
  return hipGetLastError();
}

static bool same_grid(const PassLane* lanes, int n) {
  for (int i = 1; i < n; ++i)
    if (lanes[i].a.nx != lanes[0].a.nx || lanes[i].a.ny != lanes[0].a.ny) return false;
  return true;
}

hipError_t launch_row_lanes(const PassLane* lanes, int n, int variant, hipStream_t s) {
  if (n < 1 || n > MAX_LANES || !same_grid(lanes, n)) return hipErrorInvalidValue;
  PassTable t{};
  t.n = n;
  for (int i = 0; i < n; ++i) t.l[i] = lanes[i];
  switch (lanes[0].a.nx) {
#define CASE(NN) \
  case NN: return variant ? row_launch<NN, 1>(t, s) : row_launch<NN, 0>(t, s);
    TACAW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_col_lanes(const PassLane* lanes, int n, int variant, hipStream_t s) {
  if (n < 1 || n > MAX_LANES || !same_grid(lanes, n)) return hipErrorInvalidValue;
  PassTable t{};
  t.n = n;
  for (int i = 0; i < n; ++i) t.l[i] = lanes[i];
  switch (lanes[0].a.ny) {
#define CASE(NN) \
  case NN: return variant ? col_launch<NN, 1>(t, s) : col_launch<NN, 0>(t, s);
    TACAW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_row_pass(const PassArgs& a, int mode, hipStream_t s) {
  PassLane l{};
  l.a = a;
  l.mode = mode;
  return launch_row_lanes(&l, 1, 1, s);
}

hipError_t launch_col_pass(const PassArgs& a, int mode, hipStream_t s) {
  PassLane l{};
  l.a = a;
  l.mode = mode;
  return launch_col_lanes(&l, 1, 1, s);
}

hipError_t launch_splat_lanes(const SplatLane* lanes, int n, hipStream_t s) {
  if (n < 1 || n > MAX_LANES) return hipErrorInvalidValue;
  SplatTable t{};
  t.n = n;
  int blocks = 0;
  for (int i = 0; i < n; ++i) {
    t.l[i] = lanes[i];
    t.l[i].block_start = blocks;
    const SplatArgs& a = lanes[i].a;
    blocks += a.tiles_x * a.tiles_y * lanes[i].n_slices_launch * a.fb;
  }
  hipLaunchKernelGGL(k_splat, dim3(blocks), dim3(256), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_splat(const SplatArgs& a, int n_slices_launch, hipStream_t s) {
  SplatLane l{};
  l.a = a;
  l.n_slices_launch = n_slices_launch;
  return launch_splat_lanes(&l, 1, s);
}

int time_stage_kt(int n_frames, int n_k) {
  int kt = 4;
  while (kt > 1 && (kt * n_frames > TIME_LDS_C || n_k % kt != 0)) kt >>= 1;
  return kt;
}

hipError_t launch_time_stage(const TimeArgs& a, hipStream_t s) {
  if (a.n_k % a.kt != 0 || a.kt * a.n_frames > TIME_LDS_C) return hipErrorInvalidValue;
  const size_t lds = (size_t)(a.n_frames + 2 * a.kt * a.n_frames) * sizeof(float2);
  const long blocks = (long)a.n_probes * (a.n_k / a.kt);
  dim3 grid((unsigned)blocks), block(a.kt * TIME_G);
  hipLaunchKernelGGL(k_time, grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

hipError_t launch_prop_factor(float2* out, int n, double d, double lam, double dz, double scale,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_prop_factor, dim3((n + 255) / 256), dim3(256), 0, s, out, n, d, lam, dz, scale);
  return hipGetLastError();
}

hipError_t launch_aperture_count(int* count, int nx, int ny, double dx, double dy, double lam,
                                 double alpha, hipStream_t s) {
  const int n = nx * ny;
  hipLaunchKernelGGL(k_aperture_count, dim3((n + 255) / 256), dim3(256), 0, s, count, nx, ny, dx, dy,
                     lam, alpha);
  return hipGetLastError();
}

hipError_t launch_probe_fill(float2* out, const double* rloc, const int* count, int n_probes, int nx,
                             int ny, double dx, double dy, double lam, double alpha, hipStream_t s) {
  const size_t n = (size_t)nx * ny * n_probes;
  hipLaunchKernelGGL(k_probe_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, rloc, count,
                     n_probes, nx, ny, dx, dy, lam, alpha);
  return hipGetLastError();
}

}  // namespace tacaw
