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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "fft_engine.h"
#include "tacaw_internal.h"

namespace tacaw {

// Timing events for the next main-kernel launch on this thread: when set, the
// launch records them itself (start and end of the kernel) instead of separate
// event packets around it.
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}
#define TACAW_LAUNCH(K, GRID, BLOCK, SHM, S, ...)                                   \
  do {                                                                              \
    hipEvent_t e0_ = t_ev_start, e1_ = t_ev_stop;                                   \
    t_ev_start = t_ev_stop = nullptr;                                               \
    if (e0_)                                                                        \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SHM, S, e0_, e1_, 0, __VA_ARGS__);      \
    else                                                                            \
      hipLaunchKernelGGL(K, GRID, BLOCK, SHM, S, __VA_ARGS__);                      \
  } while (0)

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
// chi(k) of the polar aberration coefficients, in radians
__device__ double aberration_chi(double kx, double ky, double lam, const Aberrations& ab) {
  constexpr int NM[N_ABERR][2] = {{1, 0}, {1, 2}, {2, 1}, {2, 3}, {3, 0}, {3, 2}, {3, 4},
                                  {4, 1}, {4, 3}, {4, 5}, {5, 0}, {5, 2}, {5, 4}, {5, 6}};
  const double alpha = lam * sqrt(kx * kx + ky * ky);
  const double phi = atan2(ky, kx);
  double chi = 0.0;
#pragma unroll
  for (int i = 0; i < N_ABERR; ++i) {
    double ap = alpha;   // alpha^(n+1)
#pragma unroll
    for (int q = 0; q < NM[i][0]; ++q) ap *= alpha;
    chi += ab.c[i] * ap / (NM[i][0] + 1) * cos(NM[i][1] * (phi - ab.phi[i]));
  }
  return 2.0 * M_PI / lam * chi;
}

__global__ void k_probe_fill(float2* out, const double* rloc, const int* count, int n_probes, int nx,
                             int ny, double dx, double dy, double lam, double alpha, Aberrations ab) {
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
    if (ab.on) {   // times exp(-i chi)
      double sa, ca;
      sincos(-aberration_chi(kx, ky, lam, ab), &sa, &ca);
      const double c2 = c * ca - s * sa;
      s = s * ca + c * sa;
      c = c2;
    }
    v = make_float2((float)(amp * c), (float)(amp * s));
  }
  out[i] = v;
}

// Orders LDS writes and reads of the lanes of one wavefront (no workgroup
// barrier needed when only that wavefront touches the memory).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exp(i phi) for the transmission function: the argument is reduced to
// [-1/2, 1/2) revolutions exactly (subtracting an integer), then the hardware
// sine and cosine (absolute error ~1.6e-7 there) are used.
__device__ __forceinline__ float2 phase_factor(float phi) {
  float rev = phi * 0.15915494309189535f;
  rev -= rintf(rev);
  return make_float2(__builtin_amdgcn_cosf(rev), __builtin_amdgcn_sinf(rev));
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
// pixel distance from grid node `node` (0 <= node < n + tile) to an atom at
// pixel ipos + fpos (0 <= ipos < n).  No integer division: node - ipos lies in
// (-n, 2n).  exp2 of an argument below -26.6 (the 1e-8 cutoff) is never
// evaluated, so the raw hardware exp2 is accurate here.
__device__ __forceinline__ float profile(int node, int ipos, float fpos, int n, float e2, float rc,
                                         int img) {
  int di = node - ipos;
  if (di >= n) di -= n;
  if (di < 0) di += n;
  if (di >= n - n / 2) di -= n;  // di in [-(n/2), n - n/2)
  const float d0 = (float)di - fpos;
  if (img == 0) return fabsf(d0) <= rc ? __builtin_amdgcn_exp2f(-e2 * d0 * d0) : 0.f;
  float g = 0.f;
  for (int k = -img; k <= img; ++k) {
    const float d = d0 + (float)(k * n);
    if (fabsf(d) <= rc) g += __builtin_amdgcn_exp2f(-e2 * d * d);
  }
  return g;
}

// Potentials: each wavefront computes one 32 x 32 tile of V for one slice
// and up to `fpw` frames (four wavefronts per workgroup, independent after the
// coefficients are staged).  V_tile = sum over the tile's candidate (atom,
// term) pairs, from the planner's per-tile lists, of outer(row profile, column
// profile): the 2D Gaussian of one term and its periodic images factor into x
// and y parts.  Pairs go in rounds of 32: lanes 0-31 build the column profiles
// and lanes 32-63 the row profiles (scaled by the term's amplitude), node-major
// in LDS; then v_mfma_f32_16x16x4f32 adds four pairs per instruction to each
// of the tile's four 16 x 16 quarters (FP32 products and sums).  Positions of
// the first rounds are prefetched one frame ahead.  Pair order and instruction
// sequence are fixed, so the result is deterministic.
// IZ: per-frame slice binning (lanes carry a frame-slice table); a separate
// instantiation keeps the check out of the default kernel.
// Profile fill of one round: NPL nodes per lane.  Lanes form 64 / NPL parts
// of NPL lanes (one pair each); the first half of the parts fill column
// profiles (unit amplitude), the second half row profiles (the term's
// amplitude), node-major in LDS.  Pairs mp .. mp4 - 1 get zeros (the MFMA
// steps take four pairs at a time); FULL: mp = NPL, no lane is idle.
template <int NPL, int PS, bool IZ, bool FULL>
__device__ __forceinline__ void splat_fill(float (*gx)[PS], float (*gy)[PS], int lane, int mp, int mp4,
                                           const AtomPos& p, const float* c, int at, const SplatArgs& a, int s,
                                           size_t frame_off, int tx0, int ty0, bool simple_x, bool simple_y) {
  const int pr = lane % NPL;                      // pair of this lane
  const int part = lane / NPL;
  const bool along_y = part >= 32 / NPL;          // lanes 0-31: column profiles, 32-63: row profiles
  const int nbase = (part % (32 / NPL)) * NPL;    // first profile node of this lane
  float* dst = along_y ? &gy[nbase][pr] : &gx[nbase][pr];   // node nbase + j at dst[j * PS]
  if (FULL || pr < mp) {   // FULL: a round of MP pairs, every lane has one
    // per-frame binning: an atom outside this slice in this frame adds nothing
    const bool gone = IZ && a.fslice != nullptr && at >= 0 && a.fslice[frame_off + at] != s;
    // lanes 0-31 and 32-63 run the same instructions on their own axis
    const int n_ax = along_y ? a.pny : a.pnx;
    const int node0 = along_y ? ty0 : tx0;
    const int ip = along_y ? p.iy : p.ix;
    const float fp = along_y ? p.fy : p.fx;
    const float amp = along_y ? c[0] : 1.f;
    const float e2 = along_y ? c[2] : c[1];
    const float rc = along_y ? c[4] : c[3];
    if (along_y ? simple_y : simple_x) {
      int o = node0 - ip;
      if (o >= n_ax - n_ax / 2) o -= n_ax;
      if (o < -(n_ax / 2)) o += n_ax;
      // node j sits at d = j - u pixels from the atom, u = f - o.  Every
      // node of a tile the term's box reaches gets the exact value (beyond
      // the radius it is below 1e-8 of the peak, or underflows to 0; only
      // this image reaches the tile), which saves the cutoff test.  The
      // value amp 2^(-e2 d^2) is 2^(A x^2 + B x + C) with x = j - NPL/2
      // (centred, so the terms stay small), A = -e2, B = 2 e2 u',
      // C = log2(amp) - e2 u'^2, u' = u - NPL/2: two FMAs and one exp2
      // per node.
      const float up = fp - (float)(o + nbase) - (float)(NPL / 2);
      const float la = along_y ? c[5] : 0.f;
      const float qa = -e2, qb = 2.f * e2 * up;
      const float qc = IZ && gone ? -INFINITY : fmaf(-e2 * up, up, la);
#pragma unroll
      for (int x = 0; x < NPL; ++x) {
        const float xc = (float)(x - NPL / 2);
        dst[x * PS] = __builtin_amdgcn_exp2f(fmaf(qa, xc * xc, fmaf(qb, xc, qc)));
      }
    } else {
      const int img = along_y ? a.img_y : a.img_x;
      const float amp_f = IZ && gone ? 0.f : amp;
      for (int x = 0; x < NPL; ++x)
        dst[x * PS] = amp_f * profile(node0 + nbase + x, ip, fp, n_ax, e2, rc, img);
    }
  } else if (pr < mp4) {
#pragma unroll
    for (int x = 0; x < NPL; ++x) dst[x * PS] = 0.f;
  }
}

// a compile-time flag handed to a generic lambda (instantiates one body per value)
template <bool B>
struct Flag {
  static constexpr bool value = B;
};

template <int MP, bool IZ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_splat(SplatTable tab) {
  // MP pairs per round (32 or 16).  Lanes split into 64 / MP parts of MP
  // lanes; each part fills NPL = MP nodes of the column (x) or row (y)
  // profiles of the round's pairs (fewer nodes per lane in a short last
  // round).
  static_assert(MP == 32 || MP == 16, "round sizes 32 and 16");
  constexpr int NPL = MP;                 // profile nodes per lane in a full round
  // profiles in LDS as [node][pair], rows of PS floats: a full round's fill
  // instruction (32 lanes: consecutive pairs of one or two nodes) and an
  // MFMA operand read (16 nodes x 2 pairs) both hit 32 distinct banks
  constexpr int PS = MP == 32 ? MP + 2 : MP + 1;
  static_assert(SPLAT_TX == 32 && SPLAT_TY == 32, "MFMA tiling assumes 32 x 32 tiles");
  __shared__ __align__(16) float gxs[4][SPLAT_TX][PS];
  __shared__ float gys[4][SPLAT_TY][PS];
  __shared__ float coef_s[SPLAT_MAX_SPECIES * N_GAUSS * COEF_STRIDE];

  // the wave index is uniform across the wavefront: keep it (and what follows
  // from it: the work item, its tile range and frame count) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  // one work item (tile, slice, group of FPW frames) per wavefront; lanes of
  // the table start on block boundaries
  const int L = find_lane(tab, blockIdx.x);
  const SplatArgs& a = tab.l[L].a;
  const int nsl = tab.l[L].n_slices_launch;
  const int n_coef = a.n_species * N_GAUSS * COEF_STRIDE;
  const bool coef_in_lds = a.n_species <= SPLAT_MAX_SPECIES;
  if (coef_in_lds)
    for (int i = threadIdx.x; i < n_coef; i += blockDim.x) coef_s[i] = a.coef[i];
  __syncthreads();  // the only workgroup barrier: everything below is per wavefront
  const float* coef = coef_in_lds ? coef_s : a.coef;
  const int n_tiles = a.tiles_x * a.tiles_y;
  const int FPW = tab.l[L].fpw;  // frames per wavefront
  const int n_fg = (a.fb + FPW - 1) / FPW;
  const int item = (blockIdx.x - tab.l[L].block_start) * 4 + wave;
  if (item >= n_tiles * nsl * n_fg) return;
  const int tile = item % n_tiles;
  const int sl = (item / n_tiles) % nsl;
  const int fl0 = (item / (n_tiles * nsl)) * FPW;
  const int nf = min(FPW, a.fb - fl0);
  const int s = a.slice0 + sl;
  const int tx0 = (tile % a.tiles_x) * SPLAT_TX;
  const int ty0 = (tile / a.tiles_x) * SPLAT_TY;
  const int cs = a.tile_start[s * n_tiles + tile];
  const int ce = a.tile_start[s * n_tiles + tile + 1];
  const bool simple_x = a.img_x == 0 && 2 * (a.rcx + SPLAT_TX + 2) < a.pnx;
  const bool simple_y = a.img_y == 0 && 2 * (a.rcy + SPLAT_TY + 2) < a.pny;
  float (*gx)[PS] = gxs[wave];
  float (*gy)[PS] = gys[wave];
  typedef float v4f __attribute__((ext_vector_type(4)));
  // A round of mp pairs fills NPL nodes per lane when mp > MP/2, else NPL/2
  // (NPL/4 when mp <= MP/4 and MP/4 >= 8): lane l holds pair l mod (that
  // node count), so a short round does a half or a quarter of the exp2 work
  auto pair_of = [&](int mp) { return lane % (mp > MP / 2 ? MP : (mp > MP / 4 || MP / 4 < 8 ? MP / 2 : MP / 4)); };

  // per round: this lane's atom and coefficients are the same for every
  // frame; positions of the first PRE = 2 rounds are prefetched one frame
  // ahead
  constexpr int PRE = 2;
  int atom_r[PRE];
  int coef_r[PRE];
  AtomPos pn[PRE];
#pragma unroll
  for (int r = 0; r < PRE; ++r) {
    atom_r[r] = -1;
    coef_r[r] = 0;
    pn[r] = AtomPos{};
    const int c0 = cs + r * MP;
    const int pr = pair_of(min(MP, ce - c0));
    if (c0 + pr < ce) {
      const int entry = a.tile_atoms[c0 + pr];
      atom_r[r] = entry >> 3;
      coef_r[r] = (a.species[entry >> 3] * N_GAUSS + (entry & 7)) * COEF_STRIDE;
    }
  }
#pragma unroll
  for (int r = 0; r < PRE; ++r)
    if (atom_r[r] >= 0 && nf > 0) pn[r] = a.pos[(size_t)(a.f0 + fl0) * a.n_atoms + atom_r[r]];

  for (int k = 0; k < nf; ++k) {
    const int fl = fl0 + k;
    const size_t frame_off = (size_t)(a.f0 + fl) * a.n_atoms;
    v4f acc[4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    // one round: pairs c0 .. c0 + mp - 1, this lane holding pair c0 + pair_of(mp)
    // (position p, coefficient offset coff, atom at)
    // (full: a round of MP pairs known at compile time, its MFMA steps unrolled)
    auto round = [&](auto full, int c0, AtomPos p, int coff, int at) {
      constexpr bool FULL = decltype(full)::value;
      const int mp = FULL ? MP : min(MP, ce - c0);
      const int mp4 = FULL ? MP : (mp + 3) & ~3;
      wave_lds_sync();  // the previous round's MFMA reads are done
      // the lane holds pair pair_of(mp) of the round
      if (FULL || mp == MP) {
        splat_fill<NPL, PS, IZ, true>(gx, gy, lane, mp, mp4, p, coef + coff, at, a, s, frame_off, tx0, ty0,
                                      simple_x, simple_y);
      } else if (mp > MP / 2) {
        splat_fill<NPL, PS, IZ, false>(gx, gy, lane, mp, mp4, p, coef + coff, at, a, s, frame_off, tx0, ty0,
                                       simple_x, simple_y);
      } else {
        if (mp > MP / 4 || MP / 4 < 8)
          splat_fill<NPL / 2, PS, IZ, false>(gx, gy, lane, mp, mp4, p, coef + coff, at, a, s, frame_off, tx0, ty0,
                                             simple_x, simple_y);
        else
          splat_fill<(MP / 4 < 8 ? 8 : NPL / 4), PS, IZ, false>(gx, gy, lane, mp, mp4, p, coef + coff, at, a, s,
                                                                frame_off, tx0, ty0, simple_x, simple_y);
      }
      wave_lds_sync();
      // V[r][c] += sum_k gy[k][r] gx[k][c] over four 16 x 16 quarters; A is 16 x 4
      // (row lane % 16, k lane / 16), B is 4 x 16 (k lane / 16, column lane % 16)
#pragma unroll
      for (int k0 = 0; k0 < (FULL ? MP : mp4); k0 += 4) {
        const int kk = k0 + lane / 16;
        const float a0 = gy[lane % 16][kk], a1 = gy[16 + lane % 16][kk];
        const float b0 = gx[lane % 16][kk], b1 = gx[16 + lane % 16][kk];
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[3], 0, 0, 0);
      }
    };
    // the first two rounds take the positions prefetched a frame ahead and
    // prefetch the next frame's; later rounds load their own
    const AtomPos p0 = pn[0], p1 = pn[1];
    if (k + 1 < nf) {
      if (atom_r[0] >= 0) pn[0] = a.pos[frame_off + a.n_atoms + atom_r[0]];
      if (atom_r[1] >= 0) pn[1] = a.pos[frame_off + a.n_atoms + atom_r[1]];
    }
    if (ce - cs >= MP)
      round(Flag<true>{}, cs, p0, coef_r[0], atom_r[0]);
    else if (cs < ce)
      round(Flag<false>{}, cs, p0, coef_r[0], atom_r[0]);
    if (cs + MP < ce) round(Flag<false>{}, cs + MP, p1, coef_r[1], atom_r[1]);
    for (int c0 = cs + 2 * MP; c0 < ce; c0 += MP) {
      AtomPos p{};
      int coff = 0, at = -1;
      const int pr = pair_of(min(MP, ce - c0));
      if (c0 + pr < ce) {
        const int entry = a.tile_atoms[c0 + pr];
        at = entry >> 3;
        p = a.pos[frame_off + at];
        coff = (a.species[at] * N_GAUSS + (entry & 7)) * COEF_STRIDE;
      }
      round(Flag<false>{}, c0, p, coff, at);
    }
    // D layout: lane holds rows 4 (lane / 16) + j, j < 4, of column lane % 16
    float* out = a.V + ((size_t)fl * nsl + sl) * a.pny * a.pnx;
    if (MP == 32 && a.pnx % 4 == 0) {
      // through this wavefront's profile buffer (32 x 32 floats, rows of 32,
      // bit 4 of the column flipped in odd quads of rows so that both 16-lane
      // groups of a write hit distinct banks), then whole 128-byte rows with
      // 16-byte stores: eight lanes per row, eight rows per instruction
      float* T = &gx[0][0];
      wave_lds_sync();  // the last round's MFMA reads are done
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 16 * (q >> 1) + 4 * (lane / 16) + j;
          const int col = 16 * (q & 1) + lane % 16;
          T[row * 32 + (col ^ (((row >> 2) & 1) << 4))] = acc[q][j];
        }
      wave_lds_sync();
      const int col = 4 * (lane % 8);
      const int x = tx0 + col;
#pragma unroll
      for (int k8 = 0; k8 < 4; ++k8) {
        const int row = lane / 8 + 8 * k8;
        const float4 v = *reinterpret_cast<const float4*>(&T[row * 32 + (col ^ (((row >> 2) & 1) << 4))]);
        const int y = ty0 + row;
        if (y < a.pny && x < a.pnx) *reinterpret_cast<float4*>(&out[(size_t)y * a.pnx + x]) = v;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int x = tx0 + 16 * (q & 1) + lane % 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int y = ty0 + 16 * (q >> 1) + 4 * (lane / 16) + j;
          if (y < a.pny && x < a.pnx) out[(size_t)y * a.pnx + x] = acc[q][j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The paper's reciprocal-space potential route: structure factors of a pair
// of slices on the MFMA units
// ---------------------------------------------------------------------------
// exp(-2 pi i m x / n) at x = ip + fp pixels (0 <= ip < n, 0 <= fp < 1):
// the integer part of m x is reduced exactly, the rest in FP32 revolutions.
// nyq: m is the Nyquist index -n/2 of an even side, which takes the cosine
// alone (the mean of the +n/2 and -n/2 terms).
__device__ __forceinline__ float2 sf_term(int m, int ip, float fp, int n, float inv_n, bool nyq) {
  // t = m ip mod n, exactly: |m ip| < 2^23, so it and its float are exact,
  // and the float quotient is at most one off (corrected)
  const int mi = m * ip;
  int t = mi - n * (int)floorf((float)mi * inv_n);
  t += t < 0 ? n : 0;
  t -= t >= n ? n : 0;
  float rev = ((float)t + (float)m * fp) * inv_n;
  rev -= rintf(rev);
  const float c = __builtin_amdgcn_cosf(rev);
  return make_float2(c, nyq ? 0.f : -__builtin_amdgcn_sinf(rev));
}

// signed frequency index of grid index i (numpy fftfreq order)
__device__ __forceinline__ int freq_index(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// sum_i a_i / (q2 + b_i) + c_i 2^(-d_i q2) for one species' coefficients
__device__ __forceinline__ float kform(const float* cf, float q2) {
  float ff = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    ff += cf[i] * __builtin_amdgcn_rcpf(q2 + cf[3 + i]) + cf[6 + i] * __builtin_amdgcn_exp2f(-cf[9 + i] * q2);
  return ff;
}

// At the corner frequency where both sides are even and both indices are
// Nyquist, the real part of f exp(-2 pi i (mx x / Lx + my y / Ly)) is
// f (cos a cos b - sin a sin b), while the per-axis cosines give the first
// product only.  Returns sum over the slice's atoms of f_z sin a sin b, to be
// subtracted there.
__device__ float corner_sin_sum(const KPotArgs& a, int f, int s, float q2c) {
  const int mx = -(a.pnx / 2), my = -(a.pny / 2);
  const float inv_nx = 1.f / (float)a.pnx, inv_ny = 1.f / (float)a.pny;
  float acc = 0.f;
  for (int z = 0; z < a.n_species; ++z) {
    const int js = a.ks_start[s * a.n_species + z], je = a.ks_start[s * a.n_species + z + 1];
    float sz = 0.f;
    for (int c = js; c < je; ++c) {
      const size_t o = (size_t)f * a.n_atoms + a.ks_atoms[c];
      if (a.fslice != nullptr && a.fslice[o] != s) continue;
      const AtomPos p = a.pos[o];
      float rx = ((float)((mx * p.ix) % a.pnx) + (float)mx * p.fx) * inv_nx;
      float ry = ((float)((my * p.iy) % a.pny) + (float)my * p.fy) * inv_ny;
      rx -= rintf(rx);
      ry -= rintf(ry);
      sz += __builtin_amdgcn_sinf(rx) * __builtin_amdgcn_sinf(ry);
    }
    if (je > js) acc += kform(a.kcoef + z * KP_NCOEF, q2c) * sz;
  }
  return acc;
}

// One workgroup computes a KP_TY x KP_TX tile (rows ky index r0 .., columns
// kx index c0 ..) of W for one frame and one slice pair.  For each slice and
// species, the tile's structure factor S(k) = sum_j Ey_j(ky) Ex_j(kx) is a
// complex product of a [rows x atoms] and an [atoms x columns] matrix, taken
// KP_K atoms at a time: the workgroup writes the stage's exponentials to LDS
// (real and imaginary planes, [row or column][atom]), then each wavefront
// runs v_mfma_f32_16x16x4f32 on its 32 x 32 part (four 16 x 16 blocks, three
// real products per complex one: Re Re, Im Im and (Re + Im)(Re + Im), whose
// combinations give the real part Re Re - Im Im and the imaginary part).  The species' form
// factor multiplies the finished sum element by element.  Atoms are taken in
// list order and the instruction sequence is fixed, so results are
// deterministic.
__global__ void __launch_bounds__(256) k_kpot(KPotArgs a) {
  constexpr int PS = KP_K + 1;   // LDS row stride (floats)
  __shared__ float eyr[KP_TY][PS], eyi[KP_TY][PS];
  __shared__ float exr[KP_TX][PS], exi[KP_TX][PS];
  typedef float v4f __attribute__((ext_vector_type(4)));
  static_assert(KP_TY == 32 && KP_TX == 128 && KP_K == 16, "tile shape of the MFMA layout below");

  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  int b = blockIdx.x;
  const int ct = b % a.col_tiles;
  b /= a.col_tiles;
  const int rt = b % a.row_tiles;
  b /= a.row_tiles;
  const int q = b % a.npairs;
  const int fl = b / a.npairs;
  const int f = a.f0 + fl;
  const int r0 = rt * KP_TY, c0 = ct * KP_TX;
  const int half_rows = a.pny / 2 + 1;   // rows 0 .. pny/2 computed here
  const float inv_nx = 1.f / (float)a.pnx, inv_ny = 1.f / (float)a.pny;
  const bool even_x = (a.pnx & 1) == 0, even_y = (a.pny & 1) == 0;

  // exponential slots of this thread: atom gj of the stage; rows gr + 16 i
  // (i < 2) and columns gr + 16 i (i < 8) of the tile
  const int gj = tid % KP_K, gr = tid / KP_K;
  int my[2], mx[8];
  bool ok_y[2], ok_x[8], nyq_y[2], nyq_x[8];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = r0 + gr + 16 * i;
    ok_y[i] = row < half_rows;
    my[i] = freq_index(row, a.pny);
    nyq_y[i] = even_y && 2 * row == a.pny;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int col = c0 + gr + 16 * i;
    ok_x[i] = col < a.pnx;
    mx[i] = freq_index(col, a.pnx);
    nyq_x[i] = even_x && 2 * col == a.pnx;
  }

  // |k|^2 of the 16 output elements of this lane: block u (rows 16 (u >> 1),
  // columns 32 wave + 16 (u & 1)), element e at row 4 (lane / 16) + e of the
  // block, column lane % 16
  float q2[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = c0 + 32 * wave + 16 * (u & 1) + lane % 16;
    const float kx = (float)freq_index(col, a.pnx) * a.kx_unit;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + 16 * (u >> 1) + 4 * (lane / 16) + e;
      const float ky = (float)freq_index(row, a.pny) * a.ky_unit;
      q2[u][e] = kx * kx + ky * ky;
    }
  }

  v4f vs[2][4][2];   // [slice of the pair][block][re, im]
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 4; ++u) vs[h][u][0] = vs[h][u][1] = v4f{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = a.slice0 + 2 * q + h;
    if (s >= a.n_slices) break;   // the last pair of an odd count has one slice
    for (int z = 0; z < a.n_species; ++z) {
      const int js = a.ks_start[s * a.n_species + z], je = a.ks_start[s * a.n_species + z + 1];
      if (js == je) continue;
      // three real products per complex one: P1 = Ar Br, P2 = Ai Bi,
      // P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2
      v4f acc[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u][0] = acc[u][1] = acc[u][2] = v4f{0.f, 0.f, 0.f, 0.f};
      for (int c = js; c < je; c += KP_K) {
        bool on = gj < je - c;
        AtomPos p{};
        if (on) {
          const int at = a.ks_atoms[c + gj];
          const size_t o = (size_t)f * a.n_atoms + at;
          p = a.pos[o];
          if (a.fslice != nullptr && a.fslice[o] != s) on = false;   // elsewhere in this frame
        }
        __syncthreads();   // the previous stage's operand reads are done
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          float2 e = make_float2(0.f, 0.f);
          if (on && ok_y[i]) e = sf_term(my[i], p.iy, p.fy, a.pny, inv_ny, nyq_y[i]);
          eyr[gr + 16 * i][gj] = e.x;
          eyi[gr + 16 * i][gj] = e.y;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          float2 e = make_float2(0.f, 0.f);
          if (on && ok_x[i]) e = sf_term(mx[i], p.ix, p.fx, a.pnx, inv_nx, nyq_x[i]);
          exr[gr + 16 * i][gj] = e.x;
          exi[gr + 16 * i][gj] = e.y;
        }
        __syncthreads();
        // A is 16 x 4 (row lane % 16, atom lane / 16), B is 4 x 16 (atom lane / 16,
        // column lane % 16); unused atom slots hold zeros
        const int kn = min(KP_K, ((je - c) + 3) & ~3);
        for (int k0 = 0; k0 < kn; k0 += 4) {
          const int kk = k0 + lane / 16;
          float ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            ar[v] = eyr[16 * v + lane % 16][kk];
            ai[v] = eyi[16 * v + lane % 16][kk];
            br[v] = exr[32 * wave + 16 * v + lane % 16][kk];
            bi[v] = exi[32 * wave + 16 * v + lane % 16][kk];
            as[v] = ar[v] + ai[v];
            bs[v] = br[v] + bi[v];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ry = u >> 1, cx = u & 1;
            acc[u][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ry], br[cx], acc[u][0], 0, 0, 0);
            acc[u][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[ry], bi[cx], acc[u][1], 0, 0, 0);
            acc[u][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[ry], bs[cx], acc[u][2], 0, 0, 0);
          }
        }
      }
      // V(k) += f_z(|k|) S_z(k): f = sum_i a_i / (q^2 + b_i) + c_i 2^(-d_i q^2)
      // (a, c carry C / A and d carries log2 e)
      const float* cf = a.kcoef + z * KP_NCOEF;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ff = kform(cf, q2[u][e]);
          const float re = acc[u][0][e] - acc[u][1][e];
          const float im = acc[u][2][e] - acc[u][0][e] - acc[u][1][e];
          vs[h][u][0][e] = fmaf(ff, re, vs[h][u][0][e]);
          vs[h][u][1][e] = fmaf(ff, im, vs[h][u][1][e]);
        }
    }
  }

  // W(k) = A + i B and W(-k) = conj A + i conj B (A, B: the pair's slices)
  float2* out = a.W + ((size_t)fl * a.npairs + q) * (size_t)a.pnx * a.pny;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = c0 + 32 * wave + 16 * (u & 1) + lane % 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + 16 * (u >> 1) + 4 * (lane / 16) + e;
      if (row >= half_rows || col >= a.pnx) continue;
      float are = vs[0][u][0][e], bre = vs[1][u][0][e];
      const float aim = vs[0][u][1][e], bim = vs[1][u][1][e];
      if (even_x && even_y && 2 * row == a.pny && 2 * col == a.pnx) {   // the corner (both Nyquist)
        const int s = a.slice0 + 2 * q;
        are -= corner_sin_sum(a, f, s, q2[u][e]);
        if (s + 1 < a.n_slices) bre -= corner_sin_sum(a, f, s + 1, q2[u][e]);
      }
      out[(size_t)row * a.pnx + col] = make_float2(are - bim, aim + bre);
      if (row > 0 && 2 * row < a.pny) {
        const int mrow = a.pny - row, mcol = col == 0 ? 0 : a.pnx - col;
        out[(size_t)mrow * a.pnx + mcol] = make_float2(are + bim, bre - aim);
      }
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

  // row ids are below 2^31 (checked at launch)
  const int total = a.n_probes * a.fb * a.ny;
  const int rid = lb * RPI + g;
  const bool active = rid < total;
  int p = 0, fl = 0, y = 0;
  float2* row = nullptr;
  if (active) {
    const int w = rid / a.ny;
    y = rid - w * a.ny;
    p = w / a.fb;
    fl = w - p * a.fb;
    row = a.exit + (((size_t)p * a.n_frames + a.f0 + fl) * a.ny + y) * (size_t)N;
  }

  // N / G values per thread; global reads go CH at a time, all in flight
  // before their LDS writes
  constexpr int PER = N / G;
  constexpr int CH = PER < 8 ? PER : 8;
  auto load_row = [&](const float2* src) {
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += CH) {
      float2 v[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i0 + i < PER) v[i] = src[t + (i0 + i) * G];
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i0 + i < PER) buf[t + (i0 + i) * G] = v[i];
    }
  };
  if (active) {
    if (mode == ROW_FIRST) {
      if (a.plane) {
        for (int x = t; x < N; x += G) buf[x] = make_float2(a.plane_amp, 0.f);
      } else {
        load_row(a.probe0 + ((size_t)p * a.ny + y) * (size_t)N);
      }
    } else {
      load_row(row);
    }
  }
  __syncthreads();
  if (mode != ROW_FIRST) StagesIP<N, G, true, 1, typename PL::R>::run(buf, tw, t);
  if (mode == ROW_INVERSE_ONLY) {
    if (active && a.vout) {
      // two real planes (reciprocal-space potentials): real part, imaginary part
      const size_t plane = (size_t)a.ny * N;
      const size_t w = (size_t)p * a.n_frames + a.f0 + fl;
      float* o0 = a.vout + 2 * w * plane + (size_t)y * N;
      float* o1 = o0 + plane;
      for (int x = t; x < N; x += G) {
        o0[x] = buf[x].x;
        o1[x] = buf[x].y;
      }
    } else if (active) {
      for (int x = t; x < N; x += G) row[x] = buf[x];
    }
    return;
  }
  if (active) {
    const int ox = a.plane ? 0 : a.origin[2 * p];
    const int oy = a.plane ? 0 : a.origin[2 * p + 1];
    int yy = oy + y;
    if (yy >= a.pny) yy -= a.pny;
    const float* vrow =
        a.V + (((size_t)fl * a.v_slices + (a.slice - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += CH) {
      float vv[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i0 + i < PER) {
          int xx = ox + t + (i0 + i) * G;
          if (xx >= a.pnx) xx -= a.pnx;
          vv[i] = vrow[xx];
        }
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (i0 + i < PER) {
          const int x = t + (i0 + i) * G;
          buf[x] = cmul(buf[x], phase_factor(a.sigma * vv[i]));
        }
    }
  }
  __syncthreads();
  StagesIP<N, G, false, 1, typename PL::R>::run(buf, tw, t);
  if (active)
    for (int x = t; x < N; x += G) row[x] = buf[x];
}

// ---------------------------------------------------------------------------
// Row pass on registers (N = 64, 128, 256, 512; radix-8 stages, then radix 4
// where N needs it): one row per G = N/8 lanes inside one wavefront; lane t
// keeps the row values at x = t + G r (r < 8) in registers,
// which is both the first Stockham stage's input layout and the last stage's
// output layout, so global loads and stores are coalesced and only S-1 LDS
// exchanges per FFT remain, synchronised within the wavefront only.  Each
// wavefront walks over rows with a grid stride; stage twiddles stay in
// registers for all its rows.
// ---------------------------------------------------------------------------
template <int N>
struct R8 {
  // stage radices, radix 8 first (so every later stage stride is a multiple
  // of 8); each divides the 8 values a lane holds
  static constexpr int S = N == 64 ? 2 : (N == 128 || N == 256 || N == 512) ? 3 : 0;
  static constexpr int radix(int j) {
    return j == 0 ? 8 : N == 128 ? 4 : (N == 256 && j == 2) ? 4 : 8;
  }
  static constexpr int stride(int j) { return j == 0 ? 1 : stride(j - 1) * radix(j - 1); }
  static constexpr int G = N / 8;            // lanes per row
  static constexpr int RPW = 64 / G;         // rows per wavefront
  static_assert(S > 0 && G <= 64 && G % 8 == 0, "register FFT sizes: 64, 128, 256, 512");
  static_assert(S < 1 || stride(S - 1) * radix(S - 1) == N, "radices multiply to N");
};

// LDS layout of a row or column in the register kernels: element i sits in
// slot i + i/8 (one pad slot after every 8 values), so that the exchanges
// (stride-8 and stride-64 writes) and the transposes spread over all banks.
// padded(n) slots hold n elements.
constexpr int padded(int n) { return n + n / 8; }

// Stage twiddles of one lane: stage j with radix R and stride P runs Q = 8/R
// butterflies b = t + G q; input r of butterfly q takes W_{PR}^{r (b mod P)},
// stored at tw[j][q (R - 1) + r - 1].  Stage 0 (P = 1) has none.
template <int N>
__device__ __forceinline__ void reg_twiddles(float2 (&tw)[R8<N>::S][7], const float2* table, int t) {
  int P = R8<N>::radix(0);
#pragma unroll
  for (int j = 1; j < R8<N>::S; P *= R8<N>::radix(j), ++j) {
    const int R = R8<N>::radix(j), Q = 8 / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k = (t + R8<N>::G * q) % P;
#pragma unroll
      for (int r = 1; r < R; ++r) tw[j][q * (R - 1) + r - 1] = table[(r * k * (N / (P * R))) % N];
    }
  }
}

// Stage J of the register FFT and the stages after it.  x[r'] holds position
// t + G r'; butterfly q of a radix-R stage takes x[q + Q r], r < R, which sit
// at b + r N/R.  Outputs go to positions (b - k) R + k + r P, k = b mod P,
// through LDS, except after the last stage, where they already sit at
// t + G (q + Q r).
template <int N, bool INV, int J>
__device__ __forceinline__ void reg_fft_stage(float2 (&x)[8], float2* lds, const float2 (&tw)[R8<N>::S][7],
                                              int t) {
  constexpr int S = R8<N>::S, G = R8<N>::G;
  constexpr int R = R8<N>::radix(J), P = R8<N>::stride(J), Q = 8 / R;
  if constexpr (J > 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[J][q * (R - 1) + r - 1];
        x[q + Q * r] = INV ? cmulc(x[q + Q * r], w) : cmul(x[q + Q * r], w);
      }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = x[q + Q * r];
    dft<R, INV>(y);
#pragma unroll
    for (int r = 0; r < R; ++r) x[q + Q * r] = y[r];
  }
  if constexpr (J < S - 1) {
    static_assert(P == 1 ? R == 8 : P % 8 == 0, "padded write offsets");
    wave_lds_sync();  // earlier reads of lds by this wavefront are done
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      // base is a multiple of 8 when P = 1, and P is a multiple of 8 otherwise:
      // slot of base + r P is base + base/8 + (P + P/8) r
      const int b = t + G * q;
      const int k = b % P;
      const int base = (b - k) * R + k;
      const int wbase = base + (base >> 3);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[wbase + r * (P + P / 8)] = x[q + Q * r];
    }
    wave_lds_sync();
    // x[r'] from position t + G r': slot t + t/8 + (G + G/8) r'
    const int rbase = t + (t >> 3);
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = lds[rbase + r * (G + G / 8)];
    reg_fft_stage<N, INV, J + 1>(x, lds, tw, t);
  }
}

// One FFT on registers: x[r] at positions t + G r in and out.  lds: this
// row's scratch of padded(N) values.
template <int N, bool INV>
__device__ __forceinline__ void fft_r8(float2 (&x)[8], float2* lds, const float2 (&tw)[R8<N>::S][7], int t) {
  reg_fft_stage<N, INV, 0>(x, lds, tw, t);
}

// DEPTH 1: the next row's reads are in flight while a row is transformed
// (five wavefronts per SIMD); DEPTH 2: the next two rows' (three rotating
// register buffers, four wavefronts per SIMD).
template <int N, int DEPTH, bool VOUT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DEPTH == 1 ? 5 : 4)))
k_row_r8(PassTable tab) {
  constexpr int G = R8<N>::G;
  constexpr int RPW = R8<N>::RPW;
  constexpr int S = R8<N>::S;
  __shared__ float2 scratch[4][RPW][padded(N)];

  // lane L owns blocks [block_start, next lane's block_start), in proportion
  // to its rows
  const int L = find_lane(tab, blockIdx.x);
  const PassArgs& a = tab.l[L].a;
  const int mode = tab.l[L].mode;
  const int lb = blockIdx.x - tab.l[L].block_start;
  const int blocks_per_lane = (L + 1 < tab.n ? tab.l[L + 1].block_start : (int)gridDim.x) - tab.l[L].block_start;
  // wavefront-uniform: with one row per wavefront the row bookkeeping below
  // runs on the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int sub = RPW == 1 ? 0 : lane / G;   // row within the wavefront
  const int t = lane % G;
  float2* lds = scratch[wave][sub];

  float2 tw[S][7];
  reg_twiddles<N>(tw, a.tw_x, t);
  // row ids are below 2^31 (checked at launch)
  const int total = a.n_probes * a.fb * a.ny;
  const int stride = blocks_per_lane * 4 * RPW;
  const bool transmit = mode != ROW_INVERSE_ONLY;

  // global reads of one row (the wave values and the potential row values);
  // `out` receives the row's place in the exit store
  auto fetch = [&](int rid, float2 (&xv)[8], float (&vv)[8], float2*& out) {
    if (rid >= total) return;
    const int w = rid / a.ny;
    const int y = rid - w * a.ny;
    const int p = w / a.fb;
    const int fl = w - p * a.fb;
    float2* row = a.exit + (((size_t)p * a.n_frames + a.f0 + fl) * a.ny + y) * (size_t)N;
    out = row;
    if (mode == ROW_FIRST) {
      if (a.plane) {
#pragma unroll
        for (int r = 0; r < 8; ++r) xv[r] = make_float2(a.plane_amp, 0.f);
      } else {
        const float2* src = a.probe0 + ((size_t)p * a.ny + y) * (size_t)N;
#pragma unroll
        for (int r = 0; r < 8; ++r) xv[r] = src[t + r * G];
      }
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) xv[r] = row[t + r * G];
    }
    if (transmit) {
      const int ox = a.plane ? 0 : a.origin[2 * p];
      const int oy = a.plane ? 0 : a.origin[2 * p + 1];
      int yy = oy + y;
      if (yy >= a.pny) yy -= a.pny;
      const float* vrow =
          a.V + (((size_t)fl * a.v_slices + (a.slice - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
      if (ox == 0 && a.pnx == N) {   // plane wave, or a window at the origin: no wrap
#pragma unroll
        for (int r = 0; r < 8; ++r) vv[r] = vrow[t + r * G];
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          int xx = ox + t + r * G;
          if (xx >= a.pnx) xx -= a.pnx;
          vv[r] = vrow[xx];
        }
      }
    }
  };

  // transform one row held in (x, v) and store it to out (inverse-only rows
  // of the reciprocal-space potentials with vout set: the real and imaginary
  // parts to the two potential planes of the wave instead)
  auto transform = [&](float2 (&x)[8], const float (&v)[8], float2* out, int rid) {
    if (mode != ROW_FIRST) fft_r8<N, true>(x, lds, tw, t);
    if (transmit) {
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = cmul(x[r], phase_factor(a.sigma * v[r]));
      fft_r8<N, false>(x, lds, tw, t);
    }
    if (rid < total) {
      if (VOUT && !transmit && a.vout) {
        const int w = rid / a.ny;
        const int y = rid - w * a.ny;
        const int p = w / a.fb;
        const int fl = w - p * a.fb;
        const size_t plane = (size_t)a.ny * N;
        float* o0 = a.vout + 2 * ((size_t)p * a.n_frames + a.f0 + fl) * plane + (size_t)y * N;
        float* o1 = o0 + plane;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          o0[t + r * G] = x[r].x;
          o1[t + r * G] = x[r].y;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) out[t + r * G] = x[r];
      }
    }
  };
  int rid0 = (lb * 4 + wave) * RPW;
  if constexpr (DEPTH == 1) {
    float2 xn[8];
    float vn[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      xn[r] = make_float2(0.f, 0.f);
      vn[r] = 0.f;
    }
    float2* out_next = nullptr;
    fetch(rid0 + sub, xn, vn, out_next);
    for (; rid0 < total; rid0 += stride) {
      float2* out = out_next;
      float2 x[8];
      float v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        x[r] = xn[r];
        v[r] = vn[r];
      }
      fetch(rid0 + stride + sub, xn, vn, out_next);  // next row's reads overlap this row's arithmetic
      transform(x, v, out, rid0 + sub);
    }
  } else {
    // rows i, i+1, i+2 of this wavefront rotate through buffers A, B, C: while
    // one is transformed, the reads of the two after it are in flight
    float2 xa[8], xb[8], xc[8];
    float va[8], vb[8], vc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      xa[r] = xb[r] = xc[r] = make_float2(0.f, 0.f);
      va[r] = vb[r] = vc[r] = 0.f;
    }
    float2 *oa = nullptr, *ob = nullptr, *oc = nullptr;
    fetch(rid0 + sub, xa, va, oa);
    fetch(rid0 + stride + sub, xb, vb, ob);
    for (; rid0 < total; rid0 += 3 * stride) {
      fetch(rid0 + 2 * stride + sub, xc, vc, oc);
      transform(xa, va, oa, rid0 + sub);
      if (rid0 + stride >= total) break;
      fetch(rid0 + 3 * stride + sub, xa, va, oa);
      transform(xb, vb, ob, rid0 + stride + sub);
      if (rid0 + 2 * stride >= total) break;
      fetch(rid0 + 4 * stride + sub, xb, vb, ob);
      transform(xc, vc, oc, rid0 + 2 * stride + sub);
    }
  }
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

  // CT x N values, N / G per thread, loaded with every load of a chunk of up
  // to 16 in flight before the LDS writes
  constexpr int THREADS = ColCfg<N, VAR>::THREADS;
  constexpr int PER = CT * N / THREADS;
  constexpr int CH = PER < 16 ? PER : 16;
  static_assert(PER * THREADS == CT * N, "whole values per thread");
#pragma unroll
  for (int i0 = 0; i0 < PER; i0 += CH) {
    float2 v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (i0 + i < PER) {
        const int e = threadIdx.x + (i0 + i) * THREADS;
        v[i] = wave[(size_t)(e / CT) * a.nx + x0 + e % CT];
      }
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (i0 + i < PER) {
        const int e = threadIdx.x + (i0 + i) * THREADS;
        cols[(e % CT) * LD + e / CT] = v[i];
      }
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
// Column pass, uniform radix 8 (N = 64 or 512).  A block owns CT adjacent
// columns of one wave: it loads them coalesced into LDS (column stride
// N + 2 keeps the transposing writes and the column reads conflict-free),
// then each column is transformed by G = N/8 lanes of one wavefront on
// registers (FFT_y, * P, iFFT_y) with wavefront-local LDS exchanges, written
// back to its LDS column and stored coalesced.  Blocks walk over tiles with a
// grid stride (XCD-contiguous order), keeping their stage twiddles in
// registers.
// ---------------------------------------------------------------------------
template <int N, int WIDE>
struct C8 {
  static constexpr int G = N / 8;               // lanes per column
  static constexpr int CPW = 64 / G;            // columns per wavefront
  static constexpr int WAVES = (N == 512 ? 8 : 4) * (WIDE ? 2 : 1);
  static constexpr int CT = WAVES * CPW;        // columns per block
  // column stride in LDS (8-byte slots).  An 8-byte LDS access serves 16
  // lanes per pass over the 32 banks, so the 16 lanes of a transpose
  // instruction must land on 16 distinct slots mod 16: two adjacent rows of 8
  // columns need LD = 2 (mod 16), one row of 16 columns an odd LD; 64-point
  // columns (two per 16 lanes in the FFT exchanges) need LD = 8 (mod 16).
  static constexpr int LD = N == 64 ? padded(N) : CT >= 16 ? padded(N) + 1 : padded(N) + 2;
  static constexpr int THREADS = WAVES * 64;
};

// DB = 1: two LDS tile buffers in turn, so a tile's transposed stores and the
// next tile's staging need no barrier between them (two barriers per tile
// instead of three).
template <int N, int WIDE, int DB>
__global__ void __launch_bounds__((C8<N, WIDE>::THREADS)) k_col_r8(PassTable tab, int total_tiles) {
  constexpr int G = C8<N, WIDE>::G;
  constexpr int CPW = C8<N, WIDE>::CPW;
  constexpr int CT = C8<N, WIDE>::CT;
  constexpr int LD = C8<N, WIDE>::LD;
  constexpr int S = R8<N>::S;
  constexpr int THREADS = C8<N, WIDE>::THREADS;
  constexpr int PER = CT * N / THREADS;  // tile values each thread moves
  __shared__ float2 cols_mem[(DB ? 2 : 1) * CT * LD];
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int cl = wave * CPW + lane / G;  // this lane's column in the tile
  const int t = lane % G;
  // padded LDS slots: this lane's FFT values (t + G r) and its transpose
  // element (column e mod CT, row e / CT, e = threadIdx.x + q THREADS; the
  // row step THREADS / CT is a multiple of 8)
  static_assert((THREADS / CT) % 8 == 0 && G % 8 == 0, "padded slots");
  const int rslot = t + (t >> 3);
  const int trow = threadIdx.x / CT;
  const int tslot = (threadIdx.x % CT) * LD + trow + (trow >> 3);

  // stage twiddles of the y transform (every lane of the table has this ny)
  float2 tw[S][7];
  reg_twiddles<N>(tw, tab.l[0].a.tw_y, t);
  // tile geometry of a logical tile index
  auto locate = [&](int it, int& L, int& x0, float2*& wp) {
    const int tile_g = xcd_remap(it, total_tiles);
    L = find_lane(tab, tile_g);
    const PassArgs& a = tab.l[L].a;
    const int tile = tile_g - tab.l[L].block_start;
    const int tiles_per_wave = a.nx / CT;
    const int w = tile / tiles_per_wave;
    x0 = (tile % tiles_per_wave) * CT;
    const int p = w / a.fb;
    const int fl = w % a.fb;
    wp = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;
  };
  float2 pre[PER];
  int L = 0, x0 = 0;
  float2* wp = nullptr;
  int it = blockIdx.x;
  if (it < total_tiles) {
    locate(it, L, x0, wp);
    const int nx = tab.l[L].a.nx;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * THREADS;
      pre[q] = wp[(size_t)(e / CT) * nx + x0 + e % CT];
    }
  }
  for (int n_done = 0; it < total_tiles; it += gridDim.x, ++n_done) {
    const PassArgs& a = tab.l[L].a;
    const int mode = tab.l[L].mode;
    const int cur_x0 = x0;
    float2* cur_wp = wp;
    float2* cols = cols_mem + (DB ? (n_done & 1) * CT * LD : 0);
    float2* lds = cols + cl * LD;
    // single buffer: the previous tile's stores from LDS must be done; two
    // buffers: this one was last read two tiles ago, before the last barrier
    if (!DB) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) cols[tslot + q * (THREADS / CT + THREADS / CT / 8)] = pre[q];
    // issue the next tile's loads; they complete during this tile's arithmetic
    const int nit = it + gridDim.x;
    if (nit < total_tiles) {
      locate(nit, L, x0, wp);
      const int nx = tab.l[L].a.nx;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * THREADS;
        pre[q] = wp[(size_t)(e / CT) * nx + x0 + e % CT];
      }
    }
    __syncthreads();
    float2 x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = lds[rslot + r * (G + G / 8)];
    if (mode == COL_INVERSE_ONLY) {
      fft_r8<N, true>(x, lds, tw, t);
    } else {
      fft_r8<N, false>(x, lds, tw, t);
      const float2 pxv = a.px[cur_x0 + cl];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = cmul(x[r], cmul(pxv, a.py[t + r * G]));
      if (mode == COL_REGULAR) fft_r8<N, true>(x, lds, tw, t);
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) lds[rslot + r * (G + G / 8)] = x[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * THREADS;
      cur_wp[(size_t)(e / CT) * a.nx + cur_x0 + e % CT] = cols[tslot + q * (THREADS / CT + THREADS / CT / 8)];
    }
  }
}

// ---------------------------------------------------------------------------
// Waves resident in LDS (square grids of 64 and 128): one workgroup holds one
// (probe, frame) wave for a run of slices, so HBM carries only the potentials
// and, at the ends of the run, the wave itself.  Per slice: every row goes
// through iFFT_x, the transmission exp(i sigma V) and FFT_x, then every column
// through FFT_y, the propagator and iFFT_y (or FFT_y and the last-slice
// propagator at the job's last slice), with a workgroup barrier after each
// phase.  Rows and columns use the register FFT of the row and column passes
// (same stages, twiddles, butterflies and products, so the same arithmetic),
// with their exchanges done in place in the resident wave.  Layout: element
// (y, x) at slot (y + y/16) PITCH + x + x/16; a 16-lane access then hits at
// most two slots per bank pair (checked by enumeration of every exchange of
// both phases).
// ---------------------------------------------------------------------------
template <int N>
struct RS {
  static constexpr int G = N / 8;                  // lanes per line
  static constexpr int RPW = 64 / G;               // lines per wavefront
  static constexpr int WAVES = N == 128 ? 16 : 8;
  static constexpr int THREADS = WAVES * 64;
  static constexpr int PITCH = N == 128 ? 145 : 67;
  static constexpr int ROWS = N + (N - 1) / 16;    // physical rows: rs_pad(N - 1) + 1
  static constexpr int ITS = N / (WAVES * RPW);    // line iterations per phase
  static constexpr size_t LDS = (size_t)ROWS * PITCH * sizeof(float2);
  static_assert(N == 64 || N == 128, "resident grids: 64 and 128");
  static_assert(PITCH >= N + (N - 1) / 16, "rows hold their padded slots");
};
__device__ __forceinline__ int rs_pad(int i) { return i + (i >> 4); }

// line handled by (iteration, wavefront, line within the wavefront): 128:
// consecutive lines per wavefront; 64: lines w + 8 sub (the two lines of a
// 16-lane group are 8 apart, which the bank check prefers)
template <int N>
__device__ __forceinline__ int rs_line(int it, int wave, int sub) {
  if constexpr (N == 128)
    return (it * RS<N>::WAVES + wave) * RS<N>::RPW + sub;
  else
    return wave + RS<N>::WAVES * sub;
}

// Stage J of the register FFT (the arithmetic of reg_fft_stage) with the
// exchanges at LDS slots addr(position).
template <int N, bool INV, int J, typename Addr>
__device__ __forceinline__ void res_fft_stage(float2 (&x)[8], float2* psi, const Addr& addr,
                                              const float2 (&tw)[R8<N>::S][7], int t) {
  constexpr int S = R8<N>::S, G = R8<N>::G;
  constexpr int R = R8<N>::radix(J), P = R8<N>::stride(J), Q = 8 / R;
  if constexpr (J > 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[J][q * (R - 1) + r - 1];
        x[q + Q * r] = INV ? cmulc(x[q + Q * r], w) : cmul(x[q + Q * r], w);
      }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = x[q + Q * r];
    dft<R, INV>(y);
#pragma unroll
    for (int r = 0; r < R; ++r) x[q + Q * r] = y[r];
  }
  if constexpr (J < S - 1) {
    wave_lds_sync();  // earlier reads of this line by the wavefront are done
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = t + G * q;
      const int k = b % P;
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) psi[addr(base + r * P)] = x[q + Q * r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = psi[addr(t + G * r)];
    res_fft_stage<N, INV, J + 1>(x, psi, addr, tw, t);
  }
}

template <int N>
__global__ void __launch_bounds__(RS<N>::THREADS) k_res(ResTable tab) {
  constexpr int G = RS<N>::G, S = R8<N>::S, PITCH = RS<N>::PITCH;
  extern __shared__ float2 psi[];
  const int L = find_lane(tab, blockIdx.x);
  const ResLane& ln = tab.l[L];
  const PassArgs& a = ln.a;
  const int w = blockIdx.x - ln.block_start;    // wave of the lane: probe p, frame f0 + fl
  const int p = w / a.fb;
  const int fl = w - p * a.fb;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int sub = lane / G, t = lane % G;
  float2* store = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * N;
  float2 tw[S][7];
  reg_twiddles<N>(tw, a.tw_x, t);   // square grid: the y transform has the same twiddles
  const int ox = a.plane ? 0 : a.origin[2 * p];
  const int oy = a.plane ? 0 : a.origin[2 * p + 1];
  const int s0 = a.slice, s1 = a.slice + ln.n_slices_launch;

  // the wave in flight ((kx, y) layout) unless the run starts at slice 0
  if (s0 > 0) {
    for (int e = threadIdx.x; e < N * N; e += RS<N>::THREADS)
      psi[rs_pad(e / N) * PITCH + rs_pad(e % N)] = store[e];
    __syncthreads();
  }
  for (int sl = s0; sl < s1; ++sl) {
    // rows: iFFT_x (not at slice 0: the incident wave is in real space),
    // transmission, FFT_x
#pragma unroll 1
    for (int it = 0; it < RS<N>::ITS; ++it) {
      const int y = rs_line<N>(it, wave, sub);
      float2* row = psi + rs_pad(y) * PITCH;
      auto addr = [](int i) { return rs_pad(i); };
      float2 x[8];
      if (sl == 0) {
        if (a.plane) {
#pragma unroll
          for (int r = 0; r < 8; ++r) x[r] = make_float2(a.plane_amp, 0.f);
        } else {
          const float2* src = a.probe0 + ((size_t)p * a.ny + y) * (size_t)N;
#pragma unroll
          for (int r = 0; r < 8; ++r) x[r] = src[t + r * G];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = row[addr(t + r * G)];
      }
      int yy = oy + y;
      if (yy >= a.pny) yy -= a.pny;
      const float* vrow = a.V + (((size_t)fl * a.v_slices + (sl - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
      float v[8];
      if (ox == 0 && a.pnx == N) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = vrow[t + r * G];
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          int xx = ox + t + r * G;
          if (xx >= a.pnx) xx -= a.pnx;
          v[r] = vrow[xx];
        }
      }
      if (sl > 0) res_fft_stage<N, true, 0>(x, row, addr, tw, t);
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = cmul(x[r], phase_factor(a.sigma * v[r]));
      res_fft_stage<N, false, 0>(x, row, addr, tw, t);
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 8; ++r) row[addr(t + r * G)] = x[r];
    }
    __syncthreads();
    // columns: FFT_y, propagator, iFFT_y (the job's last slice: FFT_y and the
    // last-slice propagator)
    const bool last = sl == a.n_slices - 1;
    const float2* px = last ? ln.px_last : a.px;
    const float2* py = last ? ln.py_last : a.py;
#pragma unroll 1
    for (int it = 0; it < RS<N>::ITS; ++it) {
      const int xc = rs_line<N>(it, wave, sub);
      const int cs = rs_pad(xc);
      auto addr = [cs](int i) { return rs_pad(i) * PITCH + cs; };
      float2 x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = psi[addr(t + r * G)];
      res_fft_stage<N, false, 0>(x, psi, addr, tw, t);
      const float2 pxv = px[xc];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = cmul(x[r], cmul(pxv, py[t + r * G]));
      if (!last) res_fft_stage<N, true, 0>(x, psi, addr, tw, t);
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 8; ++r) psi[addr(t + r * G)] = x[r];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < N * N; e += RS<N>::THREADS) store[e] = psi[rs_pad(e / N) * PITCH + rs_pad(e % N)];
}

// ---------------------------------------------------------------------------
// Column pass for ny = 512 as 512 = 8 x 64 (six-step), tiles of 8 columns.
// Lanes run along x, so a tile is read and written straight from its rows in
// 64-byte segments with no LDS transpose:
//   layout A: column c = lane % 8, r0 = 8 wave + lane / 8, values at rows
//             r0 + 64 j (j < 8): 8-point transform over j, twiddle
//             W512^(r0 k1), exchange through LDS to
//   layout B: k1 = wave, column lane / 8, u = lane % 8, values at r0 = u + 8 q:
//             8-point transform over q, twiddle W64^(u k2), a wavefront-local
//             exchange, 8-point transform over u: frequency k1 + 8 u + 64 k3
//             held as k3 < 8.
// The propagator is applied in that order, and the inverse retraces the same
// steps backwards (conjugate twiddles), ending in layout A for the store.  The
// last slice stores the spectrum straight from layout B.  Per tile: two
// exchanges across wavefronts and two within one, against two transposes and
// four exchanges in k_col_r8.  LDS slots: [k1][r0][c ^ (r0 % 8)] for the
// cross-wavefront exchanges, and, inside wavefront k1's own 512 slots,
// 64 c + 8 (u ^ (c % 2)) + (k2 ^ u) for the local ones; every 16-lane group of
// an access hits 16 distinct 8-byte slots modulo 16.
// ---------------------------------------------------------------------------
template <int R1>
__global__ void __launch_bounds__(512) k_col_6s(PassTable tab, int total_tiles) {
  static_assert(R1 == 8 || R1 == 6, "512 = 8 x 64 and 384 = 6 x 64");
  constexpr int N = 64 * R1, CT = 8;
  __shared__ float2 xs[4096];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ca = lane & 7, r0 = 8 * wave + (lane >> 3);   // layout A
  const int k1 = wave, cb = lane >> 3, u = lane & 7;      // layout B
  // layout B has R1 wavefronts (k1 < R1); at 384 rows waves 6 and 7 only
  // take part in the workgroup barriers there
  const bool in_b = k1 < R1;
  // slots
  const int sa = 8 * r0 + (ca ^ (r0 & 7));                 // + 512 k1
  const int sb = 512 * k1 + 8 * u + (cb ^ u);              // + 64 q
  float2* lw = xs + 512 * k1 + 64 * cb;                    // local exchange region
  const int lodd = cb & 1;
  // twiddles, the same for every tile (all lanes of a table have ny = N):
  // W_N^(r0 k) and W64^(u k) = W_N^(R1 u k), R1 u k < N
  float2 ta[R1], tb[8];   // entries from 1 (entry 0 is 1 and never used)
  {
    const float2* tw = tab.l[0].a.tw_y;
#pragma unroll
    for (int k = 1; k < R1; ++k) ta[k] = tw[(N & (N - 1)) == 0 ? (r0 * k) & (N - 1) : (r0 * k) % N];
#pragma unroll
    for (int k = 1; k < 8; ++k) tb[k] = tw[R1 * u * k];
  }
  auto locate = [&](int it, int& L, int& x0, float2*& wp) {
    const int tile_g = xcd_remap(it, total_tiles);
    L = find_lane(tab, tile_g);
    const PassArgs& a = tab.l[L].a;
    const int tile = tile_g - tab.l[L].block_start;
    const int tiles_per_wave = a.nx / CT;
    const int w = tile / tiles_per_wave;
    x0 = (tile % tiles_per_wave) * CT;
    const int p = w / a.fb;
    const int fl = w % a.fb;
    wp = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;
  };
  float2 pre[R1];
  int L = 0, x0 = 0;
  float2* wp = nullptr;
  int it = blockIdx.x;
  if (it < total_tiles) {
    locate(it, L, x0, wp);
    const int nx = tab.l[L].a.nx;
#pragma unroll
    for (int j = 0; j < R1; ++j) pre[j] = wp[(size_t)(r0 + 64 * j) * nx + x0 + ca];
  }
  for (; it < total_tiles; it += gridDim.x) {
    const PassArgs& a = tab.l[L].a;
    const int mode = tab.l[L].mode;
    const int nx = a.nx;
    const int cur_x0 = x0;
    float2* cur_wp = wp;
    float2 x[8];
#pragma unroll
    for (int j = 0; j < R1; ++j) x[j] = pre[j];
    // the next tile's loads complete during this tile's arithmetic
    const int nit = it + gridDim.x;
    if (nit < total_tiles) {
      locate(nit, L, x0, wp);
      const int nnx = tab.l[L].a.nx;
#pragma unroll
      for (int j = 0; j < R1; ++j) pre[j] = wp[(size_t)(r0 + 64 * j) * nnx + x0 + ca];
    }
    // layout A: R1-point transform over j, twiddle, to LDS
    dft<R1, false>(x);
#pragma unroll
    for (int k = 1; k < R1; ++k) x[k] = cmul(x[k], ta[k]);
    __syncthreads();   // the previous tile's reads of the exchange buffer are done
#pragma unroll
    for (int k = 0; k < R1; ++k) xs[512 * k + sa] = x[k];
    __syncthreads();
    const bool last = mode == COL_LAST;
    if (in_b) {
      // layout B: 8-point transform over q, twiddle, local exchange, over u
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = xs[sb + 64 * q];
      dft8<false>(x);
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], tb[k]);
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < 8; ++k) lw[8 * (u ^ lodd) + (k ^ u)] = x[k];
      wave_lds_sync();
#pragma unroll
      for (int v = 0; v < 8; ++v) x[v] = lw[8 * (v ^ lodd) + (u ^ v)];
      dft8<false>(x);   // x[k3] = psi(k1 + R1 u + 8 R1 k3) of column cur_x0 + cb
      const float2 pxv = a.px[cur_x0 + cb];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = cmul(x[k], cmul(pxv, a.py[k1 + R1 * u + 8 * R1 * k]));
      if (last) {
#pragma unroll
        for (int k = 0; k < 8; ++k) cur_wp[(size_t)(k1 + R1 * u + 8 * R1 * k) * nx + cur_x0 + cb] = x[k];
      } else {
        // inverse, the same steps backwards
        dft8<true>(x);    // over k3: x[v] at u-index v, this lane's k2 = u
        wave_lds_sync();
#pragma unroll
        for (int v = 0; v < 8; ++v) lw[8 * (v ^ lodd) + (u ^ v)] = x[v];
        wave_lds_sync();
        x[0] = lw[8 * (u ^ lodd) + u];
#pragma unroll
        for (int k = 1; k < 8; ++k) x[k] = cmulc(lw[8 * (u ^ lodd) + (k ^ u)], tb[k]);
        dft8<true>(x);    // over k2: x[q] at r0 = u + 8 q
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 8; ++q) xs[sb + 64 * q] = x[q];
      }
    }
    if (last) continue;   // the same for the whole workgroup (one lane per tile)
    __syncthreads();
    // layout A: conjugate twiddle, R1-point transform over k1, store
    x[0] = xs[sa];
#pragma unroll
    for (int k = 1; k < R1; ++k) x[k] = cmulc(xs[512 * k + sa], ta[k]);
    dft<R1, true>(x);
#pragma unroll
    for (int j = 0; j < R1; ++j) cur_wp[(size_t)(r0 + 64 * j) * nx + cur_x0 + ca] = x[j];
  }
}

// ---------------------------------------------------------------------------
// Column pass for ny = 256 as 256 = 8 x 32 (six-step) on tiles of 16 columns
// (whole 128-byte row segments), 512 threads:
//   layout A: column c = lane % 16, r0 = 4 wave + lane / 16, values at rows
//             r0 + 32 j (j < 8): 8-point transform over j, twiddle
//             W256^(r0 k1), exchange through LDS to
//   layout B: k1 = wave, column lane / 4, u = lane % 4, values at r0 = u + 4 q:
//             8-point transform over q, twiddle W32^(u k2), a wavefront-local
//             exchange that gives lane u the values of k2 = u and u + 4 for
//             every u-index, and two 4-point transforms over that index:
//             frequency k1 + 8 k2 + 64 k3 (k3 < 4).
// The propagator is applied in that order and the inverse retraces the steps
// with conjugate twiddles; the last slice stores the spectrum from layout B.
// LDS slots: 16 r0 + (c ^ 4 (r0 % 4)) within region k1 for the cross-wavefront
// exchanges, and 16 (k2 / 4) + 4 ((k2 % 4) ^ (c % 4)) + (u ^ (c % 4)) within
// column c's 32 slots of region k1 for the local ones; every 16-lane access
// hits 16 distinct 8-byte slots modulo 16 (checked by enumeration, with the
// index arithmetic checked against a reference FFT in the same enumeration).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512) k_col_6q(PassTable tab, int total_tiles) {
  constexpr int N = 256, CT = 16;
  __shared__ float2 xs[4096];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ca = lane & 15, r0 = 4 * wave + (lane >> 4);   // layout A
  const int k1 = wave, cb = lane >> 2, u = lane & 3;       // layout B
  const int sa = 16 * r0 + (ca ^ (4 * (r0 & 3)));          // + 512 k1
  const int sb = 512 * k1 + 16 * u + (cb ^ (4 * u));       // + 64 q (r0 = u + 4 q)
  float2* lw = xs + 512 * k1 + 32 * cb;                    // local exchange region
  const int cs = cb & 3;
  auto lslot = [cs](int k2, int uu) { return 16 * (k2 >> 2) + 4 * ((k2 & 3) ^ cs) + (uu ^ cs); };
  // twiddles, the same for every tile (all lanes of a table have ny = 256)
  float2 ta[8], tb[8];   // entries 1..7
  {
    const float2* tw = tab.l[0].a.tw_y;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      ta[k] = tw[(r0 * k) & (N - 1)];
      tb[k] = tw[(8 * u * k) & (N - 1)];
    }
  }
  auto locate = [&](int it, int& L, int& x0, float2*& wp) {
    const int tile_g = xcd_remap(it, total_tiles);
    L = find_lane(tab, tile_g);
    const PassArgs& a = tab.l[L].a;
    const int tile = tile_g - tab.l[L].block_start;
    const int tiles_per_wave = a.nx / CT;
    const int w = tile / tiles_per_wave;
    x0 = (tile % tiles_per_wave) * CT;
    const int p = w / a.fb;
    const int fl = w % a.fb;
    wp = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;
  };
  float2 pre[8];
  int L = 0, x0 = 0;
  float2* wp = nullptr;
  int it = blockIdx.x;
  if (it < total_tiles) {
    locate(it, L, x0, wp);
    const int nx = tab.l[L].a.nx;
#pragma unroll
    for (int j = 0; j < 8; ++j) pre[j] = wp[(size_t)(r0 + 32 * j) * nx + x0 + ca];
  }
  for (; it < total_tiles; it += gridDim.x) {
    const PassArgs& a = tab.l[L].a;
    const int mode = tab.l[L].mode;
    const int nx = a.nx;
    const int cur_x0 = x0;
    float2* cur_wp = wp;
    float2 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = pre[j];
    // the next tile's loads complete during this tile's arithmetic
    const int nit = it + gridDim.x;
    if (nit < total_tiles) {
      locate(nit, L, x0, wp);
      const int nnx = tab.l[L].a.nx;
#pragma unroll
      for (int j = 0; j < 8; ++j) pre[j] = wp[(size_t)(r0 + 32 * j) * nnx + x0 + ca];
    }
    // layout A: 8-point transform over j, twiddle, to LDS
    dft8<false>(x);
#pragma unroll
    for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], ta[k]);
    __syncthreads();   // the previous tile's reads of the exchange buffer are done
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[512 * k + sa] = x[k];
    __syncthreads();
    // layout B: 8-point transform over q, twiddle, local exchange, two
    // 4-point transforms over the u-index
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = xs[sb + 64 * q];
    dft8<false>(x);
#pragma unroll
    for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], tb[k]);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 8; ++k) lw[lslot(k, u)] = x[k];
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 8; ++v) x[v] = lw[lslot(u + 4 * (v >> 2), v & 3)];
    dft4<false>(x);
    dft4<false>(x + 4);   // x[4 h + k3] = psi(k1 + 8 (u + 4 h) + 64 k3) of column cur_x0 + cb
    const float2 pxv = a.px[cur_x0 + cb];
    const bool last = mode == COL_LAST;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k3 = 0; k3 < 4; ++k3)
        x[4 * h + k3] = cmul(x[4 * h + k3], cmul(pxv, a.py[k1 + 8 * (u + 4 * h) + 64 * k3]));
    if (last) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k3 = 0; k3 < 4; ++k3)
          cur_wp[(size_t)(k1 + 8 * (u + 4 * h) + 64 * k3) * nx + cur_x0 + cb] = x[4 * h + k3];
      continue;
    }
    // inverse, the same steps backwards
    dft4<true>(x);
    dft4<true>(x + 4);   // x[4 h + v]: u-index v of k2 = u + 4 h
    wave_lds_sync();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v) lw[lslot(u + 4 * h, v)] = x[4 * h + v];
    wave_lds_sync();
    x[0] = lw[lslot(0, u)];
#pragma unroll
    for (int k = 1; k < 8; ++k) x[k] = cmulc(lw[lslot(k, u)], tb[k]);
    dft8<true>(x);    // over k2: x[q] at r0 = u + 4 q
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 8; ++q) xs[sb + 64 * q] = x[q];
    __syncthreads();
    // layout A: conjugate twiddle, 8-point transform over k1, store
    x[0] = xs[sa];
#pragma unroll
    for (int k = 1; k < 8; ++k) x[k] = cmulc(xs[512 * k + sa], ta[k]);
    dft8<true>(x);
#pragma unroll
    for (int j = 0; j < 8; ++j) cur_wp[(size_t)(r0 + 32 * j) * nx + cur_x0 + ca] = x[j];
  }
}

// ---------------------------------------------------------------------------
// The same six-step column transform on tiles of 16 columns, so that every
// load and store instruction of a wavefront covers whole 128-byte row
// segments (4 rows x 16 columns), with 512 threads and 68 KiB of LDS per
// workgroup: two workgroups fit one CU.  A lane holds two columns' or two
// rows' worth of the 8-column kernel's values:
//   layout A: column c = lane % 16, ra = 4 wave + lane / 16; rows
//             r0 = ra + 32 h (h < 2), values at rows r0 + 64 j;
//   layout B: k1 = wave, columns cb + 8 h (cb = lane / 8), u = lane % 8,
//             values at r0 = u + 8 q.
// LDS slots of the exchanges across wavefronts: 1024 k1 + 512 (c / 8) +
// 8 (r0 ^ (c / 8)) + ((c % 8) ^ (r0 % 8)), so columns 8 h .. 8 h + 7 fill one
// half of wavefront k1's 1024 slots.  The local exchanges of column cb + 8 h
// use 64 slots of that half, 512 h + 64 cb + 8 (u ^ (cb % 2)) + (k2 ^ u): a
// half is only overwritten after this wavefront has read all of it.  Every
// 16-lane group of an access hits 16 distinct 8-byte slots modulo 16
// (checked by enumeration).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_col_6w(PassTable tab, int total_tiles) {
  constexpr int N = 512, CT = 16;
  __shared__ float2 xs[8192];
  __shared__ float2 twl[N];   // W512^m, for the layout-A twiddles
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ca = lane & 15, ra = 4 * wave + (lane >> 4);   // layout A
  const int k1 = wave, cb = lane >> 3, u = lane & 7;       // layout B
  const int sa0 = 512 * (ca >> 3) + 8 * (ra ^ (ca >> 3)) + ((ca & 7) ^ (ra & 7));   // + 1024 k1 + 256 h
  float2* lw0 = xs + 1024 * k1 + 64 * cb;                  // local regions of columns cb, cb + 8
  float2* lw1 = lw0 + 512;
  const int lodd = cb & 1;
  // slot of (k1, r0 = u + 8 q, column cb + 8 h): 1024 k1 + 512 h + 8 (u ^ h) + 64 q + (cb ^ u)
  const int sb0 = 1024 * k1 + 8 * u + (cb ^ u);
  const int sb1 = 1024 * k1 + 512 + 8 * (u ^ 1) + (cb ^ u);
  float2 tb[8];   // layout-B twiddles, entries 1..7; layout A reads W512^(r0 k) from twl
  {
    const float2* tw = tab.l[0].a.tw_y;
#pragma unroll
    for (int k = 1; k < 8; ++k) tb[k] = tw[(8 * u * k) & (N - 1)];
    for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = tw[i];
  }
  auto locate = [&](int it, int& L, int& x0, float2*& wp) {
    const int tile_g = xcd_remap(it, total_tiles);
    L = find_lane(tab, tile_g);
    const PassArgs& a = tab.l[L].a;
    const int tile = tile_g - tab.l[L].block_start;
    const int tiles_per_wave = a.nx / CT;
    const int w = tile / tiles_per_wave;
    x0 = (tile % tiles_per_wave) * CT;
    const int p = w / a.fb;
    const int fl = w % a.fb;
    wp = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;
  };
  // the two rows (layout A) or columns (layout B) of a lane go one after the
  // other, so that only 8 values per lane are live at a time
  for (int it = blockIdx.x; it < total_tiles; it += gridDim.x) {
    int L = 0, x0 = 0;
    float2* wp = nullptr;
    locate(it, L, x0, wp);
    const PassArgs& a = tab.l[L].a;
    const int mode = tab.l[L].mode;
    const int nx = a.nx;
    float2 x[8];
    __syncthreads();   // the previous tile's reads of the exchange buffer are done
    // layout A: 8-point transform over j, twiddle, to LDS
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = wp[(size_t)(ra + 32 * h + 64 * j) * nx + x0 + ca];
      dft8<false>(x);
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], twl[((ra + 32 * h) * k) & (N - 1)]);
#pragma unroll
      for (int k = 0; k < 8; ++k) xs[1024 * k + 256 * h + sa0] = x[k];
    }
    __syncthreads();
    // layout B, one column at a time: 8-point transform over q, twiddle,
    // local exchange, over u; propagator; and back
    const bool last = mode == COL_LAST;
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      const int sb = h ? sb1 : sb0;
      float2* lw = h ? lw1 : lw0;
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = xs[sb + 64 * q];
      dft8<false>(x);
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], tb[k]);
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < 8; ++k) lw[8 * (u ^ lodd) + (k ^ u)] = x[k];
      wave_lds_sync();
#pragma unroll
      for (int v = 0; v < 8; ++v) x[v] = lw[8 * (v ^ lodd) + (u ^ v)];
      dft8<false>(x);   // x[k3] = psi(k1 + 8 u + 64 k3) of column x0 + cb + 8 h
      const float2 pxv = a.px[x0 + cb + 8 * h];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = cmul(x[k], cmul(pxv, a.py[k1 + 8 * u + 64 * k]));
      if (last) {
#pragma unroll
        for (int k = 0; k < 8; ++k) wp[(size_t)(k1 + 8 * u + 64 * k) * nx + x0 + cb + 8 * h] = x[k];
        continue;
      }
      dft8<true>(x);    // over k3: x[v] at u-index v, this lane's k2 = u
      wave_lds_sync();
#pragma unroll
      for (int v = 0; v < 8; ++v) lw[8 * (v ^ lodd) + (u ^ v)] = x[v];
      wave_lds_sync();
      x[0] = lw[8 * (u ^ lodd) + u];
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmulc(lw[8 * (u ^ lodd) + (k ^ u)], tb[k]);
      dft8<true>(x);    // over k2: x[q] at r0 = u + 8 q
      wave_lds_sync();  // this wavefront's reads of the local region are done
#pragma unroll
      for (int q = 0; q < 8; ++q) xs[sb + 64 * q] = x[q];
    }
    if (last) continue;
    __syncthreads();
    // layout A: conjugate twiddle, 8-point transform over k1, store
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      x[0] = xs[256 * h + sa0];
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmulc(xs[1024 * k + 256 * h + sa0], twl[((ra + 32 * h) * k) & (N - 1)]);
      dft8<true>(x);
#pragma unroll
      for (int j = 0; j < 8; ++j) wp[(size_t)(ra + 32 * h + 64 * j) * nx + x0 + ca] = x[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Register FFTs with 12 or 16 values per lane (N = 384 and 768: 12 values,
// radices 6, 4, 4, 4 [, 2]; N = 1024: 16 values, radices 8, 8, 4, 4).  Same
// layout and wavefront-local exchanges as the 8-value kernels; the stage
// twiddles are read from a table in LDS, since the register file cannot hold
// them beside 12-16 values and their prefetch.  PAD selects the padded LDS
// slots (element i in slot i + i/8) or plain ones.
// ---------------------------------------------------------------------------
template <int N>
struct RV {
  static constexpr int V = N == 1024 ? 16 : 12;   // values per lane
  static constexpr int G = N / V;                 // lanes per row
  static constexpr int RPW = 64 / G;              // rows per wavefront
  static constexpr int S = N == 384 ? 4 : N == 768 ? 5 : N == 1024 ? 4 : 0;
  static constexpr int radix(int j) { return N == 1024 ? (j < 2 ? 8 : 4) : (j == 0 ? 6 : j < 4 ? 4 : 2); }
  static constexpr int stride(int j) { return j == 0 ? 1 : stride(j - 1) * radix(j - 1); }
  // per-lane twiddles of stages 1 .. J-1: (R - 1) Q each
  static constexpr int tw_offset(int j) {
    return j <= 1 ? 0 : tw_offset(j - 1) + (radix(j - 1) - 1) * (V / radix(j - 1));
  }
  static constexpr int NT = tw_offset(S);          // twiddles per lane
  static_assert(S > 0 && G <= 64 && G % 8 == 0, "register FFT sizes 384, 768, 1024");
  static_assert(stride(S - 1) * radix(S - 1) == N, "radices multiply to N");
};

// Per-lane stage twiddles in LDS, laid out [twiddle][lane t] (NT x G), so a
// lane reads twiddle i at a fixed offset from its own slot: entry
// tw_offset(J) + q (R - 1) + r - 1 of stage J is W_{PR}^{r (b mod P)},
// b = t + G q.  Built from the FP64-derived table `tw` (N entries).
template <int N>
__device__ __forceinline__ void build_lane_twiddles(float2* twl, const float2* tw) {
  constexpr int G = RV<N>::G, V = RV<N>::V, S = RV<N>::S;
  for (int e = threadIdx.x; e < RV<N>::NT * G; e += blockDim.x) {
    const int i = e / G, t = e % G;
    int j = 1, off = 0, P = RV<N>::radix(0);
    while (j < S - 1 && i >= off + (RV<N>::radix(j) - 1) * (V / RV<N>::radix(j))) {
      off += (RV<N>::radix(j) - 1) * (V / RV<N>::radix(j));
      P *= RV<N>::radix(j);
      ++j;
    }
    const int R = RV<N>::radix(j);
    const int q = (i - off) / (R - 1), r = (i - off) % (R - 1) + 1;
    const int k = (t + G * q) % P;
    twl[e] = tw[r * k * (N / (P * R))];
  }
}

template <int N, bool INV, bool PAD, int J>
__device__ __forceinline__ void rv_fft_stage(float2 (&x)[RV<N>::V], float2* lds, const float2* twl, int t) {
  constexpr int V = RV<N>::V, S = RV<N>::S, G = RV<N>::G;
  constexpr int R = RV<N>::radix(J), P = RV<N>::stride(J), Q = V / R;
  static_assert(V % R == 0, "the radix divides the values per lane");
  if constexpr (J > 0) {
    // input r of butterfly q takes W_{PR}^{r (b mod P)}, b = t + G q, from
    // this lane's column of the twiddle table
    constexpr int OFF = RV<N>::tw_offset(J);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = twl[(OFF + q * (R - 1) + r - 1) * G + t];
        x[q + Q * r] = INV ? cmulc(x[q + Q * r], w) : cmul(x[q + Q * r], w);
      }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float2 y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = x[q + Q * r];
    dft<R, INV>(y);
#pragma unroll
    for (int r = 0; r < R; ++r) x[q + Q * r] = y[r];
  }
  if constexpr (J < S - 1) {
    wave_lds_sync();  // earlier reads of lds by this wavefront are done
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = t + G * q;
      const int k = b % P;
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int pos = base + r * P;
        lds[PAD ? pos + (pos >> 3) : pos] = x[q + Q * r];
      }
    }
    wave_lds_sync();
    const int rbase = PAD ? t + (t >> 3) : t;
#pragma unroll
    for (int r = 0; r < V; ++r) x[r] = lds[rbase + r * (PAD ? G + G / 8 : G)];
    rv_fft_stage<N, INV, PAD, J + 1>(x, lds, twl, t);
  }
}

template <int N, bool INV, bool PAD>
__device__ __forceinline__ void fft_rv(float2 (&x)[RV<N>::V], float2* lds, const float2* twl, int t) {
  rv_fft_stage<N, INV, PAD, 0>(x, lds, twl, t);
}

// Row pass on 12- or 16-value registers: one row per G lanes, the next row
// prefetched, rows shared among the lanes of the table as in k_row_r8.
template <int N>
__global__ void __launch_bounds__(256) k_row_rv(PassTable tab) {
  constexpr int V = RV<N>::V, G = RV<N>::G, RPW = RV<N>::RPW;
  __shared__ float2 twt[RV<N>::NT * G];
  __shared__ float2 scratch[4][RPW][padded(N)];
  const int L = find_lane(tab, blockIdx.x);
  const PassArgs& a = tab.l[L].a;
  const int mode = tab.l[L].mode;
  const int lb = blockIdx.x - tab.l[L].block_start;
  const int blocks_per_lane = (L + 1 < tab.n ? tab.l[L + 1].block_start : (int)gridDim.x) - tab.l[L].block_start;
  build_lane_twiddles<N>(twt, a.tw_x);
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int sub = RPW == 1 ? 0 : lane / G;
  const int t = lane % G;
  float2* lds = scratch[wave][sub];
  const int total = a.n_probes * a.fb * a.ny;   // below 2^31 (checked at launch)
  const int stride = blocks_per_lane * 4 * RPW;
  const bool transmit = mode != ROW_INVERSE_ONLY;
  auto fetch = [&](int rid, float2 (&xv)[V], float (&vv)[V], float2*& out) {
    if (rid >= total) return;
    const int w = rid / a.ny;
    const int y = rid - w * a.ny;
    const int p = w / a.fb;
    const int fl = w - p * a.fb;
    float2* row = a.exit + (((size_t)p * a.n_frames + a.f0 + fl) * a.ny + y) * (size_t)N;
    out = row;
    if (mode == ROW_FIRST) {
      if (a.plane) {
#pragma unroll
        for (int r = 0; r < V; ++r) xv[r] = make_float2(a.plane_amp, 0.f);
      } else {
        const float2* src = a.probe0 + ((size_t)p * a.ny + y) * (size_t)N;
#pragma unroll
        for (int r = 0; r < V; ++r) xv[r] = src[t + r * G];
      }
    } else {
#pragma unroll
      for (int r = 0; r < V; ++r) xv[r] = row[t + r * G];
    }
    if (transmit) {
      const int ox = a.plane ? 0 : a.origin[2 * p];
      const int oy = a.plane ? 0 : a.origin[2 * p + 1];
      int yy = oy + y;
      if (yy >= a.pny) yy -= a.pny;
      const float* vrow =
          a.V + (((size_t)fl * a.v_slices + (a.slice - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
#pragma unroll
      for (int r = 0; r < V; ++r) {
        int xx = ox + t + r * G;
        if (xx >= a.pnx) xx -= a.pnx;
        vv[r] = vrow[xx];
      }
    }
  };
  float2 xn[V];
  float vn[V];
#pragma unroll
  for (int r = 0; r < V; ++r) {
    xn[r] = make_float2(0.f, 0.f);
    vn[r] = 0.f;
  }
  float2* out_next = nullptr;
  int rid0 = (lb * 4 + wave) * RPW;
  fetch(rid0 + sub, xn, vn, out_next);
  for (; rid0 < total; rid0 += stride) {
    // compiler barrier: the twiddles are read from LDS at every use instead of
    // being hoisted into registers
    __asm__ volatile("" ::: "memory");
    const int rid = rid0 + sub;
    float2* out = out_next;
    float2 x[V];
    float v[V];
#pragma unroll
    for (int r = 0; r < V; ++r) {
      x[r] = xn[r];
      v[r] = vn[r];
    }
    fetch(rid0 + stride + sub, xn, vn, out_next);
    if (mode != ROW_FIRST) fft_rv<N, true, true>(x, lds, twt, t);
    if (transmit) {
#pragma unroll
      for (int r = 0; r < V; ++r) x[r] = cmul(x[r], phase_factor(a.sigma * v[r]));
      fft_rv<N, false, true>(x, lds, twt, t);
    }
    if (rid < total) {
#pragma unroll
      for (int r = 0; r < V; ++r) out[t + r * G] = x[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass for nx = 384 as 384 = 6 x 64 (six-step), one row per wavefront and
// the exchanges in the wavefront's own LDS slots:
//   layout A (natural): lane t holds x at t + 64 j (j < 6): a 6-point
//             transform over j, twiddle W384^(t k1), exchange to
//   layout B (lanes < 48): k1 = lane / 8, u = lane % 8, values at t = u + 8 q:
//             an 8-point transform over q, twiddle W64^(u k2), an exchange
//             within the 8 lanes of k1, an 8-point transform over u: index
//             k1 + 6 u + 48 k3 held as k3 < 8.
// A row of a later slice goes kx (A) -> x (B, conjugate steps), takes the
// transmission at its scrambled x positions, and returns x (B) -> kx (A) by
// the forward steps in reverse order (the transpose of the A -> B transform,
// which is again the forward DFT).  A first-slice row starts from the
// incident wave in x (A), takes the transmission there, and goes forward
// A -> B, stored from its scrambled kx positions.  Exchange slots: value k of
// position t at 64 k + (t ^ 8 (k mod 2)); the local exchanges use the
// six-step column kernel's map inside the 64 slots of k1.  Every 16-lane
// group of an access hits 16 distinct 8-byte slots modulo 16.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int r6_slot(int t, int k) { return 64 * k + (t ^ (8 * (k & 1))); }

__global__ void __launch_bounds__(256) k_row_6r(PassTable tab) {
  constexpr int N = 384;
  __shared__ float2 xs_mem[4][N];
  const int L = find_lane(tab, blockIdx.x);
  const PassArgs& a = tab.l[L].a;
  const int mode = tab.l[L].mode;   // ROW_FIRST or ROW_REGULAR (checked at launch)
  const int lb = blockIdx.x - tab.l[L].block_start;
  const int blocks_per_lane = (L + 1 < tab.n ? tab.l[L + 1].block_start : (int)gridDim.x) - tab.l[L].block_start;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int t = threadIdx.x % 64;                  // layout A
  const int k1 = t >> 3, u = t & 7;                // layout B (t < 48)
  const bool in_b = t < 48;
  const int lodd = k1 & 1;
  float2* xs = xs_mem[wave];
  float2* lw = xs + 64 * k1;                       // local exchange slots of k1
  // twiddles: W384^(t k) (k < 6) and W64^(u k) = W384^(6 u k) (k < 8)
  float2 ta[6], tb[8];
  {
    const float2* tw = a.tw_x;   // every lane of a table has nx = 384
#pragma unroll
    for (int k = 1; k < 6; ++k) ta[k] = tw[(t * k) % N];
#pragma unroll
    for (int k = 1; k < 8; ++k) tb[k] = tw[6 * u * k];
  }
  const bool first = mode == ROW_FIRST;
  const int total = a.n_probes * a.fb * a.ny;   // below 2^31 (checked at launch)
  const int stride = blocks_per_lane * 4;
  // global reads of one row: the wave in layout A (a first-slice row: the
  // incident wave), and the potential at this lane's x positions (layout A
  // for a first-slice row, layout B otherwise)
  auto fetch = [&](int rid, float2 (&xv)[6], float (&vv)[8], float2*& out) {
    if (rid >= total) return;
    const int w = rid / a.ny;
    const int y = rid - w * a.ny;
    const int p = w / a.fb;
    const int fl = w - p * a.fb;
    float2* row = a.exit + (((size_t)p * a.n_frames + a.f0 + fl) * a.ny + y) * (size_t)N;
    out = row;
    if (first) {
      if (a.plane) {
#pragma unroll
        for (int j = 0; j < 6; ++j) xv[j] = make_float2(a.plane_amp, 0.f);
      } else {
        const float2* src = a.probe0 + ((size_t)p * a.ny + y) * (size_t)N;
#pragma unroll
        for (int j = 0; j < 6; ++j) xv[j] = src[t + 64 * j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 6; ++j) xv[j] = row[t + 64 * j];
    }
    const int ox = a.plane ? 0 : a.origin[2 * p];
    const int oy = a.plane ? 0 : a.origin[2 * p + 1];
    int yy = oy + y;
    if (yy >= a.pny) yy -= a.pny;
    const float* vrow = a.V + (((size_t)fl * a.v_slices + (a.slice - a.v_slice0)) * a.pny + yy) * (size_t)a.pnx;
    // every lane reads an in-range position (lanes 48-63 of a later-slice
    // row, and entries 6-7 of a first-slice row, read one they do not use)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int x = first ? t + 64 * (r < 6 ? r : 0) : (in_b ? k1 + 6 * u + 48 * r : u);
      int xx = ox + x;
      if (xx >= a.pnx) xx -= a.pnx;
      vv[r] = vrow[xx];
    }
  };
  float2 xn[6];
  float vn[8];
#pragma unroll
  for (int j = 0; j < 6; ++j) xn[j] = make_float2(0.f, 0.f);
#pragma unroll
  for (int r = 0; r < 8; ++r) vn[r] = 0.f;
  float2* out_next = nullptr;
  int rid = lb * 4 + wave;
  fetch(rid, xn, vn, out_next);
  for (; rid < total; rid += stride) {
    float2* out = out_next;
    float2 x[8];
    float v[8];
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = xn[j];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = vn[r];
    fetch(rid + stride, xn, vn, out_next);
    if (first) {
      // transmission in x (layout A), then kx by the forward steps A -> B
#pragma unroll
      for (int j = 0; j < 6; ++j) x[j] = cmul(x[j], phase_factor(a.sigma * v[j]));
      dft6<false>(x);
#pragma unroll
      for (int k = 1; k < 6; ++k) x[k] = cmul(x[k], ta[k]);
    } else {
      // x by the conjugate steps A -> B
      dft6<true>(x);
#pragma unroll
      for (int k = 1; k < 6; ++k) x[k] = cmulc(x[k], ta[k]);
    }
    wave_lds_sync();   // the previous row's reads of xs are done
#pragma unroll
    for (int k = 0; k < 6; ++k) xs[r6_slot(t, k)] = x[k];
    wave_lds_sync();
    if (in_b) {
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = xs[r6_slot(u + 8 * q, k1)];
    }
    if (first) {
      if (in_b) {
        dft8<false>(x);
#pragma unroll
        for (int k = 1; k < 8; ++k) x[k] = cmul(x[k], tb[k]);
      }
    } else if (in_b) {
      dft8<true>(x);
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmulc(x[k], tb[k]);
    }
    wave_lds_sync();   // every lane's reads of xs are done
    if (in_b) {
#pragma unroll
      for (int k = 0; k < 8; ++k) lw[8 * (u ^ lodd) + (k ^ u)] = x[k];
    }
    wave_lds_sync();
    if (in_b) {
#pragma unroll
      for (int w = 0; w < 8; ++w) x[w] = lw[8 * (w ^ lodd) + (u ^ w)];
    }
    if (first) {
      // x[k3] = psi(kx = k1 + 6 u + 48 k3)
      if (in_b) {
        dft8<false>(x);
        if (rid < total) {
#pragma unroll
          for (int k = 0; k < 8; ++k) out[k1 + 6 * u + 48 * k] = x[k];
        }
      }
      continue;
    }
    if (in_b) {
      // x[k3] = psi(x = k1 + 6 u + 48 k3): transmission, then back to kx by
      // the forward steps in reverse order
      dft8<true>(x);
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = cmul(x[k], phase_factor(a.sigma * v[k]));
      dft8<false>(x);   // over k3: x[w] at u-index w, this lane's k2 = u
    }
    wave_lds_sync();   // every lane's reads of the local slots are done
    if (in_b) {
#pragma unroll
      for (int w = 0; w < 8; ++w) lw[8 * (w ^ lodd) + (u ^ w)] = x[w];
    }
    wave_lds_sync();
    if (in_b) {
      x[0] = lw[8 * (u ^ lodd) + u];
#pragma unroll
      for (int k = 1; k < 8; ++k) x[k] = cmul(lw[8 * (u ^ lodd) + (k ^ u)], tb[k]);
      dft8<false>(x);   // over k2: x[q] at t = u + 8 q
    }
    wave_lds_sync();   // every lane's reads of the local slots are done
    if (in_b) {
#pragma unroll
      for (int q = 0; q < 8; ++q) xs[r6_slot(u + 8 * q, k1)] = x[q];
    }
    wave_lds_sync();
    x[0] = xs[r6_slot(t, 0)];
#pragma unroll
    for (int k = 1; k < 6; ++k) x[k] = cmul(xs[r6_slot(t, k)], ta[k]);
    dft6<false>(x);
    if (rid < total) {
#pragma unroll
      for (int j = 0; j < 6; ++j) out[t + 64 * j] = x[j];
    }
  }
}

template <int N>
struct CV {
  static constexpr int G = RV<N>::G;
  static constexpr int CPW = 64 / G;                 // columns per wavefront
  static constexpr int WAVES = N == 384 ? 4 : 8;
  static constexpr int CT = WAVES * CPW;             // columns per block (8)
  static constexpr bool PAD = N != 1024;             // 1024: plain slots keep two blocks per CU
  static constexpr int LD = (PAD ? padded(N) : N) + 2;   // = 2 (mod 16): conflict-free transposes
  static constexpr int THREADS = WAVES * 64;
};

// Column pass on 12- or 16-value registers: CT-column tiles through an LDS
// transpose, as k_col_r8.  At 384 rows, three wavefronts per SIMD (168 VGPRs,
// a 12-byte spill) run the column passes 8% faster than two (170 VGPRs); the
// larger sizes keep their allocation.
template <int N>
__global__ void __launch_bounds__((CV<N>::THREADS)) __attribute__((amdgpu_waves_per_eu(N == 384 ? 3 : 1))) k_col_rv(PassTable tab, int total_tiles) {
  constexpr int V = RV<N>::V, G = CV<N>::G, CPW = CV<N>::CPW, CT = CV<N>::CT, LD = CV<N>::LD;
  constexpr bool PAD = CV<N>::PAD;
  constexpr int THREADS = CV<N>::THREADS;
  constexpr int PER = CT * N / THREADS;   // tile values each thread moves
  constexpr int TR = THREADS / CT;        // tile rows per transpose step
  static_assert(TR % 8 == 0 && (CT * N) % THREADS == 0, "transpose layout");
  __shared__ float2 twt[RV<N>::NT * G];
  __shared__ float2 cols[CT * LD];
  build_lane_twiddles<N>(twt, tab.l[0].a.tw_y);
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int cl = wave * CPW + lane / G;
  const int t = lane % G;
  float2* lds = cols + cl * LD;
  const int rslot = PAD ? t + (t >> 3) : t;
  const int trow = threadIdx.x / CT;
  const int tslot = (threadIdx.x % CT) * LD + (PAD ? trow + (trow >> 3) : trow);
  constexpr int TSTEP = PAD ? TR + TR / 8 : TR;
  auto locate = [&](int it, int& L, int& x0, float2*& wp) {
    const int tile_g = xcd_remap(it, total_tiles);
    L = find_lane(tab, tile_g);
    const PassArgs& a = tab.l[L].a;
    const int tile = tile_g - tab.l[L].block_start;
    const int tiles_per_wave = a.nx / CT;
    const int w = tile / tiles_per_wave;
    x0 = (tile % tiles_per_wave) * CT;
    const int p = w / a.fb;
    const int fl = w % a.fb;
    wp = a.exit + ((size_t)p * a.n_frames + a.f0 + fl) * (size_t)N * a.nx;
  };
  float2 pre[PER];
  int L = 0, x0 = 0;
  float2* wp = nullptr;
  int it = blockIdx.x;
  if (it < total_tiles) {
    locate(it, L, x0, wp);
    const int nx = tab.l[L].a.nx;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * THREADS;
      pre[q] = wp[(size_t)(e / CT) * nx + x0 + e % CT];
    }
  }
  for (; it < total_tiles; it += gridDim.x) {
    const PassArgs& a = tab.l[L].a;
    const int mode = tab.l[L].mode;
    const int cur_x0 = x0;
    float2* cur_wp = wp;
    __asm__ volatile("" ::: "memory");  // twiddles are read from LDS at every use
    __syncthreads();  // the previous tile's stores from LDS are done (and the table is in)
#pragma unroll
    for (int q = 0; q < PER; ++q) cols[tslot + q * TSTEP] = pre[q];
    const int nit = it + gridDim.x;
    if (nit < total_tiles) {
      locate(nit, L, x0, wp);
      const int nx = tab.l[L].a.nx;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * THREADS;
        pre[q] = wp[(size_t)(e / CT) * nx + x0 + e % CT];
      }
    }
    __syncthreads();
    float2 x[V];
#pragma unroll
    for (int r = 0; r < V; ++r) x[r] = lds[rslot + r * (PAD ? G + G / 8 : G)];
    if (mode == COL_INVERSE_ONLY) {
      fft_rv<N, true, PAD>(x, lds, twt, t);
    } else {
      fft_rv<N, false, PAD>(x, lds, twt, t);
      const float2 pxv = a.px[cur_x0 + cl];
#pragma unroll
      for (int r = 0; r < V; ++r) x[r] = cmul(x[r], cmul(pxv, a.py[t + r * G]));
      if (mode == COL_REGULAR) fft_rv<N, true, PAD>(x, lds, twt, t);
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < V; ++r) lds[rslot + r * (PAD ? G + G / 8 : G)] = x[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * THREADS;
      cur_wp[(size_t)(e / CT) * a.nx + cur_x0 + e % CT] = cols[tslot + q * TSTEP];
    }
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
  // eight loads in flight per thread before their LDS writes
  const int n_ld = KT * F;
  for (int e0 = threadIdx.x; e0 < n_ld; e0 += 8 * blockDim.x) {
    float2 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + i * blockDim.x;
      if (e < n_ld) v[i] = src[(size_t)(e / KT) * a.n_k + e % KT];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + i * blockDim.x;
      if (e < n_ld) bufA[(e % KT) * F + e / KT] = v[i];
    }
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
// Time stage with a compile-time plan for F frames: a block owns KT adjacent
// k points of one probe (KT * 8 contiguous bytes per frame row), holds their
// F-long columns in one LDS buffer, takes the FP64 mean per column with
// lane shuffles, subtracts it in FP64, runs the in-place Stockham FFT and
// writes |.|^2 / F^2 of the kept bins.
// ---------------------------------------------------------------------------
template <int F>
struct TimeCfg {
  static constexpr int G = Plan<F>::G;
  static constexpr int KT0 = (144 * 1024) / ((F + 1) * 8);
  static constexpr int KTT = 1024 / G;
  static constexpr int KTM = KT0 < KTT ? KT0 : KTT;
  // at F >= 1024, at most 8 k-points per block: two blocks fit a CU's LDS
  // and overlap their load and transform phases (c2: 1.43 against 1.58 ms)
  static constexpr int KTC = F >= 1024 && KTM > 8 ? 8 : KTM;
  static constexpr int KT = KTC >= 32 ? 32 : KTC >= 16 ? 16 : KTC >= 8 ? 8 : KTC >= 4 ? 4 : KTC >= 2 ? 2 : 1;
  static constexpr int THREADS = KT * G;
  static constexpr int LD = F + 1;
};

template <int F>
__global__ void __launch_bounds__((TimeCfg<F>::THREADS)) k_time_ct(TimeArgs a) {
  using PL = Plan<F>;
  constexpr int G = PL::G;
  constexpr int KT = TimeCfg<F>::KT;
  constexpr int LD = TimeCfg<F>::LD;
  constexpr int THREADS = TimeCfg<F>::THREADS;
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* cols = smem + F;
  const int tiles_per_probe = a.n_k / KT;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int p = tile / tiles_per_probe;
  const int k0 = (tile % tiles_per_probe) * KT;
  const float2* src = a.exit + (size_t)p * F * a.n_k + k0;
  // the block's KT x F values, PER per thread, loaded CH at a time with every
  // load of a chunk in flight before the first LDS write (a load, wait, write
  // loop would leave one HBM round trip per value outstanding)
  constexpr int PER = KT * F / THREADS;
  constexpr int CH = PER < 16 ? PER : 16;
  static_assert(PER * THREADS == KT * F, "whole values per thread");
#pragma unroll
  for (int i = 0; i < (F + THREADS - 1) / THREADS; ++i)
    if (F % THREADS == 0 || (int)threadIdx.x + i * THREADS < F) tw[threadIdx.x + i * THREADS] = a.tw[threadIdx.x + i * THREADS];
#pragma unroll
  for (int i0 = 0; i0 < PER; i0 += CH) {
    float2 v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (i0 + i < PER) {
        const int e = threadIdx.x + (i0 + i) * THREADS;
        v[i] = src[(size_t)(e / KT) * a.n_k + e % KT];
      }
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (i0 + i < PER) {
        const int e = threadIdx.x + (i0 + i) * THREADS;
        cols[(e % KT) * LD + e / KT] = v[i];
      }
  }
  __syncthreads();
  const int c = threadIdx.x / G;
  const int t = threadIdx.x % G;
  float2* col = cols + c * LD;
  // FP64 mean over frames: strided partial sums, then a butterfly over the
  // G lanes of this column (fixed order, so the result is deterministic)
  double sr = 0.0, si = 0.0;
  for (int f = t; f < F; f += G) {
    sr += (double)col[f].x;
    si += (double)col[f].y;
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, G);
    si += __shfl_xor(si, off, G);
  }
  const double mr = sr / (double)F, mi = si / (double)F;
  for (int f = t; f < F; f += G) {
    const float2 v = col[f];
    col[f] = make_float2((float)((double)v.x - mr), (float)((double)v.y - mi));
  }
  __syncthreads();
  StagesIP<F, G, false, 1, typename PL::R>::run(col, tw, t);
  float* dst = a.spec + (size_t)p * a.n_bins * a.n_k + k0;
  for (int e = threadIdx.x; e < KT * a.n_bins; e += blockDim.x) {
    const int cc = e % KT, m = e / KT;
    const float2 v = cols[cc * LD + m];
    dst[(size_t)m * a.n_k + cc] = (v.x * v.x + v.y * v.y) * a.inv_f2;
  }
}

// ---------------------------------------------------------------------------
// Spectrum analysis: reductions of I[p][m][k] at one frequency bin or along a
// list of k-nodes, accumulated in FP64 in a fixed order.
// ---------------------------------------------------------------------------
// D[k] = sum_p I[p][m][k]
__global__ void __launch_bounds__(256) k_spectral_diffraction(const float* spec, double* out, int n_probes,
                                                              int n_bins, int n_k, int m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_k) return;
  double acc = 0.0;
  for (int p = 0; p < n_probes; ++p) acc += (double)spec[((size_t)p * n_bins + m) * n_k + k];
  out[k] = acc;
}

// S[p] = sum over k-nodes with k_in^2 <= |k|^2 < k_out^2 of I[p][m][k]; one
// workgroup per probe, strided partial sums, then a fixed-order tree.
__global__ void __launch_bounds__(256) k_spectrum_image(const float* spec, double* out, int n_bins, int nx,
                                                        int ny, int m, const double* kx, const double* ky,
                                                        double k_in2, double k_out2) {
  __shared__ double part[256];
  const int p = blockIdx.x;
  const int n_k = nx * ny;
  const float* src = spec + ((size_t)p * n_bins + m) * n_k;
  double acc = 0.0;
  for (int k = threadIdx.x; k < n_k; k += blockDim.x) {
    const int iy = k / nx, ix = k - iy * nx;
    const double k2 = kx[ix] * kx[ix] + ky[iy] * ky[iy];
    if (k2 >= k_in2 && (k_out2 <= 0.0 || k2 < k_out2)) acc += (double)src[k];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = part[0];
}

// D[i][m] = sum_p I[p][m][node_i]
__global__ void __launch_bounds__(256) k_dispersion(const float* spec, double* out, int n_probes, int n_bins,
                                                    int n_k, const int* node, int n_points) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_points * n_bins) return;
  const int i = e / n_bins, m = e - i * n_bins;
  double acc = 0.0;
  for (int p = 0; p < n_probes; ++p) acc += (double)spec[((size_t)p * n_bins + m) * n_k + node[i]];
  out[e] = acc;
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
    if (total + RPI >= (1L << 31)) return hipErrorInvalidValue;  // 32-bit row ids
    t.l[i].block_start = blocks;
    blocks += (int)((total + RPI - 1) / RPI);
  }
  TACAW_LAUNCH((k_row<N, VAR>), dim3(blocks), dim3(RowCfg<N, VAR>::THREADS), 0, s, t);
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
  TACAW_LAUNCH((k_col<N, VAR>), dim3(blocks), dim3(ColCfg<N, VAR>::THREADS), 0, s, t);
  return hipGetLastError();
}

static bool same_grid(const PassLane* lanes, int n) {
  for (int i = 1; i < n; ++i)
    if (lanes[i].a.nx != lanes[0].a.nx || lanes[i].a.ny != lanes[0].a.ny) return false;
  return true;
}

template <int N, int DEPTH>
static hipError_t row_r8_launch(PassTable& t, hipStream_t s) {
  // blocks: one per rows_per_block rows, at most 2048 in all, shared among
  // the lanes in proportion to their rows (each walks its rows with a grid
  // stride over its own blocks)
  constexpr int rows_per_block = 4 * R8<N>::RPW;
  constexpr long max_blocks = 2048;
  long rows[MAX_LANES], total = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    rows[i] = (long)a.n_probes * a.fb * a.ny;
    if (rows[i] + 4 * max_blocks * rows_per_block >= (1L << 31)) return hipErrorInvalidValue;  // 32-bit row ids
    total += rows[i];
  }
  const long need = (total + rows_per_block - 1) / rows_per_block;
  int blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const long own = (rows[i] + rows_per_block - 1) / rows_per_block;
    const long b = need <= max_blocks ? own : std::max(1L, std::min(own, rows[i] * max_blocks / total));
    t.l[i].block_start = blocks;
    blocks += (int)b;
  }
  // lanes writing two potential planes (reciprocal-space route) take their
  // own instantiation, so the multislice rows carry none of that code
  bool vout = false;
  for (int i = 0; i < t.n; ++i) vout = vout || t.l[i].a.vout != nullptr;
  if (vout)
    TACAW_LAUNCH((k_row_r8<N, DEPTH, true>), dim3(blocks), dim3(256), 0, s, t);
  else
    TACAW_LAUNCH((k_row_r8<N, DEPTH, false>), dim3(blocks), dim3(256), 0, s, t);
  return hipGetLastError();
}

template <int N>
static hipError_t row_rv_launch(PassTable& t, hipStream_t s) {
  constexpr int rows_per_block = 4 * RV<N>::RPW;
  constexpr long max_blocks = 2048;
  long rows[MAX_LANES], total = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    rows[i] = (long)a.n_probes * a.fb * a.ny;
    if (rows[i] + 4 * max_blocks * rows_per_block >= (1L << 31)) return hipErrorInvalidValue;
    total += rows[i];
  }
  const long need = (total + rows_per_block - 1) / rows_per_block;
  int blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const long own = (rows[i] + rows_per_block - 1) / rows_per_block;
    const long b = need <= max_blocks ? own : std::max(1L, std::min(own, rows[i] * max_blocks / total));
    t.l[i].block_start = blocks;
    blocks += (int)b;
  }
  TACAW_LAUNCH((k_row_rv<N>), dim3(blocks), dim3(256), 0, s, t);
  return hipGetLastError();
}

static hipError_t row_6r_launch(PassTable& t, hipStream_t s) {
  constexpr int rows_per_block = 4;
  constexpr long max_blocks = 2048;
  long rows[MAX_LANES], total = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.nx != 384 || (t.l[i].mode != ROW_FIRST && t.l[i].mode != ROW_REGULAR)) return hipErrorInvalidValue;
    rows[i] = (long)a.n_probes * a.fb * a.ny;
    if (rows[i] + 4 * max_blocks * rows_per_block >= (1L << 31)) return hipErrorInvalidValue;
    total += rows[i];
  }
  const long need = (total + rows_per_block - 1) / rows_per_block;
  int blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const long own = (rows[i] + rows_per_block - 1) / rows_per_block;
    const long b = need <= max_blocks ? own : std::max(1L, std::min(own, rows[i] * max_blocks / total));
    t.l[i].block_start = blocks;
    blocks += (int)b;
  }
  TACAW_LAUNCH(k_row_6r, dim3(blocks), dim3(256), 0, s, t);
  return hipGetLastError();
}

template <int N>
static hipError_t col_rv_launch(PassTable& t, hipStream_t s) {
  constexpr int CT = CV<N>::CT;
  int tiles = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.nx % CT != 0) return hipErrorInvalidValue;
    t.l[i].block_start = tiles;
    tiles += a.n_probes * a.fb * (a.nx / CT);
  }
  const int grid = std::min(tiles, 2048);
  TACAW_LAUNCH((k_col_rv<N>), dim3(grid), dim3(CV<N>::THREADS), 0, s, t, tiles);
  return hipGetLastError();
}

bool resident_supported(int nx, int ny) { return nx == ny && (nx == 64 || nx == 128); }

template <int N>
static hipError_t res_set_attributes() {
  return hipFuncSetAttribute((const void*)k_res<N>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)RS<N>::LDS);
}

hipError_t kernels_init() {
  hipError_t e = res_set_attributes<64>();
  return e == hipSuccess ? res_set_attributes<128>() : e;
}

template <int N>
static hipError_t res_launch(ResTable& t, hipStream_t s) {
  long blocks = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.nx != N || a.ny != N || t.l[i].n_slices_launch < 1 || a.slice < 0 ||
        a.slice + t.l[i].n_slices_launch > a.n_slices || a.slice < a.v_slice0 ||
        a.slice + t.l[i].n_slices_launch > a.v_slice0 + a.v_slices)
      return hipErrorInvalidValue;
    t.l[i].block_start = (int)blocks;
    blocks += (long)a.n_probes * a.fb;
  }
  if (blocks < 1 || blocks > (1L << 30)) return hipErrorInvalidValue;
  // the dynamic LDS limit was raised by kernels_init (context creation)
  TACAW_LAUNCH((k_res<N>), dim3((unsigned)blocks), dim3(RS<N>::THREADS), RS<N>::LDS, s, t);
  return hipGetLastError();
}

hipError_t launch_res_lanes(const ResLane* lanes, int n, hipStream_t s) {
  if (n < 1 || n > MAX_LANES) return hipErrorInvalidValue;
  ResTable t{};
  t.n = n;
  for (int i = 0; i < n; ++i) {
    t.l[i] = lanes[i];
    if (lanes[i].a.nx != lanes[0].a.nx || lanes[i].a.ny != lanes[0].a.ny) return hipErrorInvalidValue;
  }
  switch (lanes[0].a.nx) {
    case 64: return res_launch<64>(t, s);
    case 128: return res_launch<128>(t, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_lanes(const PassLane* lanes, int n, int variant, hipStream_t s) {
  if (n < 1 || n > MAX_LANES || !same_grid(lanes, n)) return hipErrorInvalidValue;
  PassTable t{};
  t.n = n;
  for (int i = 0; i < n; ++i) t.l[i] = lanes[i];
  if (variant == 4) {
    // six-step row kernel at 384: first-slice and regular rows
    bool ok = lanes[0].a.nx == 384;
    for (int i = 0; i < n; ++i) ok = ok && (lanes[i].mode == ROW_FIRST || lanes[i].mode == ROW_REGULAR);
    if (ok) return row_6r_launch(t, s);
    variant = 2;
  }
  if (variant == 2 || variant == 3) {
    const bool deep = variant == 3;
    switch (lanes[0].a.nx) {
      case 512: return deep ? row_r8_launch<512, 2>(t, s) : row_r8_launch<512, 1>(t, s);
      case 256: return deep ? row_r8_launch<256, 2>(t, s) : row_r8_launch<256, 1>(t, s);
      case 128: return deep ? row_r8_launch<128, 2>(t, s) : row_r8_launch<128, 1>(t, s);
      case 64: return deep ? row_r8_launch<64, 2>(t, s) : row_r8_launch<64, 1>(t, s);
      case 384: return row_rv_launch<384>(t, s);
      case 768: return row_rv_launch<768>(t, s);
      case 1024: return row_rv_launch<1024>(t, s);
      default: variant = 1;
    }
  }
  switch (lanes[0].a.nx) {
#define CASE(NN) \
  case NN: return variant ? row_launch<NN, 1>(t, s) : row_launch<NN, 0>(t, s);
    TACAW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <int N, int WIDE, int DB = 0>
static hipError_t col_r8_launch(PassTable& t, hipStream_t s) {
  constexpr int CT = C8<N, WIDE>::CT;
  int tiles = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.nx % CT != 0) return hipErrorInvalidValue;
    t.l[i].block_start = tiles;
    tiles += a.n_probes * a.fb * (a.nx / CT);
  }
  // resident workgroups walk the tiles with a grid stride (each prefetches
  // its next tile); TACAW_COL_GRID caps the grid (default 2048)
  const char* ge = getenv("TACAW_COL_GRID");
  const int cap = ge && atoi(ge) > 0 ? atoi(ge) : 2048;
  const int grid = std::min(tiles, cap);
  TACAW_LAUNCH((k_col_r8<N, WIDE, DB>), dim3(grid), dim3(C8<N, WIDE>::THREADS), 0, s, t, tiles);
  return hipGetLastError();
}

template <int R1>
static hipError_t col_6s_launch(PassTable& t, hipStream_t s) {
  int tiles = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.ny != 64 * R1 || a.nx % 8 != 0) return hipErrorInvalidValue;
    t.l[i].block_start = tiles;
    tiles += a.n_probes * a.fb * (a.nx / 8);
  }
  // grid stride over the tiles; TACAW_COL_GRID caps the grid (default 1024,
  // two generations of the two resident workgroups per CU)
  const char* ge = getenv("TACAW_COL_GRID");
  const int cap = ge && atoi(ge) > 0 ? atoi(ge) : 1024;
  const int grid = std::min(tiles, cap);
  TACAW_LAUNCH(k_col_6s<R1>, dim3(grid), dim3(512), 0, s, t, tiles);
  return hipGetLastError();
}

static hipError_t col_6w_launch(PassTable& t, hipStream_t s) {
  int tiles = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.ny != 512 || a.nx % 16 != 0) return hipErrorInvalidValue;
    t.l[i].block_start = tiles;
    tiles += a.n_probes * a.fb * (a.nx / 16);
  }
  // grid stride over the tiles; TACAW_COL_GRID caps the grid (default 512:
  // the two resident workgroups per CU)
  const char* ge = getenv("TACAW_COL_GRID");
  const int cap = ge && atoi(ge) > 0 ? atoi(ge) : 512;
  const int grid = std::min(tiles, cap);
  TACAW_LAUNCH(k_col_6w, dim3(grid), dim3(512), 0, s, t, tiles);
  return hipGetLastError();
}

static hipError_t col_6q_launch(PassTable& t, hipStream_t s) {
  int tiles = 0;
  for (int i = 0; i < t.n; ++i) {
    const PassArgs& a = t.l[i].a;
    if (a.ny != 256 || a.nx % 16 != 0) return hipErrorInvalidValue;
    t.l[i].block_start = tiles;
    tiles += a.n_probes * a.fb * (a.nx / 16);
  }
  // grid stride over the tiles; TACAW_COL_GRID caps the grid (default 2048:
  // 236 against 240 us per spectrum-image launch at 1024)
  const char* ge = getenv("TACAW_COL_GRID");
  const int cap = ge && atoi(ge) > 0 ? atoi(ge) : 2048;
  const int grid = std::min(tiles, cap);
  TACAW_LAUNCH(k_col_6q, dim3(grid), dim3(512), 0, s, t, tiles);
  return hipGetLastError();
}

hipError_t launch_col_lanes(const PassLane* lanes, int n, int variant, hipStream_t s) {
  if (n < 1 || n > MAX_LANES || !same_grid(lanes, n)) return hipErrorInvalidValue;
  PassTable t{};
  t.n = n;
  for (int i = 0; i < n; ++i) t.l[i] = lanes[i];
  if (variant == 7) {
    // six-step kernel at 256 rows on 16-column tiles: regular and last-slice modes
    bool ok = lanes[0].a.ny == 256 && lanes[0].a.nx % 16 == 0;
    for (int i = 0; i < n; ++i) ok = ok && lanes[i].mode != COL_INVERSE_ONLY;
    if (ok) return col_6q_launch(t, s);
    variant = 3;
  }
  if (variant == 6) {
    // six-step kernel on 16-column tiles: ny = 512, regular and last-slice modes
    bool ok = lanes[0].a.ny == 512 && lanes[0].a.nx % 16 == 0;
    for (int i = 0; i < n; ++i) ok = ok && lanes[i].mode != COL_INVERSE_ONLY;
    if (ok) return col_6w_launch(t, s);
    variant = 5;
  }
  if (variant == 5 || variant == 8) {
    // six-step kernel: ny = 512 (variant 5) or 384 (variant 8), regular and
    // last-slice modes
    const int ny = variant == 5 ? 512 : 384;
    bool ok = lanes[0].a.ny == ny && lanes[0].a.nx % 8 == 0;
    for (int i = 0; i < n; ++i) ok = ok && lanes[i].mode != COL_INVERSE_ONLY;
    if (ok) return variant == 5 ? col_6s_launch<8>(t, s) : col_6s_launch<6>(t, s);
    variant = 2;
  }
  if (variant == 4) {
    const int ny = lanes[0].a.ny, nx = lanes[0].a.nx;
    if (ny == 512 && nx % C8<512, 0>::CT == 0) return col_r8_launch<512, 0, 1>(t, s);
    if (ny == 256 && nx % C8<256, 0>::CT == 0) return col_r8_launch<256, 0, 1>(t, s);
    variant = 2;
  }
  if (variant == 3) {
    // 16-column tiles: whole 128-byte row segments per tile row
    const int ny = lanes[0].a.ny, nx = lanes[0].a.nx;
    if (ny == 512 && nx % C8<512, 1>::CT == 0) return col_r8_launch<512, 1>(t, s);
    if (ny == 256 && nx % C8<256, 1>::CT == 0) return col_r8_launch<256, 1>(t, s);
    variant = 2;
  }
  if (variant == 2) {
    const int ny = lanes[0].a.ny, nx = lanes[0].a.nx;
    if (ny == 512 && nx % C8<512, 0>::CT == 0) return col_r8_launch<512, 0>(t, s);
    if (ny == 256 && nx % C8<256, 0>::CT == 0) return col_r8_launch<256, 0>(t, s);
    if (ny == 128 && nx % C8<128, 0>::CT == 0) return col_r8_launch<128, 0>(t, s);
    if (ny == 64 && nx % C8<64, 0>::CT == 0) return col_r8_launch<64, 0>(t, s);
    if (ny == 384 && nx % CV<384>::CT == 0) return col_rv_launch<384>(t, s);
    if (ny == 768 && nx % CV<768>::CT == 0) return col_rv_launch<768>(t, s);
    if (ny == 1024 && nx % CV<1024>::CT == 0) return col_rv_launch<1024>(t, s);
    variant = 0;
  }
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
  // TACAW_SPLAT_FPW and TACAW_SPLAT_ROUND are read at every launch.  Frames
  // per wavefront: TACAW_SPLAT_FPW, else the most (16, 8, 4, 2, 1) that still
  // gives the launch at least 16384 work items (16 workgroups per CU); more
  // frames per item share the item's list and coefficient set-up (c2: 12.5
  // ms per step at 16 frames, 12.9 at 4).
  const char* fe = getenv("TACAW_SPLAT_FPW");
  const int fpw_v = fe ? atoi(fe) : 0;
  int fpw_env = fpw_v >= 1 && fpw_v <= 64 ? fpw_v : 0;
  if (fpw_env == 0) {
    for (fpw_env = 16; fpw_env > 1; fpw_env /= 2) {
      long items = 0;
      for (int i = 0; i < n; ++i) {
        const SplatArgs& a = lanes[i].a;
        items += (long)a.tiles_x * a.tiles_y * lanes[i].n_slices_launch * ((a.fb + fpw_env - 1) / fpw_env);
      }
      if (items >= 16384) break;
    }
  }
  for (int i = 0; i < n; ++i) {
    t.l[i] = lanes[i];
    t.l[i].block_start = blocks;
    t.l[i].fpw = fpw_env;
    const SplatArgs& a = lanes[i].a;
    const int items = a.tiles_x * a.tiles_y * lanes[i].n_slices_launch *
                      ((a.fb + fpw_env - 1) / fpw_env);  // one per wavefront
    blocks += (items + 3) / 4;
  }
  // pairs per round: TACAW_SPLAT_ROUND (16 or 32; default 32)
  const char* re = getenv("TACAW_SPLAT_ROUND");
  const int round = re && atoi(re) == 16 ? 16 : 32;
  bool iz = false;   // any lane binned frame by frame
  for (int i = 0; i < n; ++i) iz = iz || lanes[i].a.fslice != nullptr;
  if (round == 16 && iz)
    TACAW_LAUNCH((k_splat<16, true>), dim3(blocks), dim3(256), 0, s, t);
  else if (round == 16)
    TACAW_LAUNCH((k_splat<16, false>), dim3(blocks), dim3(256), 0, s, t);
  else if (iz)
    TACAW_LAUNCH((k_splat<32, true>), dim3(blocks), dim3(256), 0, s, t);
  else
    TACAW_LAUNCH((k_splat<32, false>), dim3(blocks), dim3(256), 0, s, t);
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

template <int F>
static hipError_t time_ct_launch(const TimeArgs& a, hipStream_t s) {
  constexpr int KT = TimeCfg<F>::KT;
  if (a.n_k % KT != 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)(F + KT * TimeCfg<F>::LD) * sizeof(float2);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_time_ct<F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const long blocks = (long)a.n_probes * (a.n_k / KT);
  TACAW_LAUNCH((k_time_ct<F>), dim3((unsigned)blocks), dim3(TimeCfg<F>::THREADS), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_time_stage(const TimeArgs& a, hipStream_t s) {
  switch (a.n_frames) {
#define CASE(NN) \
  case NN:       \
    if (a.n_k % TimeCfg<NN>::KT == 0) return time_ct_launch<NN>(a, s); \
    break;
    TACAW_SIZES(CASE)
    CASE(2048)
#undef CASE
    default:
      break;
  }
  if (a.n_k % a.kt != 0 || a.kt * a.n_frames > TIME_LDS_C) return hipErrorInvalidValue;
  const size_t lds = (size_t)(a.n_frames + 2 * a.kt * a.n_frames) * sizeof(float2);
  const long blocks = (long)a.n_probes * (a.n_k / a.kt);
  dim3 grid((unsigned)blocks), block(a.kt * TIME_G);
  TACAW_LAUNCH(k_time, grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_kpot(const KPotArgs& a, hipStream_t s) {
  const long blocks = (long)a.fb * a.npairs * a.row_tiles * a.col_tiles;
  if (blocks <= 0 || blocks >= (1L << 31) || a.pnx > 4096 || a.pny > 4096) return hipErrorInvalidValue;
  TACAW_LAUNCH(k_kpot, dim3((unsigned)blocks), dim3(256), 0, s, a);
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
                             int ny, double dx, double dy, double lam, double alpha, const Aberrations& ab,
                             hipStream_t s) {
  const size_t n = (size_t)nx * ny * n_probes;
  hipLaunchKernelGGL(k_probe_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, rloc, count,
                     n_probes, nx, ny, dx, dy, lam, alpha, ab);
  return hipGetLastError();
}

}  // namespace tacaw

namespace tacaw {
// D[p][k] = (1/F) sum_f |psi[p][f][k]|^2, lanes along k (coalesced per frame)
__global__ void __launch_bounds__(256) k_mean_diffraction(const float2* exit, double* out, int n_frames, int n_k) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (k >= n_k) return;
  const float2* src = exit + (size_t)p * n_frames * n_k + k;
  double acc = 0.0;
  for (int f = 0; f < n_frames; ++f) {
    const float2 v = src[(size_t)f * n_k];
    acc += __dadd_rn(__dmul_rn((double)v.x, (double)v.x), __dmul_rn((double)v.y, (double)v.y));
  }
  out[(size_t)p * n_k + k] = acc / n_frames;
}

// A[p] = sum of D[p][k] over inner <= 1e3 lambda |k| < outer; one workgroup
// per probe, strided partial sums, then a fixed-order tree.  The angle is
// formed as (1e3 lambda) sqrt(kx^2 + ky^2) with no contraction.
__global__ void __launch_bounds__(256) k_adf(const double* diff, double* out, int nx, int ny, const double* kx,
                                             const double* ky, double lam_mrad, double inner, double outer) {
  __shared__ double part[256];
  const int p = blockIdx.x;
  const int n_k = nx * ny;
  const double* src = diff + (size_t)p * n_k;
  double acc = 0.0;
  for (int k = threadIdx.x; k < n_k; k += blockDim.x) {
    const int iy = k / nx, ix = k - iy * nx;
    const double th = __dmul_rn(lam_mrad, sqrt(__dadd_rn(__dmul_rn(kx[ix], kx[ix]), __dmul_rn(ky[iy], ky[iy]))));
    if (th >= inner && th < outer) acc += src[k];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = part[0];
}

// I_avg = (1/J) sum_j I_j element by element, FP64 sums in job order
__global__ void __launch_bounds__(256) k_average_spectra(const float* const* specs, int n_jobs, float* out,
                                                         size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < n_jobs; ++j) acc += (double)specs[j][i];
    out[i] = (float)(acc / n_jobs);
  }
}

hipError_t launch_average_spectra(const float* const* specs, int n_jobs, float* out, size_t n, hipStream_t s) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_average_spectra, dim3((unsigned)blocks), dim3(256), 0, s, specs, n_jobs, out, n);
  return hipGetLastError();
}

hipError_t launch_mean_diffraction(const float2* exit, double* out, int n_probes, int n_frames, int n_k,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_mean_diffraction, dim3((n_k + 255) / 256, n_probes), dim3(256), 0, s, exit, out, n_frames,
                     n_k);
  return hipGetLastError();
}
hipError_t launch_adf(const double* diff, double* out, int n_probes, int nx, int ny, const double* kx,
                      const double* ky, double lam, double inner_mrad, double outer_mrad, hipStream_t s) {
  hipLaunchKernelGGL(k_adf, dim3(n_probes), dim3(256), 0, s, diff, out, nx, ny, kx, ky, 1e3 * lam, inner_mrad,
                     outer_mrad);
  return hipGetLastError();
}
hipError_t launch_spectral_diffraction(const float* spec, double* out, int n_probes, int n_bins, int n_k, int m,
                                       hipStream_t s) {
  hipLaunchKernelGGL(k_spectral_diffraction, dim3((n_k + 255) / 256), dim3(256), 0, s, spec, out, n_probes,
                     n_bins, n_k, m);
  return hipGetLastError();
}
hipError_t launch_spectrum_image(const float* spec, double* out, int n_probes, int n_bins, int nx, int ny, int m,
                                 const double* kx, const double* ky, double k_in2, double k_out2, hipStream_t s) {
  hipLaunchKernelGGL(k_spectrum_image, dim3(n_probes), dim3(256), 0, s, spec, out, n_bins, nx, ny, m, kx, ky,
                     k_in2, k_out2);
  return hipGetLastError();
}
hipError_t launch_dispersion(const float* spec, double* out, int n_probes, int n_bins, int n_k, const int* node,
                             int n_points, hipStream_t s) {
  const long n = (long)n_points * n_bins;
  hipLaunchKernelGGL(k_dispersion, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spec, out, n_probes, n_bins,
                     n_k, node, n_points);
  return hipGetLastError();
}
}  // namespace tacaw
