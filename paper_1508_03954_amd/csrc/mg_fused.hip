// Fused finest-level sweep: standalone kernels, tile table and launchers.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstring>

#include "mg_fused_ops.h"

namespace mg {

// Tile of a block.  Order 0: tiles in launch order (x fastest).  Order 1:
// blocks are handed to the XCDs round robin (block i runs on XCD i mod 8), so
// block i is given the (i div 8)-th tile of the i mod 8-th contiguous chunk of
// tiles numbered y fastest: the tiles an XCD runs at one time are y and x
// neighbours, and the halo rows they share are fetched into that XCD's L2 once.
// Order 2: the XCDs take y bands.  Tiles are numbered band by band (a band
// is ceil(gy / 8) y tiles high, the last one may be lower), inside a band z
// major and x fastest, and block i takes the (i div 8)-th tile of the (i mod
// 8)-th contiguous chunk of that numbering.  The tiles an XCD runs at one time
// are then the x and y neighbours of one z range: the halo rows and columns
// they share stay in its L2, and whole rows of the grid are read together
// (order 1 groups y neighbours only, and reads each row in tile-wide pieces
// far apart in time, which costs more than it saves on large grids).
// Every mapping is a bijection for any tile count; a different dispatch order
// changes only the speed.
__device__ inline void fused3_block_tile(int order, int gx, int gy, int gz, int& bx, int& by, int& bz) {
  const int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (order == 0) {
    bx = lin % gx;
    by = (lin / gx) % gy;
    bz = lin / (gx * gy);
    return;
  }
  const int N = gx * gy * gz, q = N >> 3, rem = N & 7;
  const int k = lin & 7, local = lin >> 3;
  const int t = k * q + min(k, rem) + local;
  if (order == 1) {
    by = t % gy;
    bx = (t / gy) % gx;
    bz = t / (gx * gy);
    return;
  }
  const int h = (gy + 7) >> 3;
  const int band_tiles = gx * h * gz;
  const int b = t / band_tiles;
  const int y0 = b * h;
  const int hb = min(h, gy - y0);
  const int r = t - b * band_tiles;
  bx = r % gx;
  by = y0 + (r / gx) % hb;
  bz = (r / gx) / hb;
}

// PF > 1 tiles keep PF planes of loads in flight and take more registers:
// they are meant for grids with few waves per CU, so they ask for 2 waves per SIMD.
template <class T, int TYC, int RPT, int ZC, int VAR, int PF>
__global__ __launch_bounds__(64 * (3 * TYC / RPT), PF == 1 ? 3 : 2) void k_fused3(FusedArgs<T> a) {
  __shared__ F3Lds<T, TYC, RPT, VAR == 2> sm;
  int bx, by, bz;
  fused3_block_tile(a.order, gridDim.x, gridDim.y, gridDim.z, bx, by, bz);
  // partial sums are indexed by tile, so the norm's summation order does not
  // depend on the block order
  double* part = a.partials ? a.partials + 2 * (bx + gridDim.x * (by + gridDim.y * bz)) : nullptr;
  fused3_tile<T, TYC, RPT, ZC, VAR, kSweep, PF>(a, bx, by, bz, part, sm);
}

template <class T, int ZC, bool BPX>
__global__ __launch_bounds__(64) void k_fused2(FusedArgs<T> a) {
  __shared__ cpx<T> Gz[2][F2_GX];
  __shared__ cpx<T> Sz[2][F2_GX];
  double* part = a.partials ? a.partials + 2 * (blockIdx.x + gridDim.x * blockIdx.y) : nullptr;
  fused2_wave_tile<T, ZC, BPX>(a, blockIdx.x, blockIdx.y, Gz, Sz, part);
}

// Tile variants of the fused sweep (coarse rows per block, rows per thread,
// coarse planes per block, block order, prefetch depth); the context picks one
// per problem (default table or autotuning on the device).
struct TileShape3 { int tyc, rpt, zc, order, pf; };
constexpr TileShape3 kTiles3[] = {{2, 2, 9, 0, 1},  {2, 2, 14, 0, 1}, {2, 2, 21, 0, 1}, {2, 2, 27, 0, 1},
                                  {2, 2, 28, 0, 1}, {4, 2, 14, 0, 1}, {4, 2, 21, 0, 1}, {4, 2, 28, 0, 1},
                                  {2, 1, 14, 0, 1}, {2, 1, 21, 0, 1}, {2, 2, 9, 1, 1},  {2, 2, 21, 1, 1},
                                  {4, 2, 28, 0, 2}, {4, 2, 28, 0, 3}, {2, 2, 28, 0, 2}, {2, 2, 28, 0, 3},
                                  {4, 2, 28, 1, 3}, {2, 2, 28, 1, 3}, {2, 2, 9, 2, 1},  {4, 2, 14, 2, 1},
                                  {4, 2, 28, 2, 3}, {2, 2, 28, 2, 3}, {2, 2, 3, 0, 1},  {2, 2, 3, 2, 1}};
constexpr int kTiles2[] = {2, 1, 4, 8};
constexpr int kNumTiles3 = sizeof(kTiles3) / sizeof(kTiles3[0]);
static_assert(kNumTiles3 == 24, "launch_fused has one case per entry of kTiles3");
constexpr int kNumTiles2 = sizeof(kTiles2) / sizeof(kTiles2[0]);

int fused_tile_count(int dim) { return dim == 3 ? kNumTiles3 : kNumTiles2; }

int fused_tile_index(int dim, int tyc, int rpt, int zc) {
  if (dim == 3) {
    for (int t = 0; t < kNumTiles3; ++t)
      if (kTiles3[t].tyc == tyc && kTiles3[t].rpt == rpt && kTiles3[t].zc == zc && kTiles3[t].order == 0 &&
          kTiles3[t].pf == 1)
        return t;
    return -1;
  }
  for (int t = 0; t < kNumTiles2; ++t)
    if (kTiles2[t] == zc) return t;
  return -1;
}

static dim3 fused_grid(int dim, int n, int tile) {
  const int nc = (n - 1) / 3 + 1;
  if (dim == 3) {
    const TileShape3 t = kTiles3[tile];
    return dim3(f3_xtiles(nc), (nc + t.tyc - 1) / t.tyc, (nc + t.zc - 1) / t.zc);
  }
  const int zc = kTiles2[tile];
  return dim3((nc + F2_TXC - 1) / F2_TXC, (nc + zc - 1) / zc, 1);
}

int fused_partials_blocks(int dim, int n, int tile) {
  if (n < 10 || tile < 0 || tile >= fused_tile_count(dim)) return -1;
  const dim3 g = fused_grid(dim, n, tile);
  return (int)(g.x * g.y * g.z);
}

// The sweep is launched through hipExtLaunchKernel: the optional events t0 / t1
// take the kernel's own start and end times (nullptr: no timing).
// (The case of launch_fused must instantiate the shape its tile entry names:
// the grid comes from the entry, the block's coverage from the template.)
template <class T, int TYC, int RPT, int ZC, int PF = 1>
static hipError_t launch3(const FusedArgs<T>& a0, dim3 g, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const TileShape3 e = kTiles3[a0.tile];
  if (e.tyc != TYC || e.rpt != RPT || e.zc != ZC || e.pf != PF) return hipErrorInvalidValue;
  const dim3 b(F3<T, TYC, RPT, ZC, false>::NT);
  FusedArgs<T> a = a0;
  a.order = kTiles3[a0.tile].order;
  if (a.variant == 2) hipExtLaunchKernelGGL((k_fused3<T, TYC, RPT, ZC, 2, PF>), g, b, 0, s, t0, t1, 0, a);
  else if (a.variant == 1) hipExtLaunchKernelGGL((k_fused3<T, TYC, RPT, ZC, 1, PF>), g, b, 0, s, t0, t1, 0, a);
  else hipExtLaunchKernelGGL((k_fused3<T, TYC, RPT, ZC, 0, PF>), g, b, 0, s, t0, t1, 0, a);
  return hipSuccess;
}

template <class T, int ZC>
static void launch2(const FusedArgs<T>& a, dim3 g, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (a.variant == 2) hipExtLaunchKernelGGL((k_fused2<T, ZC, true>), g, dim3(64), 0, s, t0, t1, 0, a);
  else hipExtLaunchKernelGGL((k_fused2<T, ZC, false>), g, dim3(64), 0, s, t0, t1, 0, a);
}

template <class T>
hipError_t launch_fused(int dim, const FusedArgs<T>& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (a.nc != (a.n - 1) / 3 + 1 || a.n < 10) return hipErrorInvalidValue;
  if (a.tile < 0 || a.tile >= fused_tile_count(dim)) return hipErrorInvalidValue;
  if (a.variant == 2 && (a.sic == nullptr || a.sic_out == nullptr || a.sic == a.sic_out)) return hipErrorInvalidValue;
  if (dim == 3 && a.spill == nullptr) return hipErrorInvalidValue;
  const dim3 g = fused_grid(dim, a.n, a.tile);
  if (dim == 3) {
    hipError_t e;
    switch (a.tile) {
      case 0: e = launch3<T, 2, 2, 9>(a, g, s, t0, t1); break;
      case 1: e = launch3<T, 2, 2, 14>(a, g, s, t0, t1); break;
      case 2: e = launch3<T, 2, 2, 21>(a, g, s, t0, t1); break;
      case 3: e = launch3<T, 2, 2, 27>(a, g, s, t0, t1); break;
      case 4: e = launch3<T, 2, 2, 28>(a, g, s, t0, t1); break;
      case 5: e = launch3<T, 4, 2, 14>(a, g, s, t0, t1); break;
      case 6: e = launch3<T, 4, 2, 21>(a, g, s, t0, t1); break;
      case 7: e = launch3<T, 4, 2, 28>(a, g, s, t0, t1); break;
      case 8: e = launch3<T, 2, 1, 14>(a, g, s, t0, t1); break;
      case 9: e = launch3<T, 2, 1, 21>(a, g, s, t0, t1); break;
      case 10: e = launch3<T, 2, 2, 9>(a, g, s, t0, t1); break;
      case 11: e = launch3<T, 2, 2, 21>(a, g, s, t0, t1); break;
      case 12: e = launch3<T, 4, 2, 28, 2>(a, g, s, t0, t1); break;
      case 13: e = launch3<T, 4, 2, 28, 3>(a, g, s, t0, t1); break;
      case 14: e = launch3<T, 2, 2, 28, 2>(a, g, s, t0, t1); break;
      case 15: e = launch3<T, 2, 2, 28, 3>(a, g, s, t0, t1); break;
      case 16: e = launch3<T, 4, 2, 28, 3>(a, g, s, t0, t1); break;
      case 17: e = launch3<T, 2, 2, 28, 3>(a, g, s, t0, t1); break;
      case 18: e = launch3<T, 2, 2, 9>(a, g, s, t0, t1); break;
      case 19: e = launch3<T, 4, 2, 14>(a, g, s, t0, t1); break;
      case 20: e = launch3<T, 4, 2, 28, 3>(a, g, s, t0, t1); break;
      case 21: e = launch3<T, 2, 2, 28, 3>(a, g, s, t0, t1); break;
      case 22: e = launch3<T, 2, 2, 3>(a, g, s, t0, t1); break;
      case 23: e = launch3<T, 2, 2, 3>(a, g, s, t0, t1); break;
      default: return hipErrorInvalidValue;   // every entry of kTiles3 has its case above
    }
    if (e != hipSuccess) return e;
  } else {
    switch (a.tile) {
      case 0: launch2<T, 2>(a, g, s, t0, t1); break;
      case 1: launch2<T, 1>(a, g, s, t0, t1); break;
      case 2: launch2<T, 4>(a, g, s, t0, t1); break;
      default: launch2<T, 8>(a, g, s, t0, t1); break;
    }
  }
  return hipGetLastError();
}

// Seam rows of the 3D restriction: rho_c at coarse row (s + 1) TYC gains the
// share of fine rows 3 (s + 1) TYC - 2 and - 1, restricted by y tile s into
// the same vertex of the seam array (see f3_ytiles); one addition per vertex,
// so the result does not depend on the order of the tiles.
template <class T>
__global__ __launch_bounds__(128) void k_seam3(cpx<T>* __restrict__ rhoc, const cpx<T>* __restrict__ spill, int nc,
                                               int tyc) {
  // block (s, mz): seam s of coarse plane mz, coarse row (s + 1) tyc
  const int mz = blockIdx.y, my = (blockIdx.x + 1) * tyc;
  if (mz < 1 || mz > nc - 2 || my > nc - 2) return;
  const long long row = ((long long)mz * nc + my) * nc;
  for (int mx = threadIdx.x + 1; mx <= nc - 2; mx += 128) {
    cpx<T>& d = rhoc[row + mx];
    const cpx<T> e = spill[row + mx];
    d = mk(d.re + e.re, d.im + e.im);
  }
}

template <class T>
hipError_t launch_fused_seam(int dim, const FusedArgs<T>& a, hipStream_t s) {
  if (dim != 3) return hipSuccess;
  if (a.tile < 0 || a.tile >= kNumTiles3 || a.spill == nullptr || a.rhoc == nullptr) return hipErrorInvalidValue;
  const int tyc = kTiles3[a.tile].tyc, nseam = f3_ytiles(a.nc, tyc) - 1;
  if (nseam < 1) return hipSuccess;
  hipLaunchKernelGGL(k_seam3<T>, dim3(nseam, a.nc), dim3(128), 0, s, a.rhoc, a.spill, a.nc, tyc);
  return hipGetLastError();
}

size_t fused_spill_count(int dim, int n) {
  if (dim != 3) return 0;
  const size_t nc = (n - 1) / 3 + 1;
  return nc * nc * nc;
}

// rho_c = R x (3D) with the sweep's march and restriction (no operator): the
// 4 x 2 x 28 tile with prefetch depth 3 in the y-band block order (order 2);
// the seam rows go through the seam array and k_seam3.
constexpr int kRTyc = 4, kRRpt = 2, kRZc = 28, kKrylovOrder = 2;
template <class T, int DOT>
__global__ __launch_bounds__(64 * (3 * kRTyc / kRRpt), 2) void k_restrict3(FusedArgs<T> a) {
  __shared__ F3Lds<T, kRTyc, kRRpt, false, true> sm;
  int bx, by, bz;
  fused3_block_tile(kKrylovOrder, gridDim.x, gridDim.y, gridDim.z, bx, by, bz);
  // |s|^2 partials are indexed by tile (summation order independent of the block order)
  double* part = DOT ? a.partials + (bx + gridDim.x * (by + gridDim.y * bz)) : nullptr;
  fused3_tile<T, kRTyc, kRRpt, kRZc, 1, kRestrict, 3, DOT>(a, bx, by, bz, part, sm);
}

int restrict3_blocks(int nc) { return f3_xtiles(nc) * f3_ytiles(nc, kRTyc) * ((nc + kRZc - 1) / kRZc); }

// Backtracking of a coarse level in the Galerkin form as the restriction
// march (DOT 4): rho_c = R rho with the level's update sc = ws rho (masked)
// and, for BPX (VAR 2), the injection si_c = ws rho, in one pass.
template <class T, int VAR>
__global__ __launch_bounds__(64 * (3 * kRTyc / kRRpt), 2) void k_post3(FusedArgs<T> a) {
  __shared__ F3Lds<T, kRTyc, kRRpt, VAR == 2, true> sm;
  int bx, by, bz;
  fused3_block_tile(kKrylovOrder, gridDim.x, gridDim.y, gridDim.z, bx, by, bz);
  fused3_tile<T, kRTyc, kRRpt, kRZc, VAR, kRestrict, 3, 4>(a, bx, by, bz, nullptr, sm);
}

template <class T>
hipError_t launch_post3(int nc, int variant, const cpx<T>* rho, cpx<T> ws, cpx<T>* sc, cpx<T>* sic, cpx<T>* rhoc,
                        cpx<T>* spill, hipStream_t s) {
  const int n = 3 * (nc - 1) + 1;
  // variant: 1 hierarchical basis, 2 BPX (the fused kernels' numbering)
  if (n < 10 || spill == nullptr || (variant != 1 && variant != 2)) return hipErrorInvalidValue;
  if (variant == 2 && sic == nullptr) return hipErrorInvalidValue;
  FusedArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nc = nc;
  a.b = rho;
  a.rhoc = rhoc;
  a.spill = spill;
  a.zout = sc;
  a.sic_out = sic;
  a.ws = ws;
  a.variant = variant;
  a.order = kKrylovOrder;
  const dim3 g(f3_xtiles(nc), f3_ytiles(nc, kRTyc), (nc + kRZc - 1) / kRZc);
  constexpr int NT = F3<T, kRTyc, kRRpt, kRZc, false>::NT;
  if (variant == 2) hipLaunchKernelGGL((k_post3<T, 2>), g, NT, 0, s, a);
  else hipLaunchKernelGGL((k_post3<T, 1>), g, NT, 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nseam = f3_ytiles(nc, kRTyc) - 1;
  if (nseam >= 1) hipLaunchKernelGGL(k_seam3<T>, dim3(nseam, nc), dim3(128), 0, s, rhoc, spill, nc, kRTyc);
  return hipGetLastError();
}
template hipError_t launch_post3<double>(int, int, const cpx<double>*, cpx<double>, cpx<double>*, cpx<double>*,
                                         cpx<double>*, cpx<double>*, hipStream_t);
template hipError_t launch_post3<float>(int, int, const cpx<float>*, cpx<float>, cpx<float>*, cpx<float>*,
                                        cpx<float>*, cpx<float>*, hipStream_t);

template <class T>
hipError_t launch_restrict3(int nc, const cpx<T>* x, cpx<T>* rhoc, cpx<T>* spill, hipStream_t s) {
  const int n = 3 * (nc - 1) + 1;
  if (n < 10 || spill == nullptr) return hipErrorInvalidValue;
  FusedArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nc = nc;
  a.b = x;
  a.rhoc = rhoc;
  a.spill = spill;
  a.variant = 1;
  a.order = kKrylovOrder;
  const dim3 g(f3_xtiles(nc), f3_ytiles(nc, kRTyc), (nc + kRZc - 1) / kRZc);
  constexpr int NT = F3<T, kRTyc, kRRpt, kRZc, false>::NT;
  hipLaunchKernelGGL((k_restrict3<T, 0>), g, NT, 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nseam = f3_ytiles(nc, kRTyc) - 1;
  if (nseam >= 1) hipLaunchKernelGGL(k_seam3<T>, dim3(nseam, nc), dim3(128), 0, s, rhoc, spill, nc, kRTyc);
  return hipGetLastError();
}

template <class T>
hipError_t launch_restrict3_s(int nc, const cpx<T>* r, const cpx<T>* v, cpx<double> alpha, cpx<T>* sv, cpx<T>* rhoc,
                              cpx<T>* spill, double* partials, hipStream_t s) {
  const int n = 3 * (nc - 1) + 1;
  if (n < 10 || spill == nullptr || partials == nullptr || sv == r || sv == v) return hipErrorInvalidValue;
  FusedArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nc = nc;
  a.b = r;
  a.w2 = v;
  a.alpha = alpha;
  a.zout = sv;
  a.rhoc = rhoc;
  a.spill = spill;
  a.partials = partials;
  a.variant = 1;
  a.order = kKrylovOrder;
  const dim3 g(f3_xtiles(nc), f3_ytiles(nc, kRTyc), (nc + kRZc - 1) / kRZc);
  constexpr int NT = F3<T, kRTyc, kRRpt, kRZc, false>::NT;
  hipLaunchKernelGGL((k_restrict3<T, 3>), g, NT, 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nseam = f3_ytiles(nc, kRTyc) - 1;
  if (nseam >= 1) hipLaunchKernelGGL(k_seam3<T>, dim3(nseam, nc), dim3(128), 0, s, rhoc, spill, nc, kRTyc);
  return hipGetLastError();
}

template hipError_t launch_restrict3_s<double>(int, const cpx<double>*, const cpx<double>*, cpx<double>, cpx<double>*,
                                               cpx<double>*, cpx<double>*, double*, hipStream_t);
template hipError_t launch_restrict3_s<float>(int, const cpx<float>*, const cpx<float>*, cpx<double>, cpx<float>*,
                                              cpx<float>*, cpx<float>*, double*, hipStream_t);

template <class T, int VAR, int DOT>
__global__ __launch_bounds__(64 * (3 * kRTyc / kRRpt), 2) void k_prec_apply3(FusedArgs<T> a) {
  __shared__ F3Lds<T, kRTyc, kRRpt, false, true> sm;
  int bx, by, bz;
  fused3_block_tile(kKrylovOrder, gridDim.x, gridDim.y, gridDim.z, bx, by, bz);
  // dot partials are indexed by tile, so their summation order does not depend on the block order
  constexpr int ND = DOT == 1 ? 2 : 3;
  double* part = DOT ? a.partials + ND * (bx + gridDim.x * (by + gridDim.y * bz)) : nullptr;
  fused3_tile<T, kRTyc, kRRpt, kRZc, VAR, kPrecApply, 3, DOT>(a, bx, by, bz, part, sm);
}

int prec_apply3_blocks(int n) {
  if (n < 10 || (n - 1) % 3 != 0) return -1;
  const int nc = (n - 1) / 3 + 1;
  return f3_xtiles(nc) * f3_ytiles(nc, kRTyc) * ((nc + kRZc - 1) / kRZc);
}

template <class T, int VAR>
static void launch_pa3(int dot, dim3 g, const FusedArgs<T>& a, hipStream_t s) {
  constexpr int NT = F3<T, kRTyc, kRRpt, kRZc, false>::NT;
  if (dot == 1) hipLaunchKernelGGL((k_prec_apply3<T, VAR, 1>), g, NT, 0, s, a);
  else if (dot == 2) hipLaunchKernelGGL((k_prec_apply3<T, VAR, 2>), g, NT, 0, s, a);
  else hipLaunchKernelGGL((k_prec_apply3<T, VAR, 0>), g, NT, 0, s, a);
}

template <class T>
hipError_t launch_prec_apply3(int n, const cpx<T>* coef, cpx<T> ws, int mask_c, const cpx<T>* x, const cpx<T>* gc,
                              cpx<T>* z, cpx<T>* y, int dot, const cpx<T>* v2, double* partials, hipStream_t s) {
  if (n < 10 || (n - 1) % 3 != 0 || dot < 0 || dot > 2) return hipErrorInvalidValue;
  if (dot && (v2 == nullptr || partials == nullptr)) return hipErrorInvalidValue;
  const int nc = (n - 1) / 3 + 1;
  FusedArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nc = nc;
  a.w = x;
  a.scc = gc;
  a.wout = y;
  a.zout = z;
  a.b = v2;
  a.partials = partials;
  for (int q = 0; q < 4; ++q) a.coef[q] = coef[q];
  a.ws = ws;
  a.variant = mask_c ? 1 : 0;
  a.order = kKrylovOrder;
  const dim3 g(f3_xtiles(nc), f3_ytiles(nc, kRTyc), (nc + kRZc - 1) / kRZc);
  if (mask_c) launch_pa3<T, 1>(dot, g, a, s);
  else launch_pa3<T, 0>(dot, g, a, s);
  return hipGetLastError();
}

template hipError_t launch_prec_apply3<double>(int, const cpx<double>*, cpx<double>, int, const cpx<double>*,
                                               const cpx<double>*, cpx<double>*, cpx<double>*, int,
                                               const cpx<double>*, double*, hipStream_t);
template hipError_t launch_prec_apply3<float>(int, const cpx<float>*, cpx<float>, int, const cpx<float>*,
                                              const cpx<float>*, cpx<float>*, cpx<float>*, int, const cpx<float>*,
                                              double*, hipStream_t);
template hipError_t launch_restrict3<double>(int, const cpx<double>*, cpx<double>*, cpx<double>*, hipStream_t);
template hipError_t launch_restrict3<float>(int, const cpx<float>*, cpx<float>*, cpx<float>*, hipStream_t);

// y = H x or r = b - H x (constant phi, 3D) with the sweep's march: 2 x 2
// coarse-row tiles, z extent 21, no coarse levels.
template <class T, int MODE>
__global__ __launch_bounds__(192, 3) void k_stencil3(FusedArgs<T> a) {
  __shared__ F3Lds<T, 2, 2, false, false> sm;
  double* part = a.partials ? a.partials + 2 * (blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) : nullptr;
  fused3_tile<T, 2, 2, 21, 1, MODE>(a, blockIdx.x, blockIdx.y, blockIdx.z, part, sm);
}

static dim3 stencil3_grid(int n) {
  const int nc = (n - 1) / 3 + 1;
  return dim3(f3_xtiles(nc), (nc + 1) / 2, (nc + 20) / 21);
}

int stencil3_blocks(int n) {
  if (n < 10 || (n - 1) % 3 != 0) return -1;
  const dim3 g = stencil3_grid(n);
  return (int)(g.x * g.y * g.z);
}

template <class T>
hipError_t launch_stencil3(int apply, int n, const cpx<T>* coef, const cpx<T>* b, const cpx<T>* x, cpx<T>* out,
                           double* partials, int* nparts, hipStream_t s) {
  const int blocks = stencil3_blocks(n);
  if (blocks < 0) return hipErrorInvalidValue;
  FusedArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nc = (n - 1) / 3 + 1;
  a.w = x;
  a.wout = out;
  a.b = b;
  for (int q = 0; q < 4; ++q) a.coef[q] = coef[q];
  a.partials = partials;
  a.variant = 1;
  const dim3 g = stencil3_grid(n);
  constexpr int NT = F3<T, 2, 2, 21, false>::NT;
  static_assert(NT == 192, "k_stencil3 launch bounds");
  if (apply) hipLaunchKernelGGL((k_stencil3<T, kApply>), g, NT, 0, s, a);
  else hipLaunchKernelGGL((k_stencil3<T, kResid>), g, NT, 0, s, a);
  if (nparts) *nparts = blocks;
  return hipGetLastError();
}

template hipError_t launch_stencil3<double>(int, int, const cpx<double>*, const cpx<double>*, const cpx<double>*,
                                            cpx<double>*, double*, int*, hipStream_t);
template hipError_t launch_stencil3<float>(int, int, const cpx<float>*, const cpx<float>*, const cpx<float>*,
                                           cpx<float>*, double*, int*, hipStream_t);

template hipError_t launch_fused<double>(int, const FusedArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fused<float>(int, const FusedArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fused_seam<double>(int, const FusedArgs<double>&, hipStream_t);
template hipError_t launch_fused_seam<float>(int, const FusedArgs<float>&, hipStream_t);

}  // namespace mg
