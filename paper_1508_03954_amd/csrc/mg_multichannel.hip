// Same-grid multichannel form (Section 7.5): C channels -- independent
// Helmholtz problems that share the grid and differ in phi (and load) --
// fused into one problem on one grid, every vertex holding a C^C tuple
// (array-of-structures: channel c of vertex i at i * C + c).  One cycle runs
// the pipelined additive cycle of every channel at once: the coarse-level
// traversal, the index arithmetic and the transfer weights are shared by the
// channels of a vertex.
//
// Lanes span (vertex, channel) pairs: a wavefront covers 64 / C consecutive
// vertices of one row with all C channels of each, so every load of a
// neighbour's tuple is one contiguous 1 KiB run of the wavefront (a lane per
// vertex reading its whole tuple would stride the wavefront's loads by 16 C
// bytes).  A lane's channel is fixed for the whole launch; its stencil
// weights come from a per-level table of C x 4 weights.
//
// The cycle is the Galerkin form of the single-problem engine's level passes
// (constant phi per channel and a uniform rotation): descent (sc += P sc_c,
// BPX: - P si_c off c-points), finest U = w + P g, then one pass forming
// r = b - H U with the norms of every channel and the pointwise update
// (written to the other iterate buffer) with its injections, rho_c = R r;
// then the Galerkin backtracking of the coarse levels and the coarsest
// update.  Coarse u is not stored (the Galerkin form never reads it).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "mg_common.h"
#include "mg_engine.h"

namespace mg {

constexpr int kMcMaxChannels = 16;

// Row traversal with (vertex, channel) lanes: lane l of a wavefront takes
// channel l % C of vertex x = block x-offset + l / C on the row, which is
// uniform across the wavefront; blocks of 4 wavefronts walk the rows
// grid-stride.
#define MC_ROWS(D, C, n)                                                                    \
  const int lane_ = threadIdx.x & 63;                                                        \
  const int ch_ = lane_ & ((C) - 1);                                                         \
  const int x_ = blockIdx.x * (64 / (C)) + lane_ / (C);                                      \
  const int nrows_ = (D == 3) ? (n) * (n) : (n);                                             \
  for (int row_ = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); \
       row_ < nrows_; row_ += gridDim.y * 4)

// d-linear prolongation weights and coarse indices of fine vertex j: the 2^d
// corners (a corner past a coarse vertex repeats it with weight 0).
template <int D>
__device__ inline void prolong_support(int nc, const int j[3], long long idx[8], double wt[8]) {
  int m[3] = {0, 0, 0};
  double w0[3] = {1, 1, 1}, w1[3] = {0, 0, 0};
  bool two[3] = {false, false, false};
  for (int a = 0; a < D; ++a) {
    const int q = j[a] % 3;
    m[a] = j[a] / 3;
    if (q == 1) {
      w0[a] = 2.0 / 3.0; w1[a] = 1.0 / 3.0; two[a] = true;
    } else if (q == 2) {
      w0[a] = 1.0 / 3.0; w1[a] = 2.0 / 3.0; two[a] = true;
    }
  }
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    double w = 1.0;
    int k[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int bit = (c >> a) & 1;
      w *= bit ? w1[a] : w0[a];
      k[a] = m[a] + (two[a] ? bit : 0);
    }
    idx[c] = ravel<D>(k, nc);
    wt[c] = w;
  }
}

// acc += sgn * sum over corners of wt * v[idx * C + ch]
template <int D, int C>
__device__ inline cpx<double> prolong_add(const cpx<double>* __restrict__ v, const long long idx[8],
                                          const double wt[8], double sgn, int ch, cpx<double> acc) {
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) acc = acc + (sgn * wt[c]) * v[idx[c] * C + ch];
  return acc;
}

// Descent of a coarse level: sc += P sc_c (BPX: - P si_c off c-points).  The
// iterate u += sc + sf is not stored (see the header).
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_pre(int n, cpx<double>* __restrict__ sc, const cpx<double>* __restrict__ scc,
                                                const cpx<double>* __restrict__ sic, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  MC_ROWS(D, C, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (!is_interior<D>(j, n)) continue;
    long long idx[8];
    double wt[8];
    prolong_support<D>(nc, j, idx, wt);
    const long long e = i * C + ch_;
    cpx<double> acc = prolong_add<D, C>(scc, idx, wt, 1.0, ch_, sc[e]);
    if (bpx && !is_cpoint<D>(j)) acc = prolong_add<D, C>(sic, idx, wt, -1.0, ch_, acc);
    sc[e] = acc;
  }
}

// Finest descent: U = w + P sc_c (BPX: - P si_c off c-points); 0 on the boundary.
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_fine_pre(int n, const cpx<double>* __restrict__ w,
                                                     cpx<double>* __restrict__ U, const cpx<double>* __restrict__ scc,
                                                     const cpx<double>* __restrict__ sic, int has_coarse, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  MC_ROWS(D, C, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const long long e = i * C + ch_;
    if (!is_interior<D>(j, n)) {
      U[e] = czero<double>();
      continue;
    }
    cpx<double> acc = w[e];
    if (has_coarse) {
      long long idx[8];
      double wt[8];
      prolong_support<D>(nc, j, idx, wt);
      acc = prolong_add<D, C>(scc, idx, wt, 1.0, ch_, acc);
      if (bpx && !is_cpoint<D>(j)) acc = prolong_add<D, C>(sic, idx, wt, -1.0, ch_, acc);
    }
    U[e] = acc;
  }
}

// Block sums of |r|^2 and maxima of |r|^2 per channel, fixed order: the lanes
// of one channel in a wavefront (ch, ch + C, ...) by a shuffle tree, then the
// four wavefronts in order.  partials[2 (block C + ch)] and [.. + 1].
template <int C>
__device__ inline void mc_block_norms(double s2, double mx, double* partials) {
  __shared__ double ss[4][C], sm[4][C];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int off = 32; off >= C; off >>= 1) {
    s2 += __shfl_down(s2, off, 64);
    mx = fmax(mx, __shfl_down(mx, off, 64));
  }
  if (lane < C) {
    ss[wid][lane] = s2;
    sm[wid][lane] = mx;
  }
  __syncthreads();
  if (threadIdx.x < C) {
    const int ch = threadIdx.x;
    double a = 0, b = 0;
    for (int w = 0; w < 4; ++w) {
      a += ss[w][ch];
      b = fmax(b, sm[w][ch]);
    }
    const size_t bid = blockIdx.x + (size_t)gridDim.x * blockIdx.y;
    partials[2 * (bid * C + ch)] = a;
    partials[2 * (bid * C + ch) + 1] = b;
  }
}

// (H x)_e for interior vertex j: the 3^d neighbours' values of the lane's
// channel with the weight of their offset class (0: centre, 1: face,
// 2: edge, 3: corner neighbour).
template <int D, int C>
__device__ inline cpx<double> mc_stencil(const cpx<double>* __restrict__ x, int n, const int j[3], int ch,
                                         const cpx<double> cw[4]) {
  cpx<double> acc = czero<double>();
  const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
#pragma unroll
  for (int oz = zlo; oz <= zhi; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int k[3] = {j[0] + ox, j[1] + oy, j[2] + oz};
        if (!is_interior<D>(k, n)) continue;
        const int cls = (ox != 0) + (oy != 0) + (oz != 0);
        acc = acc + cmul(cw[cls], x[ravel<D>(k, n) * C + ch]);
      }
  return acc;
}

// The finest pass: r = b - H U (0 on the boundary) with the per-block norms of
// every channel, and the pointwise update s = omega D^-1 r, sc = s (0 on
// c-points when masked), unew = U + sc (written to the other iterate buffer,
// so that neighbours still read U), at c-points sfc = sc (additive form) and
// sic = s (BPX).  coef: C x 4 stencil weights, invD: C inverse diagonals.
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_fine_step(int n, const cpx<double>* __restrict__ coef,
                                                      const cpx<double>* __restrict__ invD, cpx<double> omega,
                                                      int mask_c, const cpx<double>* __restrict__ b,
                                                      const cpx<double>* __restrict__ U, cpx<double>* __restrict__ r,
                                                      cpx<double>* __restrict__ unew, cpx<double>* __restrict__ sfc,
                                                      cpx<double>* __restrict__ sic, double* partials) {
  const int nc = (n - 1) / 3 + 1;
  double s2 = 0.0, mx = 0.0;
  {
    MC_ROWS(D, C, n) {
      int j[3];
      long long i;
      if (!row_vertex<D>(row_, x_, n, j, i)) continue;
      const long long e = i * C + ch_;
      if (!is_interior<D>(j, n)) {
        r[e] = czero<double>();
        unew[e] = czero<double>();
        continue;
      }
      cpx<double> cw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) cw[q] = coef[ch_ * 4 + q];
      const cpx<double> rv = b[e] - mc_stencil<D, C>(U, n, j, ch_, cw);
      r[e] = rv;
      const double a2 = rv.re * rv.re + rv.im * rv.im;
      s2 += a2;
      mx = fmax(mx, a2);
      const cpx<double> s = cmul(omega, cmul(invD[ch_], rv));
      const bool cp = is_cpoint<D>(j);
      const cpx<double> scv = csel(mask_c && cp, czero<double>(), s);
      unew[e] = U[e] + scv;
      if (cp && (sfc || sic)) {
        const int m[3] = {j[0] / 3, j[1] / 3, j[2] / 3};
        const long long ec = ravel<D>(m, nc) * C + ch_;
        if (sfc) sfc[ec] = scv;
        if (sic) sic[ec] = s;
      }
    }
  }
  if (partials) mc_block_norms<C>(s2, sqrt(mx), partials);
}

// The same finest pass in 3D as a march along z: a wavefront takes one row y
// and a chunk of kMcTz planes and keeps the 3 x 3 neighbourhood of its
// vertices in the planes z - 1, z and z + 1 in registers, so a step loads the
// nine values of one new plane instead of all 27 neighbours.  U is zero on
// the boundary (the finest descent writes it so), so the neighbours of an
// interior vertex need no test.
constexpr int kMcTz = 8;

template <int C>
__device__ inline void mc_plane(const cpx<double>* __restrict__ U, int n, int x, int y, int z, int ch,
                                cpx<double> v[9]) {
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
      v[3 * (dy + 1) + dx + 1] = U[(((long long)z * n + y + dy) * n + x + dx) * C + ch];
}

template <int C>
__device__ inline cpx<double> mc_plane_sum(const cpx<double> v[9], const cpx<double> cw[4], int dz) {
  cpx<double> acc = czero<double>();
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int dy = k / 3 - 1, dx = k % 3 - 1;
    acc = acc + cmul(cw[(dx != 0) + (dy != 0) + (dz != 0)], v[k]);
  }
  return acc;
}

template <int C>
__global__ __launch_bounds__(256) void k_mc_fine_step3(int n, const cpx<double>* __restrict__ coef,
                                                       const cpx<double>* __restrict__ invD, cpx<double> omega,
                                                       int mask_c, const cpx<double>* __restrict__ b,
                                                       const cpx<double>* __restrict__ U, cpx<double>* __restrict__ r,
                                                       cpx<double>* __restrict__ unew, cpx<double>* __restrict__ sfc,
                                                       cpx<double>* __restrict__ sic, double* partials) {
  const int nc = (n - 1) / 3 + 1;
  const int lane = threadIdx.x & 63, ch = lane & (C - 1);
  const int x = blockIdx.x * (64 / C) + lane / C;
  const int nzc = (n + kMcTz - 1) / kMcTz;
  cpx<double> cw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cw[q] = coef[ch * 4 + q];
  const cpx<double> di = cmul(omega, invD[ch]);
  double s2 = 0.0, mx = 0.0;
  for (int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); t < n * nzc;
       t += gridDim.y * 4) {
    const int y = t % n, zs = (t / n) * kMcTz, ze = min(zs + kMcTz, n);
    if (x >= n) continue;
    const bool in_xy = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
    const bool cpxy = x % 3 == 0 && y % 3 == 0;
    const int z0 = max(zs, 1), z1 = min(ze, n - 1);   // interior planes of the chunk
    for (int z = zs; z < ze; ++z)
      if (!in_xy || z < z0 || z >= z1) {
        const long long e = (((long long)z * n + y) * n + x) * C + ch;
        r[e] = czero<double>();
        unew[e] = czero<double>();
      }
    if (!in_xy || z0 >= z1) continue;
    cpx<double> pa[9], pb[9], pc[9];
    mc_plane<C>(U, n, x, y, z0 - 1, ch, pa);
    mc_plane<C>(U, n, x, y, z0, ch, pb);
    for (int z = z0; z < z1; ++z) {
      mc_plane<C>(U, n, x, y, z + 1, ch, pc);
      const long long e = (((long long)z * n + y) * n + x) * C + ch;
      const cpx<double> hu = mc_plane_sum<C>(pa, cw, 1) + mc_plane_sum<C>(pb, cw, 0) + mc_plane_sum<C>(pc, cw, 1);
      const cpx<double> rv = b[e] - hu;
      r[e] = rv;
      const double a2 = rv.re * rv.re + rv.im * rv.im;
      s2 += a2;
      mx = fmax(mx, a2);
      const cpx<double> sv = cmul(di, rv);
      const bool cp = cpxy && z % 3 == 0;
      const cpx<double> scv = csel(mask_c && cp, czero<double>(), sv);
      unew[e] = pb[4] + scv;
      if (cp && (sfc || sic)) {
        const long long ec = (((long long)(z / 3) * nc + y / 3) * nc + x / 3) * C + ch;
        if (sfc) sfc[ec] = scv;
        if (sic) sic[ec] = sv;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        pa[k] = pb[k];
        pb[k] = pc[k];
      }
    }
  }
  mc_block_norms<C>(s2, sqrt(mx), partials);
}

// The finest descent in 3D as a march along z (rows y, chunks of kMcTz
// planes, as the finest step): P is separable, so a lane interpolates its
// coarse corners in x and y once per coarse plane (four loads per array) and
// keeps the two coarse planes that bracket its fine z in registers; a fine
// plane then costs one load of w.  Same values as k_mc_fine_pre up to the
// order of the additions.
template <int C>
__device__ inline cpx<double> mc_xy_interp(const cpx<double>* __restrict__ v, int nc, int mz, const long long cidx[4],
                                           const double cw[4], int ch) {
  cpx<double> acc = czero<double>();
  const long long base = (long long)mz * nc * nc;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = acc + cw[k] * v[(base + cidx[k]) * C + ch];
  return acc;
}

template <int C>
__global__ __launch_bounds__(256) void k_mc_fine_pre3(int n, const cpx<double>* __restrict__ w,
                                                      cpx<double>* __restrict__ U, const cpx<double>* __restrict__ scc,
                                                      const cpx<double>* __restrict__ sic, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  const int lane = threadIdx.x & 63, ch = lane & (C - 1);
  const int x = blockIdx.x * (64 / C) + lane / C;
  const int nzc = (n + kMcTz - 1) / kMcTz;
  for (int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); t < n * nzc;
       t += gridDim.y * 4) {
    const int y = t % n, zs = (t / n) * kMcTz, ze = min(zs + kMcTz, n);
    if (x >= n) continue;
    const bool in_xy = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
    const int z0 = max(zs, 1), z1 = min(ze, n - 1);
    for (int z = zs; z < ze; ++z)
      if (!in_xy || z < z0 || z >= z1) U[(((long long)z * n + y) * n + x) * C + ch] = czero<double>();
    if (!in_xy || z0 >= z1) continue;
    // x and y corners (the second one with weight 0 on a coarse line; its
    // index stays inside the coarse grid for an interior fine vertex)
    const int mx = x / 3, qx = x % 3, my = y / 3, qy = y % 3;
    const double wx1 = qx / 3.0, wx0 = qx == 0 ? 1.0 : 1.0 - wx1;
    const double wy1 = qy / 3.0, wy0 = qy == 0 ? 1.0 : 1.0 - wy1;
    const long long cidx[4] = {(long long)my * nc + mx, (long long)my * nc + mx + 1, (long long)(my + 1) * nc + mx,
                               (long long)(my + 1) * nc + mx + 1};
    const double cwt[4] = {wy0 * wx0, wy0 * wx1, wy1 * wx0, wy1 * wx1};
    const bool cxy = qx == 0 && qy == 0;
    int mz = z0 / 3;
    cpx<double> s0 = mc_xy_interp<C>(scc, nc, mz, cidx, cwt, ch), s1 = mc_xy_interp<C>(scc, nc, mz + 1, cidx, cwt, ch);
    cpx<double> i0 = czero<double>(), i1 = czero<double>();
    if (bpx) {
      i0 = mc_xy_interp<C>(sic, nc, mz, cidx, cwt, ch);
      i1 = mc_xy_interp<C>(sic, nc, mz + 1, cidx, cwt, ch);
    }
    for (int z = z0; z < z1; ++z) {
      if (z / 3 != mz) {   // the next coarse interval: shift the bracket by one plane
        mz = z / 3;
        s0 = s1;
        s1 = mc_xy_interp<C>(scc, nc, mz + 1, cidx, cwt, ch);
        if (bpx) {
          i0 = i1;
          i1 = mc_xy_interp<C>(sic, nc, mz + 1, cidx, cwt, ch);
        }
      }
      const int qz = z % 3;
      const double wz1 = qz / 3.0, wz0 = qz == 0 ? 1.0 : 1.0 - wz1;
      const long long e = (((long long)z * n + y) * n + x) * C + ch;
      cpx<double> acc = w[e] + (wz0 * s0 + wz1 * s1);
      if (bpx && !(cxy && qz == 0)) acc = acc - (wz0 * i0 + wz1 * i1);
      U[e] = acc;
    }
  }
}

// y = H x for every channel.
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_apply(int n, const cpx<double>* __restrict__ coef,
                                                  const cpx<double>* __restrict__ x, cpx<double>* __restrict__ y) {
  MC_ROWS(D, C, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    cpx<double> acc = czero<double>();
    if (is_interior<D>(j, n)) {
      cpx<double> cw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) cw[q] = coef[ch_ * 4 + q];
      acc = mc_stencil<D, C>(x, n, j, ch_, cw);
    }
    y[i * C + ch_] = acc;
  }
}

// Pointwise post-phase of a coarse level: s = omega r / D_ch, sc_out = s (0 on
// c-points when masked); at c-points sf_c = sf + sc (if sfc), si_c = s (if sic).
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_update(int n, const cpx<double>* __restrict__ invD,
                                                   const cpx<double>* __restrict__ r, cpx<double> omega, int mask_c,
                                                   cpx<double>* __restrict__ sc_out, const cpx<double>* __restrict__ sf,
                                                   cpx<double>* __restrict__ sfc, cpx<double>* __restrict__ sic) {
  const int nc = (n - 1) / 3 + 1;
  MC_ROWS(D, C, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const long long e = i * C + ch_;
    const bool in = is_interior<D>(j, n);
    const bool cp = is_cpoint<D>(j);
    cpx<double> s = czero<double>();
    if (in) s = cmul(omega, cmul(invD[ch_], r[e]));
    const cpx<double> scv = csel(mask_c && cp, czero<double>(), s);
    sc_out[e] = scv;
    if (cp && (sfc || sic)) {
      const int m[3] = {j[0] / 3, j[1] / 3, j[2] / 3};
      const long long ec = ravel<D>(m, nc) * C + ch_;
      if (sfc) sfc[ec] = sf[e] + scv;
      if (sic) sic[ec] = s;
    }
  }
}

// (R v) at coarse vertex m for the lane's channel: weights (1 - |o|/3) per
// axis over the fine offsets o in [-2, 2]^d around 3m.
template <int D, int C>
__device__ inline cpx<double> mc_restrict_at(const cpx<double>* __restrict__ vf, int nf, const int m[3], int ch) {
  constexpr double w[5] = {1.0 / 3.0, 2.0 / 3.0, 1.0, 2.0 / 3.0, 1.0 / 3.0};
  cpx<double> acc = czero<double>();
  const int zlo = D == 3 ? -2 : 0, zhi = D == 3 ? 2 : 0;
  for (int oz = zlo; oz <= zhi; ++oz)
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) {
        const int k[3] = {3 * m[0] + ox, 3 * m[1] + oy, 3 * m[2] + oz};
        double wt = w[ox + 2] * w[oy + 2];
        if (D == 3) wt *= w[oz + 2];
        acc = acc + wt * vf[ravel<D>(k, nf) * C + ch];
      }
  return acc;
}

// rho_c = R v on the interior of the coarse level (0 on its boundary; the
// support of an interior coarse vertex lies inside the fine grid).
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_restrict(int nc, const cpx<double>* __restrict__ vf,
                                                     cpx<double>* __restrict__ vc) {
  const int nf = 3 * (nc - 1) + 1;
  MC_ROWS(D, C, nc) {
    int m[3];
    long long ic;
    if (!row_vertex<D>(row_, x_, nc, m, ic)) continue;
    vc[ic * C + ch_] = is_interior<D>(m, nc) ? mc_restrict_at<D, C>(vf, nf, m, ch_) : czero<double>();
  }
}

// The restriction in 3D as a march along coarse z: a wavefront takes one
// coarse row my and a chunk of kMcTz coarse planes; per fine plane a lane
// forms the x-y weighted sum of its 5 x 5 fine support once (25 loads), and
// a coarse plane combines five such sums with the z weights, two of them
// carried over from the previous coarse plane (75 loads per coarse value
// instead of 125).  Same values as k_mc_restrict up to the order of the
// additions.
template <int C>
__device__ inline cpx<double> mc_xy_restrict(const cpx<double>* __restrict__ vf, int nf, int fz, int fy0, int fx0,
                                             int ch) {
  constexpr double w[5] = {1.0 / 3.0, 2.0 / 3.0, 1.0, 2.0 / 3.0, 1.0 / 3.0};
  cpx<double> acc = czero<double>();
#pragma unroll
  for (int oy = 0; oy < 5; ++oy) {
    const long long row = ((long long)fz * nf + fy0 + oy) * nf + fx0;
#pragma unroll
    for (int ox = 0; ox < 5; ++ox) acc = acc + (w[oy] * w[ox]) * vf[(row + ox) * C + ch];
  }
  return acc;
}

template <int C>
__global__ __launch_bounds__(256) void k_mc_restrict3(int nc, const cpx<double>* __restrict__ vf,
                                                      cpx<double>* __restrict__ vc) {
  const int nf = 3 * (nc - 1) + 1;
  const int lane = threadIdx.x & 63, ch = lane & (C - 1);
  const int mx = blockIdx.x * (64 / C) + lane / C;
  const int nzc = (nc + kMcTz - 1) / kMcTz;
  for (int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); t < nc * nzc;
       t += gridDim.y * 4) {
    const int my = t % nc, zs = (t / nc) * kMcTz, ze = min(zs + kMcTz, nc);
    if (mx >= nc) continue;
    const bool in_xy = mx >= 1 && mx <= nc - 2 && my >= 1 && my <= nc - 2;
    const int z0 = max(zs, 1), z1 = min(ze, nc - 1);
    for (int mz = zs; mz < ze; ++mz)
      if (!in_xy || mz < z0 || mz >= z1) vc[(((long long)mz * nc + my) * nc + mx) * C + ch] = czero<double>();
    if (!in_xy || z0 >= z1) continue;
    const int fx0 = 3 * mx - 2, fy0 = 3 * my - 2;
    // sums of the fine planes 3 mz - 2 and 3 mz - 1 for the first coarse plane
    cpx<double> q0 = mc_xy_restrict<C>(vf, nf, 3 * z0 - 2, fy0, fx0, ch);
    cpx<double> q1 = mc_xy_restrict<C>(vf, nf, 3 * z0 - 1, fy0, fx0, ch);
    for (int mz = z0; mz < z1; ++mz) {
      const cpx<double> q2 = mc_xy_restrict<C>(vf, nf, 3 * mz, fy0, fx0, ch);
      const cpx<double> q3 = mc_xy_restrict<C>(vf, nf, 3 * mz + 1, fy0, fx0, ch);
      const cpx<double> q4 = mc_xy_restrict<C>(vf, nf, 3 * mz + 2, fy0, fx0, ch);
      vc[(((long long)mz * nc + my) * nc + mx) * C + ch] =
          (1.0 / 3.0) * q0 + (2.0 / 3.0) * q1 + q2 + (2.0 / 3.0) * q3 + (1.0 / 3.0) * q4;
      q0 = q3;
      q1 = q4;
    }
  }
}

// Per-channel second stage of the norms over `count` blocks: block ch adds
// its channel's partials, thread t the blocks t, t + 256, ... in order, then
// a fixed shared-memory tree (sums; maxima).
template <int C>
__global__ __launch_bounds__(256) void k_mc_finish(const double* __restrict__ partials, int count,
                                                   double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  const int ch = blockIdx.x, t = threadIdx.x;
  double a = 0, b = 0;
  for (int k = t; k < count; k += 256) {
    a += partials[2 * ((size_t)k * C + ch)];
    b = fmax(b, partials[2 * ((size_t)k * C + ch) + 1]);
  }
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      sa[t] += sa[t + h];
      sb[t] = fmax(sb[t], sb[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[2 * ch] = sa[0];
    out[2 * ch + 1] = sb[0];
  }
}

template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_copy_zero_boundary(int n, const cpx<double>* __restrict__ in,
                                                               cpx<double>* __restrict__ out) {
  MC_ROWS(D, C, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const long long e = i * C + ch_;
    out[e] = is_interior<D>(j, n) ? in[e] : czero<double>();
  }
}

// Grid of a level pass: 64 / C vertices of a row per block column, 4 rows per
// block row; at most about kMcMaxBlocks blocks (the rows loop grid-stride), so
// that the per-block norm partials of the finest pass stay a few MB.
constexpr int kMcMaxBlocks = 8192;
static dim3 mc_row_grid(int n, int dim, int C) {
  const long long rows = dim == 3 ? (long long)n * n : n;
  const int per = 64 / C;
  const long long gx = (n + per - 1) / per;
  long long gy = (rows + 3) / 4;
  gy = std::min<long long>(gy, std::max<long long>(1, kMcMaxBlocks / gx));
  return dim3((unsigned)gx, (unsigned)gy);
}

// ---------------------------------------------------------------------------
// Host engine.

struct McBase {
  virtual ~McBase() {}
  virtual int apply(const cpx<double>* x, cpx<double>* y) = 0;
  virtual int set_rhs(const cpx<double>* b) = 0;
  virtual int set_solution(const cpx<double>* u) = 0;
  virtual int cycle(int ncycles, double* res_h) = 0;
  virtual int flush(cpx<double>* u) = 0;
  int dim = 3, L = 1, lmin = 1, nchan = 1;
  hipStream_t s = nullptr;
};

template <int C>
struct McEngine : McBase {
  struct Lv {
    int n = 0;
    size_t N = 0;
    cpx<double>*b = nullptr, *sc = nullptr, *sf = nullptr, *si = nullptr;
    cpx<double>* coef = nullptr;   // C x 4 stencil weights, then C inverse diagonals
  };
  std::vector<Lv> lv;
  cpx<double>* w[2] = {nullptr, nullptr};
  int cur = 0;
  cpx<double>* tR = nullptr;
  double* partials = nullptr;
  double* hist = nullptr;
  int hist_cap = 0, iter = 0, variant = MG_BPX, scheme = MG_OMEGA_CONST, omega_L = 1, red_blocks = 0;
  complex<double> omega = 0.6;
  std::vector<void*> owned;

  ~McEngine() override {
    for (void* p : owned) (void)hipFree(p);
  }

  int alloc(cpx<double>** p, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(cpx<double>));
    if (e != hipSuccess) return fail(MG_ENOMEM, std::string("multichannel hipMalloc: ") + hipGetErrorString(e));
    owned.push_back(q);
    *p = (cpx<double>*)q;
    MG_HIP(launch_fill(q, std::max<size_t>(count, 1) * sizeof(cpx<double>), s));
    return MG_OK;
  }

  template <class K, class... A>
  int launch(K k2, K k3, int n, A... args) {
    const dim3 g = mc_row_grid(n, dim, C);
    if (dim == 3) hipLaunchKernelGGL(k3, g, dim3(256), 0, s, args...);
    else hipLaunchKernelGGL(k2, g, dim3(256), 0, s, args...);
    MG_HIP(hipGetLastError());
    return MG_OK;
  }

  const cpx<double>* invD(int l) const { return lv[l].coef + 4 * C; }

  // rho = R v from level l + 1 to level l (3D: the z march).
  int restrict_to(int l, const cpx<double>* vf) {
    const int nc = lv[l].n;
    if (dim == 3) {
      const int per = 64 / C;
      const long long gx = (nc + per - 1) / per;
      const long long items = (long long)nc * ((nc + kMcTz - 1) / kMcTz);
      long long gy = (items + 3) / 4;
      gy = std::min<long long>(gy, std::max<long long>(1, kMcMaxBlocks / gx));
      hipLaunchKernelGGL(k_mc_restrict3<C>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, nc, vf, lv[l].b);
      MG_HIP(hipGetLastError());
      return MG_OK;
    }
    return launch(k_mc_restrict<2, C>, k_mc_restrict<2, C>, nc, nc, vf, lv[l].b);
  }

  // Grid of the 3D finest march: 64 / C vertices per block column, rows times
  // z chunks walked by the block rows (at most about kMcMaxBlocks blocks).
  dim3 march_grid() const {
    const int n = lv[L].n, per = 64 / C;
    const long long gx = (n + per - 1) / per;
    const long long items = (long long)n * ((n + kMcTz - 1) / kMcTz);
    long long gy = (items + 3) / 4;
    gy = std::min<long long>(gy, std::max<long long>(1, kMcMaxBlocks / gx));
    return dim3((unsigned)gx, (unsigned)gy);
  }

  int setup(const mg_params& p, int nch, const mg_c128* phis, hipStream_t stream) {
    s = stream;
    dim = p.dim;
    lmin = p.level_min;
    L = p.level_max;
    nchan = nch;
    variant = p.variant;
    scheme = p.omega_scheme;
    omega_L = p.omega_L;
    omega = complex<double>(p.omega.re, p.omega.im);
    lv.resize(L + 1);
    for (int l = lmin; l <= L; ++l) {
      Lv& v = lv[l];
      v.n = (int)ipow(3, l) + 1;
      v.N = (size_t)ipow(v.n, dim);
      std::vector<cpx<double>> tab(5 * C);
      for (int ch = 0; ch < C; ++ch) {
        const mg_c128 ph = phis[ch];
        const OpData<double> o = make_const_op<double>(dim, l, p.theta, complex<double>(ph.re, ph.im), p.conjugate != 0);
        for (int q = 0; q < 4; ++q) tab[4 * ch + q] = o.coef[q];
        tab[4 * C + ch] = o.invD;
      }
      MG_TRY(alloc(&v.coef, tab.size()));
      MG_HIP(hipMemcpyAsync(v.coef, tab.data(), tab.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, s));
      MG_HIP(hipStreamSynchronize(s));
      const size_t NC = v.N * C;
      if (l < L) {
        MG_TRY(alloc(&v.b, NC));
        MG_TRY(alloc(&v.sc, NC));
        MG_TRY(alloc(&v.sf, NC));
        MG_TRY(alloc(&v.si, NC));
      } else {
        MG_TRY(alloc(&v.b, NC));
        MG_TRY(alloc(&w[0], NC));
        MG_TRY(alloc(&w[1], NC));
        MG_TRY(alloc(&tR, NC));
      }
    }
    const dim3 g = dim == 3 ? march_grid() : mc_row_grid(lv[L].n, dim, C);
    red_blocks = (int)(g.x * g.y);
    void* q = nullptr;
    MG_HIP(hipMalloc(&q, 2 * (size_t)red_blocks * C * sizeof(double)));
    owned.push_back(q);
    partials = (double*)q;
    return ensure_hist(64);
  }

  int ensure_hist(int cap) {
    if (cap <= hist_cap) return MG_OK;
    void* q = nullptr;
    MG_HIP(hipMalloc(&q, 2 * (size_t)cap * C * sizeof(double)));
    owned.push_back(q);
    hist = (double*)q;
    hist_cap = cap;
    return MG_OK;
  }

  int zero_helpers() {
    for (int l = lmin; l < L; ++l) {
      MG_HIP(launch_fill(lv[l].sc, lv[l].N * C * sizeof(cpx<double>), s));
      MG_HIP(launch_fill(lv[l].sf, lv[l].N * C * sizeof(cpx<double>), s));
      MG_HIP(launch_fill(lv[l].si, lv[l].N * C * sizeof(cpx<double>), s));
    }
    return MG_OK;
  }

  int copy_in(const cpx<double>* src, cpx<double>* dst) {
    return launch(k_mc_copy_zero_boundary<2, C>, k_mc_copy_zero_boundary<3, C>, lv[L].n, lv[L].n, src, dst);
  }

  int apply(const cpx<double>* x, cpx<double>* y) override {
    return launch(k_mc_apply<2, C>, k_mc_apply<3, C>, lv[L].n, lv[L].n, (const cpx<double>*)lv[L].coef, x, y);
  }

  int set_rhs(const cpx<double>* b) override {
    MG_TRY(copy_in(b, lv[L].b));
    iter = 0;
    return zero_helpers();
  }

  int set_solution(const cpx<double>* u) override {
    MG_TRY(copy_in(u, w[cur]));
    iter = 0;
    return zero_helpers();
  }

  int pre_coarse() {
    for (int l = lmin + 1; l < L; ++l)
      MG_TRY(launch(k_mc_pre<2, C>, k_mc_pre<3, C>, lv[l].n, lv[l].n, lv[l].sc, (const cpx<double>*)lv[l - 1].sc,
                    (const cpx<double>*)lv[l - 1].si, variant == MG_BPX ? 1 : 0));
    return MG_OK;
  }

  int fine_pre(cpx<double>* U) {
    const bool hc = L > lmin;
    if (dim == 3 && hc) {
      hipLaunchKernelGGL(k_mc_fine_pre3<C>, march_grid(), dim3(256), 0, s, lv[L].n, (const cpx<double>*)w[cur], U,
                         (const cpx<double>*)lv[L - 1].sc, (const cpx<double>*)lv[L - 1].si, variant == MG_BPX ? 1 : 0);
      MG_HIP(hipGetLastError());
      return MG_OK;
    }
    return launch(k_mc_fine_pre<2, C>, k_mc_fine_pre<3, C>, lv[L].n, lv[L].n, (const cpx<double>*)w[cur], U,
                  hc ? (const cpx<double>*)lv[L - 1].sc : nullptr, hc ? (const cpx<double>*)lv[L - 1].si : nullptr,
                  hc ? 1 : 0, variant == MG_BPX ? 1 : 0);
  }

  // One cycle: U = w[1 - cur] from the iterate w[cur]; the finest step reads
  // U and writes the new iterate back into w[cur] (whose old value U has
  // absorbed), so the iterate stays in w[cur].
  int cycle_once(int k) {
    ++iter;
    MG_TRY(pre_coarse());
    Lv& f = lv[L];
    const bool hc = L > lmin;
    Lv* c = hc ? &lv[L - 1] : nullptr;
    cpx<double>* U = w[1 - cur];
    MG_TRY(fine_pre(U));
    const complex<double> wL = omega_level(scheme, omega, omega_L, 0, iter);
    const int mask = (hc && variant != MG_ADD) ? 1 : 0;
    cpx<double>* sfc = (hc && variant == MG_ADD) ? c->sf : nullptr;
    cpx<double>* sic = (hc && variant == MG_BPX) ? c->si : nullptr;
    if (dim == 3) {
      hipLaunchKernelGGL(k_mc_fine_step3<C>, march_grid(), dim3(256), 0, s, f.n, (const cpx<double>*)f.coef, invD(L),
                         to_c<double>(wL), mask, (const cpx<double>*)f.b, (const cpx<double>*)U, tR, w[cur], sfc, sic,
                         partials);
      MG_HIP(hipGetLastError());
    } else {
      MG_TRY(launch(k_mc_fine_step<2, C>, k_mc_fine_step<2, C>, f.n, f.n, (const cpx<double>*)f.coef, invD(L),
                    to_c<double>(wL), mask, (const cpx<double>*)f.b, (const cpx<double>*)U, tR, w[cur], sfc, sic,
                    partials));
    }
    if (hc) MG_TRY(restrict_to(L - 1, tR));
    hipLaunchKernelGGL(k_mc_finish<C>, dim3(C), dim3(256), 0, s, (const double*)partials, red_blocks,
                       hist + 2 * (size_t)k * C);
    MG_HIP(hipGetLastError());
    // backtracking of the coarse levels (Galerkin form: the b slot holds the
    // level's residual R r of the finer one)
    for (int l = L - 1; l >= lmin; --l) {
      Lv& v = lv[l];
      const bool hcc = l > lmin;
      Lv* cc = hcc ? &lv[l - 1] : nullptr;
      const complex<double> wl = omega_level(scheme, omega, omega_L, L - l, iter);
      MG_TRY(launch(k_mc_update<2, C>, k_mc_update<3, C>, v.n, v.n, invD(l), (const cpx<double>*)v.b,
                    to_c<double>(wl), (hcc && variant != MG_ADD) ? 1 : 0, v.sc, (const cpx<double>*)v.sf,
                    (hcc && variant == MG_ADD) ? cc->sf : (cpx<double>*)nullptr,
                    (hcc && variant == MG_BPX) ? cc->si : (cpx<double>*)nullptr));
      if (hcc) MG_TRY(restrict_to(l - 1, v.b));
    }
    return MG_OK;
  }

  int cycle(int ncycles, double* res_h) override {
    if (ncycles <= 0) return MG_OK;
    MG_TRY(ensure_hist(ncycles));
    for (int k = 0; k < ncycles; ++k) MG_TRY(cycle_once(k));
    if (res_h) {
      std::vector<double> h(2 * (size_t)ncycles * C);
      MG_HIP(hipMemcpyAsync(h.data(), hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
      const double scale = std::pow(3.0, -L * dim);
      for (int k = 0; k < ncycles; ++k)
        for (int ch = 0; ch < nchan; ++ch) res_h[(size_t)k * nchan + ch] = std::sqrt(scale * h[(2 * (size_t)k) * C + 2 * ch]);
    }
    return MG_OK;
  }

  int flush(cpx<double>* u) override {
    MG_TRY(pre_coarse());
    MG_TRY(fine_pre(w[1 - cur]));
    cur = 1 - cur;
    MG_TRY(zero_helpers());
    if (u) MG_HIP(hipMemcpyAsync(u, w[cur], lv[L].N * C * sizeof(cpx<double>), hipMemcpyDeviceToDevice, s));
    return MG_OK;
  }
};

}  // namespace mg

using namespace mg;

struct mg_mc {
  McBase* impl = nullptr;
  ~mg_mc() { delete impl; }
};

extern "C" {

int mg_mc_setup(const mg_params* p, int nchan, const mg_c128* phis, void* hip_stream, mg_mc** out) {
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || !phis) return fail(MG_EINVAL, "NULL argument");
  if (p->dim != 2 && p->dim != 3) return fail(MG_EINVAL, "dim must be 2 or 3");
  if (p->level_min < 1 || p->level_max <= p->level_min) return fail(MG_EINVAL, "need 1 <= level_min < level_max");
  if (p->level_max > (p->dim == 3 ? 6 : 9)) return fail(MG_EINVAL, "level_max too large (3D: <= 6, 2D: <= 9)");
  if (nchan != 1 && nchan != 2 && nchan != 4 && nchan != 8 && nchan != 16)
    return fail(MG_EINVAL, "nchan must be 1, 2, 4, 8 or 16");
  if (p->variant < MG_ADD || p->variant > MG_BPX) return fail(MG_EINVAL, "bad variant");
  if (p->omega_scheme < MG_OMEGA_CONST || p->omega_scheme > MG_OMEGA_TWO_PHASE) return fail(MG_EINVAL, "bad omega scheme");
  if (p->phi_field || p->layer_width > 0 || p->precision != MG_FP64)
    return fail(MG_EINVAL, "multichannel problems take one constant phi per channel, FP64, no absorbing layer");
  const size_t N = (size_t)ipow(ipow(3, p->level_max) + 1, p->dim);
  if (N * (size_t)nchan >= (1ull << 31)) return fail(MG_EINVAL, "grid times channels exceeds the 32-bit element range");
  mg_mc* m = new mg_mc();
  int rc;
  switch (nchan) {
    case 1: { auto* e = new McEngine<1>(); m->impl = e; rc = e->setup(*p, nchan, phis, (hipStream_t)hip_stream); break; }
    case 2: { auto* e = new McEngine<2>(); m->impl = e; rc = e->setup(*p, nchan, phis, (hipStream_t)hip_stream); break; }
    case 4: { auto* e = new McEngine<4>(); m->impl = e; rc = e->setup(*p, nchan, phis, (hipStream_t)hip_stream); break; }
    case 8: { auto* e = new McEngine<8>(); m->impl = e; rc = e->setup(*p, nchan, phis, (hipStream_t)hip_stream); break; }
    default: { auto* e = new McEngine<16>(); m->impl = e; rc = e->setup(*p, nchan, phis, (hipStream_t)hip_stream); break; }
  }
  if (rc == MG_OK) {
    const hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("multichannel setup: ") + hipGetErrorString(e));
  }
  if (rc != MG_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return MG_OK;
}

void mg_mc_destroy(mg_mc* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->impl->s);
  delete m;
}

int mg_mc_apply(mg_mc* m, const mg_c128* x, mg_c128* y) {
  if (!m || !x || !y) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)x == (const void*)y) return fail(MG_EINVAL, "x and y must not alias");
  return m->impl->apply((const cpx<double>*)x, (cpx<double>*)y);
}

int mg_mc_set_rhs(mg_mc* m, const mg_c128* b) {
  if (!m || !b) return fail(MG_EINVAL, "NULL argument");
  return m->impl->set_rhs((const cpx<double>*)b);
}

int mg_mc_set_solution(mg_mc* m, const mg_c128* u) {
  if (!m || !u) return fail(MG_EINVAL, "NULL argument");
  return m->impl->set_solution((const cpx<double>*)u);
}

int mg_mc_cycle(mg_mc* m, int ncycles, double* res_h) {
  if (!m || ncycles < 0) return fail(MG_EINVAL, "bad argument");
  return m->impl->cycle(ncycles, res_h);
}

int mg_mc_flush(mg_mc* m, mg_c128* u) {
  if (!m) return fail(MG_EINVAL, "NULL context");
  return m->impl->flush((cpx<double>*)u);
}

}  // extern "C"
