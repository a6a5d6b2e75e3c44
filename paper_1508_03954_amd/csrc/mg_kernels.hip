// Generic level passes of the additive multilevel cycle: one thread per vertex,
// neighbours gathered through the cache hierarchy.  They cover every case
// (constant or nodal phi, FAS or Galerkin coarse right-hand sides, all levels);
// the finest level of the constant-phi case has a fused single-pass kernel in
// mg_fused.hip.
//
// Level l: n = 3^l + 1 vertices per axis, C order with x fastest.  Fields are
// zero on boundary vertices; kernels keep them so.
#include <algorithm>

#include "mg_common.h"
#include "mg_level_ops.h"

namespace mg {

// ---------------------------------------------------------------------------
// Block reduction of (sum, max) into partials[blockIdx.x][2].
__device__ inline void block_sum_max(double s, double m, double* partials) {
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    m = fmax(m, __shfl_down(m, off, 64));
  }
  __shared__ double ss[16], sm[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { ss[wid] = s; sm[wid] = m; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) { a += ss[w]; b = fmax(b, sm[w]); }
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    partials[2 * bid] = a;
    partials[2 * bid + 1] = b;
  }
}

__device__ inline void block_sum2(double s0, double s1, double* partials) {
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  __shared__ double a0[16], a1[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { a0[wid] = s0; a1[wid] = s1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0, y = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) { x += a0[w]; y += a1[w]; }
    partials[2 * blockIdx.x] = x;
    partials[2 * blockIdx.x + 1] = y;
  }
}

// N sums per block (wave shuffles, then waves in order), for the fused
// Krylov kernels: partials[N * block + k].
template <int N>
__device__ inline void block_sumN(double (&v)[N], double* partials) {
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  __shared__ double acc[N][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double x = 0;
      for (int w = 0; w < nw; ++w) x += acc[k][w];
      partials[N * blockIdx.x + k] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// (256-thread blocks, as every row kernel is launched: the bound lets the
// per-cell path keep its 3^d neighbourhood in registers.)
template <class T, int D>
__global__ __launch_bounds__(256) void k_apply(OpData<T> op, const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y) {
  MG_ROWS(D, op.n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, op.n, j, i)) continue;
    cpx<T> v = czero<T>();
    if (is_interior<D>(j, op.n)) v = apply_row<T, D>(x, op.n, j, op);
    y[i] = v;
  }
}

// Coarse-level pre-phase (descent of tdAdd / tdBPX), see pre_vertex.
template <class T, int D>
__global__ void k_pre(int n, cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc, const cpx<T>* __restrict__ sf,
                      const cpx<T>* __restrict__ scc, const cpx<T>* __restrict__ sic, int has_coarse, int bpx) {
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    pre_vertex<T, D>(n, j, i, u, sc, sf, scc, sic, has_coarse, bpx);
  }
}

// The same over a flat index (one thread per vertex, every lane busy), for 3D
// levels with n <= kFastDivMaxN whose rows do not fill whole wavefronts.
template <class T>
__global__ __launch_bounds__(256) void k_pre_flat3(int n, cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc,
                                                   const cpx<T>* __restrict__ sf, const cpx<T>* __restrict__ scc,
                                                   const cpx<T>* __restrict__ sic, int has_coarse, int bpx) {
  const unsigned N = (unsigned)n * n * n, magic = fastdiv_magic(n);
  for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < N; i += gridDim.x * 256u) {
    int j[3];
    unravel_fast<3>(i, n, magic, j);
    pre_vertex<T, 3>(n, j, i, u, sc, sf, scc, sic, has_coarse, bpx);
  }
}

// The same descent on a large 3D level as a march along z: a wavefront takes
// 64 vertices of one row and a chunk of kPreTz planes.  P is separable, so a
// lane interpolates its coarse corners in x and y once per coarse plane (four
// loads per coarse array) and keeps the two coarse planes that bracket its z
// in registers: a fine vertex then costs its own sc (and u, sf) and no
// gathered load.  Same values as pre_vertex up to the order of the additions.
constexpr int kPreTz = 8;
constexpr int kPreMarchMinN = 244;   // levels of 244^3 vertices and more (rows of >= 4 wavefronts)

template <class T>
__device__ inline cpx<T> pre_xy_interp(const cpx<T>* __restrict__ v, int nc, int mz, const long long cidx[4],
                                       const T cw[4]) {
  const long long base = (long long)mz * nc * nc;
  cpx<T> acc = czero<T>();
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = acc + cw[k] * v[base + cidx[k]];
  return acc;
}

// Modes of the prolongation march: the coarse descent sc += P scc (- P sic
// off c-points for BPX; u += sc + sf when the coarse iterate is formed), the
// finest descent out = w + P scc (- P sic off c-points), and the hierarchical
// surplus out = w - P scc.  The last two write zero off the interior.
enum { kPmPre = 0, kPmFine = 1, kPmSurplus = 2 };
constexpr int kProlongMarchMinN = 82;   // finest descent and surplus: 3D levels of 82^3 and more

template <class T, int KIND>
__global__ __launch_bounds__(256) void k_prolong_march3(int n, cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc,
                                                        const cpx<T>* __restrict__ sf,
                                                        const cpx<T>* __restrict__ scc,
                                                        const cpx<T>* __restrict__ sic, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  const int x = blockIdx.x * 64 + (int)(threadIdx.x & 63);
  const int nzc = (n + kPreTz - 1) / kPreTz;
  // kPmFine / kPmSurplus: sc is the input w, u the output
  for (int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); t < n * nzc;
       t += gridDim.y * 4) {
    const int y = t % n, zs = (t / n) * kPreTz, ze = min(zs + kPreTz, n);
    if (x >= n) continue;
    const bool in_xy = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
    const int z0 = max(zs, 1), z1 = min(ze, n - 1);
    if (KIND != kPmPre)
      for (int z = zs; z < ze; ++z)
        if (!in_xy || z < z0 || z >= z1) u[((long long)z * n + y) * n + x] = czero<T>();
    // the coarse descent leaves non-interior vertices alone
    if (!in_xy || z0 >= z1) continue;
    // x and y corners (the second with weight 0 on a coarse line; its index
    // stays inside the coarse grid for an interior vertex)
    const int mx = x / 3, qx = x % 3, my = y / 3, qy = y % 3;
    const T wx1 = T(qx) / T(3), wx0 = qx == 0 ? T(1) : T(1) - wx1;
    const T wy1 = T(qy) / T(3), wy0 = qy == 0 ? T(1) : T(1) - wy1;
    const long long cidx[4] = {(long long)my * nc + mx, (long long)my * nc + mx + 1, (long long)(my + 1) * nc + mx,
                               (long long)(my + 1) * nc + mx + 1};
    const T cwt[4] = {wy0 * wx0, wy0 * wx1, wy1 * wx0, wy1 * wx1};
    const bool cxy = qx == 0 && qy == 0;
    const bool use_i = KIND != kPmSurplus && bpx;
    int mz = z0 / 3;
    cpx<T> s0 = pre_xy_interp(scc, nc, mz, cidx, cwt), s1 = pre_xy_interp(scc, nc, mz + 1, cidx, cwt);
    cpx<T> i0 = czero<T>(), i1 = czero<T>();
    if (use_i) {
      i0 = pre_xy_interp(sic, nc, mz, cidx, cwt);
      i1 = pre_xy_interp(sic, nc, mz + 1, cidx, cwt);
    }
    for (int z = z0; z < z1; ++z) {
      if (z / 3 != mz) {   // the next coarse interval: shift the bracket by one plane
        mz = z / 3;
        s0 = s1;
        s1 = pre_xy_interp(scc, nc, mz + 1, cidx, cwt);
        if (use_i) {
          i0 = i1;
          i1 = pre_xy_interp(sic, nc, mz + 1, cidx, cwt);
        }
      }
      const int qz = z % 3;
      const T wz1 = T(qz) / T(3), wz0 = qz == 0 ? T(1) : T(1) - wz1;
      const long long e = ((long long)z * n + y) * n + x;
      const cpx<T> ps = wz0 * s0 + wz1 * s1;
      if (KIND == kPmSurplus) {
        u[e] = sc[e] - ps;
        continue;
      }
      cpx<T> v = sc[e] + ps;
      if (use_i && !(cxy && qz == 0)) v = v - (wz0 * i0 + wz1 * i1);
      if (KIND == kPmFine) {
        u[e] = v;
        continue;
      }
      sc[e] = v;
      if (u) u[e] = u[e] + v + sf[e];
    }
  }
}

template <class T, int KIND>
static hipError_t launch_prolong_march3(int n, cpx<T>* u, cpx<T>* sc, const cpx<T>* sf, const cpx<T>* scc,
                                        const cpx<T>* sic, int bpx, hipStream_t s) {
  const long long items = (long long)n * ((n + kPreTz - 1) / kPreTz);
  const dim3 g((unsigned)((n + 63) / 64), (unsigned)std::min<long long>((items + 3) / 4, 65535));
  hipLaunchKernelGGL((k_prolong_march3<T, KIND>), g, 256, 0, s, n, u, sc, sf, scc, sic, bpx);
  return hipGetLastError();
}

// Finest-level pre-phase on the folded iterate w = u + sc:
//   u = w + P sc_c (- P si_c off c-points for BPX), written to a second buffer.
template <class T, int D>
__global__ void k_fine_pre(int n, const cpx<T>* __restrict__ w, cpx<T>* __restrict__ u,
                           const cpx<T>* __restrict__ scc, const cpx<T>* __restrict__ sic, int has_coarse,
                           int bpx) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (!is_interior<D>(j, n)) { u[i] = czero<T>(); continue; }
    cpx<T> v = w[i];
    if (has_coarse) {
      v = v + prolong_at<T, D>(scc, nc, j);
      if (bpx && !is_cpoint<D>(j)) v = v - prolong_at<T, D>(sic, nc, j);
    }
    u[i] = v;
  }
}

// Hierarchical surplus uhat = u - P u_c (eq. HTMG).
template <class T, int D>
__global__ void k_uhat(int n, const cpx<T>* __restrict__ u, const cpx<T>* __restrict__ uc, cpx<T>* __restrict__ uh) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    cpx<T> v = czero<T>();
    if (is_interior<D>(j, n)) v = u[i] - prolong_at<T, D>(uc, nc, j);
    uh[i] = v;
  }
}

// r = b - H x (interior), optional norm partials.
template <class T, int D>
__global__ __launch_bounds__(256) void k_resid(OpData<T> op, const cpx<T>* __restrict__ b, const cpx<T>* __restrict__ x,
                                               cpx<T>* __restrict__ r, double* partials) {
  double s2 = 0, mx = 0;
  MG_ROWS(D, op.n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, op.n, j, i)) continue;
    cpx<T> v = czero<T>();
    if (is_interior<D>(j, op.n)) {
      v = b[i] - apply_row<T, D>(x, op.n, j, op);
      const double a2 = (double)v.re * v.re + (double)v.im * v.im;
      s2 += a2;
      mx = fmax(mx, a2);
    }
    if (r) r[i] = v;
  }
  if (partials) block_sum_max(s2, sqrt(mx), partials);
}

// r = b - H x with per-cell coefficients (varying phi, absorbing layer) in 3D
// as a march along z: a wavefront takes 64 vertices of one row and a chunk of
// kVarTz planes, keeps the 3 x 3 neighbourhoods of the planes z - 1, z, z + 1
// in registers and the coefficients of the two layers of cells around z, so a
// step loads one plane's nine values and one layer's four cells (eight with a
// per-cell stiffness) instead of stencil_var's 27 + 8 cell loads plus its
// 64 vertex loads.  The arithmetic is stencil_var's, in its order.
constexpr int kVarTz = 8;

template <class T>
__device__ inline void var_plane(const cpx<T>* __restrict__ x, int n, int xx, int y, int z, cpx<T> v[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int j[3] = {xx + k % 3 - 1, y + k / 3 - 1, z};
    v[k] = czero<T>();
    if (is_interior<3>(j, n)) v[k] = x[ravel<3>(j, n)];
  }
}

// The four cells of layer cz around (xx, y): cell (xx - bx, y - by, cz) at 2 by + bx.
template <class T, bool STIFF>
__device__ inline void var_cells(const OpData<T>& op, int n, int xx, int y, int cz, cpx<T> cm[4], cpx<T> ck[4]) {
  const int nc = n - 1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c[3] = {xx - (k & 1), y - (k >> 1), cz};
    const long long ci = ravel<3>(c, nc);
    cm[k] = op.cmass[ci];
    if (STIFF) ck[k] = op.cstiff[ci];
  }
}

// STIFF: per-cell stiffness coefficients (op.cstiff, the absorbing layer);
// otherwise the uniform stiffness op.alpha with the assembled 27-point weights.
// b == nullptr: r = H x (the operator alone, as k_apply).
template <class T, bool STIFF>
__global__ __launch_bounds__(256) void k_resid_var3(OpData<T> op, const cpx<T>* __restrict__ b,
                                                    const cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                                    double* partials) {
  const int n = op.n;
  const int xx = blockIdx.x * 64 + (int)(threadIdx.x & 63);
  const int nzc = (n + kVarTz - 1) / kVarTz;
  double s2 = 0, mx = 0;
  for (int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); t < n * nzc;
       t += gridDim.y * 4) {
    const int y = t % n, zs = (t / n) * kVarTz, ze = min(zs + kVarTz, n);
    if (xx >= n) continue;
    const bool in_xy = xx >= 1 && xx <= n - 2 && y >= 1 && y <= n - 2;
    const int z0 = max(zs, 1), z1 = min(ze, n - 1);
    if (r)
      for (int z = zs; z < ze; ++z)
        if (!in_xy || z < z0 || z >= z1) r[((long long)z * n + y) * n + xx] = czero<T>();
    if (!in_xy || z0 >= z1) continue;
    constexpr int NK = STIFF ? 4 : 1;
    cpx<T> pa[9], pb[9], pc[9], cmL[4], ckL[NK], cmU[4], ckU[NK];
    var_plane(x, n, xx, y, z0 - 1, pa);
    var_plane(x, n, xx, y, z0, pb);
    var_cells<T, STIFF>(op, n, xx, y, z0 - 1, cmL, ckL);
    for (int z = z0; z < z1; ++z) {
      var_plane(x, n, xx, y, z + 1, pc);
      var_cells<T, STIFF>(op, n, xx, y, z, cmU, ckU);
      // xv[q], q = (ox + 1) + 3 (oy + 1) + 9 (oz + 1): pa, pb, pc
      cpx<T> st = czero<T>();
      if (!STIFF) {
#pragma unroll
        for (int q = 0; q < 27; ++q) {
          const cpx<T> v = q < 9 ? pa[q] : (q < 18 ? pb[q - 9] : pc[q - 18]);
          const int cls = (q % 3 != 1) + ((q / 3) % 3 != 1) + (q / 9 != 1);
          st = st + stiff_weight<T, 3>(cls) * v;
        }
        st = cmul(op.alpha, st);
      }
      cpx<T> ms = czero<T>();
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        // cell j - bits(c): layer z - 1 for bit 2 set (cmL), z otherwise (cmU)
        cpx<T> am = czero<T>(), ak = czero<T>();
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const int q = (((kk >> 0) & 1) - ((c >> 0) & 1) + 1) + 3 * (((kk >> 1) & 1) - ((c >> 1) & 1) + 1) +
                        9 * (((kk >> 2) & 1) - ((c >> 2) & 1) + 1);
          const cpx<T> v = q < 9 ? pa[q] : (q < 18 ? pb[q - 9] : pc[q - 18]);
          am = am + elem_mass<T, 3>(c, kk) * v;
          if (STIFF) ak = ak + elem_stiff<T, 3>(c, kk) * v;
        }
        const int k4 = c & 3;
        const cpx<T> cmv = (c & 4) ? cmL[k4] : cmU[k4];
        ms = ms + cmul(cmv, am);
        if (STIFF) st = st + cmul((c & 4) ? ckL[k4 % NK] : ckU[k4 % NK], ak);
      }
      const long long e = ((long long)z * n + y) * n + xx;
      const cpx<T> v = b ? b[e] - (st - ms) : st - ms;
      if (r) r[e] = v;
      const double a2 = (double)v.re * v.re + (double)v.im * v.im;
      s2 += a2;
      mx = fmax(mx, a2);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        pa[k] = pb[k];
        pb[k] = pc[k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) cmL[k] = cmU[k];
#pragma unroll
      for (int k = 0; k < NK; ++k) ckL[k] = ckU[k];
    }
  }
  if (partials) block_sum_max(s2, sqrt(mx), partials);
}

// Post-phase pointwise part, see update_vertex.
template <class T, int D>
__global__ void k_update(OpData<T> op, const cpx<T>* __restrict__ r, cpx<T> omega, int mask_c,
                         cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc_out, const cpx<T>* __restrict__ sf,
                         cpx<T>* __restrict__ sfc, cpx<T>* __restrict__ sic) {
  MG_ROWS(D, op.n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, op.n, j, i)) continue;
    update_vertex<T, D>(op, j, i, r, omega, mask_c, u, sc_out, sf, sfc, sic);
  }
}

// Coarse post-phase with the Galerkin form, one launch per level l > l_min:
// eight lanes per coarse vertex, lanes 0..4 take the parts oo = -2..2 of its
// support (see post_galerkin_part) and a xor-shuffle sums them, so a vertex
// waits for one round of loads instead of five.
template <class T, int D>
__global__ __launch_bounds__(256) void k_post_galerkin(OpData<T> op, const cpx<T>* __restrict__ rho, cpx<T> omega,
                                                       int mask_c, cpx<T>* __restrict__ sc,
                                                       const cpx<T>* __restrict__ sf, cpx<T>* __restrict__ rhoc,
                                                       cpx<T>* __restrict__ sfc, cpx<T>* __restrict__ sic) {
  const int nc = (op.n - 1) / 3 + 1;
  const long long Nc = D == 3 ? (long long)nc * nc * nc : (long long)nc * nc;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long v = g >> 3;
  const int part = (int)(g & 7);
  int m[3] = {0, 0, 0};
  const bool valid = v < Nc;
  const long long vv = valid ? v : 0;
  if (nc <= kFastDivMaxN) unravel_fast<D>((unsigned)vv, nc, fastdiv_magic(nc), m);
  else unravel<D>(vv, nc, m);
  cpx<T> p = czero<T>();
  if (valid && part < 5) p = post_galerkin_part<T, D>(op, m, vv, part - 2, rho, omega, mask_c, sc, sf, sfc, sic);
  T re = p.re, im = p.im;
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (valid && part == 0) rhoc[vv] = csel(is_interior<D>(m, nc), mk(re, im), czero<T>());
}

// R v = P^T v (weights 1 - |o|/3 per axis around 3m; zero on the coarse
// boundary): eight lanes per coarse vertex, lanes 0..4 take the parts
// oo = -2..2, summed by a xor shuffle.
template <class T, int D>
__global__ __launch_bounds__(256) void k_restrict(int nc, const cpx<T>* __restrict__ vf, cpx<T>* __restrict__ vc) {
  const int nf = 3 * (nc - 1) + 1;
  const long long Nc = D == 3 ? (long long)nc * nc * nc : (long long)nc * nc;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long v = g >> 3;
  const int part = (int)(g & 7);
  const bool valid = v < Nc;
  const long long vv = valid ? v : 0;
  int m[3] = {0, 0, 0};
  if (nc <= kFastDivMaxN) unravel_fast<D>((unsigned)vv, nc, fastdiv_magic(nc), m);
  else unravel<D>(vv, nc, m);
  cpx<T> p = czero<T>();
  if (valid && part < 5) p = restrict_part<T, D>(vf, nf, m, part - 2);
  T re = p.re, im = p.im;
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (valid && part == 0) vc[vv] = csel(is_interior<D>(m, nc), mk(re, im), czero<T>());
}

template <class T, int D>
__global__ void k_inject(int nc, const cpx<T>* __restrict__ vf, cpx<T>* __restrict__ vc) {
  const int nf = 3 * (nc - 1) + 1;
  MG_ROWS(D, nc) {
    int m[3];
    long long i;
    if (!row_vertex<D>(row_, x_, nc, m, i)) continue;
    int j[3] = {3 * m[0], 3 * m[1], 3 * m[2]};
    vc[i] = vf[ravel<D>(j, nf)];
  }
}

// Nested iteration: vc(m) = vf(stride m) (the load sampled on a coarser level)
// and uf = P uc on the interior of the finer level, zero on its boundary.
template <class T, int D>
__global__ void k_sample(int nc, int stride, const cpx<T>* __restrict__ vf, cpx<T>* __restrict__ vc) {
  const int nf = stride * (nc - 1) + 1;
  MG_ROWS(D, nc) {
    int m[3];
    long long i;
    if (!row_vertex<D>(row_, x_, nc, m, i)) continue;
    int j[3] = {stride * m[0], stride * m[1], stride * m[2]};
    vc[i] = vf[ravel<D>(j, nf)];
  }
}

template <class T, int D>
__global__ void k_prolong(int n, const cpx<T>* __restrict__ uc, cpx<T>* __restrict__ uf) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    uf[i] = is_interior<D>(j, n) ? prolong_at<T, D>(uc, nc, j) : czero<T>();
  }
}

template <class T, int D>
__global__ void k_prec_up(OpData<T> op, const cpx<T>* __restrict__ rho, cpx<T> omega, int mask_c, int is_lmin,
                          const cpx<T>* __restrict__ gc, cpx<T>* __restrict__ z) {
  MG_ROWS(D, op.n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, op.n, j, i)) continue;
    prec_up_vertex<T, D>(op, j, i, rho, omega, mask_c, is_lmin, gc, z);
  }
}

template <class T, int D>
__global__ void k_prec_g(OpData<T> op, const cpx<T>* __restrict__ rho, cpx<T> omega, const cpx<T>* __restrict__ zc,
                         cpx<T>* __restrict__ g) {
  const int nc = (op.n - 1) / 3 + 1;
  MG_ROWS(D, nc) {
    int m[3];
    long long ic;
    if (!row_vertex<D>(row_, x_, nc, m, ic)) continue;
    prec_g_vertex<T, D>(op, m, ic, rho, omega, zc, g);
  }
}

// Per-cell coefficients: mu_c = phibar_c eta_c^d and (stiff != nullptr)
// kappa_c = eta_c^(d-2), formed in double precision.
template <class T, int D>
__global__ void k_cellcoef(int n, const cpx<T>* __restrict__ phi, cpx<T>* __restrict__ mass,
                           cpx<T>* __restrict__ stiff, CellRotation rot) {
  const int nc = n - 1;
  const long long N = total<D>(nc);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    int c[3];
    unravel<D>(i, nc, c);
    cpx<double> acc = mk(0.0, 0.0);
    for (int k = 0; k < (1 << D); ++k) {
      int v[3] = {c[0] + (k & 1), c[1] + ((k >> 1) & 1), c[2] + ((k >> 2) & 1)};
      const cpx<T> p = phi[ravel<D>(v, n)];
      acc = acc + mk((double)p.re, (double)p.im);
    }
    acc = (1.0 / (1 << D)) * acc;
    if (rot.conj) acc.im = -acc.im;
    const cpx<double> mu = cmul(acc, cell_eta_pow<D>(rot, c, nc, D));
    mass[i] = mk(T(mu.re), T(mu.im));
    if (stiff) {
      const cpx<double> ka = cell_eta_pow<D>(rot, c, nc, D - 2);
      stiff[i] = mk(T(ka.re), T(ka.im));
    }
  }
}

// 1 / D_j with D_j = sum_{c contains j} (kappa_c K_jj - mu_c M_jj), K_jj =
// d 3^(1-d) and M_jj = 3^-d on every cell (kappa_c = alpha unless per cell).
template <class T, int D>
__global__ void k_invdiag(OpData<T> op, cpx<T>* __restrict__ invDv) {
  const int n = op.n, nc = n - 1;
  const T kd = D == 3 ? T(1.0 / 3.0) : T(2.0 / 3.0);
  const T m0 = D == 3 ? T(1.0 / 27.0) : T(1.0 / 9.0);
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (!is_interior<D>(j, n)) { invDv[i] = mk(T(1), T(0)); continue; }
    cpx<T> ms = czero<T>(), ks = czero<T>();
    for (int k = 0; k < (1 << D); ++k) {
      int c[3] = {j[0] - (k & 1), j[1] - ((k >> 1) & 1), j[2] - ((k >> 2) & 1)};
      const long long ci = ravel<D>(c, nc);
      ms = ms + op.cmass[ci];
      ks = ks + (op.cstiff ? op.cstiff[ci] : op.alpha);
    }
    const cpx<T> d = kd * ks - m0 * ms;
    // 1/d computed in double for both precisions
    const double dr = d.re, di = d.im, den = dr * dr + di * di;
    invDv[i] = mk(T(dr / den), T(-di / den));
  }
}

template <class T>
__global__ void k_set_value(size_t count, cpx<T>* __restrict__ v, cpx<T> value) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    v[i] = value;
}

template <int D>
__global__ void k_rhs_cells(int n, const cpx<double>* __restrict__ chi, cpx<double>* __restrict__ b,
                            CellRotation rot) {
  const int nc = n - 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    cpx<double> out = mk(0.0, 0.0);
    if (is_interior<D>(j, n)) {
      cpx<double> w = mk(0.0, 0.0);
      for (int k = 0; k < (1 << D); ++k) {
        int c[3] = {j[0] - (k & 1), j[1] - ((k >> 1) & 1), j[2] - ((k >> 2) & 1)};
        w = w + cell_eta_pow<D>(rot, c, nc, D);
      }
      out = cmul((1.0 / (1 << D)) * w, chi[i]);
    }
    b[i] = out;
  }
}

template <class T, int D>
__global__ void k_zero_boundary_copy(int n, const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, cpx<T> scale) {
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    out[i] = csel(is_interior<D>(j, n), cmul(scale, in[i]), czero<T>());
  }
}

__global__ void k_fill(unsigned int* p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <class S, class Dt>
__global__ void k_convert(size_t count, const cpx<S>* __restrict__ in, cpx<Dt>* __restrict__ out, double scale) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<S> v = in[i];
    out[i] = mk(Dt((double)v.re * scale), Dt((double)v.im * scale));
  }
}

template <class T>
__global__ void k_dot(size_t count, const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b, double* partials) {
  double sr = 0, si = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> x = a[i], y = b[i];
    sr += (double)x.re * y.re + (double)x.im * y.im;
    si += (double)x.re * y.im - (double)x.im * y.re;
  }
  block_sum2(sr, si, partials);
}

template <class T>
__global__ void k_norm2(size_t count, const cpx<T>* __restrict__ a, double* partials) {
  double s = 0, m = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> x = a[i];
    const double v = (double)x.re * x.re + (double)x.im * x.im;
    s += v;
    m = fmax(m, v);
  }
  block_sum_max(s, sqrt(m), partials);
}

template <class T>
__global__ void k_axpby(size_t count, cpx<double> a, const cpx<T>* __restrict__ x, cpx<double> b, cpx<T>* __restrict__ y) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> xv = x[i], yv = y[i];
    const double re = a.re * xv.re - a.im * xv.im + b.re * yv.re - b.im * yv.im;
    const double im = a.re * xv.im + a.im * xv.re + b.re * yv.im + b.im * yv.re;
    y[i] = mk(T(re), T(im));
  }
}

template <class T>
__global__ void k_bicg_p(size_t count, const cpx<T>* __restrict__ r, const cpx<T>* __restrict__ v, cpx<double> beta,
                         cpx<double> w, cpx<T>* __restrict__ p) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> pv = p[i], vv = v[i], rv = r[i];
    const double tr = pv.re - (w.re * vv.re - w.im * vv.im);
    const double ti = pv.im - (w.re * vv.im + w.im * vv.re);
    p[i] = mk(T(rv.re + beta.re * tr - beta.im * ti), T(rv.im + beta.re * ti + beta.im * tr));
  }
}

template <class T>
__global__ void k_bicg_xr(size_t count, cpx<T>* __restrict__ x, const cpx<T>* __restrict__ y, const cpx<T>* __restrict__ z,
                          cpx<double> a, cpx<double> w, cpx<T>* __restrict__ r, const cpx<T>* __restrict__ sv,
                          const cpx<T>* __restrict__ t) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> xv = x[i], yv = y[i], zv = z[i], s = sv[i], tv = t[i];
    x[i] = mk(T(xv.re + a.re * yv.re - a.im * yv.im + w.re * zv.re - w.im * zv.im),
              T(xv.im + a.re * yv.im + a.im * yv.re + w.re * zv.im + w.im * zv.re));
    r[i] = mk(T(s.re - (w.re * tv.re - w.im * tv.im)), T(s.im - (w.re * tv.im + w.im * tv.re)));
  }
}

// s = r - a v, partial |s|^2.
template <class T>
__global__ void k_bicg_s(size_t count, const cpx<T>* __restrict__ r, const cpx<T>* __restrict__ v, cpx<double> a,
                         cpx<T>* __restrict__ sv, double* partials) {
  double acc[1] = {0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> rv = r[i], vv = v[i];
    const cpx<T> o = mk(T(rv.re - (a.re * vv.re - a.im * vv.im)), T(rv.im - (a.re * vv.im + a.im * vv.re)));
    sv[i] = o;
    acc[0] += (double)o.re * o.re + (double)o.im * o.im;
  }
  block_sumN<1>(acc, partials);
}

// conj(t) . s and |t|^2 in one pass.
template <class T>
__global__ void k_bicg_ts(size_t count, const cpx<T>* __restrict__ t, const cpx<T>* __restrict__ sv, double* partials) {
  double acc[3] = {0, 0, 0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> x = t[i], y = sv[i];
    acc[0] += (double)x.re * y.re + (double)x.im * y.im;
    acc[1] += (double)x.re * y.im - (double)x.im * y.re;
    acc[2] += (double)x.re * x.re + (double)x.im * x.im;
  }
  block_sumN<3>(acc, partials);
}

// x += a y + w z ; r = s - w t ; partial |r|^2 and conj(rh) . r.
template <class T>
__global__ void k_bicg_xr2(size_t count, cpx<T>* __restrict__ x, const cpx<T>* __restrict__ y,
                           const cpx<T>* __restrict__ z, cpx<double> a, cpx<double> w, cpx<T>* __restrict__ r,
                           const cpx<T>* __restrict__ sv, const cpx<T>* __restrict__ t, const cpx<T>* __restrict__ rh,
                           double* partials) {
  double acc[3] = {0, 0, 0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<T> xv = x[i], yv = y[i], zv = z[i], s = sv[i], tv = t[i], hv = rh[i];
    x[i] = mk(T(xv.re + a.re * yv.re - a.im * yv.im + w.re * zv.re - w.im * zv.im),
              T(xv.im + a.re * yv.im + a.im * yv.re + w.re * zv.im + w.im * zv.re));
    const cpx<T> o = mk(T(s.re - (w.re * tv.re - w.im * tv.im)), T(s.im - (w.re * tv.im + w.im * tv.re)));
    r[i] = o;
    acc[0] += (double)o.re * o.re + (double)o.im * o.im;
    acc[1] += (double)hv.re * o.re + (double)hv.im * o.im;
    acc[2] += (double)hv.re * o.im - (double)hv.im * o.re;
  }
  block_sumN<3>(acc, partials);
}

// Second stage of block_sumN: out[k] = sum over blocks in block order, by 256
// strided partial sums and a tree (as the other second stages).
template <int N>
__global__ void k_finishN(const double* __restrict__ partials, int count, double* out) {
  __shared__ double sh[N][256];
  const int t = threadIdx.x;
  double a[N];
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = 0;
#pragma unroll 4
  for (int i = t; i < count; i += 256)
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] += partials[N * i + k];
#pragma unroll
  for (int k = 0; k < N; ++k) sh[k][t] = a[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int k = 0; k < N; ++k) sh[k][t] += sh[k][t + w];
    __syncthreads();
  }
  if (t == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = sh[k][0];
}

__global__ void k_accum32(size_t count, const cpx<float>* __restrict__ e, double scale, cpx<double>* __restrict__ u) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const cpx<float> ev = e[i];
    const cpx<double> uv = u[i];
    u[i] = mk(uv.re + scale * (double)ev.re, uv.im + scale * (double)ev.im);
  }
}

// dJ/dV_j = -2 Re sum_{c contains j} 2^-d eta^d lam_c^H M u_c.
template <int D>
__global__ void k_grad_potential(int n, cpx<double> etad, const cpx<double>* __restrict__ u,
                                 const cpx<double>* __restrict__ lam, double* __restrict__ g) {
  const long long N = total<D>(n);
  const int nc = n - 1;
  const double m0 = D == 3 ? 1.0 / 27.0 : 1.0 / 9.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    int j[3];
    unravel<D>(i, n, j);
    double acc = 0;
    for (int c = 0; c < (1 << D); ++c) {
      int cell[3] = {0, 0, 0};
      bool ok = true;
      for (int a = 0; a < D; ++a) {
        cell[a] = j[a] - ((c >> a) & 1);
        if (cell[a] < 0 || cell[a] >= nc) ok = false;
      }
      if (!ok) continue;
      // lam_c^H M u_c
      cpx<double> cv = mk(0.0, 0.0);
      for (int k = 0; k < (1 << D); ++k) {
        int vk[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) vk[a] = cell[a] + ((k >> a) & 1);
        const cpx<double> lk = lam[ravel<D>(vk, n)];
        cpx<double> mu = mk(0.0, 0.0);
        for (int kk = 0; kk < (1 << D); ++kk) {
          int vv[3] = {0, 0, 0};
          double w = m0;
          for (int a = 0; a < D; ++a) {
            const int b = (kk >> a) & 1;
            vv[a] = cell[a] + b;
            if (b != ((k >> a) & 1)) w *= 0.5;
          }
          mu = mu + w * u[ravel<D>(vv, n)];
        }
        cv = cv + cconjmul(lk, mu);
      }
      acc += cmul(etad, cv).re;
    }
    g[i] = -2.0 * acc / (1 << D);
  }
}

// Second reduction stage, one block of 256 threads: thread t folds partials
// t, t+256, ... in order, then a fixed tree; the result does not depend on
// timing, so repeated runs agree bitwise.
// Second reduction stage, fixed order: 256 strided partial sums, then a
// tree.  Works in any block of at least 256 threads (the others only join the
// barriers).
template <bool MAX2>
__device__ inline void finish_block(const double* __restrict__ partials, int count, double* out) {
  __shared__ double s0[256], s1[256];
  const int t = threadIdx.x;
  if (t < 256) {
    double a = 0, b = 0;
    // unrolled so that the loads issue together; the sums keep index order
#pragma unroll 8
    for (int i = t; i < count; i += 256) {
      a += partials[2 * i];
      b = MAX2 ? fmax(b, partials[2 * i + 1]) : b + partials[2 * i + 1];
    }
    s0[t] = a;
    s1[t] = b;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      s0[t] += s0[t + w];
      s1[t] = MAX2 ? fmax(s1[t], s1[t + w]) : s1[t] + s1[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

template <bool MAX2>
__global__ void k_finish(const double* __restrict__ partials, int count, double* out) {
  finish_block<MAX2>(partials, count, out);
}

// The smallest coarse levels in one block (see SmallArgs).
template <class T, int D>
__device__ inline void small_unravel(long long i, int n, int j[3]) {
  unravel_fast<D>((unsigned)i, n, fastdiv_magic(n), j);   // small levels: n <= 16
}

template <class T, int D>
__device__ inline void small_pre_levels(const SmallArgs<T>& a) {
  for (int k = 0; k < a.nl; ++k) {
    const SmallLevel<T>& v = a.lv[k];
    const long long N = D == 3 ? (long long)v.n * v.n * v.n : (long long)v.n * v.n;
    const bool hc = k > 0;
    for (long long i = threadIdx.x; i < N; i += blockDim.x) {
      int j[3];
      small_unravel<T, D>(i, v.n, j);
      pre_vertex<T, D>(v.n, j, i, v.u, v.sc, v.sf, hc ? a.lv[k - 1].sc : nullptr, hc ? a.lv[k - 1].si : nullptr,
                       hc ? 1 : 0, a.variant == 2 ? 1 : 0);
    }
    __syncthreads();
  }
}

template <class T, int D>
__global__ __launch_bounds__(kSmallThreads) void k_small_pre(SmallArgs<T> a) {
  small_pre_levels<T, D>(a);
}

template <class T, int D>
__global__ __launch_bounds__(kSmallThreads) void k_small_post(SmallArgs<T> a) {
  const bool add = a.variant == 0, bpx = a.variant == 2;
  // Galerkin backtracking of levels l_min + nl - 1 .. l_min + 1: eight lanes
  // per coarse vertex, as k_post_galerkin
  for (int k = a.nl - 1; k >= 1; --k) {
    const SmallLevel<T>& v = a.lv[k];
    const SmallLevel<T>& c = a.lv[k - 1];
    const long long Nc = D == 3 ? (long long)c.n * c.n * c.n : (long long)c.n * c.n;
    for (long long g = threadIdx.x; g < 8 * Nc; g += blockDim.x) {
      const long long vv = g >> 3;
      const int part = (int)(g & 7);
      int m[3];
      small_unravel<T, D>(vv, c.n, m);
      cpx<T> p = czero<T>();
      if (part < 5)
        p = post_galerkin_part<T, D>(v.op, m, vv, part - 2, v.b, v.omega, add ? 0 : 1, v.sc, v.sf,
                                     add ? c.sf : nullptr, bpx ? c.si : nullptr);
      T re = p.re, im = p.im;
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (part == 0) c.b[vv] = csel(is_interior<D>(m, c.n), mk(re, im), czero<T>());
    }
    __syncthreads();
  }
  // coarsest level: pointwise update from its residual
  {
    const SmallLevel<T>& v = a.lv[0];
    const long long N = D == 3 ? (long long)v.n * v.n * v.n : (long long)v.n * v.n;
    for (long long i = threadIdx.x; i < N; i += blockDim.x) {
      int j[3];
      small_unravel<T, D>(i, v.n, j);
      update_vertex<T, D>(v.op, j, i, v.b, v.omega, 0, nullptr, v.sc, v.sf, nullptr, nullptr);
    }
  }
  if (a.partials) finish_block<true>(a.partials, a.nparts, a.out);
  // the next cycle starts with the pre-phase of these levels: one launch fewer
  if (a.then_pre) {
    __syncthreads();
    small_pre_levels<T, D>(a);
  }
}


// ---------------------------------------------------------------------------
// Launch wrappers.
static inline int grid_for(long long N, int threads = 256) {
  long long g = (N + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

#define MG_DISPATCH(dim, KERNEL, GRID, ...)                                         \
  do {                                                                              \
    if ((dim) == 3) hipLaunchKernelGGL((KERNEL<T, 3>), GRID, 256, 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL((KERNEL<T, 2>), GRID, 256, 0, s, __VA_ARGS__);            \
  } while (0)

static inline long long pow_n(int n, int dim) { return dim == 3 ? (long long)n * n * n : (long long)n * n; }

// Grid of the row-based kernels: x blocks of 64 columns, 4 rows per block,
// at most max_rows_blocks row blocks (grid-stride beyond).
static inline dim3 row_grid(int n, int dim, int max_row_blocks = 65535) {
  const long long rows = dim == 3 ? (long long)n * n : n;
  long long gy = (rows + 3) / 4;
  if (gy > max_row_blocks) gy = max_row_blocks;
  return dim3((n + 63) / 64, (unsigned)gy, 1);
}

template <class T>
hipError_t launch_apply(int dim, const OpData<T>& op, const cpx<T>* x, cpx<T>* y, hipStream_t s) {
  if (dim == 3 && !op.cmass && stencil3_blocks(op.n) > 0)
    return launch_stencil3<T>(1, op.n, op.coef, nullptr, x, y, nullptr, nullptr, s);
  if (dim == 3 && op.cmass) return launch_resid<T>(dim, op, nullptr, x, y, nullptr, nullptr, s);
  MG_DISPATCH(dim, k_apply, row_grid(op.n, dim), op, x, y);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pre(int dim, int n, cpx<T>* u, cpx<T>* sc, const cpx<T>* sf, const cpx<T>* scc,
                      const cpx<T>* sic, int has_coarse, int bpx, hipStream_t s) {
  if (dim == 3 && has_coarse && n >= kPreMarchMinN)
    return launch_prolong_march3<T, kPmPre>(n, u, sc, sf, scc, sic, bpx, s);
  if (dim == 3 && n <= kFastDivMaxN && n % 64 != 0) {
    const long long N = (long long)n * n * n;
    hipLaunchKernelGGL(k_pre_flat3<T>, dim3((unsigned)((N + 255) / 256)), 256, 0, s, n, u, sc, sf, scc, sic, has_coarse,
                       bpx);
    return hipGetLastError();
  }
  MG_DISPATCH(dim, k_pre, row_grid(n, dim), n, u, sc, sf, scc, sic, has_coarse, bpx);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fine_pre(int dim, int n, const cpx<T>* w, cpx<T>* u, const cpx<T>* scc, const cpx<T>* sic,
                           int has_coarse, int bpx, hipStream_t s) {
  if (dim == 3 && has_coarse && n >= kProlongMarchMinN)
    return launch_prolong_march3<T, kPmFine>(n, u, const_cast<cpx<T>*>(w), nullptr, scc, sic, bpx, s);
  MG_DISPATCH(dim, k_fine_pre, row_grid(n, dim), n, w, u, scc, sic, has_coarse, bpx);
  return hipGetLastError();
}

template <class T>
hipError_t launch_uhat(int dim, int n, const cpx<T>* u, const cpx<T>* uc, cpx<T>* uh, hipStream_t s) {
  if (dim == 3 && n >= kProlongMarchMinN)
    return launch_prolong_march3<T, kPmSurplus>(n, uh, const_cast<cpx<T>*>(u), nullptr, uc, nullptr, 0, s);
  MG_DISPATCH(dim, k_uhat, row_grid(n, dim), n, u, uc, uh);
  return hipGetLastError();
}

template <class T>
hipError_t launch_resid(int dim, const OpData<T>& op, const cpx<T>* b, const cpx<T>* x, cpx<T>* r,
                        double* partials, int* nparts, hipStream_t s) {
  const int sb = dim == 3 && !op.cmass && r ? stencil3_blocks(op.n) : -1;
  if (sb > 0 && (!partials || sb <= kRedBlocks))
    return launch_stencil3<T>(0, op.n, op.coef, b, x, r, partials, nparts, s);
  if (dim == 3 && op.cmass) {
    const int gx = (op.n + 63) / 64;
    const long long items = (long long)op.n * ((op.n + kVarTz - 1) / kVarTz);
    int gy = (int)std::min<long long>((items + 3) / 4, 65535);
    if (partials) {
      // the row kernel's block count (resid_norm_blocks); blocks past the
      // items only write zero partials
      gy = std::max(1, std::min((int)row_grid(op.n, dim).y, kRedBlocks / gx));
      if (nparts) *nparts = gx * gy;
    }
    if (op.cstiff) hipLaunchKernelGGL((k_resid_var3<T, true>), dim3(gx, gy), 256, 0, s, op, b, x, r, partials);
    else hipLaunchKernelGGL((k_resid_var3<T, false>), dim3(gx, gy), 256, 0, s, op, b, x, r, partials);
    return hipGetLastError();
  }
  dim3 g = row_grid(op.n, dim);
  if (partials) {
    const int gx = (int)g.x;
    g.y = std::max(1, std::min((int)g.y, kRedBlocks / gx));
    if (nparts) *nparts = gx * (int)g.y;
  }
  MG_DISPATCH(dim, k_resid, g, op, b, x, r, partials);
  return hipGetLastError();
}

int resid_norm_blocks(int dim, int n) {
  // (the per-cell 3D march is launched with the same count when it writes partials)
  const dim3 g = row_grid(n, dim);
  const int gx = (int)g.x;
  if (gx > kRedBlocks) return -1;
  return gx * std::max(1, std::min((int)g.y, kRedBlocks / gx));
}

template <class T>
hipError_t launch_post_galerkin(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, int mask_c,
                                cpx<T>* sc, const cpx<T>* sf, cpx<T>* rhoc, cpx<T>* sfc, cpx<T>* sic, hipStream_t s) {
  const int nc = (op.n - 1) / 3 + 1;
  const long long lanes = 8 * pow_n(nc, dim);
  MG_DISPATCH(dim, k_post_galerkin, dim3((unsigned)((lanes + 255) / 256)), op, rho, omega, mask_c, sc, sf, rhoc, sfc,
              sic);
  return hipGetLastError();
}

template <class T>
hipError_t launch_update(int dim, const OpData<T>& op, const cpx<T>* r, cpx<T> omega, int mask_c, cpx<T>* u,
                         cpx<T>* sc_out, const cpx<T>* sf, cpx<T>* sfc, cpx<T>* sic, hipStream_t s) {
  MG_DISPATCH(dim, k_update, row_grid(op.n, dim), op, r, omega, mask_c, u, sc_out, sf, sfc, sic);
  return hipGetLastError();
}

template <class T>
hipError_t launch_restrict(int dim, int nc, const cpx<T>* vf, cpx<T>* vc, hipStream_t s) {
  const long long lanes = 8 * pow_n(nc, dim);
  MG_DISPATCH(dim, k_restrict, dim3((unsigned)((lanes + 255) / 256)), nc, vf, vc);
  return hipGetLastError();
}

template <class T>
hipError_t launch_inject(int dim, int nc, const cpx<T>* vf, cpx<T>* vc, hipStream_t s) {
  MG_DISPATCH(dim, k_inject, row_grid(nc, dim), nc, vf, vc);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sample(int dim, int nc, int stride, const cpx<T>* vf, cpx<T>* vc, hipStream_t s) {
  if (nc < 2 || stride < 1) return hipErrorInvalidValue;
  MG_DISPATCH(dim, k_sample, row_grid(nc, dim), nc, stride, vf, vc);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prolong(int dim, int n, const cpx<T>* uc, cpx<T>* uf, hipStream_t s) {
  if (n < 4 || (n - 1) % 3 != 0) return hipErrorInvalidValue;
  MG_DISPATCH(dim, k_prolong, row_grid(n, dim), n, uc, uf);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prec_up(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, int mask_c, int is_lmin,
                          const cpx<T>* gc, cpx<T>* z, hipStream_t s) {
  MG_DISPATCH(dim, k_prec_up, row_grid(op.n, dim), op, rho, omega, mask_c, is_lmin, gc, z);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prec_g(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, const cpx<T>* zc, cpx<T>* g,
                         hipStream_t s) {
  const int nc = (op.n - 1) / 3 + 1;
  MG_DISPATCH(dim, k_prec_g, row_grid(nc, dim), op, rho, omega, zc, g);
  return hipGetLastError();
}

template <class T>
hipError_t launch_cellcoef(int dim, int n, const cpx<T>* phi, cpx<T>* mass, cpx<T>* stiff, CellRotation rot,
                           hipStream_t s) {
  MG_DISPATCH(dim, k_cellcoef, dim3(grid_for(pow_n(n - 1, dim))), n, phi, mass, stiff, rot);
  return hipGetLastError();
}

template <class T>
hipError_t launch_invdiag(int dim, const OpData<T>& op, cpx<T>* invDv, hipStream_t s) {
  MG_DISPATCH(dim, k_invdiag, row_grid(op.n, dim), op, invDv);
  return hipGetLastError();
}

template <class T>
hipError_t launch_zero_boundary_copy(int dim, int n, const cpx<T>* in, cpx<T>* out, cpx<T> scale, hipStream_t s) {
  MG_DISPATCH(dim, k_zero_boundary_copy, row_grid(n, dim), n, in, out, scale);
  return hipGetLastError();
}

template <class T>
hipError_t launch_set_value(size_t count, cpx<T>* v, cpx<double> value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_value<T>, dim3(grid_for((long long)count)), 256, 0, s, count, v,
                     mk(T(value.re), T(value.im)));
  return hipGetLastError();
}

hipError_t launch_rhs_cells(int dim, int n, const cpx<double>* chi, cpx<double>* b, CellRotation rot, hipStream_t s) {
  if (dim == 3) hipLaunchKernelGGL(k_rhs_cells<3>, row_grid(n, 3), 256, 0, s, n, chi, b, rot);
  else hipLaunchKernelGGL(k_rhs_cells<2>, row_grid(n, 2), 256, 0, s, n, chi, b, rot);
  return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((long long)words)), 256, 0, s, (unsigned int*)p, words);
  return hipGetLastError();
}

template <class S, class Dt>
hipError_t launch_convert(size_t count, const cpx<S>* in, cpx<Dt>* out, double scale, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<S, Dt>), dim3(grid_for((long long)count)), 256, 0, s, count, in, out, scale);
  return hipGetLastError();
}

template <class T>
hipError_t launch_dot(size_t count, const cpx<T>* a, const cpx<T>* b, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<T>, dim3(kRedBlocks), kRedThreads, 0, s, count, a, b, partials);
  return hipGetLastError();
}

template <class T>
hipError_t launch_norm2(size_t count, const cpx<T>* a, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2<T>, dim3(kRedBlocks), kRedThreads, 0, s, count, a, partials);
  return hipGetLastError();
}

template <class T>
hipError_t launch_axpby(size_t count, cpx<double> a, const cpx<T>* x, cpx<double> b, cpx<T>* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for((long long)count)), 256, 0, s, count, a, x, b, y);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_p(size_t count, const cpx<T>* r, const cpx<T>* v, cpx<double> beta, cpx<double> w,
                         cpx<T>* p, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_p<T>, dim3(grid_for((long long)count)), 256, 0, s, count, r, v, beta, w, p);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_xr(size_t count, cpx<T>* x, const cpx<T>* y, const cpx<T>* z, cpx<double> a, cpx<double> w,
                          cpx<T>* r, const cpx<T>* sv, const cpx<T>* t, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_xr<T>, dim3(grid_for((long long)count)), 256, 0, s, count, x, y, z, a, w, r, sv, t);
  return hipGetLastError();
}

hipError_t launch_accum32(size_t count, const cpx<float>* e, double scale, cpx<double>* u, hipStream_t s) {
  hipLaunchKernelGGL(k_accum32, dim3(grid_for((long long)count)), 256, 0, s, count, e, scale, u);
  return hipGetLastError();
}

hipError_t launch_grad_potential(int dim, int n, cpx<double> etad, const cpx<double>* u, const cpx<double>* lam,
                                 double* g, hipStream_t s) {
  const int grid = grid_for(pow_n(n, dim));
  if (dim == 3) hipLaunchKernelGGL(k_grad_potential<3>, dim3(grid), 256, 0, s, n, etad, u, lam, g);
  else hipLaunchKernelGGL(k_grad_potential<2>, dim3(grid), 256, 0, s, n, etad, u, lam, g);
  return hipGetLastError();
}

hipError_t launch_finish_sum_max(const double* partials, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish<true>, dim3(1), 256, 0, s, partials, count, out);
  return hipGetLastError();
}

template <class T>
hipError_t launch_small_pre(const SmallArgs<T>& a, hipStream_t s) {
  if (a.nl < 1 || a.nl > kSmallMax) return hipErrorInvalidValue;
  if (a.dim == 3) hipLaunchKernelGGL((k_small_pre<T, 3>), dim3(1), kSmallThreads, 0, s, a);
  else hipLaunchKernelGGL((k_small_pre<T, 2>), dim3(1), kSmallThreads, 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_small_post(const SmallArgs<T>& a, hipStream_t s) {
  if (a.nl < 1 || a.nl > kSmallMax) return hipErrorInvalidValue;
  if (a.dim == 3) hipLaunchKernelGGL((k_small_post<T, 3>), dim3(1), kSmallThreads, 0, s, a);
  else hipLaunchKernelGGL((k_small_post<T, 2>), dim3(1), kSmallThreads, 0, s, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_s(size_t count, const cpx<T>* r, const cpx<T>* v, cpx<double> a, cpx<T>* sv, double* partials,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_s<T>, dim3(kRedBlocks), 256, 0, s, count, r, v, a, sv, partials);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_ts(size_t count, const cpx<T>* t, const cpx<T>* sv, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_ts<T>, dim3(kRedBlocks), 256, 0, s, count, t, sv, partials);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bicg_xr2(size_t count, cpx<T>* x, const cpx<T>* y, const cpx<T>* z, cpx<double> a, cpx<double> w,
                           cpx<T>* r, const cpx<T>* sv, const cpx<T>* t, const cpx<T>* rh, double* partials,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_xr2<T>, dim3(kRedBlocks), 256, 0, s, count, x, y, z, a, w, r, sv, t, rh, partials);
  return hipGetLastError();
}

hipError_t launch_finishN(int nvals, const double* partials, int count, double* out, hipStream_t s) {
  if (nvals == 1) hipLaunchKernelGGL(k_finishN<1>, dim3(1), 256, 0, s, partials, count, out);
  else if (nvals == 3) hipLaunchKernelGGL(k_finishN<3>, dim3(1), 256, 0, s, partials, count, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_finish_sum2(const double* partials, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish<false>, dim3(1), 256, 0, s, partials, count, out);
  return hipGetLastError();
}

#define MG_INSTANTIATE(T)                                                                                        \
  template hipError_t launch_apply<T>(int, const OpData<T>&, const cpx<T>*, cpx<T>*, hipStream_t);              \
  template hipError_t launch_pre<T>(int, int, cpx<T>*, cpx<T>*, const cpx<T>*, const cpx<T>*, const cpx<T>*, int, \
                                    int, hipStream_t);                                                          \
  template hipError_t launch_fine_pre<T>(int, int, const cpx<T>*, cpx<T>*, const cpx<T>*, const cpx<T>*, int, int, \
                                         hipStream_t);                                                          \
  template hipError_t launch_uhat<T>(int, int, const cpx<T>*, const cpx<T>*, cpx<T>*, hipStream_t);             \
  template hipError_t launch_resid<T>(int, const OpData<T>&, const cpx<T>*, const cpx<T>*, cpx<T>*, double*,     \
                                      int*, hipStream_t);                                                       \
  template hipError_t launch_bicg_s<T>(size_t, const cpx<T>*, const cpx<T>*, cpx<double>, cpx<T>*, double*,      \
                                       hipStream_t);                                                            \
  template hipError_t launch_bicg_ts<T>(size_t, const cpx<T>*, const cpx<T>*, double*, hipStream_t);              \
  template hipError_t launch_bicg_xr2<T>(size_t, cpx<T>*, const cpx<T>*, const cpx<T>*, cpx<double>, cpx<double>, \
                                         cpx<T>*, const cpx<T>*, const cpx<T>*, const cpx<T>*, double*,          \
                                         hipStream_t);                                                          \
  template hipError_t launch_small_pre<T>(const SmallArgs<T>&, hipStream_t);                                     \
  template hipError_t launch_small_post<T>(const SmallArgs<T>&, hipStream_t);                                    \
  template hipError_t launch_post_galerkin<T>(int, const OpData<T>&, const cpx<T>*, cpx<T>, int, cpx<T>*,        \
                                              const cpx<T>*, cpx<T>*, cpx<T>*, cpx<T>*, hipStream_t);            \
  template hipError_t launch_update<T>(int, const OpData<T>&, const cpx<T>*, cpx<T>, int, cpx<T>*, cpx<T>*,      \
                                       const cpx<T>*, cpx<T>*, cpx<T>*, hipStream_t);                            \
  template hipError_t launch_restrict<T>(int, int, const cpx<T>*, cpx<T>*, hipStream_t);                        \
  template hipError_t launch_inject<T>(int, int, const cpx<T>*, cpx<T>*, hipStream_t);                          \
  template hipError_t launch_sample<T>(int, int, int, const cpx<T>*, cpx<T>*, hipStream_t);                     \
  template hipError_t launch_prolong<T>(int, int, const cpx<T>*, cpx<T>*, hipStream_t);                         \
  template hipError_t launch_prec_up<T>(int, const OpData<T>&, const cpx<T>*, cpx<T>, int, int, const cpx<T>*,   \
                                        cpx<T>*, hipStream_t);                                                  \
  template hipError_t launch_prec_g<T>(int, const OpData<T>&, const cpx<T>*, cpx<T>, const cpx<T>*, cpx<T>*,     \
                                       hipStream_t);                                                            \
  template hipError_t launch_cellcoef<T>(int, int, const cpx<T>*, cpx<T>*, cpx<T>*, CellRotation, hipStream_t);  \
  template hipError_t launch_set_value<T>(size_t, cpx<T>*, cpx<double>, hipStream_t);                           \
  template hipError_t launch_invdiag<T>(int, const OpData<T>&, cpx<T>*, hipStream_t);                           \
  template hipError_t launch_zero_boundary_copy<T>(int, int, const cpx<T>*, cpx<T>*, cpx<T>, hipStream_t);      \
  template hipError_t launch_dot<T>(size_t, const cpx<T>*, const cpx<T>*, double*, hipStream_t);                \
  template hipError_t launch_norm2<T>(size_t, const cpx<T>*, double*, hipStream_t);                             \
  template hipError_t launch_axpby<T>(size_t, cpx<double>, const cpx<T>*, cpx<double>, cpx<T>*, hipStream_t);   \
  template hipError_t launch_bicg_p<T>(size_t, const cpx<T>*, const cpx<T>*, cpx<double>, cpx<double>, cpx<T>*, \
                                       hipStream_t);                                                            \
  template hipError_t launch_bicg_xr<T>(size_t, cpx<T>*, const cpx<T>*, const cpx<T>*, cpx<double>, cpx<double>, \
                                        cpx<T>*, const cpx<T>*, const cpx<T>*, hipStream_t);

MG_INSTANTIATE(double)
MG_INSTANTIATE(float)
template hipError_t launch_convert<double, float>(size_t, const cpx<double>*, cpx<float>*, double, hipStream_t);
template hipError_t launch_convert<float, double>(size_t, const cpx<float>*, cpx<double>*, double, hipStream_t);
template hipError_t launch_convert<double, double>(size_t, const cpx<double>*, cpx<double>*, double, hipStream_t);

}  // namespace mg
