// Device functions of the fused finest-level sweep, shared by the standalone
// kernels (mg_fused.hip) and the batched persistent kernel (mg_batch.hip).
// Fused finest-level sweep of the pipelined additive cycle (constant phi,
// Galerkin form of the coarse right-hand side), one pass over the finest grid:
//
//   pre  (descent of tdAdd / tdBPX):  u = w + P g,  g = sc_c (- si_c off c-points for BPX)
//   post (backtracking):              r = b - H u,  s = omega r / D,
//                                     w' = u + s (s masked on c-points for hb / BPX),
//                                     rho_c = R r,  sf_c = I s (add),  si_c = I s (BPX),
//                                     partial sums of |r|^2 and max |r|.
//
// w is the finest iterate with the finest smoothing update already folded in
// (u + sc of the paper's state); only the coarse correction is pending.  With
// constant phi the Galerkin identity R H_l P = H_(l-1) turns the paper's
// R (b - H uhat) into R r + H_(l-1) u_(l-1) (its Lemma 2), so the finest level
// needs one operator application; the coarse level reads its residual from the
// restricted one.  BPX reads si_c of the previous cycle and writes the new one:
// the caller passes two different buffers.
//
// Work decomposition (3D).  A block owns a box of coarse vertices: 20 x TYC in
// the plane and ZC coarse planes.  Its fine vertices (3m .. 3m+2 per axis) are
// written by it alone.  R at a coarse vertex m needs r on fine offsets -2..2
// around 3m, so r is computed on the owned fine box extended by two vertices
// towards lower x and y, and u on one more vertex on each side: 64 columns,
// exactly one wavefront, lane l at x = x0 - 3 + l.  x-neighbours are exchanged
// with DPP wave shifts (no LDS); each thread keeps RPT consecutive rows (and
// the two rows around them) in registers; the block marches through z one fine
// plane per step.  The 27-point stencil row at plane p splits into an in-plane
// part M_p and a neighbour-plane part N_p, so H u at plane p-1 is
// M_(p-1) + N_(p-2) + N_p, carried in registers.  The next plane's w and b are
// loaded while the current plane is processed.  R: x-part by DPP shifts, y-part
// through LDS, z-part in a two-slot ring of coarse planes; one barrier a step.
#pragma once
#include "mg_internal.h"

namespace mg {


template <class T>
__device__ inline cpx<T> f_add(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <class T>
__device__ inline cpx<T> f_sub(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <class T>
__device__ inline cpx<T> f_scale(T s, cpx<T> a) { return mk(s * a.re, s * a.im); }
template <class T>
__device__ inline cpx<T> f_mul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__device__ inline cpx<T> f_mac(cpx<T> acc, cpx<T> c, cpx<T> x) {  // acc + c x
  return mk(acc.re + c.re * x.re - c.im * x.im, acc.im + c.re * x.im + c.im * x.re);
}
template <class T>
__device__ inline cpx<T> f_zero() { return mk(T(0), T(0)); }

__device__ inline int floor_div3(int p) { return p >= 0 ? p / 3 : -((-p + 2) / 3); }

// Linear interpolation weights of fine offset q in {0,1,2} inside a coarse cell,
// and restriction weights of offset o in [-2, 2].
template <class T>
__device__ inline T w_lo(int q) { return q == 0 ? T(1) : (q == 1 ? T(2.0 / 3.0) : T(1.0 / 3.0)); }
template <class T>
__device__ inline T w_hi(int q) { return q == 0 ? T(0) : (q == 1 ? T(1.0 / 3.0) : T(2.0 / 3.0)); }
template <class T>
__device__ inline T w_r(int o) { return o == 0 ? T(1) : ((o == 1 || o == -1) ? T(2.0 / 3.0) : T(1.0 / 3.0)); }

// Wave-wide lane shifts (DPP): lane l receives lane l-1 (LEFT) or l+1 (RIGHT);
// the lane falling off the wave receives 0.
constexpr int kDppLeft = 0x138;
constexpr int kDppRight = 0x130;

template <int CTRL>
__device__ inline double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo));
}
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL, class T>
__device__ inline cpx<T> dpp_c(cpx<T> v) { return mk(dpp_move<CTRL>(v.re), dpp_move<CTRL>(v.im)); }

__device__ inline void block_reduce_store(double s, double m, double* part, int nt) {
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
    for (int w = 0; w < (nt + 63) / 64; ++w) { a += ss[w]; b = fmax(b, sm[w]); }
    part[0] = a;
    part[1] = b;
  }
  __syncthreads();
}

// Wavefront-local ordering of LDS traffic (the 2D sweep runs one tile per wave).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------
// 3D
constexpr int F3_TXC = 20;     // coarse columns per block: 60 owned fine columns + 4 halo = 64 lanes

template <class T, int TYC, int RPT, int ZC, bool BPX>
struct F3 {
  static constexpr int TXC = F3_TXC, TX = 3 * TXC, TY = 3 * TYC;
  static constexpr int CY = TY + 2;            // computed rows y0-2 .. y0+TY-1
  static constexpr int W = CY / RPT;           // waves per block
  static constexpr int NT = 64 * W;
  static constexpr int IR = RPT + 2;           // rows of u a thread needs
  static constexpr int GX = TXC + 2, GY = TYC + 2, NG = GX * GY;
  static_assert(CY % RPT == 0, "rows per thread must divide the computed rows");
  static_assert(NG <= NT && TXC * TYC <= NT, "staging needs one thread per coarse point");
};

// LDS of one 3D tile: restricted x-partials of the computed rows (two planes)
// and the staged coarse corrections of two planes (BPX: also sc itself).  The
// z extent does not enter, so tiles that differ only in ZC can share it.
template <class T, int TYC, int RPT, bool BPX>
struct F3Lds {
  using G = F3<T, TYC, RPT, 1, BPX>;
  cpx<T> RX[2][G::CY][G::TXC];
  cpx<T> Gz[2][G::GY][G::GX];
  cpx<T> Sz[BPX ? 2 : 1][BPX ? G::GY : 1][BPX ? G::GX : 1];
};

// One tile (bx, by, bz) of the 3D sweep, executed by a whole block of
// F3<...>::NT threads with LDS `sm`; `part` receives the tile's
// (sum |r|^2, max |r|) or is null.
template <class T, int TYC, int RPT, int ZC, bool BPX>
__device__ inline void fused3_tile(const FusedArgs<T>& a, int bx, int by, int bz, double* part,
                                   F3Lds<T, TYC, RPT, BPX>& sm) {
  using G = F3<T, TYC, RPT, ZC, BPX>;
  constexpr int TXC = G::TXC, TX = G::TX, TY = G::TY, CY = G::CY, IR = G::IR, GX = G::GX, NG = G::NG;
  auto& RX = sm.RX;
  auto& Gz = sm.Gz;
  auto& Sz = sm.Sz;

  const int tid = threadIdx.x, lane = tid & 63;
  // the wave index is uniform across a wavefront: keeping it scalar makes every
  // y-dependent quantity (row validity, weights, row addresses) scalar too
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, nc = a.nc;
  const int n2 = n * n, nc2 = nc * nc;
  const int mx0 = bx * TXC, my0 = by * TYC, mz0 = bz * ZC;
  const int mz1 = min(mz0 + ZC, nc);
  const int x0 = 3 * mx0, y0 = 3 * my0;
  const int x = x0 - 3 + lane;
  const bool xin = x >= 1 && x <= n - 2;
  const bool xcomp = lane >= 1 && lane <= 62;
  const bool xown = x >= x0 && x <= min(x0 + TX - 1, n - 1);
  const int yfirst = y0 - 3 + wv * RPT;            // input row k sits at y = yfirst + k
  const int yown_hi = min(y0 + TY - 1, n - 1);
  const int zown_lo = 3 * mz0, zown_hi = min(3 * mz1 - 1, n - 1);
  const bool mask = a.variant != 0;
  const cpx<T> c0 = a.coef[0], c1 = a.coef[1], c2 = a.coef[2], c3 = a.coef[3];
  const cpx<T> ws = a.ws;
  // x part of the prolongation for this lane
  const int mxl = x >= 0 ? x / 3 : 0, qx = x - 3 * mxl, gxl = mxl - mx0 + 1;
  const T wx0 = w_lo<T>(qx), wx1 = w_hi<T>(qx);
  // staging point of this thread (coarse in-plane)
  const int sgx = tid % GX, sgy = tid / GX;
  const int smx = mx0 - 1 + sgx, smy = my0 - 1 + sgy;
  const bool sval = tid < NG && smx >= 0 && smx < nc && smy >= 0 && smy < nc;
  const int sidx = smy * nc + smx;

  cpx<T> wc[IR], wn[IR], bc[RPT], bn[RPT];
  cpx<T> A[RPT], Np[RPT], Cp[RPT];
  cpx<T> gsc0, gsc1, gsi0, gsi1;
  cpx<T> acc0 = f_zero<T>(), acc1 = f_zero<T>();
  double nsum = 0.0, nmax = 0.0;

  auto plane_ok = [&](int p) { return p >= 1 && p <= n - 2; };
  auto load_w = [&](int p, cpx<T>* dst) {
#pragma unroll
    for (int k = 0; k < IR; ++k) {
      const int y = yfirst + k;
      const cpx<T>* row = a.w + ((long long)p * n2 + (long long)y * n);
      dst[k] = (plane_ok(p) && y >= 1 && y <= n - 2 && xin) ? row[x] : f_zero<T>();
    }
  };
  auto load_b = [&](int q, cpx<T>* dst) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int y = yfirst + 1 + j;
      const cpx<T>* row = a.b + ((long long)q * n2 + (long long)y * n);
      dst[j] = (plane_ok(q) && y >= 1 && y <= n - 2 && xin && xcomp) ? row[x] : f_zero<T>();
    }
  };
  auto load_g = [&](int p) {
    gsc0 = gsc1 = gsi0 = gsi1 = f_zero<T>();
    if (sval && plane_ok(p)) {
      const int kz = p / 3, tz = p - 3 * kz;
      const long long c = (long long)kz * nc2 + sidx;
      gsc0 = a.scc[c];
      if (BPX) gsi0 = a.sic[c];
      if (tz != 0) {
        gsc1 = a.scc[c + nc2];
        if (BPX) gsi1 = a.sic[c + nc2];
      }
    }
  };
  auto store_g = [&](int p) {
    if (tid < NG) {
      const int kz = floor_div3(p), tz = p - 3 * kz;
      const cpx<T> g0 = BPX ? f_sub(gsc0, gsi0) : gsc0;
      const cpx<T> g1 = BPX ? f_sub(gsc1, gsi1) : gsc1;
      Gz[p & 1][sgy][sgx] = tz == 0 ? g0 : f_add(f_scale(w_lo<T>(tz), g0), f_scale(w_hi<T>(tz), g1));
      if (BPX) Sz[p & 1][sgy][sgx] = gsc0;   // used on c-points only (tz == 0)
    }
  };

  const int p0 = 3 * mz0 - 3;
  load_g(p0);
  store_g(p0);
  load_g(p0 + 1);
  load_w(p0, wc);
  load_b(p0 - 1, bc);
#pragma unroll
  for (int j = 0; j < RPT; ++j) { A[j] = f_zero<T>(); Np[j] = f_zero<T>(); Cp[j] = f_zero<T>(); }
  __syncthreads();

  for (int p = p0; p <= 3 * mz1; ++p) {
    const int q = p - 1;
    const int pb = p & 1;
    // prefetch the next plane
    load_w(p + 1, wn);
    load_b(p, bn);
    // (1) u on plane p: folded iterate plus the prolongated coarse correction
    const int kz = floor_div3(p), tz = p - 3 * kz;
    cpx<T> u[IR];
#pragma unroll
    for (int k = 0; k < IR; ++k) {
      const int y = yfirst + k;
      cpx<T> v = f_zero<T>();
      if (plane_ok(p) && xin && y >= 1 && y <= n - 2) {
        const int my = y / 3, qy = y - 3 * my, gy = my - my0 + 1;
        if (BPX && qx == 0 && qy == 0 && tz == 0) {
          v = f_add(wc[k], Sz[pb][gy][gxl]);       // BPX keeps si on c-points: sc_c itself
        } else {
          cpx<T> row0 = f_scale(wx0, Gz[pb][gy][gxl]);
          if (qx != 0) row0 = f_add(row0, f_scale(wx1, Gz[pb][gy][gxl + 1]));
          cpx<T> g = f_scale(w_lo<T>(qy), row0);
          if (qy != 0) {
            cpx<T> row1 = f_scale(wx0, Gz[pb][gy + 1][gxl]);
            if (qx != 0) row1 = f_add(row1, f_scale(wx1, Gz[pb][gy + 1][gxl + 1]));
            g = f_add(g, f_scale(w_hi<T>(qy), row1));
          }
          v = f_add(wc[k], g);
        }
      }
      u[k] = v;
    }
    // (2) in-row neighbour sums by lane shifts
    cpx<T> h[IR];
#pragma unroll
    for (int k = 0; k < IR; ++k) h[k] = f_add(dpp_c<kDppLeft>(u[k]), dpp_c<kDppRight>(u[k]));
    // (3) stencil, residual, smoothing update, folded iterate, injections
    const bool q_in = plane_ok(q);
    const bool q_own = q >= zown_lo && q <= zown_hi;
    const bool q_c = q >= 0 && (q % 3) == 0;
    cpx<T> r[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int y = yfirst + 1 + j;
      const cpx<T> C = u[j + 1];
      const cpx<T> F2 = f_add(h[j + 1], f_add(u[j], u[j + 2]));
      const cpx<T> E2 = f_add(h[j], h[j + 2]);
      const cpx<T> M = f_mac(f_mac(f_mul(c0, C), c1, F2), c2, E2);
      const cpx<T> N = f_mac(f_mac(f_mul(c1, C), c2, F2), c3, E2);
      const bool in = q_in && xin && xcomp && y >= 1 && y <= n - 2;
      const cpx<T> rv = in ? f_sub(bc[j], f_add(A[j], N)) : f_zero<T>();
      const cpx<T> s = f_mul(ws, rv);
      const bool cp = q_c && qx == 0 && x >= 0 && y >= 0 && (y % 3) == 0;
      const cpx<T> scm = (mask && cp) ? f_zero<T>() : s;
      if (q_own && xown && y >= y0 && y <= yown_hi) {
        cpx<T>* row = a.wout + ((long long)q * n2 + (long long)y * n);
        row[x] = in ? f_add(Cp[j], scm) : f_zero<T>();
        if (in) {
          const double r2 = (double)rv.re * rv.re + (double)rv.im * rv.im;
          nsum += r2;
          nmax = fmax(nmax, r2);
        }
        if (cp) {
          const long long ic = (long long)(q / 3) * nc2 + (y / 3) * nc + x / 3;
          if (a.sfc) a.sfc[ic] = scm;
          if (BPX) a.sic_out[ic] = s;
        }
      }
      r[j] = rv;
      A[j] = f_add(M, Np[j]);
      Np[j] = N;
      Cp[j] = C;
    }
    // (4) x-part of R by lane shifts; lanes 3, 6, .., 60 sit on coarse columns
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const cpx<T> l1 = dpp_c<kDppLeft>(r[j]), l2 = dpp_c<kDppLeft>(l1);
      const cpx<T> r1 = dpp_c<kDppRight>(r[j]), r2 = dpp_c<kDppRight>(r1);
      const cpx<T> rx = f_add(r[j], f_add(f_scale(T(2.0 / 3.0), f_add(l1, r1)), f_scale(T(1.0 / 3.0), f_add(l2, r2))));
      if (lane >= 3 && lane <= 60 && lane % 3 == 0) RX[pb][wv * RPT + j][lane / 3 - 1] = rx;
    }
    // (5) coarse correction of the next plane into LDS, fetch the one after
    store_g(p + 1);
    load_g(p + 2);
    __syncthreads();
    // (6) y-part of R at the owned coarse vertices, ring over coarse planes
    if (q >= 3 * mz0 - 2 && tid < TXC * TYC) {
      const int lx = tid % TXC, ly = tid / TXC;
      const int mx = mx0 + lx, my = my0 + ly;
      cpx<T> v = f_zero<T>();
#pragma unroll
      for (int oy = -2; oy <= 2; ++oy) v = f_add(v, f_scale(w_r<T>(oy), RX[pb][3 * ly + 2 + oy][lx]));
      const int k0 = floor_div3(q), t = q - 3 * k0;
      if (t == 0) {
        acc0 = f_add(acc0, v);
      } else if (t == 1) {
        acc0 = f_add(acc0, f_scale(T(2.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(1.0 / 3.0), v));
      } else {
        acc0 = f_add(acc0, f_scale(T(1.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(2.0 / 3.0), v));
        if (k0 >= mz0 && k0 < mz1 && mx < nc && my < nc) {
          const bool cin = k0 >= 1 && k0 <= nc - 2 && mx >= 1 && mx <= nc - 2 && my >= 1 && my <= nc - 2;
          a.rhoc[(long long)k0 * nc2 + my * nc + mx] = cin ? acc0 : f_zero<T>();
        }
        acc0 = acc1;
        acc1 = f_zero<T>();
      }
    }
#pragma unroll
    for (int k = 0; k < IR; ++k) wc[k] = wn[k];
#pragma unroll
    for (int j = 0; j < RPT; ++j) bc[j] = bn[j];
  }
  if (part) block_reduce_store(nsum, sqrt(nmax), part, G::NT);
}

// ----------------------------------------------------------------------------
// 2D: rows as planes, one wavefront per block marching in y.
constexpr int F2_TXC = 20;

constexpr int F2_GX = F2_TXC + 2;   // staged coarse points per row

// One tile (bx, by) of the 2D sweep, executed by one wavefront; Gz and Sz are
// that wave's LDS slices of 2 * F2_GX entries each; `part` receives the tile's
// (sum |r|^2, max |r|) or is null.
template <class T, int ZC, bool BPX>
__device__ inline void fused2_wave_tile(const FusedArgs<T>& a, int bx, int by, cpx<T> (*Gz)[F2_GX],
                                        cpx<T> (*Sz)[F2_GX], double* part) {
  constexpr int TXC = F2_TXC, TX = 3 * TXC, GX = F2_GX;
  const int lane = threadIdx.x & 63;
  const int n = a.n, nc = a.nc;
  const int mx0 = bx * TXC, my0 = by * ZC;
  const int my1 = min(my0 + ZC, nc);
  const int x0 = 3 * mx0;
  const int x = x0 - 3 + lane;
  const bool xin = x >= 1 && x <= n - 2;
  const bool xcomp = lane >= 1 && lane <= 62;
  const bool xown = x >= x0 && x <= min(x0 + TX - 1, n - 1);
  const int yown_lo = 3 * my0, yown_hi = min(3 * my1 - 1, n - 1);
  const bool mask = a.variant != 0;
  const cpx<T> c0 = a.coef[0], c1 = a.coef[1], c2 = a.coef[2];
  const cpx<T> ws = a.ws;
  const int mxl = x >= 0 ? x / 3 : 0, qx = x - 3 * mxl, gxl = mxl - mx0 + 1;
  const T wx0 = w_lo<T>(qx), wx1 = w_hi<T>(qx);
  const int smx = mx0 - 1 + lane;
  const bool sval = lane < GX && smx >= 0 && smx < nc;
  const bool ccol = lane >= 3 && lane <= 60 && lane % 3 == 0;
  const int cmx = mx0 + lane / 3 - 1;

  cpx<T> wc, wn, bc, bn, A = f_zero<T>(), Np = f_zero<T>(), Cp = f_zero<T>();
  cpx<T> gsc0, gsc1, gsi0, gsi1, acc0 = f_zero<T>(), acc1 = f_zero<T>();
  double nsum = 0.0, nmax = 0.0;
  auto row_ok = [&](int p) { return p >= 1 && p <= n - 2; };
  auto load_w = [&](int p) { return (row_ok(p) && xin) ? a.w[(long long)p * n + x] : f_zero<T>(); };
  auto load_b = [&](int q) { return (row_ok(q) && xin && xcomp) ? a.b[(long long)q * n + x] : f_zero<T>(); };
  auto load_g = [&](int p) {
    gsc0 = gsc1 = gsi0 = gsi1 = f_zero<T>();
    if (sval && row_ok(p)) {
      const int ky = p / 3, ty = p - 3 * ky;
      const long long c = (long long)ky * nc + smx;
      gsc0 = a.scc[c];
      if (BPX) gsi0 = a.sic[c];
      if (ty != 0) {
        gsc1 = a.scc[c + nc];
        if (BPX) gsi1 = a.sic[c + nc];
      }
    }
  };
  auto store_g = [&](int p) {
    if (lane < GX) {
      const int ky = floor_div3(p), ty = p - 3 * ky;
      const cpx<T> g0 = BPX ? f_sub(gsc0, gsi0) : gsc0;
      const cpx<T> g1 = BPX ? f_sub(gsc1, gsi1) : gsc1;
      Gz[p & 1][lane] = ty == 0 ? g0 : f_add(f_scale(w_lo<T>(ty), g0), f_scale(w_hi<T>(ty), g1));
      Sz[p & 1][lane] = gsc0;
    }
  };
  const int p0 = 3 * my0 - 3;
  load_g(p0);
  store_g(p0);
  load_g(p0 + 1);
  wc = load_w(p0);
  bc = load_b(p0 - 1);
  wave_sync();
  for (int p = p0; p <= 3 * my1; ++p) {
    const int q = p - 1, pb = p & 1;
    wn = load_w(p + 1);
    bn = load_b(p);
    const int ky = floor_div3(p), ty = p - 3 * ky;
    cpx<T> u = f_zero<T>();
    if (row_ok(p) && xin) {
      if (BPX && qx == 0 && ty == 0) {
        u = f_add(wc, Sz[pb][gxl]);
      } else {
        cpx<T> g = f_scale(wx0, Gz[pb][gxl]);
        if (qx != 0) g = f_add(g, f_scale(wx1, Gz[pb][gxl + 1]));
        u = f_add(wc, g);
      }
    }
    const cpx<T> h = f_add(dpp_c<kDppLeft>(u), dpp_c<kDppRight>(u));
    const cpx<T> M = f_mac(f_mul(c0, u), c1, h);
    const cpx<T> N = f_mac(f_mul(c1, u), c2, h);
    const bool in = row_ok(q) && xin && xcomp;
    const cpx<T> rv = in ? f_sub(bc, f_add(A, N)) : f_zero<T>();
    const cpx<T> s = f_mul(ws, rv);
    const bool cp = q >= 0 && (q % 3) == 0 && qx == 0 && x >= 0;
    const cpx<T> scm = (mask && cp) ? f_zero<T>() : s;
    if (q >= yown_lo && q <= yown_hi && xown) {
      a.wout[(long long)q * n + x] = in ? f_add(Cp, scm) : f_zero<T>();
      if (in) {
        const double r2 = (double)rv.re * rv.re + (double)rv.im * rv.im;
        nsum += r2;
        nmax = fmax(nmax, r2);
      }
      if (cp) {
        const long long ic = (long long)(q / 3) * nc + x / 3;
        if (a.sfc) a.sfc[ic] = scm;
        if (BPX) a.sic_out[ic] = s;
      }
    }
    A = f_add(M, Np);
    Np = N;
    Cp = u;
    // R: x-part by lane shifts, y-part in a two-slot ring held by the coarse-column lanes
    const cpx<T> l1 = dpp_c<kDppLeft>(rv), l2 = dpp_c<kDppLeft>(l1);
    const cpx<T> r1 = dpp_c<kDppRight>(rv), r2 = dpp_c<kDppRight>(r1);
    const cpx<T> v = f_add(rv, f_add(f_scale(T(2.0 / 3.0), f_add(l1, r1)), f_scale(T(1.0 / 3.0), f_add(l2, r2))));
    if (q >= 3 * my0 - 2 && ccol) {
      const int k0 = floor_div3(q), t = q - 3 * k0;
      if (t == 0) {
        acc0 = f_add(acc0, v);
      } else if (t == 1) {
        acc0 = f_add(acc0, f_scale(T(2.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(1.0 / 3.0), v));
      } else {
        acc0 = f_add(acc0, f_scale(T(1.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(2.0 / 3.0), v));
        if (k0 >= my0 && k0 < my1 && cmx < nc) {
          const bool cin = k0 >= 1 && k0 <= nc - 2 && cmx >= 1 && cmx <= nc - 2;
          a.rhoc[(long long)k0 * nc + cmx] = cin ? acc0 : f_zero<T>();
        }
        acc0 = acc1;
        acc1 = f_zero<T>();
      }
    }
    store_g(p + 1);
    load_g(p + 2);
    wave_sync();
    wc = wn;
    bc = bn;
  }
  if (part) {
    double s2 = nsum, m2 = sqrt(nmax);
    for (int off = 32; off > 0; off >>= 1) {
      s2 += __shfl_down(s2, off, 64);
      m2 = fmax(m2, __shfl_down(m2, off, 64));
    }
    if (lane == 0) {
      part[0] = s2;
      part[1] = m2;
    }
  }
}

}  // namespace mg
