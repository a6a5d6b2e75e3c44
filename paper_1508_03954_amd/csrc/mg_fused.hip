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
// needs one operator application and the coarse level adds H_(l-1) u_(l-1)
// implicitly by reading its residual from the restricted one.
//
// Work decomposition.  A block owns a box of coarse vertices: TXC x TYC in the
// plane and ZC coarse planes in z.  Its fine vertices (3m .. 3m+2 per axis)
// are written by it alone.  R at a coarse vertex m needs r on fine offsets
// -2..2 around 3m, so r is computed on the owned fine box extended by two
// vertices towards lower indices, and u on that box extended by one more
// vertex on each side.  The block marches through z one fine plane at a time:
// plane p of u is staged in LDS, the in-plane 3x3 neighbour sums of the
// 27-point stencil are formed there, and the out-of-plane part is carried in
// registers (the stencil row of plane p splits into a centre-plane part M_p and
// a neighbour-plane part N_p, H u at plane p-1 = M_(p-1) + N_(p-2) + N_p).
// r of plane p-1 is restricted in the plane from LDS and accumulated over z in
// a two-slot ring of coarse planes.
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
// acc + c * x
template <class T>
__device__ inline cpx<T> f_mac(cpx<T> acc, cpx<T> c, cpx<T> x) {
  return mk(acc.re + c.re * x.re - c.im * x.im, acc.im + c.re * x.im + c.im * x.re);
}
template <class T>
__device__ inline cpx<T> f_zero() { return mk(T(0), T(0)); }

__device__ inline int floor_div3(int p) { return p >= 0 ? p / 3 : -((-p + 2) / 3); }

// Linear interpolation weights of a fine offset q in {0,1,2} inside a coarse cell.
template <class T>
__device__ inline T w_lo(int q) { return q == 0 ? T(1) : (q == 1 ? T(2.0 / 3.0) : T(1.0 / 3.0)); }
template <class T>
__device__ inline T w_hi(int q) { return q == 0 ? T(0) : (q == 1 ? T(1.0 / 3.0) : T(2.0 / 3.0)); }
template <class T>
__device__ inline T w_r(int o) { return o == 0 ? T(1) : ((o == 1 || o == -1) ? T(2.0 / 3.0) : T(1.0 / 3.0)); }

template <class T>
__device__ inline void fused_reduce(double s, double m, double* partials, int bid, int nt) {
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
    partials[2 * bid] = a;
    partials[2 * bid + 1] = b;
  }
}

// ----------------------------------------------------------------------------
// 3D
constexpr int F3_TXC = 10, F3_TYC = 6, F3_ZC = 9, F3_NT = 256;

template <class T, int TXC, int TYC, int ZC, int NT>
__global__ __launch_bounds__(NT) void k_fused3(FusedArgs<T> a) {
  constexpr int TX = 3 * TXC, TY = 3 * TYC;
  constexpr int IX = TX + 4, IY = TY + 4;   // u staged on [x0-3, x0+TX] x [y0-3, y0+TY]
  constexpr int CX = TX + 2, CY = TY + 2;   // r computed on [x0-2, x0+TX-1] x [y0-2, y0+TY-1]
  constexpr int GX = TXC + 2, GY = TYC + 2; // coarse g on [mx0-1, mx0+TXC] x [my0-1, my0+TYC]
  constexpr int NCP = CX * CY;
  constexpr int K = (NCP + NT - 1) / NT;
  __shared__ cpx<T> Ub[IY][IX];
  __shared__ cpx<T> Rb[CY][CX];
  __shared__ cpx<T> Gz[GY][GX];

  const int tid = threadIdx.x;
  const int n = a.n, nc = a.nc;
  const long long n2 = (long long)n * n, nc2 = (long long)nc * nc;
  const int mx0 = blockIdx.x * TXC, my0 = blockIdx.y * TYC, mz0 = blockIdx.z * ZC;
  const int mz1 = min(mz0 + ZC, nc);
  const int x0 = 3 * mx0, y0 = 3 * my0;
  const int zown_lo = 3 * mz0, zown_hi = min(3 * mz1 - 1, n - 1);
  const int xown_hi = min(x0 + TX - 1, n - 1), yown_hi = min(y0 + TY - 1, n - 1);
  const bool bpx = a.variant == 2, mask = a.variant != 0;
  const cpx<T> c0 = a.coef[0], c1 = a.coef[1], c2 = a.coef[2], c3 = a.coef[3];

  cpx<T> A[K], Np[K], Cp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) { A[k] = f_zero<T>(); Np[k] = f_zero<T>(); Cp[k] = f_zero<T>(); }
  cpx<T> acc0 = f_zero<T>(), acc1 = f_zero<T>();
  double nsum = 0.0, nmax = 0.0;

  for (int p = 3 * mz0 - 3; p <= 3 * mz1; ++p) {
    const int q = p - 1;
    const int kz = floor_div3(p), tz = p - 3 * kz;
    const bool plane_in = p >= 1 && p <= n - 2;
    // (1) coarse correction interpolated to fine plane p (coarse in-plane points)
    for (int i = tid; i < GX * GY; i += NT) {
      const int gx = i % GX, gy = i / GX;
      const int mx = mx0 - 1 + gx, my = my0 - 1 + gy;
      cpx<T> v = f_zero<T>();
      if (plane_in && mx >= 0 && mx < nc && my >= 0 && my < nc) {
        const long long c = (long long)kz * nc2 + (long long)my * nc + mx;
        v = a.scc[c];
        if (bpx) v = f_sub(v, a.sic[c]);
        if (tz != 0) {
          cpx<T> v1 = a.scc[c + nc2];
          if (bpx) v1 = f_sub(v1, a.sic[c + nc2]);
          v = f_add(f_scale(w_lo<T>(tz), v), f_scale(w_hi<T>(tz), v1));
        }
      }
      Gz[gy][gx] = v;
    }
    __syncthreads();
    // (2) u on plane p: folded iterate plus the prolongated coarse correction
    for (int i = tid; i < IX * IY; i += NT) {
      const int ix = i % IX, iy = i / IX;
      const int x = x0 - 3 + ix, y = y0 - 3 + iy;
      cpx<T> u = f_zero<T>();
      if (plane_in && x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2) {
        u = a.w[(long long)p * n2 + (long long)y * n + x];
        const int mx = x / 3, qx = x - 3 * mx, my = y / 3, qy = y - 3 * my;
        const int gx = mx - mx0 + 1, gy = my - my0 + 1;
        const T wx0 = w_lo<T>(qx), wx1 = w_hi<T>(qx), wy0 = w_lo<T>(qy), wy1 = w_hi<T>(qy);
        cpx<T> row0 = f_scale(wx0, Gz[gy][gx]);
        if (qx != 0) row0 = f_add(row0, f_scale(wx1, Gz[gy][gx + 1]));
        cpx<T> g = f_scale(wy0, row0);
        if (qy != 0) {
          cpx<T> row1 = f_scale(wx0, Gz[gy + 1][gx]);
          if (qx != 0) row1 = f_add(row1, f_scale(wx1, Gz[gy + 1][gx + 1]));
          g = f_add(g, f_scale(wy1, row1));
        }
        u = f_add(u, g);
        // BPX keeps the coarse si on c-points (the P si term applies off c-points only)
        if (bpx && qx == 0 && qy == 0 && tz == 0) u = f_add(u, a.sic[(long long)kz * nc2 + (long long)my * nc + mx]);
      }
      Ub[iy][ix] = u;
    }
    __syncthreads();
    // (3) stencil, residual, smoothing update, folded iterate, injections
    const bool q_in = q >= 1 && q <= n - 2;
    const bool q_own = q >= zown_lo && q <= zown_hi;
    const bool q_c = (q % 3) == 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ci = tid + k * NT;
      if (ci < NCP) {
        const int cx = ci % CX, cy = ci / CX;
        const int ix = cx + 1, iy = cy + 1;
        const int x = x0 - 2 + cx, y = y0 - 2 + cy;
        const cpx<T> C = Ub[iy][ix];
        const cpx<T> F2 = f_add(f_add(Ub[iy][ix - 1], Ub[iy][ix + 1]), f_add(Ub[iy - 1][ix], Ub[iy + 1][ix]));
        const cpx<T> E2 = f_add(f_add(Ub[iy - 1][ix - 1], Ub[iy - 1][ix + 1]), f_add(Ub[iy + 1][ix - 1], Ub[iy + 1][ix + 1]));
        const cpx<T> M = f_mac(f_mac(f_mul(c0, C), c1, F2), c2, E2);
        const cpx<T> N = f_mac(f_mac(f_mul(c1, C), c2, F2), c3, E2);
        const cpx<T> Hu = f_add(A[k], N);
        cpx<T> r = f_zero<T>();
        const bool in = q_in && x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
        if (in) r = f_sub(a.b[(long long)q * n2 + (long long)y * n + x], Hu);
        const cpx<T> s = f_mul(a.ws, r);
        const bool cp = q_c && (x % 3) == 0 && (y % 3) == 0;
        const cpx<T> scm = (mask && cp) ? f_zero<T>() : s;
        if (q_own && x >= x0 && x <= xown_hi && y >= y0 && y <= yown_hi) {
          a.wout[(long long)q * n2 + (long long)y * n + x] = in ? f_add(Cp[k], scm) : f_zero<T>();
          if (in) {
            const double r2 = (double)r.re * r.re + (double)r.im * r.im;
            nsum += r2;
            nmax = fmax(nmax, r2);
          }
          if (cp) {
            const long long ic = (long long)(q / 3) * nc2 + (long long)(y / 3) * nc + x / 3;
            if (a.sfc) a.sfc[ic] = scm;
            if (a.sic_out) a.sic_out[ic] = s;
          }
        }
        Rb[cy][cx] = r;
        A[k] = f_add(M, Np[k]);
        Np[k] = N;
        Cp[k] = C;
      }
    }
    __syncthreads();
    // (4) in-plane restriction at the owned coarse vertices, ring over coarse planes
    if (q >= 3 * mz0 - 2 && tid < TXC * TYC) {
      const int lx = tid % TXC, ly = tid / TXC;
      const int mx = mx0 + lx, my = my0 + ly;
      cpx<T> v = f_zero<T>();
#pragma unroll
      for (int oy = -2; oy <= 2; ++oy) {
        cpx<T> rowv = f_zero<T>();
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) rowv = f_add(rowv, f_scale(w_r<T>(ox), Rb[3 * ly + 2 + oy][3 * lx + 2 + ox]));
        v = f_add(v, f_scale(w_r<T>(oy), rowv));
      }
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
          a.rhoc[(long long)k0 * nc2 + (long long)my * nc + mx] = cin ? acc0 : f_zero<T>();
        }
        acc0 = acc1;
        acc1 = f_zero<T>();
      }
    }
  }
  if (a.partials) {
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    fused_reduce<T>(nsum, sqrt(nmax), a.partials, bid, NT);
  }
}

// ----------------------------------------------------------------------------
// 2D: the same sweep with rows as planes (march in y, tiles along x).
constexpr int F2_TXC = 20, F2_ZC = 3, F2_NT = 64;

template <class T, int TXC, int ZC, int NT>
__global__ __launch_bounds__(NT) void k_fused2(FusedArgs<T> a) {
  constexpr int TX = 3 * TXC;
  constexpr int IX = TX + 4, CX = TX + 2, GX = TXC + 2;
  constexpr int K = (CX + NT - 1) / NT;
  __shared__ cpx<T> Ub[IX];
  __shared__ cpx<T> Rb[CX];
  __shared__ cpx<T> Gz[GX];

  const int tid = threadIdx.x;
  const int n = a.n, nc = a.nc;
  const int mx0 = blockIdx.x * TXC, my0 = blockIdx.y * ZC;
  const int my1 = min(my0 + ZC, nc);
  const int x0 = 3 * mx0;
  const int yown_lo = 3 * my0, yown_hi = min(3 * my1 - 1, n - 1);
  const int xown_hi = min(x0 + TX - 1, n - 1);
  const bool bpx = a.variant == 2, mask = a.variant != 0;
  const cpx<T> c0 = a.coef[0], c1 = a.coef[1], c2 = a.coef[2];

  cpx<T> A[K], Np[K], Cp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) { A[k] = f_zero<T>(); Np[k] = f_zero<T>(); Cp[k] = f_zero<T>(); }
  cpx<T> acc0 = f_zero<T>(), acc1 = f_zero<T>();
  double nsum = 0.0, nmax = 0.0;

  for (int p = 3 * my0 - 3; p <= 3 * my1; ++p) {
    const int q = p - 1;
    const int ky = floor_div3(p), ty = p - 3 * ky;
    const bool row_in = p >= 1 && p <= n - 2;
    for (int i = tid; i < GX; i += NT) {
      const int mx = mx0 - 1 + i;
      cpx<T> v = f_zero<T>();
      if (row_in && mx >= 0 && mx < nc) {
        const long long c = (long long)ky * nc + mx;
        v = a.scc[c];
        if (bpx) v = f_sub(v, a.sic[c]);
        if (ty != 0) {
          cpx<T> v1 = a.scc[c + nc];
          if (bpx) v1 = f_sub(v1, a.sic[c + nc]);
          v = f_add(f_scale(w_lo<T>(ty), v), f_scale(w_hi<T>(ty), v1));
        }
      }
      Gz[i] = v;
    }
    __syncthreads();
    for (int ix = tid; ix < IX; ix += NT) {
      const int x = x0 - 3 + ix;
      cpx<T> u = f_zero<T>();
      if (row_in && x >= 1 && x <= n - 2) {
        u = a.w[(long long)p * n + x];
        const int mx = x / 3, qx = x - 3 * mx, gx = mx - mx0 + 1;
        cpx<T> g = f_scale(w_lo<T>(qx), Gz[gx]);
        if (qx != 0) g = f_add(g, f_scale(w_hi<T>(qx), Gz[gx + 1]));
        u = f_add(u, g);
        if (bpx && qx == 0 && ty == 0) u = f_add(u, a.sic[(long long)ky * nc + mx]);
      }
      Ub[ix] = u;
    }
    __syncthreads();
    const bool q_in = q >= 1 && q <= n - 2;
    const bool q_own = q >= yown_lo && q <= yown_hi;
    const bool q_c = (q % 3) == 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int cx = tid + k * NT;
      if (cx < CX) {
        const int ix = cx + 1, x = x0 - 2 + cx;
        const cpx<T> C = Ub[ix];
        const cpx<T> F1 = f_add(Ub[ix - 1], Ub[ix + 1]);
        const cpx<T> M = f_mac(f_mul(c0, C), c1, F1);
        const cpx<T> N = f_mac(f_mul(c1, C), c2, F1);
        const cpx<T> Hu = f_add(A[k], N);
        cpx<T> r = f_zero<T>();
        const bool in = q_in && x >= 1 && x <= n - 2;
        if (in) r = f_sub(a.b[(long long)q * n + x], Hu);
        const cpx<T> s = f_mul(a.ws, r);
        const bool cp = q_c && (x % 3) == 0;
        const cpx<T> scm = (mask && cp) ? f_zero<T>() : s;
        if (q_own && x >= x0 && x <= xown_hi) {
          a.wout[(long long)q * n + x] = in ? f_add(Cp[k], scm) : f_zero<T>();
          if (in) {
            const double r2 = (double)r.re * r.re + (double)r.im * r.im;
            nsum += r2;
            nmax = fmax(nmax, r2);
          }
          if (cp) {
            const long long ic = (long long)(q / 3) * nc + x / 3;
            if (a.sfc) a.sfc[ic] = scm;
            if (a.sic_out) a.sic_out[ic] = s;
          }
        }
        Rb[cx] = r;
        A[k] = f_add(M, Np[k]);
        Np[k] = N;
        Cp[k] = C;
      }
    }
    __syncthreads();
    if (q >= 3 * my0 - 2 && tid < TXC) {
      const int mx = mx0 + tid;
      cpx<T> v = f_zero<T>();
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) v = f_add(v, f_scale(w_r<T>(ox), Rb[3 * tid + 2 + ox]));
      const int k0 = floor_div3(q), t = q - 3 * k0;
      if (t == 0) {
        acc0 = f_add(acc0, v);
      } else if (t == 1) {
        acc0 = f_add(acc0, f_scale(T(2.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(1.0 / 3.0), v));
      } else {
        acc0 = f_add(acc0, f_scale(T(1.0 / 3.0), v));
        acc1 = f_add(acc1, f_scale(T(2.0 / 3.0), v));
        if (k0 >= my0 && k0 < my1 && mx < nc) {
          const bool cin = k0 >= 1 && k0 <= nc - 2 && mx >= 1 && mx <= nc - 2;
          a.rhoc[(long long)k0 * nc + mx] = cin ? acc0 : f_zero<T>();
        }
        acc0 = acc1;
        acc1 = f_zero<T>();
      }
    }
  }
  if (a.partials) {
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    fused_reduce<T>(nsum, sqrt(nmax), a.partials, bid, NT);
  }
}

static dim3 fused_grid(int dim, int n) {
  const int nc = (n - 1) / 3 + 1;
  if (dim == 3)
    return dim3((nc + F3_TXC - 1) / F3_TXC, (nc + F3_TYC - 1) / F3_TYC, (nc + F3_ZC - 1) / F3_ZC);
  return dim3((nc + F2_TXC - 1) / F2_TXC, (nc + F2_ZC - 1) / F2_ZC, 1);
}

int fused_partials_blocks(int dim, int n) {
  if (n < 4) return -1;
  const dim3 g = fused_grid(dim, n);
  return (int)(g.x * g.y * g.z);
}

template <class T>
hipError_t launch_fused(int dim, const FusedArgs<T>& a, hipStream_t s) {
  if (a.nc != (a.n - 1) / 3 + 1 || a.n < 4) return hipErrorInvalidValue;
  const dim3 g = fused_grid(dim, a.n);
  if (dim == 3) hipLaunchKernelGGL((k_fused3<T, F3_TXC, F3_TYC, F3_ZC, F3_NT>), g, F3_NT, 0, s, a);
  else hipLaunchKernelGGL((k_fused2<T, F2_TXC, F2_ZC, F2_NT>), g, F2_NT, 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_fused<double>(int, const FusedArgs<double>&, hipStream_t);
template hipError_t launch_fused<float>(int, const FusedArgs<float>&, hipStream_t);

}  // namespace mg
