// Per-vertex operations of the coarse levels, shared by the level kernels and
// the batched persistent kernel.
#pragma once
#include "mg_common.h"

namespace mg {

// Coarse-level pre-phase (descent of tdAdd / tdBPX) at vertex j:
//   sc += P sc_c ;  BPX: sc -= P si_c off c-points ;  u += sc + sf.
// u == nullptr: the coarse iterate is not formed (the Galerkin form of the
// coarse right-hand side never reads it), and sf is not read either.
template <class T, int D>
__device__ inline void pre_vertex(int n, const int j[3], long long i, cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc,
                                  const cpx<T>* __restrict__ sf, const cpx<T>* __restrict__ scc,
                                  const cpx<T>* __restrict__ sic, int has_coarse, int bpx) {
  if (!is_interior<D>(j, n)) return;
  const int nc = (n - 1) / 3 + 1;
  cpx<T> s = sc[i];
  if (has_coarse) {
    s = s + prolong_at<T, D>(scc, nc, j);
    if (bpx && !is_cpoint<D>(j)) s = s - prolong_at<T, D>(sic, nc, j);
    sc[i] = s;
  }
  if (u) u[i] = u[i] + s + sf[i];
}

// Post-phase pointwise part at vertex j: s = omega r / D, sc = s (0 at c-points
// if mask_c); finest: u += sc in place; coarse: sc_out = sc.  Injection to the
// coarser level at c-points: sf_c = sf + sc, si_c = s.
template <class T, int D>
__device__ inline void update_vertex(const OpData<T>& op, const int j[3], long long i, const cpx<T>* __restrict__ r,
                                     cpx<T> omega, int mask_c, cpx<T>* __restrict__ u, cpx<T>* __restrict__ sc_out,
                                     const cpx<T>* __restrict__ sf, cpx<T>* __restrict__ sfc,
                                     cpx<T>* __restrict__ sic) {
  const int n = op.n;
  const int nc = (n - 1) / 3 + 1;
  const bool in = is_interior<D>(j, n);
  cpx<T> s = czero<T>();
  if (in) {
    cpx<T> id = op.invD;
    if (op.invDv) id = op.invDv[i];
    s = cmul(omega, cmul(id, r[i]));
  }
  const bool cp = is_cpoint<D>(j);
  const cpx<T> scv = csel(mask_c && cp, czero<T>(), s);
  if (u) {
    if (in) u[i] = u[i] + scv;
  }
  if (sc_out) sc_out[i] = scv;
  if (cp && (sfc || sic)) {
    int m[3] = {j[0] / 3, j[1] / 3, j[2] / 3};
    const long long ic = ravel<D>(m, nc);
    if (sfc) {
      cpx<T> f = czero<T>();
      if (sf) f = sf[i];
      sfc[ic] = f + scv;
    }
    if (sic) sic[ic] = s;
  }
}

// Coarse post-phase with the Galerkin form at coarse vertex m of level l-1
// (op: level l).  The vertex owns the fine vertices 3m + q, q in {0,1,2}^d, of
// level l and walks the restriction support 3m + o, o in [-2, 2]^d, once:
// every value enters rho_c(m) = (R rho)(m), and on its owned vertices it also
// forms s = omega rho / D, sc = s (0 on c-points when masked) and the
// injections sf_c = sf + sc (add), si_c = s (BPX) at 3m.
//
// post_galerkin_part does this for the offsets whose outermost component (z in
// 3D, y in 2D) equals `oo` and returns their part of rho_c(m); all its loads
// are independent (indices clamped into the grid, values masked by weight).
template <class T, int D>
__device__ inline cpx<T> post_galerkin_part(const OpData<T>& op, const int m[3], long long ic, int oo,
                                            const cpx<T>* __restrict__ rho, cpx<T> omega, int mask_c,
                                            cpx<T>* __restrict__ sc, const cpx<T>* __restrict__ sf,
                                            cpx<T>* __restrict__ sfc, cpx<T>* __restrict__ sic) {
  const int n = op.n, nc = (n - 1) / 3 + 1;
  constexpr T w[5] = {T(1.0 / 3.0), T(2.0 / 3.0), T(1), T(2.0 / 3.0), T(1.0 / 3.0)};
  const bool cin = is_interior<D>(m, nc);
  constexpr int IL = D == 3 ? -2 : 0, IH = D == 3 ? 2 : 0;   // the inner y range in 3D
  cpx<T> acc = czero<T>();
#pragma unroll
  for (int oi = IL; oi <= IH; ++oi) {
#pragma unroll
    for (int ox = -2; ox <= 2; ++ox) {
      const int o[3] = {ox, D == 3 ? oi : oo, oo};
      int j[3] = {0, 0, 0};
      bool inside = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int t = 3 * m[a] + o[a];
        inside = inside && t >= 0 && t < n;
        j[a] = min(max(t, 0), n - 1);
      }
      const unsigned i = (unsigned)ravel<D>(j, n);   // a level below the finest has < 2^31 vertices
      const cpx<T> v = rho[i];
      T wt = w[o[0] + 2] * w[o[1] + 2];
      if (D == 3) wt *= w[o[2] + 2];
      acc = acc + ((cin && inside) ? wt : T(0)) * v;
      bool owned = inside;
#pragma unroll
      for (int a = 0; a < D; ++a) owned = owned && o[a] >= 0;
      if (owned) {
        const bool in = is_interior<D>(j, n);
        cpx<T> sv = czero<T>();
        if (in) {
          cpx<T> id = op.invD;
          if (op.invDv) id = op.invDv[i];
          sv = cmul(omega, cmul(id, v));
        }
        bool cp = true;
#pragma unroll
        for (int a = 0; a < D; ++a) cp = cp && o[a] == 0;
        const cpx<T> scm = csel(mask_c && cp, czero<T>(), sv);
        sc[i] = scm;
        if (cp) {
          if (sfc) sfc[ic] = sf[i] + scm;
          if (sic) sic[ic] = sv;
        }
      }
    }
  }
  return acc;
}

// The five parts combined in a fixed order (the order of a xor-shuffle
// reduction over eight lanes holding parts oo = -2..2 in lanes 0..4), so the
// per-vertex form and the lane-split kernel give identical sums.
template <class T>
__device__ inline cpx<T> post_galerkin_combine(const cpx<T> p[5]) {
  return (((p[0] + p[4]) + p[2]) + (p[1] + p[3]));
}

template <class T, int D>
__device__ inline void post_galerkin_vertex(const OpData<T>& op, const int m[3], long long ic,
                                            const cpx<T>* __restrict__ rho, cpx<T> omega, int mask_c,
                                            cpx<T>* __restrict__ sc, const cpx<T>* __restrict__ sf,
                                            cpx<T>* __restrict__ rhoc, cpx<T>* __restrict__ sfc,
                                            cpx<T>* __restrict__ sic) {
  const int nc = (op.n - 1) / 3 + 1;
  cpx<T> p[5];
#pragma unroll 1
  for (int k = 0; k < 5; ++k) p[k] = post_galerkin_part<T, D>(op, m, ic, k - 2, rho, omega, mask_c, sc, sf, sfc, sic);
  rhoc[ic] = csel(is_interior<D>(m, nc), post_galerkin_combine(p), czero<T>());
}

// R v = P^T v: per axis weights 1 - |o|/3 for fine offsets o in [-2, 2] around 3m;
// zero on the coarse boundary.
// Part of (R v)(m) over the offsets whose outermost component (z in 3D, y in
// 2D) is oo; all loads independent (indices clamped, boundary m gives 0 later).
template <class T, int D>
__device__ inline cpx<T> restrict_part(const cpx<T>* __restrict__ vf, int nf, const int m[3], int oo) {
  constexpr T w[5] = {T(1.0 / 3.0), T(2.0 / 3.0), T(1), T(2.0 / 3.0), T(1.0 / 3.0)};
  constexpr int IL = D == 3 ? -2 : 0, IH = D == 3 ? 2 : 0;
  cpx<T> acc = czero<T>();
#pragma unroll
  for (int oi = IL; oi <= IH; ++oi) {
    cpx<T> accx = czero<T>();
#pragma unroll
    for (int ox = -2; ox <= 2; ++ox) {
      const int o[3] = {ox, D == 3 ? oi : oo, oo};
      int j[3] = {0, 0, 0};
#pragma unroll
      for (int q = 0; q < D; ++q) j[q] = min(max(3 * m[q] + o[q], 0), nf - 1);
      accx = accx + w[ox + 2] * vf[(unsigned)ravel<D>(j, nf)];
    }
    acc = acc + (D == 3 ? w[oi + 2] * w[oo + 2] : w[oo + 2]) * accx;
  }
  return acc;
}

// Zero-start cycle (the preconditioner B v), one level going up, at vertex j
// of level l (op): z = Lop(omega D^-1 rho) + P g with g the coarse correction
// (BPX: already minus I s, see prec_g_vertex); hb masks s on c-points
// (mask_c); the coarsest level has no g.
template <class T, int D>
__device__ inline void prec_up_vertex(const OpData<T>& op, const int j[3], long long i,
                                      const cpx<T>* __restrict__ rho, cpx<T> omega, int mask_c, int is_lmin,
                                      const cpx<T>* __restrict__ gc, cpx<T>* __restrict__ z) {
  const int n = op.n;
  const int nc = (n - 1) / 3 + 1;
  cpx<T> out = czero<T>();
  if (is_interior<D>(j, n)) {
    cpx<T> id = op.invD;
    if (op.invDv) id = op.invDv[i];
    cpx<T> s = cmul(omega, cmul(id, rho[i]));
    if (!is_lmin) {
      s = csel(mask_c && is_cpoint<D>(j), czero<T>(), s);
      s = s + prolong_at<T, D>(gc, nc, j);
    }
    out = s;
  }
  z[i] = out;
}

// BPX coarse correction of the zero-start cycle at level l (op), coarse vertex
// m: g = z_c(m) - (I s)(m) with s = omega D^-1 rho at 3m, so that
// z = s + P g = s - P I s + P z_c.
template <class T, int D>
__device__ inline void prec_g_vertex(const OpData<T>& op, const int m[3], long long ic,
                                     const cpx<T>* __restrict__ rho, cpx<T> omega, const cpx<T>* __restrict__ zc,
                                     cpx<T>* __restrict__ g) {
  const int n = op.n;
  const int j[3] = {3 * m[0], 3 * m[1], D == 3 ? 3 * m[2] : 0};
  cpx<T> q = czero<T>();
  if (is_interior<D>(j, n)) {
    const long long i = ravel<D>(j, n);
    cpx<T> id = op.invD;
    if (op.invDv) id = op.invDv[i];
    q = cmul(omega, cmul(id, rho[i]));
  }
  g[ic] = zc[ic] - q;
}

}  // namespace mg
