// Per-vertex operations of the coarse levels, shared by the level kernels and
// the batched persistent kernel.
#pragma once
#include "mg_common.h"

namespace mg {

// Coarse-level pre-phase (descent of tdAdd / tdBPX) at vertex j:
//   sc += P sc_c ;  BPX: sc -= P si_c off c-points ;  u += sc + sf.
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
  u[i] = u[i] + s + sf[i];
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
template <class T, int D>
__device__ inline void post_galerkin_vertex(const OpData<T>& op, const int m[3], long long ic,
                                            const cpx<T>* __restrict__ rho, cpx<T> omega, int mask_c,
                                            cpx<T>* __restrict__ sc, const cpx<T>* __restrict__ sf,
                                            cpx<T>* __restrict__ rhoc, cpx<T>* __restrict__ sfc,
                                            cpx<T>* __restrict__ sic) {
  const int n = op.n, nc = (n - 1) / 3 + 1;
  const T w[5] = {T(1.0 / 3.0), T(2.0 / 3.0), T(1), T(2.0 / 3.0), T(1.0 / 3.0)};
  const bool cin = is_interior<D>(m, nc);
  cpx<T> acc = czero<T>();
  const int zlo = D == 3 ? -2 : 0, zhi = D == 3 ? 2 : 0;
  for (int oz = zlo; oz <= zhi; ++oz) {
    for (int oy = -2; oy <= 2; ++oy) {
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) {
        int j[3] = {3 * m[0] + ox, 3 * m[1] + oy, 3 * m[2] + oz};
        const bool owned = ox >= 0 && oy >= 0 && oz >= 0;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) inside = inside && j[a] >= 0 && j[a] < n;
        if (!inside || !(cin || owned)) continue;
        const long long i = ravel<D>(j, n);
        const cpx<T> v = rho[i];
        acc = acc + (w[ox + 2] * w[oy + 2] * (D == 3 ? w[oz + 2] : T(1))) * v;
        if (owned) {
          const bool in = is_interior<D>(j, n);
          cpx<T> sv = czero<T>();
          if (in) {
            cpx<T> id = op.invD;
            if (op.invDv) id = op.invDv[i];
            sv = cmul(omega, cmul(id, v));
          }
          const bool cp = ox == 0 && oy == 0 && oz == 0;
          const cpx<T> scm = csel(mask_c && cp, czero<T>(), sv);
          sc[i] = scm;
          if (cp) {
            if (sfc) sfc[ic] = sf[i] + scm;
            if (sic) sic[ic] = sv;
          }
        }
      }
    }
  }
  rhoc[ic] = csel(cin, acc, czero<T>());
}

}  // namespace mg
