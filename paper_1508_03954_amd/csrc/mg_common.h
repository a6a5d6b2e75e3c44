// Device helpers shared by the level kernels and the batched persistent
// kernel: complex arithmetic, level indexing, prolongation and the operator row.
// Level l: n = 3^l + 1 vertices per axis, C order with x fastest.
#pragma once
#include "mg_internal.h"

namespace mg {

template <class T>
__device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <class T>
__device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <class T>
__device__ inline cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.re, s * a.im); }
template <class T>
__device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__device__ inline cpx<T> cconjmul(cpx<T> a, cpx<T> b) {  // conj(a) * b
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class T>
__device__ inline cpx<T> czero() { return mk(T(0), T(0)); }
// Component-wise select.  (A conditional expression on the struct itself may
// be lowered through private memory, whose accesses share the vector-memory
// counter with global loads and so force waits on every load in flight.)
template <class T>
__device__ inline cpx<T> csel(bool c, cpx<T> a, cpx<T> b) { return mk(c ? a.re : b.re, c ? a.im : b.im); }

// Level sizes are capped so that every vertex index fits 32 bits (the host
// checks level_max), which keeps the index arithmetic in 32-bit integers.
template <int D>
__device__ inline void unravel(long long ii, int n, int j[3]) {
  unsigned i = (unsigned)ii;
  const unsigned un = (unsigned)n;
  const unsigned t = i / un;
  j[0] = (int)(i - t * un);
  if (D == 3) {
    const unsigned z = t / un;
    j[1] = (int)(t - z * un);
    j[2] = (int)z;
  } else {
    j[1] = (int)t;
    j[2] = 0;
  }
}

// Division by a level's vertex count per axis n through a multiply-high:
// floor(i / n) = umulhi(i, m) with m = ceil(2^32 / n) is exact for
// i < 2^32 / n, so unravel_fast (two such divisions) covers levels with
// n^4 < 2^32, i.e. n <= 255.
__host__ __device__ inline unsigned fastdiv_magic(int n) { return 0xFFFFFFFFu / (unsigned)n + 1u; }
template <int D>
__device__ inline void unravel_fast(unsigned i, int n, unsigned magic, int j[3]) {
  const unsigned t = __umulhi(i, magic);
  j[0] = (int)(i - t * (unsigned)n);
  if (D == 3) {
    const unsigned z = __umulhi(t, magic);
    j[1] = (int)(t - z * (unsigned)n);
    j[2] = (int)z;
  } else {
    j[1] = (int)t;
    j[2] = 0;
  }
}
constexpr int kFastDivMaxN = 255;

template <int D>
__device__ inline long long ravel(const int j[3], int n) {
  return D == 3 ? ((long long)j[2] * n + j[1]) * n + j[0] : (long long)j[1] * n + j[0];
}

template <int D>
__device__ inline bool is_interior(const int j[3], int n) {
  for (int a = 0; a < D; ++a)
    if (j[a] <= 0 || j[a] >= n - 1) return false;
  return true;
}

template <int D>
__device__ inline bool is_cpoint(const int j[3]) {
  for (int a = 0; a < D; ++a)
    if (j[a] % 3 != 0) return false;
  return true;
}

template <int D>
__device__ inline long long total(int n) {
  return D == 3 ? (long long)n * n * n : (long long)n * n;
}

// Row-based traversal of a level: a wavefront covers 64 consecutive x of one
// row (y, z); the row index is uniform across the wave, blocks of 4 waves walk
// the rows grid-stride.  No per-vertex integer division.
#define MG_ROWS(D, n)                                                                       \
  const int lane_ = threadIdx.x & 63;                                                        \
  const int x_ = blockIdx.x * 64 + lane_;                                                    \
  const int nrows_ = (D == 3) ? (n) * (n) : (n);                                             \
  for (int row_ = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + (threadIdx.x >> 6))); \
       row_ < nrows_; row_ += gridDim.y * 4)

// Inside MG_ROWS: vertex multi-index j and linear index i; false when x is past the row.
template <int D>
__device__ inline bool row_vertex(int row, int x, int n, int j[3], long long& i) {
  if (x >= n) return false;
  j[0] = x;
  if (D == 3) {
    j[2] = row / n;
    j[1] = row - j[2] * n;
  } else {
    j[1] = row;
    j[2] = 0;
  }
  i = (long long)row * n + x;
  return true;
}

// (P v)_j: d-linear interpolation from the coarse level (nc per axis).  Per axis
// a fine index j = 3m + q takes m with weight 1 (q = 0), or m and m+1 with
// weights (2/3, 1/3) (q = 1) and (1/3, 2/3) (q = 2).
template <class T, int D>
__device__ cpx<T> prolong_at(const cpx<T>* __restrict__ vc, int nc, const int j[3]) {
  const T third = T(1.0 / 3.0), two3 = T(2.0 / 3.0);
  int m[3] = {0, 0, 0};
  T w0[3] = {1, 1, 1}, w1[3] = {0, 0, 0};
  bool two[3] = {false, false, false};
  for (int a = 0; a < D; ++a) {
    const int q = j[a] % 3;
    m[a] = j[a] / 3;
    if (q == 1) {
      w0[a] = two3; w1[a] = third; two[a] = true;
    } else if (q == 2) {
      w0[a] = third; w1[a] = two3; two[a] = true;
    }
  }
  // all 2^d corners are read (a corner past a coarse vertex repeats it with
  // weight 0), so the loads are independent and issue together
  cpx<T> acc = czero<T>();
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    T w = T(1);
    int k[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int bit = (c >> a) & 1;
      w *= bit ? w1[a] : w0[a];
      k[a] = m[a] + (two[a] ? bit : 0);
    }
    acc = acc + w * vc[ravel<D>(k, nc)];
  }
  return acc;
}

// Constant-phi operator row at an interior vertex: the assembled 3^d stencil of
// the d-linear element matrices has one weight per number of nonzero offsets
// (centre, face, edge, corner).  Boundary neighbours count as zero.
template <class T, int D>
__device__ cpx<T> stencil_const(const cpx<T>* __restrict__ x, int n, const int j[3], const OpData<T>& op) {
  cpx<T> s[4] = {czero<T>(), czero<T>(), czero<T>(), czero<T>()};
  const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
  for (int oz = zlo; oz <= zhi; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        int k[3] = {j[0] + ox, j[1] + oy, j[2] + oz};
        if (!is_interior<D>(k, n)) continue;
        const int cls = (ox != 0) + (oy != 0) + (oz != 0);
        s[cls] = s[cls] + x[ravel<D>(k, n)];
      }
  cpx<T> r = czero<T>();
  for (int c = 0; c <= D; ++c) r = r + cmul(op.coef[c], s[c]);
  return r;
}

// Stiffness-only stencil weights S_K by class (real), used with per-cell
// mass coefficients and a uniform stiffness.
template <class T, int D>
__device__ inline T stiff_weight(int cls) {
  if (D == 3) {
    const T w[4] = {T(8.0 / 3.0), T(0), T(-1.0 / 6.0), T(-1.0 / 12.0)};
    return w[cls];
  } else {
    const T w[3] = {T(8.0 / 3.0), T(-1.0 / 3.0), T(-1.0 / 3.0)};
    return w[cls];
  }
}

// Entries of the reference-cell element matrices between local vertices a
// and b (bit k of a local index: offset along axis k):
//   mass      M_ab = prod_k (1/3 if a_k == b_k else 1/6),
//   stiffness K_ab = sum_k (+-1 along k) prod_(k' != k) (1/3 or 1/6),
// the tensor products of the 1D hat-function matrices [[1,-1],[-1,1]] and
// [[1/3,1/6],[1/6,1/3]].
template <class T, int D>
__device__ inline T elem_mass(int a, int b) {
  const int diff = __builtin_popcount((unsigned)(a ^ b));
  return T(1.0 / (D == 3 ? 27.0 : 9.0)) * T(1.0 / (1 << diff));
}
template <class T, int D>
__device__ inline T elem_stiff(int a, int b) {
  T acc = T(0);
  for (int k = 0; k < D; ++k) {
    T t = ((a ^ b) >> k) & 1 ? T(-1) : T(1);
    for (int q = 0; q < D; ++q)
      if (q != k) t *= ((a ^ b) >> q) & 1 ? T(1.0 / 6.0) : T(1.0 / 3.0);
    acc += t;
  }
  return acc;
}

// Operator row with per-cell coefficients:
//   (H x)_j = sum_{cells c containing j} (kappa_c (K x_c)_loc(j) - mu_c (M x_c)_loc(j)),
// with kappa_c = alpha for every cell unless op.cstiff is given (then the
// assembled S_K stencil is replaced by the cell loop).
template <class T, int D>
__device__ cpx<T> stencil_var(const cpx<T>* __restrict__ x, int n, const int j[3], const OpData<T>& op) {
  // the 3^d neighbourhood of j, loaded once (zero outside the interior);
  // neighbour (ox, oy, oz) at index (ox + 1) + 3 (oy + 1) + 9 (oz + 1)
  constexpr int NB = D == 3 ? 27 : 9;
  cpx<T> xv[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int k[3] = {j[0] + q % 3 - 1, j[1] + (q / 3) % 3 - 1, D == 3 ? j[2] + q / 9 - 1 : 0};
    xv[q] = czero<T>();
    if (is_interior<D>(k, n)) xv[q] = x[ravel<D>(k, n)];
  }
  cpx<T> st = czero<T>();
  if (!op.cstiff) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int cls = (q % 3 != 1) + ((q / 3) % 3 != 1) + (D == 3 ? (q / 9 != 1) : 0);
      st = st + stiff_weight<T, D>(cls) * xv[q];
    }
    st = cmul(op.alpha, st);
  }
  cpx<T> ms = czero<T>();
  const int nc = n - 1;
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    // cell j - bits(c); j is its local vertex c
    int cell[3] = {0, 0, 0};
    bool ok = true;
    for (int a = 0; a < D; ++a) {
      cell[a] = j[a] - ((c >> a) & 1);
      if (cell[a] < 0 || cell[a] >= nc) ok = false;
    }
    if (!ok) continue;
    cpx<T> am = czero<T>(), ak = czero<T>();
#pragma unroll
    for (int kk = 0; kk < (1 << D); ++kk) {
      // local vertex kk of the cell sits at offset bits(kk) - bits(c) from j
      int q = 0, stride = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        q += (((kk >> a) & 1) - ((c >> a) & 1) + 1) * stride;
        stride *= 3;
      }
      am = am + elem_mass<T, D>(c, kk) * xv[q];
      if (op.cstiff) ak = ak + elem_stiff<T, D>(c, kk) * xv[q];
    }
    const long long ci = ravel<D>(cell, nc);
    ms = ms + cmul(op.cmass[ci], am);
    if (op.cstiff) st = st + cmul(op.cstiff[ci], ak);
  }
  return st - ms;
}

// Rotation angle of cell c on a level with m cells per axis.
template <int D>
__device__ inline double cell_angle(const CellRotation& r, const int c[3], int m) {
  if (r.width > 0) {
    for (int a = 0; a < D; ++a) {
      const double centre = (c[a] + 0.5) / m;
      if (((r.faces >> (2 * a)) & 1) && centre < r.width) return r.layer_theta;
      if (((r.faces >> (2 * a + 1)) & 1) && 1.0 - centre < r.width) return r.layer_theta;
    }
  }
  return r.theta;
}

// eta_c^p (p = 0 .. 3) of cell c: (h exp(i theta_c))^p, conjugated in
// conjugate mode.
template <int D>
__device__ inline cpx<double> cell_eta_pow(const CellRotation& r, const int c[3], int m, int p) {
  const double t = cell_angle<D>(r, c, m);
  const cpx<double> eta = mk(r.h * cos(t), r.conj ? -r.h * sin(t) : r.h * sin(t));
  cpx<double> out = mk(1.0, 0.0);
  for (int k = 0; k < p; ++k) out = cmul(out, eta);
  return out;
}

template <class T, int D>
__device__ inline cpx<T> apply_row(const cpx<T>* x, int n, const int j[3], const OpData<T>& op) {
  return op.cmass ? stencil_var<T, D>(x, n, j, op) : stencil_const<T, D>(x, n, j, op);
}


}  // namespace mg
