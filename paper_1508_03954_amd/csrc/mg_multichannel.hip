// Same-grid multichannel form (Section 7.5): C channels -- independent
// Helmholtz problems that share the grid and differ in phi (and load) --
// fused into one problem on one grid, every vertex holding a C^C tuple
// (array-of-structures: channel c of vertex i at i * C + c).  One cycle runs
// the pipelined additive cycle of every channel at once: the index
// arithmetic, the stencil and transfer weights and the coarse-level
// traversal are computed once per vertex and applied to all C channels, and
// every vertex is read as one contiguous run of 16 C bytes.
//
// The cycle is the Galerkin form of the single-problem engine's separate
// level passes (constant phi per channel and a uniform rotation): descent
// (sc += P sc_c, BPX: - P si_c off c-points), finest U = w + P g, r = b - H U
// with the norms of every channel, the pointwise update with its
// injections, rho_c = R r; then the Galerkin backtracking of the coarse
// levels and the coarsest update.  The finest level keeps the folded iterate
// (u + sc) in two ping-pong buffers; coarse u is not stored (the Galerkin
// form never reads it).
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

// Per-level operator data of every channel (passed by value).
template <int C>
struct McOp {
  int n;
  cpx<double> coef[C][4];   // stencil weight by number of nonzero offsets
  cpx<double> invD[C];      // 1 / diagonal
};

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

// acc[ch] += sum over corners of wt * v[idx * C + ch]
template <int D, int C>
__device__ inline void prolong_add(const cpx<double>* __restrict__ v, const long long idx[8], const double wt[8],
                                   double sgn, cpx<double> acc[C]) {
#pragma unroll
  for (int c = 0; c < (1 << D); ++c) {
    const double w = sgn * wt[c];
    const cpx<double>* p = v + idx[c] * C;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = acc[ch] + w * p[ch];
  }
}

// Descent of a coarse level: sc += P sc_c (BPX: - P si_c off c-points).  The
// iterate u += sc + sf is not stored (see the header).
template <int D, int C>
__global__ void k_mc_pre(int n, cpx<double>* __restrict__ sc, const cpx<double>* __restrict__ scc,
                         const cpx<double>* __restrict__ sic, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (!is_interior<D>(j, n)) continue;
    long long idx[8];
    double wt[8];
    prolong_support<D>(nc, j, idx, wt);
    cpx<double> acc[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = sc[i * C + ch];
    prolong_add<D, C>(scc, idx, wt, 1.0, acc);
    if (bpx && !is_cpoint<D>(j)) prolong_add<D, C>(sic, idx, wt, -1.0, acc);
#pragma unroll
    for (int ch = 0; ch < C; ++ch) sc[i * C + ch] = acc[ch];
  }
}

// Finest descent: U = w + P sc_c (BPX: - P si_c off c-points); 0 on the boundary.
template <int D, int C>
__global__ void k_mc_fine_pre(int n, const cpx<double>* __restrict__ w, cpx<double>* __restrict__ U,
                              const cpx<double>* __restrict__ scc, const cpx<double>* __restrict__ sic,
                              int has_coarse, int bpx) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    cpx<double> acc[C];
    if (!is_interior<D>(j, n)) {
#pragma unroll
      for (int ch = 0; ch < C; ++ch) U[i * C + ch] = czero<double>();
      continue;
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = w[i * C + ch];
    if (has_coarse) {
      long long idx[8];
      double wt[8];
      prolong_support<D>(nc, j, idx, wt);
      prolong_add<D, C>(scc, idx, wt, 1.0, acc);
      if (bpx && !is_cpoint<D>(j)) prolong_add<D, C>(sic, idx, wt, -1.0, acc);
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) U[i * C + ch] = acc[ch];
  }
}

// Block sums of |r|^2 and maxima of |r| per channel, fixed order.
template <int C>
__device__ inline void mc_block_norms(double s2[C], double mx[C], double* partials) {
  __shared__ double ss[C][4], sm[C][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) {
    double a = s2[ch], b = mx[ch];
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b = fmax(b, __shfl_down(b, off, 64));
    }
    if (lane == 0) {
      ss[ch][wid] = a;
      sm[ch][wid] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < C) {
    const int ch = threadIdx.x;
    double a = 0, b = 0;
    for (int w = 0; w < 4; ++w) {
      a += ss[ch][w];
      b = fmax(b, sm[ch][w]);
    }
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    partials[(2 * (size_t)bid) * C + 2 * ch] = a;
    partials[(2 * (size_t)bid) * C + 2 * ch + 1] = b;
  }
}

// r = b - H x for every channel (interior; 0 on the boundary) with the
// per-block norms of each channel.  The 3^d neighbour offsets and their
// classes are formed once per vertex.
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_resid(McOp<C> op, const cpx<double>* __restrict__ b,
                                                  const cpx<double>* __restrict__ x, cpx<double>* __restrict__ r,
                                                  double* partials) {
  const int n = op.n;
  double s2[C], mx[C];
#pragma unroll
  for (int ch = 0; ch < C; ++ch) s2[ch] = mx[ch] = 0.0;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (!is_interior<D>(j, n)) {
#pragma unroll
      for (int ch = 0; ch < C; ++ch) r[i * C + ch] = czero<double>();
      continue;
    }
    cpx<double> acc[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = b[i * C + ch];
    const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
    for (int oz = zlo; oz <= zhi; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int k[3] = {j[0] + ox, j[1] + oy, j[2] + oz};
          if (!is_interior<D>(k, n)) continue;
          const int cls = (ox != 0) + (oy != 0) + (oz != 0);
          const cpx<double>* p = x + ravel<D>(k, n) * C;
#pragma unroll
          for (int ch = 0; ch < C; ++ch) acc[ch] = acc[ch] - cmul(op.coef[ch][cls], p[ch]);
        }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
      r[i * C + ch] = acc[ch];
      const double a2 = acc[ch].re * acc[ch].re + acc[ch].im * acc[ch].im;
      s2[ch] += a2;
      mx[ch] = fmax(mx[ch], a2);
    }
  }
#pragma unroll
  for (int ch = 0; ch < C; ++ch) mx[ch] = sqrt(mx[ch]);
  if (partials) mc_block_norms<C>(s2, mx, partials);
}

// y = H x for every channel.
template <int D, int C>
__global__ __launch_bounds__(256) void k_mc_apply(McOp<C> op, const cpx<double>* __restrict__ x,
                                                  cpx<double>* __restrict__ y) {
  const int n = op.n;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    cpx<double> acc[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[ch] = czero<double>();
    if (is_interior<D>(j, n)) {
      const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
      for (int oz = zlo; oz <= zhi; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox) {
            const int k[3] = {j[0] + ox, j[1] + oy, j[2] + oz};
            if (!is_interior<D>(k, n)) continue;
            const int cls = (ox != 0) + (oy != 0) + (oz != 0);
            const cpx<double>* p = x + ravel<D>(k, n) * C;
#pragma unroll
            for (int ch = 0; ch < C; ++ch) acc[ch] = acc[ch] + cmul(op.coef[ch][cls], p[ch]);
          }
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) y[i * C + ch] = acc[ch];
  }
}

// Pointwise post-phase of a level: s = omega r / D_ch, sc = s (0 on c-points
// when masked); finest: u += sc in place; coarse: sc_out = sc.  At c-points:
// sf_c = sf + sc (if sfc), si_c = s (if sic).
template <int D, int C>
__global__ void k_mc_update(McOp<C> op, const cpx<double>* __restrict__ r, cpx<double> omega, int mask_c,
                            cpx<double>* __restrict__ u, cpx<double>* __restrict__ sc_out,
                            const cpx<double>* __restrict__ sf, cpx<double>* __restrict__ sfc,
                            cpx<double>* __restrict__ sic) {
  const int n = op.n, nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const bool in = is_interior<D>(j, n);
    const bool cp = is_cpoint<D>(j);
    long long ic = 0;
    if (cp) {
      const int m[3] = {j[0] / 3, j[1] / 3, j[2] / 3};
      ic = ravel<D>(m, nc);
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
      cpx<double> s = czero<double>();
      if (in) s = cmul(omega, cmul(op.invD[ch], r[i * C + ch]));
      const cpx<double> scv = csel(mask_c && cp, czero<double>(), s);
      if (u && in) u[i * C + ch] = u[i * C + ch] + scv;
      if (sc_out) sc_out[i * C + ch] = scv;
      if (cp && sfc) sfc[ic * C + ch] = (sf ? sf[i * C + ch] : czero<double>()) + scv;
      if (cp && sic) sic[ic * C + ch] = s;
    }
  }
}

// R v at coarse vertex m for every channel: weights (1 - |o|/3) per axis over
// the fine offsets o in [-2, 2]^d around 3m; 0 on the coarse boundary.
template <int D, int C>
__device__ inline void mc_restrict_at(const cpx<double>* __restrict__ vf, int nf, const int m[3], cpx<double> acc[C]) {
  constexpr double w[5] = {1.0 / 3.0, 2.0 / 3.0, 1.0, 2.0 / 3.0, 1.0 / 3.0};
#pragma unroll
  for (int ch = 0; ch < C; ++ch) acc[ch] = czero<double>();
  const int zlo = D == 3 ? -2 : 0, zhi = D == 3 ? 2 : 0;
  for (int oz = zlo; oz <= zhi; ++oz)
    for (int oy = -2; oy <= 2; ++oy)
      for (int ox = -2; ox <= 2; ++ox) {
        const int k[3] = {3 * m[0] + ox, 3 * m[1] + oy, 3 * m[2] + oz};
        bool inside = true;
        for (int a = 0; a < D; ++a) inside = inside && k[a] >= 0 && k[a] < nf;
        if (!inside) continue;
        double wt = w[ox + 2] * w[oy + 2];
        if (D == 3) wt *= w[oz + 2];
        const cpx<double>* p = vf + ravel<D>(k, nf) * C;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[ch] = acc[ch] + wt * p[ch];
      }
}

template <int D, int C>
__global__ void k_mc_restrict(int nc, const cpx<double>* __restrict__ vf, cpx<double>* __restrict__ vc) {
  const int nf = 3 * (nc - 1) + 1;
  MG_ROWS(D, nc) {
    int m[3];
    long long ic;
    if (!row_vertex<D>(row_, x_, nc, m, ic)) continue;
    cpx<double> acc[C];
    if (is_interior<D>(m, nc)) {
      mc_restrict_at<D, C>(vf, nf, m, acc);
    } else {
#pragma unroll
      for (int ch = 0; ch < C; ++ch) acc[ch] = czero<double>();
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) vc[ic * C + ch] = acc[ch];
  }
}

// Per-channel second stage of the norms over `count` blocks, block order.
template <int C>
__global__ void k_mc_finish(const double* __restrict__ partials, int count, double* __restrict__ out) {
  const int ch = threadIdx.x;
  if (ch >= C) return;
  double a = 0, b = 0;
  for (int k = 0; k < count; ++k) {
    a += partials[(2 * (size_t)k) * C + 2 * ch];
    b = fmax(b, partials[(2 * (size_t)k) * C + 2 * ch + 1]);
  }
  out[2 * ch] = a;
  out[2 * ch + 1] = b;
}

template <int D, int C>
__global__ void k_mc_copy_zero_boundary(int n, const cpx<double>* __restrict__ in, cpx<double>* __restrict__ out) {
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const bool in_ = is_interior<D>(j, n);
#pragma unroll
    for (int ch = 0; ch < C; ++ch) out[i * C + ch] = in_ ? in[i * C + ch] : czero<double>();
  }
}

static dim3 mc_row_grid(int n, int dim, int max_row_blocks = 65535) {
  const long long rows = dim == 3 ? (long long)n * n : n;
  long long gy = (rows + 3) / 4;
  if (gy > max_row_blocks) gy = max_row_blocks;
  return dim3((unsigned)((n + 63) / 64), (unsigned)gy);
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
    McOp<C> op;
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
  int launch(K k2, K k3, dim3 g, A... args) {
    if (dim == 3) hipLaunchKernelGGL(k3, g, dim3(256), 0, s, args...);
    else hipLaunchKernelGGL(k2, g, dim3(256), 0, s, args...);
    MG_HIP(hipGetLastError());
    return MG_OK;
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
      v.op.n = v.n;
      for (int ch = 0; ch < C; ++ch) {
        const mg_c128 ph = phis[ch];
        const OpData<double> o = make_const_op<double>(dim, l, p.theta, complex<double>(ph.re, ph.im), p.conjugate != 0);
        for (int q = 0; q < 4; ++q) v.op.coef[ch][q] = o.coef[q];
        v.op.invD[ch] = o.invD;
      }
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
    const dim3 g = mc_row_grid(lv[L].n, dim);
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
    return launch(k_mc_copy_zero_boundary<2, C>, k_mc_copy_zero_boundary<3, C>, mc_row_grid(lv[L].n, dim),
                  lv[L].n, src, dst);
  }

  int apply(const cpx<double>* x, cpx<double>* y) override {
    return launch(k_mc_apply<2, C>, k_mc_apply<3, C>, mc_row_grid(lv[L].n, dim), lv[L].op, x, y);
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
      MG_TRY(launch(k_mc_pre<2, C>, k_mc_pre<3, C>, mc_row_grid(lv[l].n, dim), lv[l].n, lv[l].sc,
                    (const cpx<double>*)lv[l - 1].sc, (const cpx<double>*)lv[l - 1].si, variant == MG_BPX ? 1 : 0));
    return MG_OK;
  }

  int fine_pre(cpx<double>* U) {
    const bool hc = L > lmin;
    return launch(k_mc_fine_pre<2, C>, k_mc_fine_pre<3, C>, mc_row_grid(lv[L].n, dim), lv[L].n,
                  (const cpx<double>*)w[cur], U, hc ? (const cpx<double>*)lv[L - 1].sc : nullptr,
                  hc ? (const cpx<double>*)lv[L - 1].si : nullptr, hc ? 1 : 0, variant == MG_BPX ? 1 : 0);
  }

  int cycle_once(int k) {
    ++iter;
    MG_TRY(pre_coarse());
    Lv& f = lv[L];
    const bool hc = L > lmin;
    Lv* c = hc ? &lv[L - 1] : nullptr;
    cpx<double>* U = w[1 - cur];
    MG_TRY(fine_pre(U));
    MG_TRY(launch(k_mc_resid<2, C>, k_mc_resid<3, C>, mc_row_grid(f.n, dim), f.op, (const cpx<double>*)f.b,
                  (const cpx<double>*)U, tR, partials));
    const complex<double> wL = omega_level(scheme, omega, omega_L, 0, iter);
    const int mask = (hc && variant != MG_ADD) ? 1 : 0;
    MG_TRY(launch(k_mc_update<2, C>, k_mc_update<3, C>, mc_row_grid(f.n, dim), f.op, (const cpx<double>*)tR,
                  to_c<double>(wL), mask, U, (cpx<double>*)nullptr, (const cpx<double>*)nullptr,
                  (hc && variant == MG_ADD) ? c->sf : nullptr, (hc && variant == MG_BPX) ? c->si : nullptr));
    if (hc)
      MG_TRY(launch(k_mc_restrict<2, C>, k_mc_restrict<3, C>, mc_row_grid(c->n, dim), c->n, (const cpx<double>*)tR,
                    c->b));
    cur = 1 - cur;
    hipLaunchKernelGGL(k_mc_finish<C>, dim3(1), dim3(64), 0, s, (const double*)partials, red_blocks,
                       hist + 2 * (size_t)k * C);
    MG_HIP(hipGetLastError());
    // backtracking of the coarse levels (Galerkin form: the b slot holds the
    // level's residual R r of the finer one)
    for (int l = L - 1; l >= lmin; --l) {
      Lv& v = lv[l];
      const bool hcc = l > lmin;
      Lv* cc = hcc ? &lv[l - 1] : nullptr;
      const complex<double> wl = omega_level(scheme, omega, omega_L, L - l, iter);
      MG_TRY(launch(k_mc_update<2, C>, k_mc_update<3, C>, mc_row_grid(v.n, dim), v.op, (const cpx<double>*)v.b,
                    to_c<double>(wl), (hcc && variant != MG_ADD) ? 1 : 0, (cpx<double>*)nullptr, v.sc,
                    (const cpx<double>*)v.sf, (hcc && variant == MG_ADD) ? cc->sf : nullptr,
                    (hcc && variant == MG_BPX) ? cc->si : nullptr));
      if (hcc)
        MG_TRY(launch(k_mc_restrict<2, C>, k_mc_restrict<3, C>, mc_row_grid(cc->n, dim), cc->n,
                      (const cpx<double>*)v.b, cc->b));
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
