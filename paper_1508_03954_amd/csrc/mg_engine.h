// Host-side engine: per-level storage, cycle and solve drivers of one problem.
// Shared by the C-ABI entry points (mg_api.hip) and the batched driver
// (mg_batch.hip).
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mg.h"
#include "mg_internal.h"

using std::complex;

namespace mg {

// Default relative residual of a complex64 inner solve in FP64 residual
// refinement (mg_params.inner_rtol = 0).  Restarting the inner BiCGStab after
// each factor of about 3 keeps its recursive residual close to the true one
// under complex64 rounding; measured on the 3D k = 40 problem and the
// 96-problem batch, tighter targets (1e-2 .. 1e-4) took 1.3-9 times longer
// because the inner solves stall well above their target.
constexpr double kInnerRtolDefault = 0.3;

// Coarse levels of at least this many vertices per axis (3D) take the
// backtracking as a streaming update pass plus the restriction march instead
// of k_post_galerkin, whose gathered restriction support runs at about 40 % of
// the streaming rate on such a level (244^3: 221 µs).
constexpr int kPostSplitMinN = 244;

inline thread_local std::string g_err;

inline int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define MG_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      return fail(MG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
    }                                                                                  \
  } while (0)

#define MG_TRY(call)          \
  do {                        \
    int rc_ = (call);         \
    if (rc_ != MG_OK) return rc_; \
  } while (0)

template <class T>
inline cpx<T> to_c(complex<double> z) {
  return mk(T(z.real()), T(z.imag()));
}

inline long long ipow(long long b, int e) {
  long long r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// Assembled stencil weights of the d-linear element matrices by number of
// nonzero offsets: stiffness S_K and mass S_M (rows sum to 0 and 1).
inline void stencil_weights(int dim, double sk[4], double sm[4]) {
  if (dim == 3) {
    const double k[4] = {8.0 / 3.0, 0.0, -1.0 / 6.0, -1.0 / 12.0};
    const double m[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
    std::copy(k, k + 4, sk);
    std::copy(m, m + 4, sm);
  } else {
    const double k[4] = {8.0 / 3.0, -1.0 / 3.0, -1.0 / 3.0, 0.0};
    const double m[4] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 0.0};
    std::copy(k, k + 4, sk);
    std::copy(m, m + 4, sm);
  }
}

struct LevelScalars {
  complex<double> eta, alpha, etad;
};

inline LevelScalars level_scalars(int dim, int lev, double theta, bool conj) {
  LevelScalars s;
  s.eta = std::pow(3.0, -lev) * std::exp(complex<double>(0.0, theta));
  if (conj) s.eta = std::conj(s.eta);
  s.alpha = std::pow(s.eta, dim - 2);
  s.etad = std::pow(s.eta, dim);
  return s;
}

template <class T>
inline OpData<T> make_const_op(int dim, int lev, double theta, complex<double> phi, bool conj) {
  OpData<T> op;
  std::memset(&op, 0, sizeof(op));
  op.n = (int)ipow(3, lev) + 1;
  const LevelScalars ls = level_scalars(dim, lev, theta, conj);
  if (conj) phi = std::conj(phi);
  double sk[4], sm[4];
  stencil_weights(dim, sk, sm);
  for (int c = 0; c < 4; ++c) op.coef[c] = to_c<T>(ls.alpha * sk[c] - phi * ls.etad * sm[c]);
  op.alpha = to_c<T>(ls.alpha);
  op.etad = to_c<T>(ls.etad);
  const complex<double> D = ls.alpha * (2.0 * dim * std::pow(2.0 / 3.0, dim - 1)) -
                            phi * ls.etad * std::pow(2.0 / 3.0, dim);
  op.invD = to_c<T>(1.0 / D);
  op.cmass = nullptr;
  op.cstiff = nullptr;
  op.invDv = nullptr;
  return op;
}

inline complex<double> omega_level(int scheme, complex<double> w, int omega_L, int succ, int iteration) {
  switch (scheme) {
    case MG_OMEGA_CONST: return w;
    case MG_OMEGA_JACOBI: return succ == 0 ? w : 0.0;
    case MG_OMEGA_LGRID: return succ <= omega_L ? w : 0.0;
    case MG_OMEGA_EXP: return std::pow(w, (double)(succ + 1));
    case MG_OMEGA_TWO_PHASE: return std::max(iteration, 1) % 2 == 1 ? w : -std::conj(w);
    default: return std::pow(w, (1.0 - 1.0 / std::max(iteration, 1)) * (succ + 1));
  }
}

// Cell rotations of level l (the absorbing layer only when its width is set).
inline CellRotation rotation(const mg_params& p, int l) {
  CellRotation r;
  r.h = std::pow(3.0, -l);
  r.theta = p.theta;
  r.layer_theta = p.layer_theta;
  r.width = p.layer_width > 0 ? p.layer_width : 0.0;
  r.faces = p.layer_faces;
  r.conj = p.conjugate != 0;
  return r;
}

template <class T>
struct Level {
  int lev = 0, n = 0;
  size_t N = 0;
  cpx<T>*u = nullptr, *b = nullptr, *sc = nullptr, *sf = nullptr, *si = nullptr;
  cpx<T>*phi = nullptr, *cmass = nullptr, *cstiff = nullptr, *invDv = nullptr;
  cpx<T>*pr = nullptr, *pz = nullptr;  // zero-start cycle scratch (coarse levels)
  OpData<T> op;
};

template <class T>
struct Engine {
  int dim = 3, lmin = 1, L = 1, variant = MG_BPX, scheme = MG_OMEGA_CONST, omega_L = 1;
  complex<double> omega = 0.6;
  bool galerkin = true, fused = false, varying = false, layered = false;
  hipStream_t s = nullptr;
  std::vector<Level<T>> lv;
  cpx<T>* w[2] = {nullptr, nullptr};
  int cur = 0;
  cpx<T>* si_alt = nullptr;    // second si buffer of level L-1 (fused BPX sweep reads old, writes new)
  cpx<T>* tune_c = nullptr;    // coarse scratch for the autotuner
  cpx<T>* spill = nullptr;     // seam rows of the 3D fused sweep's restriction
  bool small_pre_done = false; // the small levels' pre-phase of the next cycle has run
  cpx<T>*tA = nullptr, *tR = nullptr, *tRh = nullptr;
  double* partials = nullptr;  // 2 * max(kRedBlocks, fused blocks)
  double* red = nullptr;       // 4 doubles
  double* hist = nullptr;      // 2 * hist_cap
  int hist_cap = 0;
  int iter = 0;
  int fused_blocks = 0;
  int partials_cap = 0;        // capacity of `partials` in (sum, max) pairs
  size_t partials_doubles = 0; // capacity of `partials` in doubles
  std::vector<cpx<T>*> kv;     // Krylov vectors
  std::vector<void*> owned;
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs around finest sweeps
  size_t ev_used = 0;

  ~Engine() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (void* p : owned) (void)hipFree(p);
  }

  int mark(bool start) {
    if (!timing) return MG_OK;
    if (ev_used == ev.size()) {
      hipEvent_t e;
      MG_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    MG_HIP(hipEventRecord(ev[ev_used++], s));
    (void)start;
    return MG_OK;
  }

  // The next event pair of the record for a launch that takes its events
  // itself (both nullptr when not timing).
  int event_pair(hipEvent_t* t0, hipEvent_t* t1) {
    *t0 = *t1 = nullptr;
    if (!timing) return MG_OK;
    while (ev.size() < ev_used + 2) {
      hipEvent_t e;
      MG_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    *t0 = ev[ev_used++];
    *t1 = ev[ev_used++];
    return MG_OK;
  }

  int alloc(void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(MG_ENOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    owned.push_back(*p);
    return MG_OK;
  }
  template <class P>
  int alloc_c(P** p, size_t count) {
    void* q = nullptr;
    MG_TRY(alloc(&q, count * sizeof(P)));
    MG_HIP(launch_fill(q, count * sizeof(P), s));
    *p = (P*)q;
    return MG_OK;
  }

  size_t NL() const { return lv[L].N; }

  // op_only: keep the finest-level operator data only (no cycle state); used
  // for the FP64 residual of the refinement loop.
  int setup(const mg_params& p, hipStream_t stream, const cpx<double>* phi_field, bool op_only = false) {
    s = stream;
    dim = p.dim;
    lmin = p.level_min;
    L = p.level_max;
    variant = p.variant;
    scheme = p.omega_scheme;
    omega_L = p.omega_L;
    omega = complex<double>(p.omega.re, p.omega.im);
    // per-cell coefficients for a nodal phi or an absorbing layer
    layered = p.layer_width > 0;
    varying = phi_field != nullptr || layered;
    const bool conj = p.conjugate != 0;
    galerkin = !varying;
    if (p.restrict_form == MG_RESTRICT_FAS) galerkin = false;
    if (p.restrict_form == MG_RESTRICT_GALERKIN) {
      if (varying) return fail(MG_EINVAL, "GALERKIN restriction needs a constant phi and no absorbing layer");
      galerkin = true;
    }
    if (op_only) lmin = L;
    const bool fused_ok = fused_partials_blocks(dim, (int)ipow(3, L) + 1, 0) > 0;
    fused = galerkin && !varying && L > lmin && p.sweep != MG_SWEEP_GENERIC && fused_ok && !op_only;
    if (p.sweep == MG_SWEEP_FUSED && !fused)
      return fail(MG_EINVAL, "FUSED sweep needs constant phi, GALERKIN form, level_max > level_min "
                             "and a built fused kernel");
    lv.resize(L + 1);
    for (int l = lmin; l <= L; ++l) {
      Level<T>& v = lv[l];
      v.lev = l;
      v.n = (int)ipow(3, l) + 1;
      v.N = (size_t)ipow(v.n, dim);
      v.op = make_const_op<T>(dim, l, p.theta, complex<double>(p.phi.re, p.phi.im), conj);
      if (l < L) {
        MG_TRY(alloc_c(&v.u, v.N));
        MG_TRY(alloc_c(&v.b, v.N));
        MG_TRY(alloc_c(&v.sc, v.N));
        MG_TRY(alloc_c(&v.sf, v.N));
        MG_TRY(alloc_c(&v.si, v.N));
        MG_TRY(alloc_c(&v.pr, v.N));
        MG_TRY(alloc_c(&v.pz, v.N));
      } else if (!op_only) {
        MG_TRY(alloc_c(&v.b, v.N));
        MG_TRY(alloc_c(&w[0], v.N));
        MG_TRY(alloc_c(&w[1], v.N));
      }
    }
    if (varying) {
      // nodal phi on every level by injection (a constant phi with a layer:
      // the constant on every vertex), per-cell coefficients with each level's
      // own cell rotations, accumulated diagonal
      for (int l = L; l >= lmin; --l) {
        Level<T>& v = lv[l];
        MG_TRY(alloc_c(&v.phi, v.N));
        if (!phi_field) {
          MG_HIP(launch_set_value<T>(v.N, v.phi, mk(p.phi.re, p.phi.im), s));
        } else if (l == L) {
          MG_HIP((launch_convert<double, T>(v.N, phi_field, v.phi, 1.0, s)));
        } else {
          MG_HIP(launch_inject<T>(dim, v.n, lv[l + 1].phi, v.phi, s));
        }
      }
      for (int l = lmin; l <= L; ++l) {
        Level<T>& v = lv[l];
        const size_t cells = (size_t)ipow(v.n - 1, dim);
        MG_TRY(alloc_c(&v.cmass, cells));
        // the stiffness scale eta_c^(d-2) varies over the cells only in 3D
        if (layered && dim == 3) MG_TRY(alloc_c(&v.cstiff, cells));
        MG_TRY(alloc_c(&v.invDv, v.N));
        MG_HIP(launch_cellcoef<T>(dim, v.n, v.phi, v.cmass, v.cstiff, rotation(p, l), s));
        v.op.cmass = v.cmass;
        v.op.cstiff = v.cstiff;
        MG_HIP(launch_invdiag<T>(dim, v.op, v.invDv, s));
        v.op.invDv = v.invDv;
      }
    }
    if (fused && variant == MG_BPX) MG_TRY(alloc_c(&si_alt, lv[L - 1].N));
    if (fused && dim == 3) MG_TRY(alloc_c(&spill, fused_spill_count(dim, lv[L].n)));
    int max_blocks = kRedBlocks;
    if (fused) {
      for (int t = 0; t < fused_tile_count(dim); ++t)
        max_blocks = std::max(max_blocks, fused_partials_blocks(dim, lv[L].n, t));
      set_tile(default_tile());
    }
    // (sum, max) pairs per block, or up to four sums per block of the fused
    // Krylov kernels
    partials_doubles = std::max<size_t>(2 * (size_t)max_blocks, 4 * (size_t)kRedBlocks);
    MG_TRY(alloc_c(&partials, partials_doubles));
    partials_cap = max_blocks;
    MG_TRY(alloc_c(&red, 4));
    MG_TRY(ensure_hist(64));
    return MG_OK;
  }

  int tile = 0;

  // Default tile: short z chunks while the grid is small (more blocks and
  // shorter marches: on 28^3 and 82^3 the march of 3 coarse planes takes about
  // half the time of one of 9), otherwise 2 coarse rows by 21 coarse planes.
  int default_tile() const {
    if (dim == 2) return lv[L].n <= 250 ? 1 : 0;
    return fused_tile_index(3, 2, 2, lv[L].n <= 82 ? 3 : 21);
  }
  void set_tile(int t) {
    tile = t;
    fused_blocks = fused_partials_blocks(dim, lv[L].n, t);
  }

  int ensure_hist(int cap) {
    if (cap <= hist_cap) return MG_OK;
    MG_TRY(alloc_c(&hist, 2 * (size_t)cap));
    hist_cap = cap;
    return MG_OK;
  }

  int ensure_scratch() {
    if (!tA) {
      MG_TRY(alloc_c(&tA, NL()));
      MG_TRY(alloc_c(&tR, NL()));
      MG_TRY(alloc_c(&tRh, NL()));
    }
    return MG_OK;
  }

  int ensure_krylov() {
    if (kv.empty()) {
      kv.resize(8);
      for (auto& p : kv) MG_TRY(alloc_c(&p, NL()));
    }
    return MG_OK;
  }

  int zero_helpers() {
    small_pre_done = false;
    for (int l = lmin; l < L; ++l) {
      MG_HIP(launch_fill(lv[l].sc, lv[l].N * sizeof(cpx<T>), s));
      MG_HIP(launch_fill(lv[l].sf, lv[l].N * sizeof(cpx<T>), s));
      MG_HIP(launch_fill(lv[l].si, lv[l].N * sizeof(cpx<T>), s));
    }
    if (si_alt) MG_HIP(launch_fill(si_alt, lv[L - 1].N * sizeof(cpx<T>), s));
    return MG_OK;
  }

  // A new right-hand side or iterate starts the iteration afresh: helpers
  // and the cycle counter of the iteration-dependent relaxation schemes.  A
  // flush clears the helpers only, so the schemes continue where they were.
  int set_rhs(const cpx<T>* b) {
    MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, b, lv[L].b, mk(T(1), T(0)), s));
    iter = 0;
    return zero_helpers();
  }

  // Coarse iterate of level l < L, or nullptr in the Galerkin form: there the
  // coarse b slot holds the restricted residual itself, so no step reads the
  // coarse iterates and they are not formed.
  cpx<T>* coarse_u(int l) const { return galerkin ? nullptr : lv[l].u; }

  int set_solution(const cpx<T>* u) {
    MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, u, w[cur], mk(T(1), T(0)), s));
    for (int l = L; l > lmin && !galerkin; --l) {
      const cpx<T>* src = l == L ? w[cur] : lv[l].u;
      MG_HIP(launch_inject<T>(dim, lv[l - 1].n, src, lv[l - 1].u, s));
    }
    iter = 0;
    return zero_helpers();
  }

  // Number of coarsest levels (from l_min) handled by the single-block small-
  // level kernels: at most kSmallVertices vertices each, never the finest; 0
  // when fewer than two qualify or when the coarse right-hand side is not in
  // the Galerkin form.
  int small_levels() const {
    if (!galerkin) return 0;
    int k = 0;
    while (k < kSmallMax && lmin + k < L && lv[lmin + k].N <= (size_t)kSmallVertices) ++k;
    return k >= 2 ? k : 0;
  }

  SmallArgs<T> small_args(int nl) const {
    SmallArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.dim = dim;
    a.nl = nl;
    a.variant = variant;
    for (int k = 0; k < nl; ++k) {
      const Level<T>& v = lv[lmin + k];
      a.lv[k].n = v.n;
      a.lv[k].u = coarse_u(lmin + k);
      a.lv[k].b = v.b;
      a.lv[k].sc = v.sc;
      a.lv[k].sf = v.sf;
      a.lv[k].si = v.si;
      a.lv[k].op = v.op;
      a.lv[k].omega = to_c<T>(omega_level(scheme, omega, omega_L, L - (lmin + k), iter));
    }
    return a;
  }

  // Descent (pre-phase) on the coarse levels l_min .. L-1.
  int pre_coarse() {
    int l0 = lmin;
    const int ns = small_levels();
    if (ns) {
      if (!small_pre_done) MG_HIP(launch_small_pre<T>(small_args(ns), s));
      small_pre_done = false;
      l0 = lmin + ns;
    }
    for (int l = l0; l < L; ++l) {
      Level<T>& v = lv[l];
      const bool hc = l > lmin;
      MG_HIP(launch_pre<T>(dim, v.n, coarse_u(l), v.sc, v.sf, hc ? lv[l - 1].sc : nullptr,
                           hc ? lv[l - 1].si : nullptr, hc ? 1 : 0, variant == MG_BPX ? 1 : 0, s));
    }
    return MG_OK;
  }

  // more: another cycle follows in the same call (its small-level pre-phase
  // then runs in this cycle's last launch)
  int cycle_once(int k, bool more = false) {
    ++iter;
    MG_TRY(ensure_hist(k + 1));
    MG_TRY(pre_coarse());
    Level<T>& f = lv[L];
    const bool hc = L > lmin;
    Level<T>* c = hc ? &lv[L - 1] : nullptr;
    const complex<double> wL = omega_level(scheme, omega, omega_L, 0, iter);
    const int mask = (hc && variant != MG_ADD) ? 1 : 0;
    int nparts = kRedBlocks;
    if (fused) {
      // the event pair takes the sweep kernel's own start and end
      hipEvent_t t0, t1;
      MG_TRY(event_pair(&t0, &t1));
      FusedArgs<T> a = fused_args(w[1 - cur], c->b, c->sf, si_alt, wL.real(), wL.imag());
      MG_HIP(launch_fused<T>(dim, a, s, t0, t1));
      MG_HIP(launch_fused_seam<T>(dim, a, s));
      if (variant == MG_BPX) std::swap(c->si, si_alt);
      nparts = fused_blocks;
    } else {
      MG_TRY(ensure_scratch());
      MG_TRY(mark(true));
      cpx<T>* U = w[1 - cur];
      MG_HIP(launch_fine_pre<T>(dim, f.n, w[cur], U, hc ? c->sc : nullptr, hc ? c->si : nullptr, hc ? 1 : 0,
                                variant == MG_BPX ? 1 : 0, s));
      if (!galerkin && hc) MG_HIP(launch_uhat<T>(dim, f.n, U, c->u, tA, s));
      MG_HIP(launch_resid<T>(dim, f.op, f.b, U, tR, partials, &nparts, s));
      if (!galerkin && hc) MG_HIP(launch_resid<T>(dim, f.op, f.b, tA, tRh, nullptr, nullptr, s));
      MG_HIP(launch_update<T>(dim, f.op, tR, to_c<T>(wL), mask, U, nullptr, nullptr,
                              (hc && variant == MG_ADD) ? c->sf : nullptr, (hc && variant == MG_BPX) ? c->si : nullptr,
                              s));
      if (hc) MG_HIP(launch_restrict<T>(dim, c->n, galerkin ? tR : tRh, c->b, s));
      MG_TRY(mark(false));
    }
    cur = 1 - cur;
    const int ns = small_levels();
    if (!ns) MG_HIP(launch_finish_sum_max(partials, nparts, hist + 2 * k, s));
    // Backtracking (post-phase) on the coarse levels L-1 .. l_min; the smallest
    // ones, the coarsest update and the norm's second stage in one block.
    for (int l = L - 1; l >= lmin; --l) {
      if (ns && l < lmin + ns) {
        SmallArgs<T> a = small_args(ns);
        a.partials = partials;
        a.nparts = nparts;
        a.out = hist + 2 * k;
        a.then_pre = more ? 1 : 0;
        MG_HIP(launch_small_post<T>(a, s));
        small_pre_done = more;
        break;
      }
      Level<T>& v = lv[l];
      const bool hcc = l > lmin;
      Level<T>* cc = hcc ? &lv[l - 1] : nullptr;
      const complex<double> wl = omega_level(scheme, omega, omega_L, L - l, iter);
      const cpx<T>* r;
      if (galerkin && hcc) {
        if (dim == 3 && spill && v.n >= kPostSplitMinN) {
          // a large level: the restriction march of its b slot (the seam array
          // is free once the finest sweep's seam pass has run), which forms the
          // pointwise update on the way for hb and BPX; the additive variant,
          // whose injection also reads sf, takes the update as a pass of its own
          if (variant != MG_ADD) {
            const cpx<T> wsl = to_c<T>(wl * complex<double>(v.op.invD.re, v.op.invD.im));
            MG_HIP(launch_post3<T>(cc->n, variant, v.b, wsl, v.sc, variant == MG_BPX ? cc->si : nullptr, cc->b,
                                   spill, s));
            continue;
          }
          MG_HIP(launch_update<T>(dim, v.op, v.b, to_c<T>(wl), 0, nullptr, v.sc, v.sf, cc->sf, nullptr, s));
          MG_HIP(launch_restrict3<T>(cc->n, v.b, cc->b, spill, s));
          continue;
        }
        MG_HIP(launch_post_galerkin<T>(dim, v.op, v.b, to_c<T>(wl), variant != MG_ADD ? 1 : 0, v.sc, v.sf, cc->b,
                                       variant == MG_ADD ? cc->sf : nullptr, variant == MG_BPX ? cc->si : nullptr, s));
        continue;
      }
      if (galerkin) {
        r = v.b;
      } else {
        MG_TRY(ensure_scratch());
        if (hcc) MG_HIP(launch_uhat<T>(dim, v.n, v.u, cc->u, tA, s));
        MG_HIP(launch_resid<T>(dim, v.op, v.b, v.u, tR, nullptr, nullptr, s));
        if (hcc) MG_HIP(launch_resid<T>(dim, v.op, v.b, tA, tRh, nullptr, nullptr, s));
        r = tR;
      }
      MG_HIP(launch_update<T>(dim, v.op, r, to_c<T>(wl), (hcc && variant != MG_ADD) ? 1 : 0, nullptr, v.sc, v.sf,
                              (hcc && variant == MG_ADD) ? cc->sf : nullptr,
                              (hcc && variant == MG_BPX) ? cc->si : nullptr, s));
      if (hcc) MG_HIP(launch_restrict<T>(dim, cc->n, galerkin ? v.b : tRh, cc->b, s));
    }
    return MG_OK;
  }

  FusedArgs<T> fused_args(cpx<T>* wout, cpx<T>* rhoc, cpx<T>* sfc, cpx<T>* sic_out, double wL_re, double wL_im) {
    Level<T>& f = lv[L];
    Level<T>* c = &lv[L - 1];
    FusedArgs<T> a;
    a.n = f.n;
    a.nc = c->n;
    a.w = w[cur];
    a.wout = wout;
    a.b = f.b;
    a.scc = c->sc;
    a.sic = variant == MG_BPX ? c->si : nullptr;
    a.rhoc = rhoc;
    a.sfc = variant == MG_ADD ? sfc : nullptr;
    a.sic_out = variant == MG_BPX ? sic_out : nullptr;
    for (int q = 0; q < 4; ++q) a.coef[q] = f.op.coef[q];
    a.ws = to_c<T>(complex<double>(wL_re, wL_im) * complex<double>(f.op.invD.re, f.op.invD.im));
    a.partials = partials;
    a.variant = variant;
    a.spill = spill;
    a.tile = tile;
    a.order = 0;
    return a;
  }

  // Times every tile variant of the fused sweep (with its seam pass) on scratch
  // outputs; keeps the best.  Each timed launch follows a fill of two
  // finest-size scratch arrays, so that it starts with the caches holding
  // other data, as a sweep inside a cycle does.
  int autotune(int reps, int* best_tile, double* best_us, double* times) {
    if (!fused) return fail(MG_EINVAL, "the context has no fused sweep");
    MG_TRY(ensure_scratch());
    if (!tune_c) {
      MG_TRY(alloc_c(&tune_c, lv[L - 1].N));
    }
    Level<T>* c = &lv[L - 1];
    const int saved = tile;
    reps = std::max(reps, 1);
    std::vector<hipEvent_t> ev2(2 * (size_t)reps, nullptr);
    for (auto& e : ev2) MG_HIP(hipEventCreate(&e));
    int best = saved;
    double best_t = 1e300;
    const size_t flush_bytes = NL() * sizeof(cpx<T>);
    for (int t = 0; t < fused_tile_count(dim); ++t) {
      set_tile(t);
      FusedArgs<T> a = fused_args(tA, c->pr, tune_c, c->pz, omega.real(), omega.imag());
      MG_HIP(launch_fused<T>(dim, a, s));  // warm-up
      MG_HIP(launch_fused_seam<T>(dim, a, s));
      for (int k = 0; k < reps; ++k) {
        MG_HIP(launch_fill(tR, flush_bytes, s));
        MG_HIP(launch_fill(tRh, flush_bytes, s));
        MG_HIP(hipEventRecord(ev2[2 * k], s));
        MG_HIP(launch_fused<T>(dim, a, s));
        MG_HIP(launch_fused_seam<T>(dim, a, s));
        MG_HIP(hipEventRecord(ev2[2 * k + 1], s));
      }
      MG_HIP(hipEventSynchronize(ev2[2 * reps - 1]));
      double total = 0;
      for (int k = 0; k < reps; ++k) {
        float ms = 0;
        MG_HIP(hipEventElapsedTime(&ms, ev2[2 * k], ev2[2 * k + 1]));
        total += ms;
      }
      const double us = 1e3 * total / reps;
      if (times) times[t] = us;
      if (us < best_t) {
        best_t = us;
        best = t;
      }
    }
    for (auto& e : ev2) (void)hipEventDestroy(e);
    set_tile(best);
    if (best_tile) *best_tile = best;
    if (best_us) *best_us = best_t;
    return MG_OK;
  }

  // ||r||_h of cycle k from the history (host, after sync).
  double hnorm_scale() const { return std::pow(3.0, -L * dim); }

  int cycles(int ncycles, double* res_h, double* res_max) {
    MG_TRY(ensure_hist(ncycles));
    for (int k = 0; k < ncycles; ++k) MG_TRY(cycle_once(k, k + 1 < ncycles));
    if (res_h || res_max) {
      std::vector<double> h(2 * (size_t)ncycles);
      MG_HIP(hipMemcpyAsync(h.data(), hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < ncycles; ++k) {
        if (res_h) res_h[k] = std::sqrt(hnorm_scale() * h[2 * k]);
        if (res_max) res_max[k] = h[2 * k + 1];
      }
    }
    return MG_OK;
  }

  int flush(cpx<T>* u_out_T) {
    MG_TRY(pre_coarse());
    const bool hc = L > lmin;
    Level<T>* c = hc ? &lv[L - 1] : nullptr;
    MG_HIP(launch_fine_pre<T>(dim, lv[L].n, w[cur], w[1 - cur], hc ? c->sc : nullptr, hc ? c->si : nullptr,
                              hc ? 1 : 0, variant == MG_BPX ? 1 : 0, s));
    cur = 1 - cur;
    MG_TRY(zero_helpers());
    if (u_out_T) MG_HIP(hipMemcpyAsync(u_out_T, w[cur], NL() * sizeof(cpx<T>), hipMemcpyDeviceToDevice, s));
    return MG_OK;
  }

  const cpx<T>* field(int level, int f) const {
    const Level<T>& v = lv[level];
    if (level == L) {
      if (f == MG_FIELD_U) return w[cur];
      if (f == MG_FIELD_B) return v.b;
      return nullptr;
    }
    switch (f) {
      case MG_FIELD_U: return coarse_u(level);
      case MG_FIELD_B: return v.b;
      case MG_FIELD_SC: return v.sc;
      case MG_FIELD_SF: return v.sf;
      default: return v.si;
    }
  }

  // z = B v (zero-start cycle); v, z finest-size T buffers.  v's boundary is
  // ignored, unless `clean` promises it is zero already (then v is read in place).
  // Zero-start cycle below the finest level: the restriction chain of rhoL
  // and the coarse levels l_min .. L-1; *gc receives the coarse correction
  // the finest level prolongs (z_(L-1), or z_(L-1) - I s_L for BPX).
  // With s_r != nullptr (the restriction march only), rhoL is first formed as
  // s_r - s_alpha s_v inside the finest restriction, and |rhoL|^2 per block
  // goes to s_part.
  int precondition_coarse(const cpx<T>* rhoL, const cpx<T>** gc, const cpx<T>* s_r = nullptr,
                          const cpx<T>* s_v = nullptr, cpx<double> s_alpha = cpx<double>(), double* s_part = nullptr) {
    const int it = 1;
    for (int l = L; l > lmin; --l) {
      const cpx<T>* src = l == L ? rhoL : lv[l].pr;
      // the finest restriction moves most of the bytes: in 3D it takes the
      // sweep's march (the seam array is free outside the fused sweep)
      if (l == L && s_r)
        MG_HIP(launch_restrict3_s<T>(lv[l - 1].n, s_r, s_v, s_alpha, const_cast<cpx<T>*>(rhoL), lv[l - 1].pr, spill,
                                     s_part, s));
      else if (l == L && dim == 3 && spill && lv[L].n >= 10)
        MG_HIP(launch_restrict3<T>(lv[l - 1].n, src, lv[l - 1].pr, spill, s));
      else
        MG_HIP(launch_restrict<T>(dim, lv[l - 1].n, src, lv[l - 1].pr, s));
    }
    *gc = nullptr;
    for (int l = lmin; l <= L; ++l) {
      const complex<double> wl = omega_level(scheme, omega, omega_L, L - l, it);
      const cpx<T>* rho = l == L ? rhoL : lv[l].pr;
      const cpx<T>* g = nullptr;
      if (l > lmin) {
        g = lv[l - 1].pz;
        if (variant == MG_BPX) {
          // rho_(l-1) (in pr) has been used by now: it holds g
          MG_HIP(launch_prec_g<T>(dim, lv[l].op, rho, to_c<T>(wl), lv[l - 1].pz, lv[l - 1].pr, s));
          g = lv[l - 1].pr;
        }
      }
      if (l == L) {
        *gc = g;
        break;
      }
      MG_HIP(launch_prec_up<T>(dim, lv[l].op, rho, to_c<T>(wl), variant == MG_HB ? 1 : 0, l == lmin ? 1 : 0, g,
                               lv[l].pz, s));
    }
    return MG_OK;
  }

  int precondition(const cpx<T>* v, cpx<T>* z, bool clean = false) {
    const cpx<T>* rhoL = v;
    if (!clean) {
      MG_TRY(ensure_scratch());
      MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, v, tR, mk(T(1), T(0)), s));
      rhoL = tR;
    }
    const cpx<T>* gc = nullptr;
    MG_TRY(precondition_coarse(rhoL, &gc));
    const complex<double> wL = omega_level(scheme, omega, omega_L, 0, 1);
    MG_HIP(launch_prec_up<T>(dim, lv[L].op, rhoL, to_c<T>(wL), variant == MG_HB ? 1 : 0, L == lmin ? 1 : 0, gc, z, s));
    return MG_OK;
  }

  // As precondition_apply for a v whose boundary entries may be nonzero.
  int precondition_apply_any(const cpx<T>* v, cpx<T>* z, cpx<T>* y) {
    MG_TRY(ensure_scratch());
    MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, v, tR, mk(T(1), T(0)), s));
    return precondition_apply(tR, z, y);
  }

  // The Krylov step's finest passes run as marches in 3D with constant phi;
  // their per-tile partials (3 per block of the preconditioner-apply march,
  // then 1 per block of the restriction march) must fit the partials buffer.
  bool krylov_marches() const {
    if (dim != 3 || varying || L == lmin || lv[L].n < 10 || !spill) return false;
    const size_t need = 3 * (size_t)prec_apply3_blocks(lv[L].n) + (size_t)restrict3_blocks(lv[L - 1].n);
    return need <= partials_doubles;
  }
  size_t s_partials_offset() const { return 3 * (size_t)prec_apply3_blocks(lv[L].n); }

  // z = M^-1 v (v with zero boundary) and y = H z.  In 3D with constant phi
  // the finest level of M^-1 and the operator run as one march.  dot 1 also
  // returns h[0..1] = conj(v2) y, dot 2 h[0..2] = conj(y) v2 and |y|^2 (both
  // synchronise; in the march they are summed on the fly).
  int precondition_apply(const cpx<T>* v, cpx<T>* z, cpx<T>* y, int dot = 0, const cpx<T>* v2 = nullptr,
                         double* h = nullptr) {
    MG_TRY(precondition_apply_enqueue(v, z, y, dot, v2));
    if (dot) {
      MG_HIP(hipMemcpyAsync(h, red, (dot == 1 ? 2 : 3) * sizeof(double), hipMemcpyDeviceToHost, s));
      MG_HIP(hipStreamSynchronize(s));
    }
    return MG_OK;
  }

  // The same without synchronising: the dots stay in red[0..2] on the device.
  int precondition_apply_enqueue(const cpx<T>* v, cpx<T>* z, cpx<T>* y, int dot, const cpx<T>* v2) {
    if (!krylov_marches()) {
      MG_TRY(precondition(v, z, true));
      MG_HIP(launch_apply<T>(dim, lv[L].op, z, y, s));
      if (dot == 1) {
        MG_HIP(launch_dot<T>(NL(), v2, y, partials, s));
        MG_HIP(launch_finish_sum2(partials, kRedBlocks, red, s));
      } else if (dot == 2) {
        MG_HIP(launch_bicg_ts<T>(NL(), y, v2, partials, s));
        MG_HIP(launch_finishN(3, partials, kRedBlocks, red, s));
      }
    } else {
      const cpx<T>* gc = nullptr;
      MG_TRY(precondition_coarse(v, &gc));
      MG_TRY(finest_prec_apply(v, gc, z, y, dot, v2));
    }
    return MG_OK;
  }

  int finest_prec_apply(const cpx<T>* v, const cpx<T>* gc, cpx<T>* z, cpx<T>* y, int dot, const cpx<T>* v2) {
    const complex<double> wL = omega_level(scheme, omega, omega_L, 0, 1);
    const Level<T>& f = lv[L];
    const cpx<T> ws = to_c<T>(wL * complex<double>(f.op.invD.re, f.op.invD.im));
    MG_HIP(launch_prec_apply3<T>(f.n, f.op.coef, ws, variant == MG_HB ? 1 : 0, v, gc, z, y, dot, v2, partials, s));
    const int nb = prec_apply3_blocks(f.n);
    if (dot == 1) MG_HIP(launch_finish_sum2(partials, nb, red, s));
    else if (dot == 2) MG_HIP(launch_finishN(3, partials, nb, red, s));
    return MG_OK;
  }

  // The second half-step of BiCGStab: sv = r - alpha v, z = M^-1 sv, t = H z;
  // h[0] = |sv|^2, h[1..2] = conj(t) sv, h[3] = |t|^2 (synchronises).  With
  // the marches, sv is formed inside the finest restriction.
  int s_half_step(const cpx<T>* r, const cpx<T>* v, complex<double> alpha, cpx<T>* sv, cpx<T>* z, cpx<T>* t,
                  double* h) {
    if (!krylov_marches()) {
      MG_HIP(launch_bicg_s<T>(NL(), r, v, to_c<double>(alpha), sv, partials, s));
      MG_TRY(finish(1, h));
      if (std::sqrt(h[0]) == 0.0) return MG_OK;   // the caller stops at s
      return precondition_apply(sv, z, t, 2, sv, h + 1);
    }
    double* ps = partials + s_partials_offset();
    const cpx<T>* gc = nullptr;
    MG_TRY(precondition_coarse(sv, &gc, r, v, to_c<double>(alpha), ps));
    MG_TRY(finest_prec_apply(sv, gc, z, t, 2, sv));
    MG_HIP(launch_finishN(1, ps, restrict3_blocks(lv[L - 1].n), red + 3, s));
    double q[4];
    MG_HIP(hipMemcpyAsync(q, red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    h[0] = q[3];
    h[1] = q[0];
    h[2] = q[1];
    h[3] = q[2];
    return MG_OK;
  }

  int dot(const cpx<T>* a, const cpx<T>* b, complex<double>* out) {
    MG_HIP(launch_dot<T>(NL(), a, b, partials, s));
    MG_HIP(launch_finish_sum2(partials, kRedBlocks, red, s));
    double h[2];
    MG_HIP(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    *out = complex<double>(h[0], h[1]);
    return MG_OK;
  }

  int norm2(const cpx<T>* a, double* out) {
    MG_HIP(launch_norm2<T>(NL(), a, partials, s));
    MG_HIP(launch_finish_sum_max(partials, kRedBlocks, red, s));
    double h[2];
    MG_HIP(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    *out = std::sqrt(h[0]);
    return MG_OK;
  }

  // Reduced values of a fused Krylov kernel (nvals sums over kRedBlocks blocks).
  int finish(int nvals, double* h) {
    MG_HIP(launch_finishN(nvals, partials, kRedBlocks, red, s));
    MG_HIP(hipMemcpyAsync(h, red, nvals * sizeof(double), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    return MG_OK;
  }

  // Right-preconditioned BiCGStab (van der Vorst) on H x = b, T-precision vectors,
  // FP64 scalars.  b, x finest-size T buffers (x: initial guess in, result out).
  // Per iteration: two zero-start cycles, two operator applications and four
  // fused vector passes, each returning its scalars to the host.
  int bicgstab(const cpx<T>* b_in, cpx<T>* x, double rtol, int maxit, int* its, double* relres) {
    MG_TRY(ensure_krylov());
    MG_TRY(ensure_scratch());
    cpx<T>*r = kv[0], *rh = kv[1], *p = kv[2], *v = kv[3], *sv = kv[4], *t = kv[5], *y = kv[6], *z = kv[7];
    const size_t N = NL();
    const OpData<T>& op = lv[L].op;
    cpx<T>* b = tRh;  // boundary-cleaned copy of b
    MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, b_in, b, mk(T(1), T(0)), s));
    MG_HIP(launch_zero_boundary_copy<T>(dim, lv[L].n, x, x, mk(T(1), T(0)), s));
    double bnorm;
    MG_TRY(norm2(b, &bnorm));
    if (bnorm == 0.0) {
      MG_HIP(launch_fill(x, N * sizeof(cpx<T>), s));
      if (its) *its = 0;
      if (relres) *relres = 0.0;
      return MG_OK;
    }
    MG_HIP(launch_resid<T>(dim, op, b, x, r, nullptr, nullptr, s));
    MG_HIP(hipMemcpyAsync(rh, r, N * sizeof(cpx<T>), hipMemcpyDeviceToDevice, s));
    MG_HIP(launch_fill(p, N * sizeof(cpx<T>), s));
    MG_HIP(launch_fill(v, N * sizeof(cpx<T>), s));
    complex<double> rho = 1.0, alpha = 1.0, om = 1.0;
    double rn;
    MG_TRY(norm2(r, &rn));
    complex<double> rho_new = rn * rn;   // (rh, r) with rh = r
    double rel = rn / bnorm;
    const double r0 = rel;
    int it = 0;
    int status = MG_ENOTCONV;
    if (rel <= rtol) status = MG_OK;
    const bool met_at_start = status == MG_OK;
    double h[3];
    for (it = 1; it <= maxit && status == MG_ENOTCONV; ++it) {
      const complex<double> beta = (rho_new / rho) * (alpha / om);
      MG_HIP(launch_bicg_p<T>(N, r, v, to_c<double>(beta), to_c<double>(om), p, s));
      // y = M^-1 p, v = H y and (rh, v)
      MG_TRY(precondition_apply(p, y, v, 1, rh, h));
      alpha = rho_new / complex<double>(h[0], h[1]);
      // s = r - alpha v and |s|, z = M^-1 s, t = H z, (t, s) and |t|^2
      double h4[4];
      MG_TRY(s_half_step(r, v, alpha, sv, z, t, h4));
      const double sn = std::sqrt(h4[0]);
      if (sn / bnorm <= rtol) {
        MG_HIP(launch_axpby<T>(N, to_c<double>(alpha), y, mk(1.0, 0.0), x, s));
        rel = sn / bnorm;
        status = MG_OK;
        break;
      }
      om = complex<double>(h4[1], h4[2]) / h4[3];
      // x += alpha y + om z; r = s - om t; |r| and (rh, r) for the next step
      MG_HIP(launch_bicg_xr2<T>(N, x, y, z, to_c<double>(alpha), to_c<double>(om), r, sv, t, rh, partials, s));
      MG_TRY(finish(3, h));
      rho = rho_new;
      rho_new = complex<double>(h[1], h[2]);
      rn = std::sqrt(h[0]);
      rel = rn / bnorm;
      if (!std::isfinite(rel) || rel > 1e8 * std::max(r0, 1e-300)) {
        status = MG_EDIVERGED;
        break;
      }
      if (rel <= rtol) {
        status = MG_OK;
        break;
      }
    }
    if (its) *its = met_at_start ? 0 : std::min(it, maxit);
    if (relres) *relres = rel;
    return status;
  }

  // Residual h-norm of (u, b) on the finest level: ||b - H u||_h.
  int resid_norm(const cpx<T>* u, const cpx<T>* b, double* res_h, double* res_max) {
    MG_TRY(ensure_scratch());
    int np = 0;
    MG_HIP(launch_resid<T>(dim, lv[L].op, b, u, tA, partials, &np, s));
    MG_HIP(launch_finish_sum_max(partials, np, red, s));
    double h[2];
    MG_HIP(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (res_h) *res_h = std::sqrt(hnorm_scale() * h[0]);
    if (res_max) *res_max = h[1];
    return MG_OK;
  }

  // Stationary driver (the paper's iteration, one cycle per traversal).  Cycle
  // n reports the residual of iterate n - 1; the driver stops after the first
  // cycle whose reported residual meets ||r||_h <= rtol ||b||_h, or at maxit,
  // then flushes, so u holds the iterate after the cycles run (one beyond the
  // one that met the target) and *its their count.  Status: MG_EDIVERGED on a
  // non-finite residual or one above 1e8 times the first; otherwise MG_OK
  // when the returned iterate's own residual meets rtol, MG_ENOTCONV when it
  // does not (maxit reached, or the last cycle moved away from the target).
  int stationary(const cpx<T>* b, cpx<T>* u, double rtol, int maxit, int* its, double* relres) {
    MG_TRY(set_rhs(b));
    MG_TRY(set_solution(u));
    double bh;
    {
      MG_TRY(ensure_scratch());
      MG_HIP(launch_fill(tRh, NL() * sizeof(cpx<T>), s));
      MG_TRY(resid_norm(tRh, lv[L].b, &bh, nullptr));
    }
    if (bh == 0.0) {
      MG_HIP(launch_fill(u, NL() * sizeof(cpx<T>), s));
      if (its) *its = 0;
      if (relres) *relres = 0;
      return MG_OK;
    }
    int done = 0;
    bool diverged = false;
    double r0 = -1;
    while (done < maxit) {
      double rh;
      MG_TRY(cycles(1, &rh, nullptr));
      ++done;
      if (r0 < 0) r0 = rh;
      if (!std::isfinite(rh) || rh > 1e8 * r0) {
        diverged = true;
        break;
      }
      if (rh / bh <= rtol) break;
    }
    MG_TRY(flush(u));
    double fin;
    MG_TRY(resid_norm(u, lv[L].b, &fin, nullptr));
    if (its) *its = done;
    if (relres) *relres = fin / bh;
    if (diverged || !std::isfinite(fin)) return MG_EDIVERGED;
    return fin / bh <= rtol ? MG_OK : MG_ENOTCONV;
  }
};

}  // namespace mg

using namespace mg;

struct mg_ctx {
  mg_params p;
  hipStream_t s = nullptr;
  int device = 0;                 // the device current at setup (the stream's)
  Engine<double>* e64 = nullptr;  // FP64 engine (precision FP64) or FP64 finest operator holder
  Engine<float>* e32 = nullptr;   // complex64 corrections (precision FP32_REFINE)
  cpx<double>* phi64 = nullptr;   // copy of the nodal phi field (FP64 operator with FP32 engine)
  std::vector<void*> owned;
  // FP64 finest operator and scratch for the refinement loop
  OpData<double> op64;
  cpx<double>*r64 = nullptr, *b64 = nullptr;
  cpx<float>*r32 = nullptr, *e32v = nullptr;
  // nested solves: a context per coarser level (level_max = l) with its load,
  // rhs and solution buffers, made on first use and kept
  struct Nested {
    mg_ctx* ctx = nullptr;
    mg_c128 *chi = nullptr, *b = nullptr, *u = nullptr;
  };
  std::vector<Nested> nested;
  mg_c128* nested_b = nullptr;    // finest rhs of a nested solve
  ~mg_ctx();
};

