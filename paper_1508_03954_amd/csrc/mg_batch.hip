// Batched form: many independent problems (right-hand sides, wavenumbers,
// dimensions and grid depths) advanced by one pipelined cycle each in ONE
// persistent kernel launch.
//
// Work items are (problem, phase, tile).  The phases of one problem's cycle
// are its coarse pre-phases (levels l_min .. L-1), the fused finest sweep (in
// 3D followed by the seam rows of its restriction), the coarse Galerkin post-phases (levels L-1 .. l_min+1), the coarsest update and
// the residual-norm reduction; each phase depends on all tiles of the
// previous phase of the same problem and on nothing else.  A resident grid of
// workgroups pulls items from an atomic queue ordered so that every item comes
// after the items it waits for, so the waits always end: a waiting workgroup
// only waits for items claimed earlier by workgroups that are resident and
// whose own waits point further back.  Completion is published per
// (problem, phase) with an agent-scope release, one write-back of the XCD's L2
// per item; waiters poll with relaxed loads and acquire at agent scope (each
// XCD has its own L2) once per dependency and workgroup.  Every wait is
// bounded; a timeout sets an error flag and the kernel still drains.
//
// The per-vertex and per-tile code is the same as in the single-problem
// kernels (mg_level_ops.h, mg_fused_ops.h), so a problem advanced in a batch
// ends in the same state as the same problem advanced alone with the same tile.
#include <array>

#include "mg_engine.h"
#include "mg_fused_ops.h"
#include "mg_level_ops.h"

namespace mg {

enum BatchKind { BK_PRE = 0, BK_FUSED3 = 1, BK_FUSED2 = 2, BK_POST = 3, BK_UPDATE = 4, BK_NORM = 5, BK_SEAM = 6 };
constexpr int kBMaxPhases = 16;
constexpr int kBMaxLevels = 8;
constexpr int kBWaves = 3;
constexpr int kBThreads = 64 * kBWaves;
// rows of a coarse level per item, 8 per wavefront: every item publishes with
// a write-back of its XCD's L2, so items this size ran the 96-problem cycle
// faster than 4 (7 %), 16 (2 %) or 32 (12 %) rows per wavefront
constexpr int kBRows = 8 * kBWaves;
// 3D tiles of a 3-wave workgroup: coarse rows 2, rows per thread 2; z extent
// selectable.  2D: one tile per wavefront, three per item.
constexpr int kBZc3[] = {9, 3};
constexpr int kBZc2[] = {1, 2, 4, 8};
// configurations: z extent (3D) x z extent (2D) x queue order
constexpr int kBatchConfigs = 2 * 4 * 2;

template <class T>
struct BLevel {
  int n;
  cpx<T>*u, *b, *sc, *sf, *si;
  OpData<T> op;
  cpx<T> omega;
};

template <class T>
struct BProb {
  int dim, L, lmin, variant, nphase;
  int zc3, zc2;                     // indices into kBZc3 / kBZc2
  int ftiles;                       // fused tiles of the finest sweep
  int fgx, fgy;                     // fused tile grid extents (x, y)
  int parw, pars;                   // ping-pong parity of w and of si at level L-1 at launch 0
  int phase_items[kBMaxPhases];
  int phase_kind[kBMaxPhases];
  int phase_level[kBMaxPhases];
  BLevel<T> lv[kBMaxLevels];
  cpx<T>* w[2];
  cpx<T>* si2[2];
  cpx<T>* spill;                    // seam rows of the 3D sweep's restriction
  cpx<T> wsL;
  double* part;
};

struct BItem {
  int prob, phase, tile;
};

template <class T>
struct BatchArgs {
  const BItem* items;
  int nitems;
  const BProb<T>* probs;
  int* done;        // [nprob][kBMaxPhases]
  int* queue;
  int* err;
  double* hist;     // [nprob][2] of this cycle
  int cyc;          // cycle index within the call (flips the ping-pong parity)
  unsigned spin_limit;
  unsigned long long* trace;  // per item: claim-to-ready wait start, ready, done (wall clock), XCD << 16 | block; or null
};

__device__ inline unsigned xcc_id() {
  unsigned x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & 0xf;
}

// Coarse-level row items: wave w handles rows tile*kBRows + w + kBWaves k.
template <class T, int D, class F>
__device__ inline void for_rows(int n, int tile, F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nrows = D == 3 ? n * n : n;
  for (int k = 0; k < kBRows / kBWaves; ++k) {
    const int row = tile * kBRows + wv + kBWaves * k;
    if (row >= nrows) break;
    for (int x = lane; x < n; x += 64) {
      int j[3];
      long long i;
      row_vertex<D>(row, x, n, j, i);
      f(j, i);
    }
  }
}

// Wave-uniform copies of values read from a problem descriptor.  The
// descriptors are read with vector loads (the kernel also writes global
// memory, so the scalar cache may not be used for them), which leaves every
// field in vector registers; readfirstlane moves them to scalar registers,
// where the sweep's per-plane address arithmetic and constants belong.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class P>
__device__ inline P* uni(P* p) {
  const unsigned long long b = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return reinterpret_cast<P*>(((unsigned long long)hi << 32) | lo);
}
__device__ inline float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline double uni(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class T>
__device__ inline cpx<T> uni(cpx<T> c) { return mk(uni(c.re), uni(c.im)); }

template <class T>
__device__ inline FusedArgs<T> batch_fused_args(const BProb<T>& P, int cyc) {
  const int L = uni(P.L);
  const int variant = uni(P.variant);
  const bool bpx = variant == MG_BPX, add = variant == MG_ADD;
  const int pw = (uni(P.parw) + cyc) & 1, ps = (uni(P.pars) + cyc) & 1;
  FusedArgs<T> f;
  f.n = uni(P.lv[L].n);
  f.nc = uni(P.lv[L - 1].n);
  f.w = uni(P.w[pw]);
  f.wout = uni(P.w[1 - pw]);
  f.b = uni(P.lv[L].b);
  f.scc = uni(P.lv[L - 1].sc);
  f.sic = bpx ? uni(P.si2[ps]) : nullptr;
  f.rhoc = uni(P.lv[L - 1].b);
  f.sfc = add ? uni(P.lv[L - 1].sf) : nullptr;
  f.sic_out = bpx ? uni(P.si2[1 - ps]) : nullptr;
  f.spill = uni(P.spill);
  for (int q = 0; q < 4; ++q) f.coef[q] = uni(P.lv[L].op.coef[q]);
  f.ws = uni(P.wsL);
  f.partials = nullptr;
  f.variant = variant;
  f.tile = 0;
  f.order = 0;
  return f;
}

template <class T>
__device__ inline void batch_fused3(const BProb<T>* Pp, int cyc, int tile, F3Lds<T, 2, 2, true>& sm) {
  const BProb<T>& P = *Pp;
  const FusedArgs<T> f = batch_fused_args(P, cyc);
  const bool bpx = P.variant == MG_BPX;
  const int bx = tile % P.fgx, by = (tile / P.fgx) % P.fgy, bz = tile / (P.fgx * P.fgy);
  double* part = P.part + 2 * tile;
  // the non-BPX layout is a prefix of the BPX one
  auto& sm0 = reinterpret_cast<F3Lds<T, 2, 2, false>&>(sm);
  const bool add = P.variant == MG_ADD;
  if (P.zc3 == 0) {
    if (bpx) fused3_tile<T, 2, 2, 9, 2>(f, bx, by, bz, part, sm);
    else if (add) fused3_tile<T, 2, 2, 9, 0>(f, bx, by, bz, part, sm0);
    else fused3_tile<T, 2, 2, 9, 1>(f, bx, by, bz, part, sm0);
  } else {
    if (bpx) fused3_tile<T, 2, 2, 3, 2>(f, bx, by, bz, part, sm);
    else if (add) fused3_tile<T, 2, 2, 3, 0>(f, bx, by, bz, part, sm0);
    else fused3_tile<T, 2, 2, 3, 1>(f, bx, by, bz, part, sm0);
  }
}

template <class T>
__device__ inline void batch_fused2(const BProb<T>* Pp, int cyc, int id, cpx<T> (*Gz)[F2_GX],
                                          cpx<T> (*Sz)[F2_GX]) {
  const BProb<T>& P = *Pp;
  const FusedArgs<T> f = batch_fused_args(P, cyc);
  const bool bpx = P.variant == MG_BPX;
  const int bx = id % P.fgx, by = id / P.fgx;
  double* part = P.part + 2 * id;
  switch (P.zc2) {
    case 0:
      if (bpx) fused2_wave_tile<T, 1, true>(f, bx, by, Gz, Sz, part);
      else fused2_wave_tile<T, 1, false>(f, bx, by, Gz, Sz, part);
      break;
    case 1:
      if (bpx) fused2_wave_tile<T, 2, true>(f, bx, by, Gz, Sz, part);
      else fused2_wave_tile<T, 2, false>(f, bx, by, Gz, Sz, part);
      break;
    case 2:
      if (bpx) fused2_wave_tile<T, 4, true>(f, bx, by, Gz, Sz, part);
      else fused2_wave_tile<T, 4, false>(f, bx, by, Gz, Sz, part);
      break;
    default:
      if (bpx) fused2_wave_tile<T, 8, true>(f, bx, by, Gz, Sz, part);
      else fused2_wave_tile<T, 8, false>(f, bx, by, Gz, Sz, part);
      break;
  }
}

// Inlined on purpose: as a called function (its default for the 3D instance)
// it received the kernel arguments through scratch memory and saved registers
// there, and its items ran 2-5x slower.
template <class T, int D>
__device__ __attribute__((always_inline)) inline void batch_item(const BatchArgs<T>& A, const BProb<T>& P, int prob,
                                                                 int phase, int tile,
                           cpx<T> (*Gz2)[2][F2_GX], cpx<T> (*Sz2)[2][F2_GX], F3Lds<T, 2, 2, true>* f3lds) {
  const int kind = P.phase_kind[phase], lev = P.phase_level[phase];
  const bool bpx = P.variant == MG_BPX, add = P.variant == MG_ADD;
  if (kind == BK_PRE) {
    const BLevel<T>& v = P.lv[lev];
    const bool hc = lev > P.lmin;
    const cpx<T>* scc = hc ? P.lv[lev - 1].sc : nullptr;
    const cpx<T>* sic = hc ? P.lv[lev - 1].si : nullptr;
    for_rows<T, D>(v.n, tile, [&](const int j[3], long long i) {
      pre_vertex<T, D>(v.n, j, i, v.u, v.sc, v.sf, scc, sic, hc ? 1 : 0, bpx ? 1 : 0);
    });
  } else if (kind == BK_POST) {
    const BLevel<T>& v = P.lv[lev];
    const BLevel<T>& c = P.lv[lev - 1];
    for_rows<T, D>(c.n, tile, [&](const int m[3], long long ic) {
      post_galerkin_vertex<T, D>(v.op, m, ic, v.b, v.omega, add ? 0 : 1, v.sc, v.sf, c.b, add ? c.sf : nullptr,
                                 bpx ? c.si : nullptr);
    });
  } else if (kind == BK_UPDATE) {
    const BLevel<T>& v = P.lv[lev];
    for_rows<T, D>(v.n, tile, [&](const int j[3], long long i) {
      update_vertex<T, D>(v.op, j, i, v.b, v.omega, 0, nullptr, v.sc, v.sf, nullptr, nullptr);
    });
  } else if (kind == BK_SEAM) {
    // rho_c += the seam rows of the 3D restriction (rows (s + 1) 2 of each coarse plane)
    const BLevel<T>& c = P.lv[P.L - 1];
    const int nc = c.n, nseam = P.fgy - 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < kBRows / kBWaves; ++k) {
      const int row = tile * kBRows + wv + kBWaves * k;
      if (row >= nc * nseam) break;
      const int mz = row / nseam, sidx = row - mz * nseam, my = 2 * (sidx + 1);
      if (mz < 1 || mz > nc - 2 || my > nc - 2) continue;
      for (int mx = lane; mx < nc; mx += 64) {
        if (mx < 1 || mx > nc - 2) continue;
        cpx<T>& d = c.b[((long long)mz * nc + my) * nc + mx];
        const cpx<T> e = P.spill[((long long)mz * nc + my) * nc + mx];
        d = mk(d.re + e.re, d.im + e.im);
      }
    }
  } else if (kind == BK_NORM) {
    // the fixed-order second stage of the single-problem path (a tree over
    // 256 entries, the last 64 zero)
    __shared__ double s0[256], s1[256];
    const int t = threadIdx.x;
    double a = 0, b = 0;
    for (int i = t; i < P.ftiles; i += kBThreads) {
      a += P.part[2 * i];
      b = fmax(b, P.part[2 * i + 1]);
    }
    s0[t] = a;
    s1[t] = b;
    if (t < 256 - kBThreads) {
      s0[kBThreads + t] = 0.0;
      s1[kBThreads + t] = 0.0;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        s0[t] += s0[t + w];
        s1[t] = fmax(s1[t], s1[t + w]);
      }
      __syncthreads();
    }
    if (t == 0) {
      A.hist[2 * prob] = s0[0];
      A.hist[2 * prob + 1] = s1[0];
    }
  } else {
    if (kind == BK_FUSED3) {
      if (D == 3) batch_fused3<T>(&P, A.cyc, tile, *f3lds);
    } else if (D == 2) {
      const int wv = threadIdx.x >> 6;
      const int id = kBWaves * tile + wv;
      if (id < P.ftiles) batch_fused2<T>(&P, A.cyc, id, Gz2[wv], Sz2[wv]);
    }
  }
}

// Occupancy hints by precision, chosen on the compiler's output with every
// item type inlined into the kernel: complex128 takes 227 registers (2 waves
// per SIMD; a hint of 3 fitted 168 but spilled 352 bytes per lane to
// scratch), complex64 165 (3 waves per SIMD).
template <class T>
constexpr int kBatchWavesHint = 2;

template <class T>
__global__ __launch_bounds__(kBThreads, kBatchWavesHint<T>) void k_batch_cycle(BatchArgs<T> A) {
  __shared__ int s_item, s_ok, s_acq;
  int acq_prob = -1, acq_phase = -1;  // thread 0: the dependency this workgroup last acquired
  __shared__ cpx<T> Gz2[kBWaves][2][F2_GX];
  __shared__ cpx<T> Sz2[kBWaves][2][F2_GX];
  __shared__ F3Lds<T, 2, 2, true> f3lds;
  // Thread 0 claims items and publishes completions; every step it takes is
  // followed by a workgroup barrier before any other thread depends on it, and
  // the loop exit is decided on a value every thread reads after a barrier.
  // (Keeping "publish" and "claim" in one block before one barrier also keeps
  // the loop's back edge uniform: no lane may take a different path around it.)
  if (threadIdx.x == 0) s_item = atomicAdd(A.queue, 1);
  __syncthreads();
  for (;;) {
    // item indices are uniform over the workgroup: keep them (and every
    // descriptor field read through them) in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= A.nitems) break;
    BItem w = A.items[it];
    w.prob = __builtin_amdgcn_readfirstlane(w.prob);
    w.phase = __builtin_amdgcn_readfirstlane(w.phase);
    w.tile = __builtin_amdgcn_readfirstlane(w.tile);
    const BProb<T>& P = A.probs[w.prob];
    unsigned long long t_wait = 0, t_ready = 0;
    if (threadIdx.x == 0) {
      if (A.trace) t_wait = wall_clock64();
      int ok = 1, acq = 0;
      // phase 0 depends on the previous launch only; a dependency this
      // workgroup has already waited for and acquired needs neither again
      // (completion counts only grow, and an acquire invalidates caches
      // under every item running on the XCD)
      if (w.phase > 0 && (w.prob != acq_prob || w.phase != acq_phase)) {
        acq = 1;
        const int need = P.phase_items[w.phase - 1];
        int* cnt = A.done + w.prob * kBMaxPhases + w.phase - 1;
        unsigned spins = 0;
        // relaxed polling: an acquiring load would invalidate caches on every
        // poll, under the items other workgroups are running; the acquire is
        // the fence after the barrier below
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++spins > A.spin_limit) {
            ok = 0;
            atomicOr(A.err, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (ok) {
          acq_prob = w.prob;
          acq_phase = w.phase;
        }
      }
      s_ok = ok;
      s_acq = acq;
      if (A.trace) t_ready = wall_clock64();
    }
    __syncthreads();
    if (s_acq) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (s_ok) {
      if (P.dim == 3) batch_item<T, 3>(A, P, w.prob, w.phase, w.tile, Gz2, Sz2, &f3lds);
      else batch_item<T, 2>(A, P, w.prob, w.phase, w.tile, Gz2, Sz2, &f3lds);
    }
    // Publication: every wave waits until its stores have reached the L2,
    // then thread 0's releasing add writes the XCD's L2 back once for the
    // whole workgroup (a release fence in every wave would write it back once
    // per wave).
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      if (A.trace) {
        unsigned long long* t = A.trace + 4 * (size_t)it;
        t[0] = t_wait;
        t[1] = t_ready;
        t[2] = wall_clock64();
        t[3] = ((unsigned long long)xcc_id() << 16) | blockIdx.x;
      }
      __hip_atomic_fetch_add(A.done + w.prob * kBMaxPhases + w.phase, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(A.queue, 1);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batched Krylov solve.  BiCGStab advances every problem of the batch in
// lockstep.  Per iteration each of the two preconditioner applications,
// with the operator on its result and the dot products of the step, runs for
// every problem in one persistent launch (k_batch_prec), and each vector
// update of every problem in one plain launch (k_batch_vec).  The
// preconditioner is one additive cycle from a zero start, the operator of
// Engine::precondition: the restriction chain down to level l_min, then
// z_l = Lop(omega_l D_l^-1 rho_l) + P g going up (BPX: g = z_(l-1) - I s_l),
// and on the finest level z and y = H z.  Items and waits work as in the
// cycle kernel: a problem's phase depends on all items of its previous phase.

enum PrecKind { PK_R3 = 0, PK_SEAM = 1, PK_R = 2, PK_UP = 3, PK_G = 4, PK_PA3 = 5, PK_APPLY = 6, PK_DOT = 7 };
constexpr int kPMaxPhases = 24;

template <class T>
struct PProb {
  int dim, L, lmin, variant, nphase, zc3, fgx, fgy, ftiles, nslots, nslots_cap;
  int phase_items[kPMaxPhases];
  int phase_kind[kPMaxPhases];
  int phase_level[kPMaxPhases];
  OpData<T> op[kBMaxLevels];
  cpx<T> omega[kBMaxLevels];   // omega_l of a zero-start cycle (the scheme at n = 1)
  cpx<T>* pr[kBMaxLevels];     // coarse rho, then g (BPX)
  cpx<T>* pz[kBMaxLevels];     // coarse z
  cpx<T>* spill;               // seam rows of the 3D finest restriction
  cpx<T> wsL;                  // omega_L / D_L
  double* part;                // 3 dot partials per slot (finest tile in 3D, apply item in 2D)
};

// Per problem and call: input v, outputs z = B v and y = H z, the partner v2
// of the dots and where their sums go; inactive problems' items do nothing.
template <class T>
struct PIO {
  const cpx<T>* v;
  cpx<T>* z;
  cpx<T>* y;
  const cpx<T>* v2;
  double* out;
  int active;
};

template <class T>
struct PrecArgs {
  const BItem* items;
  int nitems;
  const PProb<T>* probs;
  const PIO<T>* io;
  int* done;          // [nprob][kPMaxPhases]
  int* queue;
  int* err;
  int dot;            // 1: conj(v2) y (2 values); 2: conj(y) v2 and |y|^2 (3 values)
  unsigned spin_limit;
};

// Fixed-order block sums of three values (waves in order after a wave
// shuffle); thread 0 returns them.
__device__ inline void block_sum3(double (&v)[3], double* out) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  __shared__ double s3[3][kBWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 3; ++k) s3[k][wv] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      double a = 0;
      for (int w = 0; w < kBWaves; ++w) a += s3[k][w];
      out[k] = a;
    }
  __syncthreads();
}

// The dots of the finest level from y and v2 at one vertex (DOT 1: conj(v2) y;
// DOT 2: conj(y) v2 and |y|^2).
template <class T>
__device__ inline void dot_terms(int dot, cpx<T> y, cpx<T> v2, double (&acc)[3]) {
  const double yr = y.re, yi = y.im, vr = v2.re, vi = v2.im;
  if (dot == 1) {
    acc[0] += vr * yr + vi * yi;
    acc[1] += vr * yi - vi * yr;
  } else {
    acc[0] += yr * vr + yi * vi;
    acc[1] += yr * vi - yi * vr;
    acc[2] += yr * yr + yi * yi;
  }
}

template <class T, int DOT, int VAR>
__device__ inline void prec_pa3(const FusedArgs<T>& f, int zc3, int bx, int by, int bz, double* part,
                                F3Lds<T, 2, 2, false>& sm0) {
  if (zc3 == 0) fused3_tile<T, 2, 2, 9, VAR, kPrecApply, 1, DOT>(f, bx, by, bz, part, sm0);
  else fused3_tile<T, 2, 2, 3, VAR, kPrecApply, 1, DOT>(f, bx, by, bz, part, sm0);
}

template <class T, int D>
__device__ __attribute__((always_inline)) inline void prec_item(const PrecArgs<T>& A, const PProb<T>& P,
                                                                const PIO<T>& io, int phase, int tile,
                                                                F3Lds<T, 2, 2, true>* f3lds) {
  const int kind = P.phase_kind[phase], lev = P.phase_level[phase];
  const int L = P.L, lmin = P.lmin;
  const bool bpx = P.variant == MG_BPX, hb = P.variant == MG_HB;
  auto& sm0 = reinterpret_cast<F3Lds<T, 2, 2, false>&>(*f3lds);
  if (kind == PK_R) {
    // rho_(lev-1) = R (v on the finest level, rho_lev below it)
    const int nc = P.op[lev - 1].n, nf = P.op[lev].n;
    const cpx<T>* src = lev == L ? io.v : P.pr[lev];
    cpx<T>* dst = P.pr[lev - 1];
    for_rows<T, D>(nc, tile, [&](const int m[3], long long ic) {
      cpx<T> p[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) p[k] = restrict_part<T, D>(src, nf, m, k - 2);
      dst[ic] = csel(is_interior<D>(m, nc), post_galerkin_combine(p), czero<T>());
    });
  } else if (kind == PK_UP) {
    const cpx<T>* rho = lev == L ? io.v : P.pr[lev];
    const cpx<T>* gc = lev > lmin ? (bpx ? P.pr[lev - 1] : P.pz[lev - 1]) : nullptr;
    cpx<T>* z = lev == L ? io.z : P.pz[lev];
    for_rows<T, D>(P.op[lev].n, tile, [&](const int j[3], long long i) {
      prec_up_vertex<T, D>(P.op[lev], j, i, rho, P.omega[lev], hb ? 1 : 0, lev == lmin ? 1 : 0, gc, z);
    });
  } else if (kind == PK_G) {
    const cpx<T>* rho = lev == L ? io.v : P.pr[lev];
    for_rows<T, D>(P.op[lev - 1].n, tile, [&](const int m[3], long long ic) {
      prec_g_vertex<T, D>(P.op[lev], m, ic, rho, P.omega[lev], P.pz[lev - 1], P.pr[lev - 1]);
    });
  } else if (kind == PK_APPLY) {
    // y = H z on the finest level (2D) with the dot partials of this item
    const int n = P.op[L].n;
    double acc[3] = {0.0, 0.0, 0.0};
    for_rows<T, D>(n, tile, [&](const int j[3], long long i) {
      cpx<T> yv = czero<T>();
      if (is_interior<D>(j, n)) yv = stencil_const<T, D>(io.z, n, j, P.op[L]);   // batches have constant phi
      io.y[i] = yv;
      dot_terms(A.dot, yv, io.v2[i], acc);
    });
    block_sum3(acc, P.part + 3 * tile);
  } else if (kind == PK_DOT) {
    // fixed-order second stage over the problem's slots
    __shared__ double s0[3][kBThreads];
    const int t = threadIdx.x;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = t; i < P.nslots; i += kBThreads)
      for (int k = 0; k < 3; ++k) a[k] += P.part[3 * i + k];
    for (int k = 0; k < 3; ++k) s0[k][t] = a[k];
    __syncthreads();
    if (t == 0) {
      for (int k = 0; k < 3; ++k) {
        double q = 0.0;
        for (int w = 0; w < kBThreads; ++w) q += s0[k][w];
        io.out[k] = q;
      }
    }
    __syncthreads();
  } else if (kind == PK_SEAM) {
    // rho_(L-1) += the seam rows of the 3D finest restriction (tiles of 2 coarse rows)
    const int nc = P.op[L - 1].n, nseam = P.fgy - 1;
    cpx<T>* dst = P.pr[L - 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < kBRows / kBWaves; ++k) {
      const int row = tile * kBRows + wv + kBWaves * k;
      if (row >= nc * nseam) break;
      const int mz = row / nseam, sidx = row - mz * nseam, my = 2 * (sidx + 1);
      if (mz < 1 || mz > nc - 2 || my > nc - 2) continue;
      for (int mx = lane; mx < nc; mx += 64) {
        if (mx < 1 || mx > nc - 2) continue;
        cpx<T>& d = dst[((long long)mz * nc + my) * nc + mx];
        const cpx<T> e = P.spill[((long long)mz * nc + my) * nc + mx];
        d = mk(d.re + e.re, d.im + e.im);
      }
    }
  } else if (D == 3) {
    const int bx = tile % P.fgx, by = (tile / P.fgx) % P.fgy, bz = tile / (P.fgx * P.fgy);
    FusedArgs<T> f = {};
    f.n = P.op[L].n;
    f.nc = P.op[L - 1].n;
    if (kind == PK_R3) {
      f.b = io.v;
      f.rhoc = P.pr[L - 1];
      f.spill = P.spill;
      f.variant = 1;
      if (P.zc3 == 0) fused3_tile<T, 2, 2, 9, 1, kRestrict>(f, bx, by, bz, nullptr, sm0);
      else fused3_tile<T, 2, 2, 3, 1, kRestrict>(f, bx, by, bz, nullptr, sm0);
    } else {   // PK_PA3: z = s + P g, y = H z and the dot partials of the tile
      f.w = io.v;
      f.scc = bpx ? P.pr[L - 1] : P.pz[L - 1];
      f.zout = io.z;
      f.wout = io.y;
      f.b = io.v2;
      for (int q = 0; q < 4; ++q) f.coef[q] = P.op[L].coef[q];
      f.ws = P.wsL;
      f.variant = hb ? 1 : 0;
      double* part = P.part + 3 * tile;
      if (A.dot == 1) {
        if (hb) prec_pa3<T, 1, 1>(f, P.zc3, bx, by, bz, part, sm0);
        else prec_pa3<T, 1, 0>(f, P.zc3, bx, by, bz, part, sm0);
      } else {
        if (hb) prec_pa3<T, 2, 1>(f, P.zc3, bx, by, bz, part, sm0);
        else prec_pa3<T, 2, 0>(f, P.zc3, bx, by, bz, part, sm0);
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBThreads, 2) void k_batch_prec(PrecArgs<T> A) {
  __shared__ int s_item, s_ok, s_acq;
  int acq_prob = -1, acq_phase = -1;
  __shared__ F3Lds<T, 2, 2, true> f3lds;
  // the claim / wait / publish protocol of k_batch_cycle (see there)
  if (threadIdx.x == 0) s_item = atomicAdd(A.queue, 1);
  __syncthreads();
  for (;;) {
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= A.nitems) break;
    BItem w = A.items[it];
    w.prob = __builtin_amdgcn_readfirstlane(w.prob);
    w.phase = __builtin_amdgcn_readfirstlane(w.phase);
    w.tile = __builtin_amdgcn_readfirstlane(w.tile);
    const PProb<T>& P = A.probs[w.prob];
    const PIO<T>& io = A.io[w.prob];
    if (threadIdx.x == 0) {
      int ok = 1, acq = 0;
      if (w.phase > 0 && (w.prob != acq_prob || w.phase != acq_phase)) {
        acq = 1;
        const int need = P.phase_items[w.phase - 1];
        int* cnt = A.done + w.prob * kPMaxPhases + w.phase - 1;
        unsigned spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++spins > A.spin_limit) {
            ok = 0;
            atomicOr(A.err, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (ok) {
          acq_prob = w.prob;
          acq_phase = w.phase;
        }
      }
      s_ok = ok && io.active;
      s_acq = acq;
    }
    __syncthreads();
    if (s_acq) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (s_ok) {
      if (P.dim == 3) prec_item<T, 3>(A, P, io, w.phase, w.tile, &f3lds);
      else prec_item<T, 2>(A, P, io, w.phase, w.tile, &f3lds);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(A.done + w.prob * kPMaxPhases + w.phase, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(A.queue, 1);
    }
    __syncthreads();
  }
}

// Vector updates of BiCGStab for every active problem in one launch: block b
// works on chunk b - first[p] of problem p (VB elements per block) and
// writes three partial sums to part[3 b]; k_batch_vec_finish adds each
// problem's partials in block order.
constexpr int kVecChunk = 8 * kBThreads;
enum VecOp { VO_INIT = 0, VO_P = 1, VO_S = 2, VO_XR = 3 };

template <class T>
struct VSet {
  cpx<T>*r, *rh, *p, *v, *s, *t, *y, *z, *x;
  const cpx<T>* b;
  long long N;
  cpx<double> alpha, beta, omega;
  int active;
};

template <class T>
__global__ __launch_bounds__(kBThreads) void k_batch_vec(const VSet<T>* __restrict__ vs,
                                                         const int* __restrict__ blk_prob,
                                                         const int* __restrict__ blk_first, int op, double* part) {
  const int b = blockIdx.x;
  const int pi = blk_prob[b];
  const VSet<T>& V = vs[pi];
  double acc[3] = {0.0, 0.0, 0.0};
  if (V.active) {
    const long long base = (long long)(b - blk_first[pi]) * kVecChunk;
    const long long end = min(base + (long long)kVecChunk, V.N);
    for (long long i = base + threadIdx.x; i < end; i += kBThreads) {
      if (op == VO_INIT) {
        // x = 0; r = rh = b; p = v = 0; |r|^2
        const cpx<T> bv = V.b[i];
        V.x[i] = czero<T>();
        V.r[i] = bv;
        V.rh[i] = bv;
        V.p[i] = czero<T>();
        V.v[i] = czero<T>();
        acc[0] += (double)bv.re * bv.re + (double)bv.im * bv.im;
      } else if (op == VO_P) {
        // p = r + beta (p - omega v), in double precision
        const cpx<T> rv = V.r[i], pv = V.p[i], vv = V.v[i];
        const double qr = pv.re - (V.omega.re * vv.re - V.omega.im * vv.im);
        const double qi = pv.im - (V.omega.re * vv.im + V.omega.im * vv.re);
        V.p[i] = mk(T(rv.re + V.beta.re * qr - V.beta.im * qi), T(rv.im + V.beta.re * qi + V.beta.im * qr));
      } else if (op == VO_S) {
        // s = r - alpha v and |s|^2
        const cpx<T> rv = V.r[i], vv = V.v[i];
        const cpx<T> sv = mk(T(rv.re - (V.alpha.re * vv.re - V.alpha.im * vv.im)),
                             T(rv.im - (V.alpha.re * vv.im + V.alpha.im * vv.re)));
        V.s[i] = sv;
        acc[0] += (double)sv.re * sv.re + (double)sv.im * sv.im;
      } else {
        // x += alpha y + omega z; r = s - omega t; |r|^2 and conj(rh) r
        const cpx<T> yv = V.y[i], zv = V.z[i], xv = V.x[i], sv = V.s[i], tv = V.t[i], hv = V.rh[i];
        const double xr = xv.re + V.alpha.re * yv.re - V.alpha.im * yv.im + V.omega.re * zv.re - V.omega.im * zv.im;
        const double xi = xv.im + V.alpha.re * yv.im + V.alpha.im * yv.re + V.omega.re * zv.im + V.omega.im * zv.re;
        V.x[i] = mk(T(xr), T(xi));
        const cpx<T> rv = mk(T(sv.re - (V.omega.re * tv.re - V.omega.im * tv.im)),
                             T(sv.im - (V.omega.re * tv.im + V.omega.im * tv.re)));
        V.r[i] = rv;
        acc[0] += (double)rv.re * rv.re + (double)rv.im * rv.im;
        acc[1] += (double)hv.re * rv.re + (double)hv.im * rv.im;
        acc[2] += (double)hv.re * rv.im - (double)hv.im * rv.re;
      }
    }
  }
  block_sum3(acc, part + 3 * b);
}

// One wavefront per problem: lane t adds the partials of blocks t, t + 64, ...
// in order, then a shuffle tree adds the lanes (a fixed order, so the sums do
// not change from run to run).
template <class T>
__global__ __launch_bounds__(64) void k_batch_vec_finish(const VSet<T>* __restrict__ vs, const int* __restrict__ blk_first,
                                                         const double* __restrict__ part, double* out) {
  const int pi = blockIdx.x;
  if (!vs[pi].active) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = blk_first[pi] + (int)threadIdx.x; b < blk_first[pi + 1]; b += 64)
    for (int k = 0; k < 3; ++k) a[k] += part[3 * b + k];
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_down(a[k], off, 64);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out[3 * pi + k] = a[k];
}

// ---------------------------------------------------------------------------
// Host driver.

template <class T>
static Engine<T>* engine_of(mg_ctx* c);
template <>
Engine<double>* engine_of<double>(mg_ctx* c) { return c->e64; }
template <>
Engine<float>* engine_of<float>(mg_ctx* c) { return c->e32; }

// Finest-level size (vertices) from which a problem of a batched Krylov solve
// applies its preconditioner with the engine's own launches: such a level
// fills the device by itself, and the engine's marches (deeper tiles, more
// waves per SIMD) then run its finest passes about three times faster than
// the persistent kernel's items; smaller problems stay in the persistent
// launch, where launch latency is what they would otherwise pay.
constexpr long long kBOwnVertices = 1ll << 22;
// Their 3D fused-sweep tile: 4 coarse rows of 2 rows per thread, 28 coarse
// planes, y-band block order, prefetch depth 3 (the autotuner's choice for
// the 244^3 and 730^3 grids); mg_batch_autotune retunes it per problem.
constexpr int kBOwnTile3 = 20;
// Side streams the large problems' cycles are spread over (with the batch
// stream, four hardware queues).
constexpr int kBSideStreams = 3;

// Polls of one dependency wait before it gives up: the default bounds a wait
// to about a second; the settable maximum to about a minute.
constexpr unsigned kDefaultSpinLimit = 1u << 20;
constexpr long long kMaxSpinLimit = 1ll << 26;

struct BatchBase {
  virtual ~BatchBase() {}
  virtual void set_spin_limit(unsigned v) = 0;
  virtual int cycle(int ncycles, double* res) = 0;
  virtual int autotune(int reps, int* best, double* best_us, double* times) = 0;
  virtual int set_trace(bool on) = 0;
  virtual int get_trace(long long* out, int cap, int* count) = 0;
  virtual int solve(const cpx<double>* const* bs, cpx<double>* const* us, double rtol, int maxit, int* iters,
                    double* relres) = 0;
  virtual int precondition_apply(const cpx<double>* const* vs, cpx<double>* const* zs, cpx<double>* const* ys) = 0;
  virtual int set_config(int cfg) = 0;
  std::vector<mg_ctx*> ctx;
  hipStream_t s = nullptr;
};

template <class T>
struct Batch : BatchBase {
  int np = 0, zc3 = 0, zc2 = 1, schedule = 0;
  std::vector<BProb<T>> hp;
  BProb<T>* dp = nullptr;
  BItem* ditems = nullptr;
  int nitems = 0;
  int* ddone = nullptr;
  int* dq = nullptr;
  double* dhist = nullptr;
  int hist_cap = 0;
  int grid = 0;
  unsigned spin_limit = kDefaultSpinLimit;
  std::vector<void*> owned;

  ~Batch() override {
    for (void* p : owned) (void)hipFree(p);
    for (mg_ctx* c : ctx) mg_destroy(c);
    for (hipEvent_t e : side_ev) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
  }

  // Side streams of the large problems' own cycles (default priority): a
  // call forks them from the batch stream with an event and joins them back,
  // so one problem's latency-bound coarse launches overlap another's sweep
  // and the persistent launch of the small problems.
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_ev;   // [0]: fork; [1 + q]: join of side stream q

  int ensure_side(int nown) {
    const int want = std::min(nown, kBSideStreams);
    while ((int)side.size() < want) {
      hipStream_t q;
      MG_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      side.push_back(q);
    }
    while ((int)side_ev.size() < 1 + (int)side.size()) {
      hipEvent_t e;
      MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      side_ev.push_back(e);
    }
    return MG_OK;
  }

  // ncycles of every large problem on the side streams (round robin), forked
  // from and joined back into the batch stream by the caller's two calls.
  int own_cycles_fork(int ncycles, int* nused) {
    int nown = 0;
    for (int i = 0; i < np; ++i) nown += own[i];
    *nused = 0;
    if (!nown) return MG_OK;
    MG_TRY(ensure_side(nown));
    const int nq = (int)side.size();
    MG_HIP(hipEventRecord(side_ev[0], s));
    for (int q = 0; q < nq; ++q) MG_HIP(hipStreamWaitEvent(side[q], side_ev[0], 0));
    int k = 0;
    for (int i = 0; i < np; ++i) {
      if (!own[i]) continue;
      Engine<T>& E = *engine_of<T>(ctx[i]);
      E.s = side[k++ % nq];
      const int rc = E.cycles(ncycles, nullptr, nullptr);
      E.s = s;
      MG_TRY(rc);
    }
    *nused = std::min(nown, nq);
    return MG_OK;
  }

  int own_cycles_join(int nused) {
    for (int q = 0; q < nused; ++q) {
      MG_HIP(hipEventRecord(side_ev[1 + q], side[q]));
      MG_HIP(hipStreamWaitEvent(s, side_ev[1 + q], 0));
    }
    return MG_OK;
  }

  template <class P>
  int dalloc(P** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(P));
    if (e != hipSuccess) return fail(MG_ENOMEM, std::string("batch hipMalloc: ") + hipGetErrorString(e));
    owned.push_back(q);
    *p = (P*)q;
    return MG_OK;
  }

  // Per-problem descriptor (static parts); tile choices from zc3 / zc2.
  int describe(int i, BProb<T>& P) {
    Engine<T>& E = *engine_of<T>(ctx[i]);
    std::memset(&P, 0, sizeof(P));
    P.dim = E.dim;
    P.L = E.L;
    P.lmin = E.lmin;
    P.variant = E.variant;
    if (!E.fused) return fail(MG_EINVAL, "batched problems need the fused finest sweep (constant phi, level_max > level_min)");
    if (E.scheme == MG_OMEGA_TRANSITION || E.scheme == MG_OMEGA_TWO_PHASE)
      return fail(MG_EINVAL, "batched cycles need an iteration-independent omega scheme");
    if (E.L >= kBMaxLevels) return fail(MG_EINVAL, "level_max too large for a batch");
    for (int l = E.lmin; l <= E.L; ++l) {
      BLevel<T>& v = P.lv[l];
      v.n = E.lv[l].n;
      v.u = l < E.L ? E.coarse_u(l) : E.lv[l].u;
      v.b = E.lv[l].b;
      v.sc = E.lv[l].sc;
      v.sf = E.lv[l].sf;
      v.si = E.lv[l].si;
      v.op = E.lv[l].op;
      v.omega = to_c<T>(omega_level(E.scheme, E.omega, E.omega_L, E.L - l, 1));
    }
    P.w[0] = E.w[0];
    P.w[1] = E.w[1];
    P.spill = E.spill;
    P.si2[0] = E.lv[E.L - 1].si;
    P.si2[1] = E.si_alt ? E.si_alt : E.lv[E.L - 1].si;
    P.parw = E.cur;
    P.pars = 0;
    const complex<double> wL = omega_level(E.scheme, E.omega, E.omega_L, 0, 1);
    P.wsL = to_c<T>(wL * complex<double>(E.lv[E.L].op.invD.re, E.lv[E.L].op.invD.im));
    P.part = E.partials;
    P.zc3 = zc3;
    P.zc2 = zc2;
    // the context's own tile follows the batch tiling, so that a standalone
    // cycle on it partitions the finest sweep (and its norm) identically
    const int same = E.dim == 3 ? fused_tile_index(3, 2, 2, kBZc3[zc3]) : fused_tile_index(2, 0, 0, kBZc2[zc2]);
    if (same < 0) return fail(MG_EINVAL, "batch tiling has no standalone counterpart");
    if (!own[i]) E.set_tile(same);
    const int nL = E.lv[E.L].n, nc = E.lv[E.L - 1].n;
    int k = 0;
    auto rows_items = [&](int n) { const int rows = E.dim == 3 ? n * n : n; return (rows + kBRows - 1) / kBRows; };
    for (int l = E.lmin; l < E.L; ++l) {
      P.phase_kind[k] = BK_PRE;
      P.phase_level[k] = l;
      P.phase_items[k++] = rows_items(E.lv[l].n);
    }
    if (E.dim == 3) {
      P.fgx = f3_xtiles(nc);
      P.fgy = f3_ytiles(nc, 2);
      const int gz = (nc + kBZc3[zc3] - 1) / kBZc3[zc3];
      P.ftiles = P.fgx * P.fgy * gz;
      P.phase_kind[k] = BK_FUSED3;
      P.phase_items[k] = P.ftiles;
      P.phase_level[k++] = E.L;
      P.phase_kind[k] = BK_SEAM;
      P.phase_items[k] = (nc * (P.fgy - 1) + kBRows - 1) / kBRows;
    } else {
      P.fgx = (nc + F2_TXC - 1) / F2_TXC;
      P.fgy = (nc + kBZc2[zc2] - 1) / kBZc2[zc2];
      P.ftiles = P.fgx * P.fgy;
      P.phase_kind[k] = BK_FUSED2;
      P.phase_items[k] = (P.ftiles + kBWaves - 1) / kBWaves;
    }
    (void)nL;
    P.phase_level[k++] = E.L;
    for (int l = E.L - 1; l > E.lmin; --l) {
      P.phase_kind[k] = BK_POST;
      P.phase_level[k] = l;
      P.phase_items[k++] = rows_items(E.lv[l - 1].n);
    }
    P.phase_kind[k] = BK_UPDATE;
    P.phase_level[k] = E.lmin;
    P.phase_items[k++] = rows_items(E.lv[E.lmin].n);
    P.phase_kind[k] = BK_NORM;
    P.phase_level[k] = E.L;
    P.phase_items[k++] = 1;
    P.nphase = k;
    if (k > kBMaxPhases) return fail(MG_EINVAL, "too many phases for a batch");
    // the single-problem partials buffer must hold this tiling
    if (P.ftiles > E.partials_cap) return fail(MG_EINVAL, "partials buffer too small for the batch tiling");
    return MG_OK;
  }

  // Queue order: schedule 0 = phase-major; 1 = phases aligned on each problem's
  // fused sweep.  Within a step, larger problems first.
  int build_items() {
    std::vector<std::array<long long, 4>> keys;  // sort key, prob, phase, tile
    int maxf = 0;
    for (int i = 0; i < np; ++i) maxf = std::max(maxf, hp[i].L - hp[i].lmin);
    for (int i = 0; i < np; ++i) {
      if (own[i]) continue;   // cycled with the engine's own launches
      const BProb<T>& P = hp[i];
      const long long size = (long long)P.lv[P.L].n * P.lv[P.L].n * (P.dim == 3 ? P.lv[P.L].n : 1);
      for (int ph = 0; ph < P.nphase; ++ph) {
        const int step = schedule == 0 ? ph : ph - (P.L - P.lmin) + maxf;
        for (int t = 0; t < P.phase_items[ph]; ++t)
          keys.push_back({((long long)step << 40) - size, i, ph, t});
      }
    }
    std::stable_sort(keys.begin(), keys.end(), [](const std::array<long long, 4>& a, const std::array<long long, 4>& b) {
      return a[0] < b[0];
    });
    std::vector<BItem>& items = hitems;
    items.resize(keys.size());
    for (size_t k = 0; k < keys.size(); ++k) items[k] = BItem{(int)keys[k][1], (int)keys[k][2], (int)keys[k][3]};
    nitems = (int)items.size();
    if (!ditems || nitems > item_cap) {
      MG_TRY(dalloc(&ditems, items.size()));
      item_cap = nitems;
    }
    if (tracing) MG_TRY(ensure_trace());
    MG_HIP(hipMemcpy(ditems, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice));
    return MG_OK;
  }
  int item_cap = 0;
  std::vector<BItem> hitems;
  bool tracing = false;
  unsigned long long* dtrace = nullptr;
  int trace_cap = 0;

  int ensure_trace() {
    if (nitems > trace_cap) {
      MG_TRY(dalloc(&dtrace, 4 * (size_t)nitems));
      trace_cap = nitems;
    }
    return MG_OK;
  }

  void set_spin_limit(unsigned v) override { spin_limit = v; }

  int set_trace(bool on) override {
    tracing = on;
    return on ? ensure_trace() : MG_OK;
  }

  // per item: prob, phase, tile, kind, wait start, ready, done, XCD << 16 | block
  int get_trace(long long* out, int cap, int* count) override {
    if (count) *count = nitems;
    if (!out || !dtrace) return MG_OK;
    const int m = std::min(cap, nitems);
    std::vector<unsigned long long> t(4 * (size_t)nitems);
    MG_HIP(hipMemcpyAsync(t.data(), dtrace, t.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < m; ++k) {
      const BItem& w = hitems[k];
      long long* o = out + 8 * (size_t)k;
      o[0] = w.prob;
      o[1] = w.phase;
      o[2] = w.tile;
      o[3] = hp[w.prob].phase_kind[w.phase];
      for (int q = 0; q < 4; ++q) o[4 + q] = (long long)t[4 * (size_t)k + q];
    }
    return MG_OK;
  }

  int setup(const mg_params* ps, int count, hipStream_t stream) {
    s = stream;
    np = count;
    for (int i = 0; i < count; ++i) {
      mg_params q = ps[i];
      q.sweep = MG_SWEEP_FUSED;
      mg_ctx* c = nullptr;
      MG_TRY(mg_setup(&q, stream, &c));
      ctx.push_back(c);
    }
    own.assign(np, 0);
    for (int i = 0; i < np; ++i) {
      Engine<T>& E = *engine_of<T>(ctx[i]);
      own[i] = (long long)E.NL() >= kBOwnVertices;
      if (own[i] && E.dim == 3) E.set_tile(kBOwnTile3);
    }
    hp.resize(np);
    for (int i = 0; i < np; ++i) MG_TRY(describe(i, hp[i]));
    MG_TRY(dalloc(&dp, np));
    MG_TRY(dalloc(&ddone, (size_t)np * kBMaxPhases + 2));
    dq = ddone + (size_t)np * kBMaxPhases;
    int dev = 0, ncu = 0, per = 0;
    MG_HIP(hipGetDevice(&dev));
    MG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_cycle<T>, kBThreads, 0));
    if (per < 1) return fail(MG_EDEVICE, "the batched kernel cannot be resident");
    grid = per * ncu;
    return build_items();
  }

  int ensure_hist(int n) {
    if (n > hist_cap) {
      MG_TRY(dalloc(&dhist, (size_t)2 * np * n));
      hist_cap = n;
    }
    return MG_OK;
  }

  int cycle(int ncycles, double* res) override {
    if (ncycles <= 0) return MG_OK;
    MG_TRY(ensure_hist(ncycles));
    // the error word collects the waits that gave up in any launch of this
    // call: cleared once here, not with the per-launch counters below
    MG_HIP(launch_fill(dq + 1, sizeof(int), s));
    // parities of the ping-pong buffers at this call
    for (int i = 0; i < np; ++i) {
      Engine<T>& E = *engine_of<T>(ctx[i]);
      hp[i].parw = E.cur;
      hp[i].pars = E.lv[E.L - 1].si == hp[i].si2[0] ? 0 : 1;
      hp[i].w[0] = E.w[0];
      hp[i].w[1] = E.w[1];
    }
    MG_HIP(hipMemcpyAsync(dp, hp.data(), hp.size() * sizeof(BProb<T>), hipMemcpyHostToDevice, s));
    // the large problems: the engine's own cycles (fused sweep with its tile,
    // coarse chain) on the side streams, norms in the engine's history
    int nside = 0;
    MG_TRY(own_cycles_fork(ncycles, &nside));
    for (int k = 0; k < ncycles && nitems > 0; ++k) {
      // completion counters and the queue head (not the error word after them)
      MG_HIP(launch_fill(ddone, ((size_t)np * kBMaxPhases + 1) * sizeof(int), s));
      BatchArgs<T> A;
      A.items = ditems;
      A.nitems = nitems;
      A.probs = dp;
      A.done = ddone;
      A.queue = dq;
      A.err = dq + 1;
      A.hist = dhist + (size_t)2 * np * k;
      A.cyc = k;
      A.spin_limit = spin_limit;
      A.trace = tracing ? dtrace : nullptr;
      hipLaunchKernelGGL(k_batch_cycle<T>, dim3(grid), dim3(kBThreads), 0, s, A);
      MG_HIP(hipGetLastError());
    }
    MG_TRY(own_cycles_join(nside));
    int err = 0;
    MG_HIP(hipMemcpyAsync(&err, dq + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<double> h, ho;
    if (res) {
      h.resize((size_t)2 * np * ncycles);
      ho.resize((size_t)2 * np * ncycles);
      if (nitems > 0) MG_HIP(hipMemcpyAsync(h.data(), dhist, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      for (int i = 0; i < np; ++i)
        if (own[i])
          MG_HIP(hipMemcpyAsync(ho.data() + (size_t)2 * ncycles * i, engine_of<T>(ctx[i])->hist,
                                (size_t)2 * ncycles * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    MG_HIP(hipStreamSynchronize(s));
    // the engines advance with the device state (the own problems' engines
    // have advanced themselves)
    for (int i = 0; i < np; ++i) {
      if (own[i]) continue;
      Engine<T>& E = *engine_of<T>(ctx[i]);
      if (ncycles & 1) {
        E.cur = 1 - E.cur;
        if (E.si_alt) std::swap(E.lv[E.L - 1].si, E.si_alt);
      }
      E.iter += ncycles;
    }
    if (err) return fail(MG_EDEVICE, "batched cycle: a dependency wait exceeded its bound");
    if (res) {
      for (int k = 0; k < ncycles; ++k)
        for (int i = 0; i < np; ++i) {
          Engine<T>& E = *engine_of<T>(ctx[i]);
          const double h2 = own[i] ? ho[(size_t)2 * ncycles * i + 2 * k] : h[(size_t)2 * (np * k + i)];
          res[(size_t)k * np + i] = std::sqrt(E.hnorm_scale() * h2);
        }
    }
    return MG_OK;
  }

  int configure(int z3, int z2, int sch) {
    zc3 = z3;
    zc2 = z2;
    schedule = sch;
    for (int i = 0; i < np; ++i) MG_TRY(describe(i, hp[i]));
    kready = false;   // the Krylov marches take the batch's z extent
    return build_items();
  }

  int set_config(int cfg) override {
    const int n3 = (int)(sizeof(kBZc3) / sizeof(kBZc3[0])), n2 = (int)(sizeof(kBZc2) / sizeof(kBZc2[0]));
    if (cfg < 0 || cfg >= n3 * n2 * 2) return fail(MG_EINVAL, "configuration out of range");
    return configure(cfg % n3, (cfg / n3) % n2, cfg / (n3 * n2));
  }

  // ---- batched Krylov solve --------------------------------------------
  std::vector<PProb<T>> hpp;
  PProb<T>* dpp = nullptr;
  std::vector<PIO<T>> hio;
  PIO<T>* dio = nullptr;
  int* dpdone = nullptr;               // [np][kPMaxPhases], queue, error word
  BItem* dpitems = nullptr;
  int npitems = 0, pgrid = 0;
  std::vector<BItem> hpitems_all;      // every problem's items in queue order
  int pitem_cap = 0;
  std::vector<int> pitems_active;      // the active set the device list was built for
  std::vector<VSet<T>> hvs;
  VSet<T>* dvs = nullptr;
  int* dblk_prob = nullptr;
  int* dblk_first = nullptr;
  int nvblocks = 0;
  double* dvpart = nullptr;            // 3 per vector block
  double* dvout = nullptr;             // 3 per problem
  double* dpout = nullptr;             // 3 per problem
  std::vector<cpx<T>*> xbuf, bbuf;     // inner solution and right-hand side per problem
  std::vector<int> own;                // problems of kBOwnVertices or more: the engine's own launches
  bool kready = false;

  int rows_items(int dim, int n) const {
    const int rows = dim == 3 ? n * n : n;
    return (rows + kBRows - 1) / kBRows;
  }

  // Phases of one preconditioner application with the operator (see PK_*).
  int describe_prec(int i, PProb<T>& P, double* part = nullptr, int part_cap = 0) {
    Engine<T>& E = *engine_of<T>(ctx[i]);
    std::memset(&P, 0, sizeof(P));
    P.dim = E.dim;
    P.L = E.L;
    P.lmin = E.lmin;
    P.variant = E.variant;
    P.zc3 = zc3;
    const int L = E.L, lmin = E.lmin, d = E.dim;
    const bool bpx = E.variant == MG_BPX;
    for (int l = lmin; l <= L; ++l) {
      P.op[l] = E.lv[l].op;
      P.omega[l] = to_c<T>(omega_level(E.scheme, E.omega, E.omega_L, L - l, 1));
      if (l < L) {
        P.pr[l] = E.lv[l].pr;
        P.pz[l] = E.lv[l].pz;
      }
    }
    P.spill = E.spill;
    const complex<double> wL = omega_level(E.scheme, E.omega, E.omega_L, 0, 1);
    P.wsL = to_c<T>(wL * complex<double>(E.lv[L].op.invD.re, E.lv[L].op.invD.im));
    const int nc = E.lv[L - 1].n;
    int k = 0;
    auto add = [&](int kind, int lev, int items) {
      P.phase_kind[k] = kind;
      P.phase_level[k] = lev;
      P.phase_items[k++] = items;
    };
    if (d == 3) {
      if (!E.spill) return fail(MG_EINVAL, "batched solve: a 3D problem without the fused sweep's seam array");
      P.fgx = f3_xtiles(nc);
      P.fgy = f3_ytiles(nc, 2);
      P.ftiles = P.fgx * P.fgy * ((nc + kBZc3[zc3] - 1) / kBZc3[zc3]);
      add(PK_R3, L, P.ftiles);
      if (P.fgy > 1) add(PK_SEAM, L - 1, (nc * (P.fgy - 1) + kBRows - 1) / kBRows);
    } else {
      add(PK_R, L, rows_items(d, nc));
    }
    for (int l = L - 1; l > lmin; --l) add(PK_R, l, rows_items(d, E.lv[l - 1].n));
    add(PK_UP, lmin, rows_items(d, E.lv[lmin].n));
    for (int l = lmin + 1; l < L; ++l) {
      if (bpx) add(PK_G, l, rows_items(d, E.lv[l - 1].n));
      add(PK_UP, l, rows_items(d, E.lv[l].n));
    }
    if (bpx) add(PK_G, L, rows_items(d, nc));
    if (d == 3) {
      add(PK_PA3, L, P.ftiles);
      P.nslots = P.ftiles;
    } else {
      add(PK_UP, L, rows_items(d, E.lv[L].n));
      add(PK_APPLY, L, rows_items(d, E.lv[L].n));
      P.nslots = rows_items(d, E.lv[L].n);
    }
    add(PK_DOT, L, 1);
    P.nphase = k;
    if (k > kPMaxPhases) return fail(MG_EINVAL, "too many phases for a batched preconditioner");
    if (part && P.nslots <= part_cap) {
      P.part = part;
      P.nslots_cap = part_cap;
    } else {
      MG_TRY(dalloc(&P.part, 3 * (size_t)P.nslots));
      P.nslots_cap = P.nslots;
    }
    MG_HIP(launch_fill(P.part, 3 * (size_t)P.nslots * sizeof(double), s));
    return MG_OK;
  }

  int krylov_setup() {
    if (kready) return MG_OK;
    if (dpp) {
      // rebuilt after a configuration change: descriptors and items only
      std::vector<std::array<long long, 4>> keys;
      for (int i = 0; i < np; ++i) {
        double* part = hpp[i].part;
        const int cap = hpp[i].nslots_cap;
        MG_TRY(describe_prec(i, hpp[i], part, cap));
        if (own[i]) continue;
        const long long size = (long long)engine_of<T>(ctx[i])->NL();
        for (int ph = 0; ph < hpp[i].nphase; ++ph)
          for (int t = 0; t < hpp[i].phase_items[ph]; ++t) keys.push_back({((long long)ph << 40) - size, i, ph, t});
      }
      std::stable_sort(keys.begin(), keys.end(),
                       [](const std::array<long long, 4>& a, const std::array<long long, 4>& b) { return a[0] < b[0]; });
      hpitems_all.resize(keys.size());
      for (size_t k = 0; k < keys.size(); ++k)
        hpitems_all[k] = BItem{(int)keys[k][1], (int)keys[k][2], (int)keys[k][3]};
      if ((int)hpitems_all.size() > pitem_cap) {
        MG_TRY(dalloc(&dpitems, hpitems_all.size()));
        pitem_cap = (int)hpitems_all.size();
      }
      MG_HIP(hipMemcpy(dpp, hpp.data(), np * sizeof(PProb<T>), hipMemcpyHostToDevice));
      pitems_active.clear();
      kready = true;
      return MG_OK;
    }
    hpp.resize(np);
    hio.resize(np);
    hvs.resize(np);
    xbuf.resize(np);
    bbuf.resize(np);
    std::vector<std::array<long long, 4>> keys;
    std::vector<int> blk_prob, blk_first(np + 1, 0);
    for (int i = 0; i < np; ++i) {
      Engine<T>& E = *engine_of<T>(ctx[i]);
      MG_TRY(E.ensure_krylov());
      MG_TRY(E.ensure_scratch());
      MG_TRY(describe_prec(i, hpp[i]));
      MG_TRY(dalloc(&xbuf[i], E.NL()));
      MG_TRY(dalloc(&bbuf[i], E.NL()));
      const PProb<T>& P = hpp[i];
      const long long size = (long long)E.NL();
      for (int ph = 0; ph < P.nphase && !own[i]; ++ph)
        for (int t = 0; t < P.phase_items[ph]; ++t) keys.push_back({((long long)ph << 40) - size, i, ph, t});
      VSet<T>& V = hvs[i];
      std::memset(&V, 0, sizeof(V));
      V.r = E.kv[0];
      V.rh = E.kv[1];
      V.p = E.kv[2];
      V.v = E.kv[3];
      V.s = E.kv[4];
      V.t = E.kv[5];
      V.y = E.kv[6];
      V.z = E.kv[7];
      V.x = xbuf[i];
      V.b = bbuf[i];
      V.N = (long long)E.NL();
      const int nb = (int)((V.N + kVecChunk - 1) / kVecChunk);
      blk_first[i] = (int)blk_prob.size();
      for (int q = 0; q < nb; ++q) blk_prob.push_back(i);
    }
    blk_first[np] = (int)blk_prob.size();
    nvblocks = (int)blk_prob.size();
    std::stable_sort(keys.begin(), keys.end(),
                     [](const std::array<long long, 4>& a, const std::array<long long, 4>& b) { return a[0] < b[0]; });
    hpitems_all.resize(keys.size());
    for (size_t k = 0; k < keys.size(); ++k)
      hpitems_all[k] = BItem{(int)keys[k][1], (int)keys[k][2], (int)keys[k][3]};
    MG_TRY(dalloc(&dpitems, hpitems_all.size()));
    pitem_cap = (int)hpitems_all.size();
    pitems_active.clear();
    MG_TRY(dalloc(&dpp, np));
    MG_HIP(hipMemcpy(dpp, hpp.data(), np * sizeof(PProb<T>), hipMemcpyHostToDevice));
    MG_TRY(dalloc(&dio, np));
    MG_TRY(dalloc(&dpdone, (size_t)np * kPMaxPhases + 2));
    MG_HIP(launch_fill(dpdone, ((size_t)np * kPMaxPhases + 2) * sizeof(int), s));
    MG_TRY(dalloc(&dvs, np));
    MG_TRY(dalloc(&dblk_prob, nvblocks));
    MG_TRY(dalloc(&dblk_first, np + 1));
    MG_HIP(hipMemcpy(dblk_prob, blk_prob.data(), nvblocks * sizeof(int), hipMemcpyHostToDevice));
    MG_HIP(hipMemcpy(dblk_first, blk_first.data(), (np + 1) * sizeof(int), hipMemcpyHostToDevice));
    MG_TRY(dalloc(&dvpart, 3 * (size_t)nvblocks));
    MG_TRY(dalloc(&dvout, 3 * (size_t)np));
    MG_TRY(dalloc(&dpout, 3 * (size_t)np));
    int dev = 0, ncu = 0, per = 0;
    MG_HIP(hipGetDevice(&dev));
    MG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_prec<T>, kBThreads, 0));
    if (per < 1) return fail(MG_EDEVICE, "the batched preconditioner kernel cannot be resident");
    pgrid = per * ncu;
    kready = true;
    return MG_OK;
  }

  // The device queue holds the items of the active problems only (in the
  // global queue order, which keeps every item after its dependencies):
  // rebuilt when the active set changes, so that the late iterations of a
  // lockstep solve, with few problems left, walk only their items.
  int select_items() {
    std::vector<int> act(np);
    for (int i = 0; i < np; ++i) act[i] = hio[i].active;
    if (act == pitems_active) return MG_OK;
    std::vector<BItem> items;
    items.reserve(hpitems_all.size());
    for (const BItem& w : hpitems_all)
      if (act[w.prob]) items.push_back(w);
    npitems = (int)items.size();
    if (npitems) {
      MG_HIP(hipStreamSynchronize(s));
      MG_HIP(hipMemcpyAsync(dpitems, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice, s));
      MG_HIP(hipStreamSynchronize(s));
    }
    pitems_active = act;
    return MG_OK;
  }

  // One preconditioner application with the operator for every active
  // problem: io[i] set by the caller (dot 1 or 2), sums in dpout.
  int prec_apply(int dot) {
    // problems with a finest level of kBOwnVertices or more: the engine's own
    // launches on the side streams (forked from and joined back into the
    // batch stream), dots copied into the batch's slots
    int nown = 0, nused = 0;
    for (int i = 0; i < np; ++i) nown += own[i] && hio[i].active;
    if (nown) {
      MG_TRY(ensure_side(nown));
      nused = std::min(nown, (int)side.size());
      MG_HIP(hipEventRecord(side_ev[0], s));
      for (int q = 0; q < nused; ++q) MG_HIP(hipStreamWaitEvent(side[q], side_ev[0], 0));
      int k = 0;
      for (int i = 0; i < np; ++i) {
        if (!own[i] || !hio[i].active) continue;
        Engine<T>& E = *engine_of<T>(ctx[i]);
        hipStream_t q = side[k++ % nused];
        E.s = q;
        const int rc = E.precondition_apply_enqueue(hio[i].v, hio[i].z, hio[i].y, dot, hio[i].v2);
        E.s = s;
        MG_TRY(rc);
        if (dot) MG_HIP(hipMemcpyAsync(dpout + 3 * i, E.red, 3 * sizeof(double), hipMemcpyDeviceToDevice, q));
      }
    }
    const int rc = prec_apply_small(dot);
    MG_TRY(own_cycles_join(nused));
    return rc;
  }

  // The persistent launch of the problems below kBOwnVertices.
  int prec_apply_small(int dot) {
    MG_TRY(select_items());
    if (npitems == 0) return MG_OK;
    MG_HIP(hipMemcpyAsync(dio, hio.data(), np * sizeof(PIO<T>), hipMemcpyHostToDevice, s));
    MG_HIP(launch_fill(dpdone, ((size_t)np * kPMaxPhases + 2) * sizeof(int), s));
    PrecArgs<T> A;
    A.items = dpitems;
    A.nitems = npitems;
    A.probs = dpp;
    A.io = dio;
    A.done = dpdone;
    A.queue = dpdone + (size_t)np * kPMaxPhases;
    A.err = A.queue + 1;
    A.dot = dot;
    A.spin_limit = spin_limit;
    hipLaunchKernelGGL(k_batch_prec<T>, dim3(pgrid), dim3(kBThreads), 0, s, A);
    MG_HIP(hipGetLastError());
    return MG_OK;
  }

  int vec(int op) {
    MG_HIP(hipMemcpyAsync(dvs, hvs.data(), np * sizeof(VSet<T>), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_batch_vec<T>, dim3(nvblocks), dim3(kBThreads), 0, s, dvs, dblk_prob, dblk_first, op, dvpart);
    MG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_batch_vec_finish<T>, dim3(np), dim3(64), 0, s, dvs, dblk_first, dvpart, dvout);
    MG_HIP(hipGetLastError());
    return MG_OK;
  }

  int fetch(double* hv, double* hp) {
    if (hv) MG_HIP(hipMemcpyAsync(hv, dvout, 3 * (size_t)np * sizeof(double), hipMemcpyDeviceToHost, s));
    int err = 0;
    if (hp) {
      MG_HIP(hipMemcpyAsync(hp, dpout, 3 * (size_t)np * sizeof(double), hipMemcpyDeviceToHost, s));
      MG_HIP(hipMemcpyAsync(&err, dpdone + (size_t)np * kPMaxPhases + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    MG_HIP(hipStreamSynchronize(s));
    if (err) return fail(MG_EDEVICE, "batched preconditioner: a dependency wait exceeded its bound");
    return MG_OK;
  }

  // BiCGStab in the engines' precision for the problems with act[i], right-hand
  // side bbuf[i], solution xbuf[i] (from zero), each to |r| <= tol[i] |b|, all
  // in lockstep (the same steps as Engine::bicgstab).  its[i]: iterations,
  // st[i]: MG_OK / MG_ENOTCONV / MG_EDIVERGED.
  int krylov_inner(std::vector<int> act, const std::vector<double>& tol, int maxit, std::vector<int>& its,
                   std::vector<int>& st) {
    std::vector<double> hv(3 * (size_t)np), hpo(3 * (size_t)np), bn(np, 0.0), r0(np, 1.0);
    std::vector<complex<double>> rho(np, 1.0), rho_new(np, 1.0), alpha(np, 1.0), om(np, 1.0);
    std::vector<int> at_s(np, 0);
    its.assign(np, 0);
    st.assign(np, MG_OK);
    for (int i = 0; i < np; ++i) hvs[i].active = act[i];
    MG_TRY(vec(VO_INIT));
    MG_TRY(fetch(hv.data(), nullptr));
    int nact = 0;
    for (int i = 0; i < np; ++i) {
      if (!act[i]) continue;
      bn[i] = std::sqrt(hv[3 * i]);
      rho_new[i] = hv[3 * i];   // (rh, r) with rh = r
      if (bn[i] == 0.0 || 1.0 <= tol[i]) {
        act[i] = 0;
        continue;
      }
      ++nact;
    }
    for (int it = 1; it <= maxit && nact > 0; ++it) {
      for (int i = 0; i < np; ++i) {
        hvs[i].active = act[i];
        hio[i].active = act[i];
        if (!act[i]) continue;
        const complex<double> beta = (rho_new[i] / rho[i]) * (alpha[i] / om[i]);
        hvs[i].beta = to_c<double>(beta);
        hvs[i].omega = to_c<double>(om[i]);
      }
      MG_TRY(vec(VO_P));
      // y = B p, v = H y and (rh, v)
      for (int i = 0; i < np; ++i) {
        const VSet<T>& V = hvs[i];
        hio[i] = PIO<T>{V.p, V.y, V.v, V.rh, dpout + 3 * i, act[i]};
      }
      MG_TRY(prec_apply(1));
      MG_TRY(fetch(nullptr, hpo.data()));
      for (int i = 0; i < np; ++i) {
        if (!act[i]) continue;
        alpha[i] = rho_new[i] / complex<double>(hpo[3 * i], hpo[3 * i + 1]);
        hvs[i].alpha = to_c<double>(alpha[i]);
      }
      // s = r - alpha v, |s|^2; z = B s, t = H z, (t, s) and |t|^2
      MG_TRY(vec(VO_S));
      for (int i = 0; i < np; ++i) {
        const VSet<T>& V = hvs[i];
        hio[i] = PIO<T>{V.s, V.z, V.t, V.s, dpout + 3 * i, act[i]};
      }
      MG_TRY(prec_apply(2));
      MG_TRY(fetch(hv.data(), hpo.data()));
      for (int i = 0; i < np; ++i) {
        if (!act[i]) continue;
        const double sn = std::sqrt(hv[3 * i]);
        if (sn / bn[i] <= tol[i]) {
          at_s[i] = 1;
          om[i] = 0.0;   // x += alpha y, r = s
        } else {
          om[i] = complex<double>(hpo[3 * i], hpo[3 * i + 1]) / hpo[3 * i + 2];
        }
        hvs[i].omega = to_c<double>(om[i]);
      }
      MG_TRY(vec(VO_XR));
      MG_TRY(fetch(hv.data(), nullptr));
      for (int i = 0; i < np; ++i) {
        if (!act[i]) continue;
        rho[i] = rho_new[i];
        rho_new[i] = complex<double>(hv[3 * i + 1], hv[3 * i + 2]);
        const double rel = std::sqrt(hv[3 * i]) / bn[i];
        if (it == 1) r0[i] = rel;
        if (at_s[i] || rel <= tol[i]) {
          its[i] = it;
          act[i] = 0;
          --nact;
        } else if (!std::isfinite(rel) || rel > 1e8 * std::max(r0[i], 1e-300)) {
          its[i] = it;
          st[i] = MG_EDIVERGED;
          act[i] = 0;
          --nact;
        }
      }
    }
    for (int i = 0; i < np; ++i)
      if (act[i]) {
        its[i] = maxit;
        st[i] = MG_ENOTCONV;
      }
    return MG_OK;
  }

  // z_i = B_i v_i and y_i = H_i z_i for every problem in one persistent
  // launch (inputs and outputs complex128; complex64 batches convert).
  int precondition_apply(const cpx<double>* const* vs, cpx<double>* const* zs, cpx<double>* const* ys) override {
    MG_TRY(krylov_setup());
    for (int i = 0; i < np; ++i) {
      Engine<T>& E = *engine_of<T>(ctx[i]);
      const int n = E.lv[E.L].n;
      MG_HIP((launch_convert<double, T>(E.NL(), vs[i], E.kv[4], 1.0, s)));
      MG_HIP(launch_zero_boundary_copy<T>(E.dim, n, E.kv[4], bbuf[i], mk(T(1), T(0)), s));
      hio[i] = PIO<T>{bbuf[i], xbuf[i], E.kv[6], bbuf[i], dpout + 3 * i, 1};
    }
    MG_TRY(prec_apply(1));
    for (int i = 0; i < np; ++i) {
      Engine<T>& E = *engine_of<T>(ctx[i]);
      MG_HIP((launch_convert<T, double>(E.NL(), xbuf[i], zs[i], 1.0, s)));
      MG_HIP((launch_convert<T, double>(E.NL(), E.kv[6], ys[i], 1.0, s)));
    }
    std::vector<double> sums(3 * (size_t)np);
    return fetch(nullptr, sums.data());
  }

  // Residual refinement in FP64 around the batched inner solve: for every
  // problem r = b - H u and rho = |r| in FP64, the inner solve of H e = r / rho
  // in the engines' precision (complex64 corrections to their inner
  // tolerance; an FP64 batch solves to the final tolerance directly), then
  // u += rho e in FP64, until |r| <= rtol |b| or maxit inner iterations.
  int solve(const cpx<double>* const* bs, cpx<double>* const* us, double rtol, int maxit, int* iters,
            double* relres) override {
    MG_TRY(krylov_setup());
    std::vector<double> bn(np, 0.0), rn(np, 0.0), rel(np, 1.0), rel0(np, -1.0);
    std::vector<int> act(np, 1), total(np, 0), status(np, MG_ENOTCONV);
    std::vector<double> hr(4 * (size_t)np);
    auto norms = [&](std::vector<double>& out, bool residual) -> int {
      for (int i = 0; i < np; ++i) {
        if (!act[i]) continue;
        mg_ctx* c = ctx[i];
        Engine<double>& E = *c->e64;
        const cpx<double>* v = E.tRh;
        if (residual) {
          MG_HIP(launch_resid<double>(c->p.dim, c->op64, E.tRh, us[i], E.tR, nullptr, nullptr, s));
          v = E.tR;
        }
        MG_HIP(launch_norm2<double>(E.NL(), v, E.partials, s));
        MG_HIP(launch_finish_sum_max(E.partials, kRedBlocks, E.red, s));
        MG_HIP(hipMemcpyAsync(&hr[4 * i], E.red, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      }
      MG_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < np; ++i)
        if (act[i]) out[i] = std::sqrt(hr[4 * i]);
      return MG_OK;
    };
    for (int i = 0; i < np; ++i) {
      mg_ctx* c = ctx[i];
      Engine<double>& E = *c->e64;
      MG_TRY(E.ensure_scratch());
      const int n = E.lv[E.L].n;
      MG_HIP(launch_zero_boundary_copy<double>(E.dim, n, us[i], us[i], mk(1.0, 0.0), s));
      MG_HIP(launch_zero_boundary_copy<double>(E.dim, n, bs[i], E.tRh, mk(1.0, 0.0), s));
    }
    MG_TRY(norms(bn, false));
    for (int i = 0; i < np; ++i)
      if (bn[i] == 0.0) {
        MG_HIP(launch_fill(us[i], ctx[i]->e64->NL() * sizeof(cpx<double>), s));
        act[i] = 0;
        rel[i] = 0.0;
        status[i] = MG_OK;
      }
    for (int outer = 0; outer < 100; ++outer) {
      MG_TRY(norms(rn, true));
      std::vector<int> inner(np, 0);
      std::vector<double> tol(np, 1.0);
      int any = 0;
      for (int i = 0; i < np; ++i) {
        if (!act[i]) continue;
        rel[i] = rn[i] / bn[i];
        if (rel0[i] < 0) rel0[i] = rel[i];
        if (!std::isfinite(rel[i]) || rel[i] > 1e8 * std::max(rel0[i], 1e-300)) {
          status[i] = MG_EDIVERGED;
          act[i] = 0;
        } else if (rel[i] <= rtol) {
          status[i] = MG_OK;
          act[i] = 0;
        } else if (total[i] >= maxit) {
          status[i] = MG_ENOTCONV;
          act[i] = 0;
        } else {
          inner[i] = 1;
          any = 1;
          const double it_tol = ctx[i]->p.inner_rtol > 0 ? ctx[i]->p.inner_rtol : kInnerRtolDefault;
          tol[i] = std::is_same<T, float>::value ? it_tol : std::max(0.5 * rtol / rel[i], 1e-15);
          const mg_ctx* c = ctx[i];
          MG_HIP((launch_convert<double, T>(c->e64->NL(), c->e64->tR, bbuf[i], 1.0 / rn[i], s)));
        }
      }
      if (!any) break;
      int budget = 1;
      for (int i = 0; i < np; ++i)
        if (inner[i]) budget = std::max(budget, maxit - total[i]);
      std::vector<int> its, st;
      MG_TRY(krylov_inner(inner, tol, budget, its, st));
      for (int i = 0; i < np; ++i) {
        if (!inner[i]) continue;
        total[i] += std::max(its[i], 1);
        if (st[i] == MG_EDIVERGED) {
          status[i] = MG_EDIVERGED;
          act[i] = 0;
          continue;
        }
        mg_ctx* c = ctx[i];
        const size_t N = c->e64->NL();
        if (std::is_same<T, float>::value)
          MG_HIP(launch_accum32(N, reinterpret_cast<const cpx<float>*>(xbuf[i]), rn[i], us[i], s));
        else
          MG_HIP(launch_axpby<double>(N, mk(rn[i], 0.0), reinterpret_cast<const cpx<double>*>(xbuf[i]),
                                      mk(1.0, 0.0), us[i], s));
      }
    }
    int worst = MG_OK;
    for (int i = 0; i < np; ++i) {
      if (act[i]) status[i] = MG_ENOTCONV;
      if (iters) iters[i] = total[i];
      if (relres) relres[i] = rel[i];
      if (status[i] == MG_EDIVERGED) worst = MG_EDIVERGED;
      else if (status[i] == MG_ENOTCONV && worst == MG_OK) worst = MG_ENOTCONV;
    }
    MG_HIP(hipStreamSynchronize(s));
    return worst;
  }

  int autotune(int reps, int* best, double* best_us, double* times) override {
    hipEvent_t e0, e1;
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    int bcfg = 0;
    double bt = 1e300;
    // the large problems keep the fused-sweep tile their own autotuner picks
    for (int i = 0; i < np; ++i)
      if (own[i]) MG_TRY(engine_of<T>(ctx[i])->autotune(reps, nullptr, nullptr, nullptr));
    const int n3 = (int)(sizeof(kBZc3) / sizeof(kBZc3[0])), n2 = (int)(sizeof(kBZc2) / sizeof(kBZc2[0]));
    for (int cfg = 0; cfg < n3 * n2 * 2; ++cfg) {
      MG_TRY(configure(cfg % n3, (cfg / n3) % n2, cfg / (n3 * n2)));
      MG_TRY(cycle(1, nullptr));
      MG_HIP(hipEventRecord(e0, s));
      MG_TRY(cycle(reps, nullptr));
      MG_HIP(hipEventRecord(e1, s));
      MG_HIP(hipEventSynchronize(e1));
      float ms = 0;
      MG_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1e3 * ms / reps;
      if (times) times[cfg] = us;
      if (us < bt) {
        bt = us;
        bcfg = cfg;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MG_TRY(configure(bcfg % n3, (bcfg / n3) % n2, bcfg / (n3 * n2)));
    if (best) *best = bcfg;
    if (best_us) *best_us = bt;
    return MG_OK;
  }
};

}  // namespace mg

using namespace mg;

struct mg_batch {
  BatchBase* impl = nullptr;
  ~mg_batch() { delete impl; }
};

extern "C" {

int mg_batch_setup(const mg_params* ps, int count, void* hip_stream, mg_batch** out) {
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ps || count < 1) return fail(MG_EINVAL, "need at least one problem");
  const int prec = ps[0].precision;
  for (int i = 1; i < count; ++i)
    if (ps[i].precision != prec) return fail(MG_EINVAL, "all problems of a batch share one precision");
  mg_batch* b = new mg_batch();
  int rc;
  if (prec == MG_FP64) {
    auto* impl = new Batch<double>();
    b->impl = impl;
    rc = impl->setup(ps, count, (hipStream_t)hip_stream);
  } else {
    auto* impl = new Batch<float>();
    b->impl = impl;
    rc = impl->setup(ps, count, (hipStream_t)hip_stream);
  }
  if (rc != MG_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return MG_OK;
}

void mg_batch_destroy(mg_batch* b) {
  if (!b) return;
  if (b->impl) (void)hipStreamSynchronize(b->impl->s);
  delete b;
}

int mg_batch_problem(mg_batch* b, int i, mg_ctx** ctx) {
  if (!b || !ctx || i < 0 || i >= (int)b->impl->ctx.size()) return fail(MG_EINVAL, "bad problem index");
  *ctx = b->impl->ctx[i];
  return MG_OK;
}

int mg_batch_cycle(mg_batch* b, int ncycles, double* res_h) {
  if (!b || ncycles < 0) return fail(MG_EINVAL, "bad argument");
  return b->impl->cycle(ncycles, res_h);
}

int mg_batch_autotune(mg_batch* b, int reps, int* config, double* us_per_cycle, double* times_us) {
  if (!b || reps < 1) return fail(MG_EINVAL, "bad argument");
  return b->impl->autotune(reps, config, us_per_cycle, times_us);
}

int mg_batch_configs(void) { return kBatchConfigs; }

int mg_batch_set_config(mg_batch* b, int config) {
  if (!b) return fail(MG_EINVAL, "NULL batch");
  return b->impl->set_config(config);
}

int mg_batch_set_spin_limit(mg_batch* b, long long polls) {
  if (!b || polls < 0 || polls > kMaxSpinLimit) return fail(MG_EINVAL, "spin limit out of range");
  b->impl->set_spin_limit((unsigned)polls);
  return MG_OK;
}

int mg_batch_trace(mg_batch* b, int enable) {
  if (!b) return fail(MG_EINVAL, "NULL batch");
  return b->impl->set_trace(enable != 0);
}

int mg_batch_get_trace(mg_batch* b, long long* out, int cap, int* count) {
  if (!b || cap < 0) return fail(MG_EINVAL, "bad argument");
  return b->impl->get_trace(out, cap, count);
}

int mg_batch_precondition_apply(mg_batch* b, const mg_c128* const* vs, mg_c128* const* zs, mg_c128* const* ys) {
  if (!b || !vs || !zs || !ys) return fail(MG_EINVAL, "NULL argument");
  for (size_t i = 0; i < b->impl->ctx.size(); ++i) {
    if (!vs[i] || !zs[i] || !ys[i]) return fail(MG_EINVAL, "NULL problem vector");
    if ((const void*)vs[i] == (const void*)zs[i] || (const void*)vs[i] == (const void*)ys[i] ||
        (const void*)zs[i] == (const void*)ys[i])
      return fail(MG_EINVAL, "v, z and y of a problem must not alias");
  }
  return b->impl->precondition_apply(reinterpret_cast<const cpx<double>* const*>(vs),
                                     reinterpret_cast<cpx<double>* const*>(zs), reinterpret_cast<cpx<double>* const*>(ys));
}

int mg_batch_solve(mg_batch* b, const mg_c128* const* bs, mg_c128* const* us, double rtol, int maxit, int driver,
                   int* iters, double* relres) {
  if (!b || !bs || !us) return fail(MG_EINVAL, "NULL argument");
  if (!(rtol > 0) || maxit < 1) return fail(MG_EINVAL, "need rtol > 0 and maxit >= 1");
  if (driver != MG_STATIONARY && driver != MG_BICGSTAB) return fail(MG_EINVAL, "bad driver");
  for (size_t i = 0; i < b->impl->ctx.size(); ++i)
    if (!bs[i] || !us[i]) return fail(MG_EINVAL, "NULL problem vector");
  if (driver == MG_BICGSTAB)
    return b->impl->solve(reinterpret_cast<const cpx<double>* const*>(bs), reinterpret_cast<cpx<double>* const*>(us),
                          rtol, maxit, iters, relres);
  // the stationary driver solves problem by problem
  int worst = MG_OK;
  for (size_t i = 0; i < b->impl->ctx.size(); ++i) {
    int it = 0;
    double rr = 0;
    const int rc = mg_solve(b->impl->ctx[i], bs[i], us[i], rtol, maxit, driver, &it, &rr);
    if (rc != MG_OK && rc != MG_ENOTCONV && rc != MG_EDIVERGED) return rc;
    if (rc != MG_OK && worst == MG_OK) worst = rc;
    if (iters) iters[i] = it;
    if (relres) relres[i] = rr;
  }
  return worst;
}

}  // extern "C"
