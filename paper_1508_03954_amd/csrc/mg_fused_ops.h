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
// around 3m.  Along x and z, r is computed on the owned fine box extended by
// two vertices towards lower x and z, and u on one more vertex on each side:
// 64 columns, exactly one wavefront, lane l at x = x0 - 3 + l.  Along y, r is
// computed on the owned rows only (u on one more row each side); the share of
// the two rows above the tile in R at its first coarse row is restricted by
// the tile above and handed over through a seam array.  x-neighbours are
// exchanged with DPP wave shifts (no LDS); each thread keeps RPT consecutive
// rows in registers; the block marches through z one fine plane per step.
// The 27-point stencil row at plane p splits into an in-plane part M_p and a
// neighbour-plane part N_p, so H u at plane p-1 is M_(p-1) + N_(p-2) + N_p,
// carried in registers.  The next plane's w and b are loaded while the
// current plane is processed.  R: x and y parts through LDS, z part in a
// two-plane register ring; one barrier a step.
#pragma once
#include <type_traits>

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
// Component-wise select.  (A conditional expression on the struct itself may
// be lowered through private memory, whose accesses share the vector-memory
// counter with global loads and so force waits on every load in flight.)
template <class T>
__device__ inline cpx<T> f_sel(bool c, cpx<T> a, cpx<T> b) { return mk(c ? a.re : b.re, c ? a.im : b.im); }

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

// N sums over the block, in a fixed order (wave shuffles, then waves in order).
template <int N>
__device__ inline void block_reduce_sums(double (&v)[N], double* part, int nt) {
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  __shared__ double ss[N][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) ss[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = 0;
      for (int w = 0; w < (nt + 63) / 64; ++w) a += ss[k][w];
      part[k] = a;
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

// x tiling of the 3D sweep.  An interior tile owns 20 coarse columns (60 fine
// columns, lanes at x0-3 .. x0+60).  The coarse columns on the domain
// boundary need no restriction (rho is zero there), so the first tile owns
// columns 0..20 with its lanes at x = 0..63 and the last tile the final 21
// columns with its lanes ending at x = n-1: 82 coarse columns (the 244^3
// grid) take 4 tiles instead of 5.
__host__ __device__ inline int f3_xtiles(int nc) {
  if (nc <= 22) return 1;
  if (nc <= 41) return 2;
  return 2 + (nc - 42 + F3_TXC - 1) / F3_TXC;
}
// owned coarse columns [lo, hi) of x tile bx and the x of its lane 0
__host__ __device__ inline void f3_xtile(int nc, int bx, int& lo, int& hi, int& xs) {
  const int nt = f3_xtiles(nc), n = 3 * (nc - 1) + 1;
  if (nt == 1) {
    lo = 0;
    hi = nc;
    xs = 0;
  } else if (bx == 0) {
    lo = 0;
    hi = 21;
    xs = 0;
  } else if (bx == nt - 1) {
    lo = max(nc - 21, 21);
    hi = nc;
    xs = n - 64;
  } else {
    lo = 21 + (bx - 1) * F3_TXC;
    hi = min(lo + F3_TXC, nc - 21);
    xs = 3 * lo - 3;
  }
}

template <class T, int TYC, int RPT, int ZC, bool BPX>
struct F3 {
  static constexpr int TXC = F3_TXC, TX = 3 * TXC, TY = 3 * TYC;
  static constexpr int W = TY / RPT;           // waves per block: wave k computes rows y0 + k RPT ..
  static constexpr int NT = 64 * W;
  static constexpr int GX = TXC + 2, GY = TYC + 2;
  static constexpr int TXR = TXC + 1;          // owned coarse columns of an edge tile
  static_assert(TY % RPT == 0, "rows per thread must divide the owned rows");
  static_assert(W >= 2, "the first and the last wave form one halo row each");
  static_assert(RPT <= 4, "the x part of R stages a wave's rows in its UH slot");
  static_assert(GX <= 32, "coarse staging: one coarse row per half wave");
};

// LDS of one 3D tile, two slots of everything (steps alternate):
//   RX  x-restricted residual of the owned rows of one plane, at rows 2 ..
//       TY+1 between zero rows (two above, three below), so that the y part
//       of R reads five rows at fixed offsets for every coarse row of the tile,
//   Gz  z-interpolated coarse correction of one plane (BPX: sc - si),
//   Sz  (BPX) sc of one coarse plane, used on c-points,
//   UH  u and its in-row neighbour sum h of each wave's first and last row,
//       exchanged so that every row of u is formed by one wave only.
// The z extent does not enter, so tiles that differ only in ZC can share it.
// Without SWEEP (the plain operator marches) only UH is used; the others
// shrink to one entry.
template <class T, int TYC, int RPT, bool BPX, bool SWEEP = true>
struct F3Lds {
  using G = F3<T, TYC, RPT, 1, BPX>;
  cpx<T> RX[SWEEP ? 2 : 1][SWEEP ? G::TY + 5 : 1][SWEEP ? G::TXR : 1];
  cpx<T> Gz[SWEEP ? 2 : 1][SWEEP ? G::GY : 1][SWEEP ? G::GX : 1];
  cpx<T> Sz[BPX && SWEEP ? 2 : 1][BPX && SWEEP ? G::GY : 1][BPX && SWEEP ? G::GX : 1];
  cpx<T> UH[2][G::W][RPT == 1 ? 1 : 2][2][64];
};

// Raw buffer access through a descriptor per plane.  The descriptor's size
// bounds every access: an offset at or past it loads zero and drops a store
// (the hardware range check), so the sweep masks by offset instead of by
// branches.  A fixed sequence of memory instructions per step is what lets
// the compiler wait for exactly the load a value comes from, and not for the
// prefetches behind it.
constexpr unsigned kOOB = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;   // raw (untyped) buffer, 32-bit data format

// Every operand is wave-uniform; readfirstlane keeps the descriptor in scalar
// registers even where the compiler has parked a value in a vector register
// (a descriptor in vector registers would need a loop over its distinct values).
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes) {
  const unsigned long long b = reinterpret_cast<unsigned long long>(base);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  void* p = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), kRawBufferWord3);
}
// CP: the access's cache policy bits (0, or kStream for data used once).
constexpr int kStream = 2;   // non-temporal
template <int CP = 0>
__device__ inline cpx<double> bload(cpx<double>*, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, CP);
  cpx<double> c;
  __builtin_memcpy(&c, &v, sizeof(c));
  return c;
}
template <int CP = 0>
__device__ inline cpx<float> bload(cpx<float>*, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, CP);
  cpx<float> c;
  __builtin_memcpy(&c, &v, sizeof(c));
  return c;
}
template <int CP = 0>
__device__ inline void bstore(cpx<double> c, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __attribute__((ext_vector_type(4))) unsigned v;
  __builtin_memcpy(&v, &c, sizeof(c));
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, CP);
}
template <int CP = 0>
__device__ inline void bstore(cpx<float> c, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __attribute__((ext_vector_type(2))) unsigned v;
  __builtin_memcpy(&v, &c, sizeof(c));
  __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, CP);
}

// Seam array of the 3D sweep's restriction.  A tile computes r on its own
// rows only, so R at its first coarse row 3 my0 misses fine rows 3 my0 - 2 and
// 3 my0 - 1, which belong to the tile above (by - 1).  That tile restricts
// them to coarse row my0 (its "seam row") and stores the result in the seam
// array at the same coarse vertex; a second pass (k_seam3) adds it to rho_c
// at the seam rows.  The seam array has the layout of a coarse level (only
// its seam rows are written), so both stores share one offset per point.
__host__ __device__ inline int f3_ytiles(int nc, int tyc) { return (nc + tyc - 1) / tyc; }

// One tile (bx, by, bz) of the 3D sweep, executed by a whole block of
// F3<...>::NT threads with LDS `sm`; VAR is the variant (0 add, 1 hb, 2 BPX);
// `part` receives the tile's (sum |r|^2, max |r|) or is null.
//
// Step p of the march (one barrier each) works on two planes: before the
// barrier it forms u and h on plane p for the thread's rows, starts loading w
// of plane p+1, publishes the wave's edge rows and stages the coarse
// correction of plane p+1; after the barrier it completes the stencil rows of
// plane p, which closes the residual of plane q = p-1 (update, store, norms,
// injections, x part of R), starts loading b of plane p and the coarse values
// of plane p+2, and runs the y and z parts of R for plane q-1, whose x part
// the previous step left in LDS.  Every load is issued where its register is
// free, so no prefetch is live through the stencil beyond one plane of w and
// b: that keeps the register count (and so the occupancy) down.
// Rows: the block computes r on its TY owned rows only, and u on one more row
// on each side (formed by the first and the last wave).  Work that not every
// wave needs goes to different waves: the y and z parts of R (the tile's
// owned coarse rows and the seam row below them) to the fewest middle waves
// that hold all its coarse points, the coarse staging to the other waves, two
// coarse rows each (one per half wave).
// MODE kSweep: the fused sweep.  kResid / kApply: the same march without the
// coarse levels, storing r = b - H w (with its partial norms) or y = H w.
// kRestrict: the restriction R x of the vector in b alone (rho_c and the seam
// rows), with the sweep's R and no operator.  kPrecApply: the finest level of
// the zero-start cycle and the operator on its result in one pass: from x in
// w and the coarse correction g in scc, z = s + P g with s = ws x (zero on
// c-points for VAR 1), stored to zout, and y = H z, stored to wout; with DOT
// it also sums, over the owned vertices, conj(v2) y (DOT 1, 2 values) or
// conj(y) v2 and |y|^2 (DOT 2, 3 values) for the vector v2 in b, into the
// tile's slot of part.  kRestrict with DOT 3 restricts s = b - alpha w2 (the
// BiCGStab update of its second half-step, formed in double precision, which
// keeps the cancellation in s exact for complex64 vectors) instead of b,
// stores s to zout and sums |s|^2 over the owned vertices into part.
// kRestrict with DOT 4 is the backtracking of a coarse level in the Galerkin
// form: rho_c = R rho of the level's b slot (in b), and on the way the
// pointwise update sc = ws rho (zero on c-points for VAR 1 and 2) stored to
// zout, with s = ws rho injected into sic_out at c-points for VAR 2.
constexpr int kSweep = 0, kResid = 1, kApply = 2, kRestrict = 3, kPrecApply = 4;
constexpr bool f3_full_lds(int mode) { return mode == kSweep || mode == kRestrict || mode == kPrecApply; }

// PF: prefetch depth of w and b in planes (1, 2 or 3).  With PF > 1 each wave
// keeps the loads of PF planes in flight (PF register sets used in turn): for
// grids whose tiles leave few waves per CU, latency is hidden per wave.
template <class T, int TYC, int RPT, int ZC, int VAR, int MODE = kSweep, int PF = 1, int DOT = 0>
__device__ inline void fused3_tile(const FusedArgs<T>& a, int bx, int by, int bz, double* part,
                                   F3Lds<T, TYC, RPT, VAR == 2, f3_full_lds(MODE)>& sm) {
  constexpr bool BPX = VAR == 2;
  using G = F3<T, TYC, RPT, ZC, BPX>;
  constexpr int TXR = G::TXR, TY = G::TY, W = G::W, GX = G::GX, GY = G::GY;
  constexpr unsigned CB = sizeof(cpx<T>);
  // coarse points of R: the TYC owned coarse rows and the seam row, taken by
  // NWR waves in the middle of the block (the edge waves form the halo rows)
  constexpr int NPT = TXR * (TYC + 1), NWR = (NPT + 63) / 64, WR0 = (W - NWR) / 2;
  static_assert(NWR <= W, "coarse points of R per block");
  static_assert(RPT * TXR <= 64, "x part of R: one lane per row and coarse column");
  static_assert(GY <= 2 * (W - NWR), "coarse staging: two coarse rows per wave without R points");
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index and everything derived from rows is wavefront-uniform (scalar)
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, nc = a.nc;
  const long long n2 = (long long)n * n, nc2 = (long long)nc * nc;
  const unsigned pbytes = (unsigned)(n2 * CB), cpbytes = (unsigned)(nc2 * CB);
  int cx_lo, cx_hi, xs;
  f3_xtile(nc, bx, cx_lo, cx_hi, xs);
  const int my0 = by * TYC, mz0 = bz * ZC;
  const int mz1 = min(mz0 + ZC, nc);
  const int y0 = 3 * my0;
  const int x = xs + lane;
  const bool xin = x >= 1 && x <= n - 2;
  const bool xcomp = lane >= 1 && lane <= 62;
  const bool xown = x >= 3 * cx_lo && x <= min(3 * cx_hi - 1, n - 1);
  const int ybase = y0 + wv * RPT;                // first row of this wave
  const int yown_hi = min(y0 + TY - 1, n - 1);
  const int zown_lo = 3 * mz0, zown_hi = min(3 * mz1 - 1, n - 1);
  const cpx<T> c0 = a.coef[0], c1 = a.coef[1], c2 = a.coef[2], c3 = a.coef[3];
  const cpx<T> ws = a.ws;
  // x part of the prolongation for this lane (the second weight is zero on
  // coarse columns; its index is clamped so that the read stays in the row)
  const int smx0 = xs / 3;                        // first staged coarse column
  const int mxl = x / 3, qx = x - 3 * mxl, gxl = mxl - smx0;
  const int gxl1 = min(gxl + 1, GX - 1);
  const T wx0 = w_lo<T>(qx), wx1 = w_hi<T>(qx);
  const bool ccol = qx == 0;
  auto row_ok = [&](int y) { return y >= 1 && y <= n - 2; };
  auto plane_ok = [&](int p) { return p >= 1 && p <= n - 2; };
  // offsets inside a plane: interior vertices for loads, owned ones for stores
  unsigned vld[RPT], vst[RPT], vcp[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int y = ybase + j;
    const unsigned off = (unsigned)((y * n + x) * (int)CB);
    vld[j] = (row_ok(y) && xin) ? off : kOOB;
    vst[j] = (y <= yown_hi && xown) ? off : kOOB;
    // c-point injections: coarse offset inside a coarse plane
    vcp[j] = (y <= yown_hi && xown && ccol && y % 3 == 0 && x >= 0)
                 ? (unsigned)(((y / 3) * nc + x / 3) * (int)CB) : kOOB;
  }
  const bool top = wv == 0, bot = wv == W - 1;
  const int yhalo = top ? y0 - 1 : y0 + TY;       // extra row formed by the edge waves
  const unsigned vldh = ((top || bot) && row_ok(yhalo) && xin) ? (unsigned)((yhalo * n + x) * (int)CB) : kOOB;
  // coarse staging by the waves that take no R points: staging wave k (in
  // wave order) stages coarse rows my0 - 1 + 2k and 2k + 1, one per half wave
  const bool rwave = wv >= WR0 && wv < WR0 + NWR;   // wave-uniform
  const int sidx = wv < WR0 ? wv : wv - NWR;
  const bool swave = !rwave && 2 * sidx < GY;       // wave-uniform
  const int sr = 2 * sidx + (lane >> 5), sx = lane & 31;
  const int smx = smx0 + sx, smy = my0 - 1 + sr;
  const bool stager = swave && sr < GY && sx < GX;
  const unsigned vsg = (stager && smx >= 0 && smx < nc && smy >= 0 && smy < nc)
                           ? (unsigned)((smy * nc + smx) * (int)CB) : kOOB;
  // y and z parts of R: coarse point pi of the tile (rows ly < TYC owned, ly == TYC the seam row)
  const int pi = (wv - WR0) * 64 + lane;
  const bool rpt = rwave && pi < NPT;
  const int lx = rpt ? pi % TXR : 0, ly = rpt ? pi / TXR : 0;
  const int rmx = cx_lo + lx, rmy = my0 + ly;
  const bool rcin = rmx >= 1 && rmx <= nc - 2 && rmy >= 1 && rmy <= nc - 2;
  // x part of R: lane l takes row xr_j = l / TXR of its wave and owned coarse
  // column cx_lo + xr_c, whose fine column sits at lane xr_l of that row
  const int xr_j = lane / TXR, xr_c = lane - xr_j * TXR, xr_l = 3 * (cx_lo + xr_c) - xs;
  const bool xr_ok = xr_j < RPT && cx_lo + xr_c < cx_hi && xr_l >= 2 && xr_l <= 61;
  const int xr_at = 64 * min(xr_j, RPT - 1) + min(max(xr_l, 2), 61);
  const bool rcol = rpt && rmx < cx_hi;
  const unsigned vrho = (rcol && ly < TYC && rmy < nc) ? (unsigned)((rmy * nc + rmx) * (int)CB) : kOOB;
  const unsigned vspl = (rcol && ly == TYC && rmy <= nc - 2) ? (unsigned)((rmy * nc + rmx) * (int)CB) : kOOB;

  // Plane descriptors.  A plane that is not accessed gets size zero, so its
  // base address is never used (it may lie outside the array).
  const long long pstride = n2 * CB, cstride = nc2 * CB;
  auto at = [](const void* base, long long ofs) {
    return reinterpret_cast<const void*>(reinterpret_cast<uintptr_t>(base) + (uintptr_t)ofs);
  };
  auto frs = [&](const cpx<T>* base, long long ofs, bool ok) { return plane_rsrc(at(base, ofs), ok ? pbytes : 0u); };
  auto crs = [&](const cpx<T>* base, long long ofs, bool ok) { return plane_rsrc(at(base, ofs), ok ? cpbytes : 0u); };
  cpx<T>* tagT = nullptr;

  static_assert(PF >= 1 && PF <= 3, "prefetch depth (a divisor of the six-step group)");
  cpx<T> Wr[PF][RPT], Wh[PF], Br[PF][RPT];
  cpx<T> A[RPT], Np[RPT], Cp[RPT];
  // coarse prefetch depth: with PF > 1 the coarse values of two planes are in
  // flight (register set = parity of the fine plane relative to p0)
  constexpr int GF = PF == 1 ? 1 : 2;
  cpx<T> gsc0[GF], gsc1[GF], gsi0[GF], gsi1[GF];
  cpx<T> acc0 = f_zero<T>(), acc1 = f_zero<T>();
  double nsum = 0.0, nmax = 0.0;
  // dots of the preconditioner-apply march: v2 of plane P is loaded at step P
  // (register set = parity of P relative to p0) and used one step later
  static_assert(DOT == 0 || (MODE == kPrecApply && DOT <= 2) || (MODE == kRestrict && (DOT == 3 || DOT == 4)),
                "dots of the preconditioner-apply march, the s update or the backtracking of the restriction march");
  constexpr int ND = DOT == 0 || DOT >= 3 ? 1 : (DOT == 1 ? 2 : 3);
  double dacc[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) dacc[k] = 0.0;
  cpx<T> Dv[2][RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) Dv[0][j] = Dv[1][j] = f_zero<T>();

  // The march runs over fine planes p = p0 .. plast with p0 = 3 (mz0 - 1), so
  // p mod 3 is known from the step's position in a group of six (which also
  // fixes the LDS slot); kb = coarse plane of the group's first fine plane.
  const int p0 = 3 * mz0 - 3, plast = 3 * mz1;
  // planes past the tile's last use are not fetched (zero-size descriptors)
  auto load_w = [&](int p, long long ofs, cpx<T>* dst, cpx<T>& dh) {
    const auto r = frs(a.w, ofs, plane_ok(p) && p <= plast);
#pragma unroll
    for (int j = 0; j < RPT; ++j) dst[j] = bload(tagT, r, vld[j]);
    dh = bload(tagT, r, vldh);
  };
  // the first residual plane used is p0 + 1 (the lowest fine plane of R at coarse plane mz0)
  auto load_b = [&](int p, long long ofs, cpx<T>* dst) {
    const auto r = frs(a.b, ofs, plane_ok(p) && p > p0 && p < plast);
#pragma unroll
    for (int j = 0; j < RPT; ++j) dst[j] = bload<kStream>(tagT, r, vld[j]);
  };
  // the second input of the s update (kRestrict, DOT 3), with the same planes
  cpx<T> Vr[DOT == 3 ? PF : 1][RPT];
  auto load_v2 = [&](int p, long long ofs, cpx<T>* dst) {
    const auto r = frs(a.w2, ofs, plane_ok(p) && p > p0 && p < plast);
#pragma unroll
    for (int j = 0; j < RPT; ++j) dst[j] = bload(tagT, r, vld[j]);
  };
  // coarse values of fine plane p = 3 kz + TZ: planes kz and kz+1 (the second
  // only off coarse planes); coarse boundary planes hold zeros
  auto load_g = [&](auto TZ_, auto G_, int p, long long kofs) {
    constexpr int TZ = decltype(TZ_)::value, G = decltype(G_)::value;
    const bool ok = plane_ok(p) && p <= plast;
    gsc0[G] = bload(tagT, crs(a.scc, kofs, ok), vsg);
    gsc1[G] = bload(tagT, crs(a.scc, kofs + cstride, ok && TZ != 0), vsg);
    if (BPX) {
      gsi0[G] = bload(tagT, crs(a.sic, kofs, ok), vsg);
      gsi1[G] = bload(tagT, crs(a.sic, kofs + cstride, ok && TZ != 0), vsg);
    }
  };
  auto store_g = [&](auto TZ_, auto G_, int slot) {
    constexpr int TZ = decltype(TZ_)::value, G = decltype(G_)::value;
    if (stager) {
      const cpx<T> g0 = BPX ? f_sub(gsc0[G], gsi0[G]) : gsc0[G];
      const cpx<T> g1 = BPX ? f_sub(gsc1[G], gsi1[G]) : gsc1[G];
      sm.Gz[slot][sr][sx] = TZ == 0 ? g0 : f_add(f_scale(w_lo<T>(TZ), g0), f_scale(w_hi<T>(TZ), g1));
      if (BPX) sm.Sz[slot][sr][sx] = gsc0[G];   // used on c-points only (TZ == 0)
    }
  };
  // u = w + P g on plane p (p mod 3 = PT) at row y (zero off the interior);
  // kPrecApply: u = s + P g with s = ws w, masked on c-points for VAR 1
  auto form_u = [&](auto PT_, int p, int slot, int y, cpx<T> w) {
    constexpr int PT = decltype(PT_)::value;
    if (MODE != kSweep && MODE != kPrecApply) return w;   // loads already vanish off the interior
    const int my = floor_div3(y), qy = y - 3 * my, gy = min(max(my - my0 + 1, 0), GY - 1);
    if (MODE == kPrecApply) {
      const cpx<T> sv = f_mul(ws, w);
      w = VAR == 1 && PT == 0 ? f_sel(qy == 0 && ccol, f_zero<T>(), sv) : sv;
    }
    cpx<T> g = f_add(f_scale(wx0, sm.Gz[slot][gy][gxl]), f_scale(wx1, sm.Gz[slot][gy][gxl1]));
    if (qy != 0) {
      const int gy1 = min(gy + 1, GY - 1);
      const cpx<T> g1 = f_add(f_scale(wx0, sm.Gz[slot][gy1][gxl]), f_scale(wx1, sm.Gz[slot][gy1][gxl1]));
      g = f_add(f_scale(w_lo<T>(qy), g), f_scale(w_hi<T>(qy), g1));
    } else if (BPX && PT == 0) {
      // BPX keeps si on c-points: there the correction is sc_c itself
      g = f_sel(ccol, sm.Sz[slot][gy][gxl], g);
    }
    return f_sel(plane_ok(p) && row_ok(y) && xin, f_add(w, g), f_zero<T>());
  };
  auto hsum = [&](cpx<T> u) { return f_add(dpp_c<kDppLeft>(u), dpp_c<kDppRight>(u)); };

  // y and z parts of R for fine plane 3 k0 + TQ, whose x part is in RX[slot]
  // (fine rows outside the tile read the zero rows: the seam row takes the
  // tile's last two)
  auto rest_yz = [&](auto TQ_, int k0, long long kofs, int slot) {
    constexpr int TQ = decltype(TQ_)::value;
    cpx<T> v = f_zero<T>();
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy) v = f_add(v, f_scale(w_r<T>(oy), sm.RX[slot][3 * ly + 2 + oy][lx]));
    if (TQ == 0) {
      acc0 = f_add(acc0, v);
    } else if (TQ == 1) {
      acc0 = f_add(acc0, f_scale(T(2.0 / 3.0), v));
      acc1 = f_add(acc1, f_scale(T(1.0 / 3.0), v));
    } else {
      acc0 = f_add(acc0, f_scale(T(1.0 / 3.0), v));
      acc1 = f_add(acc1, f_scale(T(2.0 / 3.0), v));
      // coarse plane k0 is complete after its last fine plane
      const bool done = k0 >= mz0 && k0 < mz1;
      const cpx<T> val = f_sel(rcin && k0 >= 1 && k0 <= nc - 2, acc0, f_zero<T>());
      bstore(val, crs(a.rhoc, kofs, done), vrho);
      bstore(val, crs(a.spill, kofs, done), vspl);
      acc0 = acc1;
      acc1 = f_zero<T>();
    }
  };

  if (MODE == kSweep || MODE == kPrecApply) {
    const long long k0ofs = (long long)(mz0 - 1) * cstride;
    if (swave) {
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, GF - 1>;
      load_g(I0(), I0(), p0, k0ofs);
      store_g(I0(), I0(), 0);
      load_g(std::integral_constant<int, 1>(), I1(), p0 + 1, k0ofs);
      if (GF == 2) load_g(std::integral_constant<int, 2>(), I0(), p0 + 2, k0ofs);
    }
  }
  if (MODE != kRestrict) {
#pragma unroll
    for (int i = 0; i < PF; ++i) load_w(p0 + i, (long long)(p0 + i) * pstride, Wr[i], Wh[i]);
  }
  if (MODE != kApply && MODE != kPrecApply) {
#pragma unroll
    for (int i = 0; i < PF; ++i) load_b(p0 - 1 + i, (long long)(p0 - 1 + i) * pstride, Br[i]);
  }
  if (DOT == 3) {
#pragma unroll
    for (int i = 0; i < PF; ++i) load_v2(p0 - 1 + i, (long long)(p0 - 1 + i) * pstride, Vr[DOT == 3 ? i : 0]);
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) { A[j] = f_zero<T>(); Np[j] = f_zero<T>(); Cp[j] = f_zero<T>(); }
  if (MODE == kSweep || MODE == kRestrict) {
    // the zero rows of RX (both slots); nothing writes them later
    constexpr int NZ = 2 * 5 * TXR;
    for (int i = tid; i < NZ; i += G::NT) {
      const int sl = i / (5 * TXR), k = (i / TXR) % 5, c = i % TXR;
      sm.RX[sl][k < 2 ? k : TY + k][c] = f_zero<T>();
    }
  }
  __syncthreads();

  // Step K of a group (p = p0 + 6i + K, kb = mz0 - 1 + 2i): LDS slot S = K & 1;
  // at its start Wr[E] holds w of plane p, Br[E] b of plane p-1 (the other
  // PF - 1 sets have the loads of the next planes in flight), and the coarse
  // registers the values of plane p+1
  // R of the residual r of plane q = p - 1 of step K: (5) x part at the owned
  // coarse columns (the boundary columns need none): the wave's rows go to
  // this wave's slot of the other UH buffer (free during this half step: it
  // is refilled by this wave only, at the next step), and lane l reads row
  // l / TXR around coarse column l % TXR; (6) y and z parts of plane q-1 = p-2
  // (its x part is in slot S)
  auto restrict_r = [&](auto K_, const cpx<T>* r, int kb, long long kofs) {
    constexpr int K = decltype(K_)::value;
    constexpr int S = K & 1;
    cpx<T>* rr = &sm.UH[1 - S][wv][0][0][0];
#pragma unroll
    for (int j = 0; j < RPT; ++j) rr[64 * j + lane] = r[j];
    if (xr_ok) {
      const cpx<T>* row = rr + xr_at;
      const cpx<T> s1 = f_add(row[-1], row[1]), s2 = f_add(row[-2], row[2]);
      const cpx<T> rx = f_add(row[0], f_add(f_scale(T(2.0 / 3.0), s1), f_scale(T(1.0 / 3.0), s2)));
      sm.RX[1 - S][2 + wv * RPT + xr_j][xr_c] = rx;
    }
    constexpr int KR = K < 2 ? -1 : (K < 5 ? 0 : 1);   // floor((K - 2) / 3)
    if (rwave) rest_yz(std::integral_constant<int, (K + 1) % 3>(), kb + KR, kofs + KR * cstride, S);
  };

  auto step = [&](auto K_, int p, int kb) {
    constexpr int K = decltype(K_)::value;
    constexpr int S = K & 1, PT = K % 3;
    constexpr int E = K % PF;   // register set of w(p) and b(p-1)
    const int q = p - 1;
    const long long pofs = (long long)p * pstride, kofs = (long long)kb * cstride;
    if (MODE == kRestrict) {
      // the input of plane q is in Br[E] (and Vr[E]); the barrier orders the LDS slots
      __syncthreads();
      cpx<T> r[RPT];
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const bool in = plane_ok(q) && row_ok(ybase + j) && xin && xcomp;
        if (DOT == 3) {
          const cpx<T> bv = Br[E][j], vv = Vr[DOT == 3 ? E : 0][j];
          const double sre = (double)bv.re - (a.alpha.re * (double)vv.re - a.alpha.im * (double)vv.im);
          const double sim = (double)bv.im - (a.alpha.re * (double)vv.im + a.alpha.im * (double)vv.re);
          r[j] = f_sel(in, mk(T(sre), T(sim)), f_zero<T>());
        } else {
          r[j] = f_sel(in, Br[E][j], f_zero<T>());
        }
      }
      if (DOT == 3) {
        const bool q_own = q >= zown_lo && q <= zown_hi;
        const auto so = frs(a.zout, pofs - pstride, q_own);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          bstore<kStream>(r[j], so, vst[j]);
          if (q_own && vst[j] != kOOB) dacc[0] += (double)r[j].re * r[j].re + (double)r[j].im * r[j].im;
        }
        load_v2(p + PF - 1, pofs + (PF - 1) * pstride, Vr[DOT == 3 ? E : 0]);
      }
      if (DOT == 4) {
        // the level's pointwise update on the way (owned vertices of plane q)
        const bool q_own = q >= zown_lo && q <= zown_hi;
        constexpr bool q_c = K % 3 == 1;
        const auto so = frs(a.zout, pofs - pstride, q_own);
        const auto co = crs(a.sic_out, kofs + (K / 3) * cstride, q_own && q_c && VAR == 2);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int y = ybase + j;
          const cpx<T> sv = f_mul(ws, r[j]);
          const bool cp = q_c && q >= 0 && ccol && x >= 0 && (y % 3) == 0;
          bstore<kStream>(f_sel(VAR != 0 && cp, f_zero<T>(), sv), so, vst[j]);
          if (VAR == 2) bstore(sv, co, vcp[j]);
        }
      }
      load_b(p + PF - 1, pofs + (PF - 1) * pstride, Br[E]);
      restrict_r(K_, r, kb, kofs);
      return;
    }
    cpx<T> u[RPT], h[RPT], uh = f_zero<T>(), hh = f_zero<T>();
    // (1) u and h on plane p
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      u[j] = form_u(std::integral_constant<int, PT>(), p, S, ybase + j, Wr[E][j]);
      h[j] = hsum(u[j]);
    }
    if (top || bot) {
      uh = form_u(std::integral_constant<int, PT>(), p, S, yhalo, Wh[E]);
      hh = hsum(uh);
    }
    constexpr int LE = RPT == 1 ? 0 : 1;   // slot of the last row (the first row when RPT == 1)
    if (MODE == kPrecApply) {
      const auto zo = frs(a.zout, pofs, p >= zown_lo && p <= zown_hi);
#pragma unroll
      for (int j = 0; j < RPT; ++j) bstore<kStream>(u[j], zo, vst[j]);
    }
    sm.UH[S][wv][0][0][lane] = u[0];
    sm.UH[S][wv][0][1][lane] = h[0];
    if (LE) {
      sm.UH[S][wv][LE][0][lane] = u[RPT - 1];
      sm.UH[S][wv][LE][1][lane] = h[RPT - 1];
    }
    // (2) refill w with plane p+PF; stage plane p+1's correction
    load_w(p + PF, pofs + PF * pstride, Wr[E], Wh[E]);
    if (DOT != 0) {
      const auto rd = frs(a.b, pofs, p >= zown_lo && p <= zown_hi);
#pragma unroll
      for (int j = 0; j < RPT; ++j) Dv[K & 1][j] = bload(tagT, rd, vst[j]);
    }
    if ((MODE == kSweep || MODE == kPrecApply) && swave)
      store_g(std::integral_constant<int, (K + 1) % 3>(), std::integral_constant<int, (K + 1) % GF>(), 1 - S);
    __syncthreads();
    // (3) neighbour rows across the wave edges
    cpx<T> ua = uh, ha = hh, ub = uh, hb = hh;
    if (!top) {
      ua = sm.UH[S][wv - 1][LE][0][lane];
      ha = sm.UH[S][wv - 1][LE][1][lane];
    }
    if (!bot) {
      ub = sm.UH[S][wv + 1][0][0][lane];
      hb = sm.UH[S][wv + 1][0][1][lane];
    }
    // (4) stencil rows of plane p close the residual of plane q (a c-plane when K % 3 == 1)
    const bool q_own = q >= zown_lo && q <= zown_hi;
    constexpr bool q_c = K % 3 == 1;
    const auto wo = frs(a.wout, pofs - pstride, q_own);
    const auto co = crs(VAR == 0 ? a.sfc : a.sic_out, kofs + (K / 3) * cstride, q_own && q_c && VAR != 1);
    cpx<T> r[RPT];
    double s2 = 0.0, m2 = 0.0;   // this plane's share of the norms
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int y = ybase + j;
      const int jm = j > 0 ? j - 1 : 0, jp = j < RPT - 1 ? j + 1 : RPT - 1;
      cpx<T> um = u[jm], hm = h[jm], up = u[jp], hp = h[jp];
      if (j == 0) {
        um = ua;
        hm = ha;
      }
      if (j == RPT - 1) {
        up = ub;
        hp = hb;
      }
      const cpx<T> C = u[j];
      const cpx<T> F2 = f_add(h[j], f_add(um, up));
      const cpx<T> E2 = f_add(hm, hp);
      const cpx<T> M = f_mac(f_mac(f_mul(c0, C), c1, F2), c2, E2);
      const cpx<T> N = f_mac(f_mac(f_mul(c1, C), c2, F2), c3, E2);
      const bool in = plane_ok(q) && row_ok(y) && xin && xcomp;
      if (MODE == kApply || MODE == kPrecApply) {
        const cpx<T> yv = f_sel(in, f_add(A[j], N), f_zero<T>());
        bstore<kStream>(yv, wo, vst[j]);
        if (DOT != 0) {
          // owned vertices of plane q only (v2 of other vertices loads as zero)
          const cpx<T> d = Dv[(K + 1) & 1][j];
          if (DOT == 1) {
            dacc[0] += (double)d.re * yv.re + (double)d.im * yv.im;
            dacc[ND > 1 ? 1 : 0] += (double)d.re * yv.im - (double)d.im * yv.re;
          } else {
            dacc[0] += (double)yv.re * d.re + (double)yv.im * d.im;
            dacc[ND > 1 ? 1 : 0] += (double)yv.re * d.im - (double)yv.im * d.re;
            if (q_own && vst[j] != kOOB) dacc[ND - 1] += (double)yv.re * yv.re + (double)yv.im * yv.im;
          }
        }
        A[j] = f_add(M, Np[j]);
        Np[j] = N;
        continue;
      }
      const cpx<T> rv = f_sel(in, f_sub(Br[E][j], f_add(A[j], N)), f_zero<T>());
      if (MODE == kSweep) {
        const cpx<T> s = f_mul(ws, rv);
        const bool cp = q_c && q >= 0 && ccol && x >= 0 && (y % 3) == 0;
        const cpx<T> scm = f_sel(VAR != 0 && cp, f_zero<T>(), s);
        // off the interior u, r and s vanish, so the stored value is zero there
        bstore<kStream>(f_add(Cp[j], scm), wo, vst[j]);
        if (VAR != 1 && q_c) bstore(VAR == 0 ? scm : s, co, vcp[j]);
      } else {
        bstore<kStream>(rv, wo, vst[j]);
      }
      const double r2 = vst[j] != kOOB ? (double)rv.re * rv.re + (double)rv.im * rv.im : 0.0;
      s2 += r2;
      m2 = r2 > m2 ? r2 : m2;
      r[j] = rv;
      A[j] = f_add(M, Np[j]);
      Np[j] = N;
      Cp[j] = C;
    }
    if (MODE == kApply) return;
    if (MODE == kPrecApply) {
      if (swave)
        load_g(std::integral_constant<int, (K + 1 + GF) % 3>(), std::integral_constant<int, (K + 1) % GF>(), p + 1 + GF,
               kofs + ((K + 1 + GF) / 3) * cstride);
      return;
    }
    if (q_own) {
      nsum += s2;
      nmax = m2 > nmax ? m2 : nmax;
    }
    // refill b with plane p+PF-1, the coarse registers with plane p+1+GF
    load_b(p + PF - 1, pofs + (PF - 1) * pstride, Br[E]);
    if (MODE != kSweep) return;
    if (swave)
      load_g(std::integral_constant<int, (K + 1 + GF) % 3>(), std::integral_constant<int, (K + 1) % GF>(), p + 1 + GF,
             kofs + ((K + 1 + GF) / 3) * cstride);
    // (5), (6) the parts of R
    restrict_r(K_, r, kb, kofs);
  };
  // six steps per iteration, so that plane phases, slots and register roles
  // are constants; the slot left holding the x part of R of plane plast-1
  int p = p0, kb = mz0 - 1, last = 0;
  for (;;) {
    step(std::integral_constant<int, 0>(), p, kb);
    if (p + 1 > plast) { last = 1; break; }
    step(std::integral_constant<int, 1>(), p + 1, kb);
    if (p + 2 > plast) { last = 0; break; }
    step(std::integral_constant<int, 2>(), p + 2, kb);
    if (p + 3 > plast) { last = 1; break; }
    step(std::integral_constant<int, 3>(), p + 3, kb);
    if (p + 4 > plast) { last = 0; break; }
    step(std::integral_constant<int, 4>(), p + 4, kb);
    if (p + 5 > plast) { last = 1; break; }
    step(std::integral_constant<int, 5>(), p + 5, kb);
    p += 6;
    kb += 2;
    if (p > plast) { last = 0; break; }
  }
  // R of the last plane plast - 1 = 3 (mz1 - 1) + 2
  if (MODE == kSweep || MODE == kRestrict) {
    __syncthreads();
    if (rwave) rest_yz(std::integral_constant<int, 2>(), mz1 - 1, (long long)(mz1 - 1) * cstride, last);
  }
  if (DOT != 0) {
    if (part) block_reduce_sums<ND>(dacc, part, G::NT);
  } else if (part) {
    block_reduce_store(nsum, sqrt(nmax), part, G::NT);
  }
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
  auto load_w = [&](int p) {
    cpx<T> v = f_zero<T>();
    if (row_ok(p) && xin) v = a.w[(long long)p * n + x];
    return v;
  };
  auto load_b = [&](int q) {
    cpx<T> v = f_zero<T>();
    if (row_ok(q) && xin && xcomp) v = a.b[(long long)q * n + x];
    return v;
  };
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
      Gz[p & 1][lane] = f_sel(ty == 0, g0, f_add(f_scale(w_lo<T>(ty), g0), f_scale(w_hi<T>(ty), g1)));
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
    const cpx<T> rv = f_sel(in, f_sub(bc, f_add(A, N)), f_zero<T>());
    const cpx<T> s = f_mul(ws, rv);
    const bool cp = q >= 0 && (q % 3) == 0 && qx == 0 && x >= 0;
    const cpx<T> scm = f_sel(mask && cp, f_zero<T>(), s);
    if (q >= yown_lo && q <= yown_hi && xown) {
      a.wout[(long long)q * n + x] = f_sel(in, f_add(Cp, scm), f_zero<T>());
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
          a.rhoc[(long long)k0 * nc + cmx] = f_sel(cin, acc0, f_zero<T>());
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
