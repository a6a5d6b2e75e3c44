// Feature-based dynamic adaptivity (Section 5.3) with hanging vertices
// (Section 4) on a dense envelope of levels.
//
// The spacetree is held as one byte per cell and level ("refined into the 3^d
// cells of the next level") over the full regular grid of every level, plus
// one class byte per vertex (absent / persistent / hanging / boundary).  Every
// pass is then a coalesced sweep over a regular array: no pointer chasing, no
// per-vertex index tables (the envelope of a 3D level-6 hierarchy, 389 M
// vertices, takes 1.2 GB of class and mark bytes).  The classification and
// the decision pass cost the level's envelope; on a 3D level the criterion
// passes and the interpolation march over chunks of planes and skip, on one
// byte of a per-level activity map or on the chunk's class bytes, the chunks
// that hold nothing to do, so that they cost what is present.
//
// Marking one level: the criterion s = max_a |u(j+e_a) - 2u(j) + u(j-e_a)| of
// every persistent vertex is formed twice -- a first pass reduces its range,
// a second bins it into equal subranges of that range (a per-wavefront ballot
// count per bin, one global integer atomic per bin and block), and a byte pass
// turns bins into marks once the numbers of top and bottom bins are chosen:
// the top bins whose count comes closest to the refine percentage, the bottom
// bins closest to the erase percentage.  Counts are integers, so the marks do
// not depend on the order in which blocks run.  The file is compiled without
// floating-point contraction, so |.|^2, s and the bin index are rounded the
// same way as the plain-arithmetic definition (one rounding per operation).
//
// Adapting: the refined-cell bytes of the levels are updated from the finest
// level of cells up (a refine mark refines the cells around the vertex; an
// erase mark returns them to leaves unless a refine mark also touches the cell
// or one of its children stays refined), then the vertex classes of every
// level are derived from the presence of the adjacent cells (a cell is present
// on the coarsest level, and below it where its parent is refined).  Finally
// a vertex that is hanging or became persistent takes P u of the coarser
// level, one that became absent or boundary is set to zero.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mg_common.h"
#include "mg_engine.h"

namespace mg {
namespace {

constexpr int kAmrMaxBins = 64;
constexpr uint8_t kNotCand = 0x40, kVetoBit = 0x80, kBinMask = 0x3F;
enum : uint8_t { kAbsent = 0, kPersistent = 1, kHanging = 2, kBoundary = 3 };
enum : uint8_t { kKeep = 0, kRefine = 1, kErase = 2 };
constexpr int kAmrMaxParts = 4096;

// Row grid of a level: 64 x per wavefront, 4 rows per block, at most
// kAmrMaxParts blocks (the range pass writes one partial per block).
dim3 amr_grid(int n, int dim) {
  const int gx = (n + 63) / 64;
  const long long rows = dim == 3 ? (long long)n * n : n;
  const long long gy = std::max<long long>(1, std::min<long long>((rows + 3) / 4, kAmrMaxParts / gx));
  return dim3((unsigned)gx, (unsigned)gy);
}

// Largest |Delta_a u|^2 over the axes at interior vertex i.
template <int D>
__device__ inline double amr_s2(const cpx<double>* __restrict__ u, int n, long long i) {
  const cpx<double> c = u[i];
  const double cr = c.re + c.re, ci = c.im + c.im;
  double best = 0;
  long long st = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const cpx<double> p = u[i + st], m = u[i - st];
    const double dr = (p.re + m.re) - cr, di = (p.im + m.im) - ci;
    const double m2 = dr * dr + di * di;
    best = m2 > best ? m2 : best;
    st *= n;
  }
  return best;
}

__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Range of s^2 over the persistent vertices: (min, max, count) per block.
template <int D>
__global__ __launch_bounds__(256) void k_amr_range(int n, const cpx<double>* __restrict__ u,
                                                   const uint8_t* __restrict__ cls, double* __restrict__ part) {
  double lo = HUGE_VAL, hi = -HUGE_VAL, cnt = 0;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    if (cls[i] != kPersistent) continue;   // persistent vertices are interior
    const double s2 = amr_s2<D>(u, n, i);
    lo = fmin(lo, s2);
    hi = fmax(hi, s2);
    cnt += 1;
  }
  __shared__ double sh[3][4];
  lo = wave_min(lo);
  hi = wave_max(hi);
  cnt = wave_sum(cnt);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = lo;
    sh[1][w] = hi;
    sh[2][w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long b = blockIdx.y * (long long)gridDim.x + blockIdx.x;
    part[3 * b + 0] = fmin(fmin(sh[0][0], sh[0][1]), fmin(sh[0][2], sh[0][3]));
    part[3 * b + 1] = fmax(fmax(sh[1][0], sh[1][1]), fmax(sh[1][2], sh[1][3]));
    part[3 * b + 2] = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
  }
}

// The two criterion passes on a 3D level as a march along z: a wavefront
// takes 64 x of one row and a chunk of kAmrTz planes.  A chunk without a
// candidate is skipped on one byte of the level's activity map (kept by the
// classification).  The class bytes of an active chunk are read first (one
// round trip); a plane in which no lane of the
// wavefront holds a candidate costs nothing more.  On the others the
// wavefront reads its row of u and keeps the rows z-1, z, z+1 in registers,
// takes x-1 and x+1 from the neighbouring lanes (the two end lanes read
// theirs), and reads the rows y-1 and y+1 and the residual for its
// candidates; when the next plane has candidates too, its reads are issued
// before this plane is evaluated, so that they are in flight meanwhile.  The
// differences are formed in the same order as amr_s2.  MODE 0: range
// partials (as k_amr_range); MODE 1: bins, veto bits and bin counts (as
// k_amr_bin).  DG: the veto compares with a per-vertex diagonal (an instance
// of its own, so that the constant-diagonal pass carries no extra registers).
constexpr int kAmrTz = 8;
constexpr int kLaneLeft = 0x138;    // wave shift: lane l receives lane l-1 (0 at lane 0)
constexpr int kLaneRight = 0x130;   // lane l receives lane l+1 (0 at lane 63)

template <int CTRL>
__device__ inline double lane_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo));
}

__device__ inline double axis_m2(cpx<double> p, cpx<double> m, double cr, double ci) {
  const double dr = (p.re + m.re) - cr, di = (p.im + m.im) - ci;
  return dr * dr + di * di;
}

dim3 amr_march_grid(int n) {
  const int gx = (n + 63) / 64;
  const long long items = (long long)n * ((n + kAmrTz - 1) / kAmrTz);
  const long long gy = std::max<long long>(1, std::min<long long>((items + 3) / 4, kAmrMaxParts / gx));
  return dim3((unsigned)gx, (unsigned)gy);
}

// XCD-aware walk over the march's items, item = (chunk * n + y) * gx + x
// block.  Blocks are dealt to the 8 XCDs in turn (block b on XCD b % 8), and
// each XCD has its own L2.  The items are cut into groups of 16 rows
// (16 gx consecutive items) that are dealt to the XCDs in turn, and the
// blocks of an XCD walk its groups in order, four items apart per block: the
// rows a wavefront reads as y - 1 and y + 1 are then mostly read on the same
// XCD at about the same time (measured on a regular 244^3 level: the range
// pass moves 1.33x instead of 2.01x its algorithmic bytes), while a region with work spreads over
// all XCDs (contiguous bands per XCD left a local refinement to one or two).
// With fewer than 8 blocks there are as many bands as blocks.  Every item is
// visited once; the items of a band increase along the walk, so it ends at
// the first item past the level.
struct AmrWalk {
  int q, step, band, bands, group;
  __device__ int item() const { return ((q / group) * bands + band) * group + q % group; }
};

__device__ inline AmrWalk amr_walk(int gx) {
  const int nb = (int)(gridDim.x * gridDim.y), b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  AmrWalk w;
  w.bands = nb < 8 ? nb : 8;
  w.band = b % w.bands;
  const int local = b / w.bands, nbk = (nb - w.band + w.bands - 1) / w.bands;
  w.q = __builtin_amdgcn_readfirstlane(local * 4 + (int)(threadIdx.x >> 6));
  w.step = nbk * 4;
  w.group = 16 * gx;
  return w;
}

template <int MODE, bool DG>
__global__ __launch_bounds__(256) void k_amr_crit3(int n, const cpx<double>* __restrict__ u,
                                                   const cpx<double>* __restrict__ r,
                                                   const cpx<double>* __restrict__ dg, double veto2,
                                                   const uint8_t* __restrict__ cls,
                                                   const uint8_t* __restrict__ act_map, double* __restrict__ part,
                                                   const double* __restrict__ stats, int nb,
                                                   uint8_t* __restrict__ marks,
                                                   unsigned long long* __restrict__ hist) {
  const int lane = threadIdx.x & 63;
  const int nzc = (n + kAmrTz - 1) / kAmrTz, gx = (n + 63) / 64;
  const long long plane = (long long)n * n;
  const long long safe = plane + n + 1;   // vertex (1, 1, 1): reads of lanes without a candidate go there
  __shared__ unsigned sh[kAmrMaxBins];
  __shared__ double shr[3][4];
  double smin = 0, smax = 0, thr = 0, range = 1, dnb = (double)nb;
  bool spread = false;
  if (MODE == 1) {
    for (int t = threadIdx.x; t < kAmrMaxBins; t += 256) sh[t] = 0;
    __syncthreads();
    smin = stats[0];
    smax = stats[1];
    thr = stats[3];
    spread = smax > smin;
    range = smax - smin;
  }
  double lo = HUGE_VAL, hi = -HUGE_VAL, cnt = 0;
  unsigned mine = 0;
  const int items = gx * n * nzc;
  for (AmrWalk w = amr_walk(gx);; w.q += w.step) {
    const int it = w.item();
    if (it >= items) break;
    if (!act_map[it]) continue;   // no candidate in the chunk
    const int bx = it % gx, t = it / gx;
    const int y = t % n, zs = (t / n) * kAmrTz, ze = min(zs + kAmrTz, n);
    const int x = bx * 64 + lane;
    const bool xin = x < n;
    const int xc = xin ? x : n - 1;   // lanes past the row read a valid vertex and hold no candidate
    // the end lanes' extra read: x-1 for lane 0, x+1 for lane 63 (0 where it would leave the row)
    const int hoff = (lane == 0 && xc > 0) ? -1 : ((lane == 63 && xc < n - 1) ? 1 : 0);
    const long long row = (long long)y * n + xc;
    bool cand[kAmrTz];
    unsigned act = 0;   // bit q: plane zs + q has a candidate in the wavefront
#pragma unroll
    for (int q = 0; q < kAmrTz; ++q) {
      const int z = min(zs + q, ze - 1);
      cand[q] = xin && cls[(long long)z * plane + row] == kPersistent;
      if (zs + q < ze && __ballot(cand[q]) != 0) act |= 1u << q;
    }
    bool ready = false;
    cpx<double> cm = czero<double>(), c0 = czero<double>(), cp = czero<double>();
    cpx<double> ym = czero<double>(), yp = czero<double>(), h = czero<double>(), rv = czero<double>();
    cpx<double> dv = czero<double>();
#pragma unroll
    for (int q = 0; q < kAmrTz; ++q) {
      const int z = zs + q;
      if (z >= ze) break;
      const long long i = (long long)z * plane + row;
      if (!(act & (1u << q))) {
        ready = false;
        if (MODE == 1 && xin) marks[i] = kNotCand;
        continue;
      }
      const bool p = cand[q];
      if (!ready) {
        const long long k = p ? i : safe;
        cm = u[i - (z > 0 ? plane : 0)];
        c0 = u[i];
        cp = u[i + (z < n - 1 ? plane : 0)];
        ym = u[k - n];
        yp = u[k + n];
        h = u[i + hoff];
        if (MODE == 1 && r) rv = r[k];
        if (DG && r) dv = dg[k];
      }
      // the next plane's reads, issued before this plane is evaluated
      const bool nxt = q + 1 < kAmrTz && (act & (2u << q));
      cpx<double> cp1 = czero<double>(), ym1 = czero<double>(), yp1 = czero<double>(), h1 = czero<double>(),
                  rv1 = czero<double>(), dv1 = czero<double>();
      if (nxt) {
        const long long i1 = i + plane;
        const long long k1 = cand[q + 1] ? i1 : safe;
        cp1 = u[i1 + (z + 2 <= n - 1 ? plane : 0)];
        ym1 = u[k1 - n];
        yp1 = u[k1 + n];
        h1 = u[i1 + hoff];
        if (MODE == 1 && r) rv1 = r[k1];
        if (DG && r) dv1 = dg[k1];
      }
      cpx<double> xm = mk(lane_move<kLaneLeft>(c0.re), lane_move<kLaneLeft>(c0.im));
      cpx<double> xp = mk(lane_move<kLaneRight>(c0.re), lane_move<kLaneRight>(c0.im));
      if (lane == 0) xm = h;
      if (lane == 63) xp = h;
      const double cr = c0.re + c0.re, ci = c0.im + c0.im;
      double s2 = axis_m2(xp, xm, cr, ci);
      const double my = axis_m2(yp, ym, cr, ci), mz = axis_m2(cp, cm, cr, ci);
      s2 = my > s2 ? my : s2;
      s2 = mz > s2 ? mz : s2;
      if (MODE == 0) {
        if (p) {
          lo = fmin(lo, s2);
          hi = fmax(hi, s2);
          cnt += 1;
        }
      } else {
        const double sv = sqrt(s2);
        int b = 0;
        if (spread) {
          const double qq = floor(((sv - smin) / range) * dnb);
          b = qq >= dnb - 1 ? nb - 1 : (int)qq;
        }
        const bool v = r && (rv.re * rv.re + rv.im * rv.im > (DG ? veto2 * (dv.re * dv.re + dv.im * dv.im) : thr));
        if (xin) marks[i] = p ? (uint8_t)(b | (v ? kVetoBit : 0)) : kNotCand;
        const int bp = p ? b : -1;
        for (int k = 0; k < nb; ++k) {
          const unsigned long long bm = __ballot(bp == k);
          if (lane == k) mine += (unsigned)__popcll(bm);
        }
      }
      ready = nxt;
      if (nxt) {
        cm = c0;
        c0 = cp;
        cp = cp1;
        ym = ym1;
        yp = yp1;
        h = h1;
        rv = rv1;
        dv = dv1;
      }
    }
  }
  if (MODE == 0) {
    lo = wave_min(lo);
    hi = wave_max(hi);
    cnt = wave_sum(cnt);
    const int w = threadIdx.x >> 6;
    if (lane == 0) {
      shr[0][w] = lo;
      shr[1][w] = hi;
      shr[2][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const long long b = blockIdx.y * (long long)gridDim.x + blockIdx.x;
      part[3 * b + 0] = fmin(fmin(shr[0][0], shr[0][1]), fmin(shr[0][2], shr[0][3]));
      part[3 * b + 1] = fmax(fmax(shr[1][0], shr[1][1]), fmax(shr[1][2], shr[1][3]));
      part[3 * b + 2] = (shr[2][0] + shr[2][1]) + (shr[2][2] + shr[2][3]);
    }
  } else {
    if (lane < nb && mine) atomicAdd(&sh[lane], mine);
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += 256)
      if (sh[q]) atomicAdd(&hist[q], (unsigned long long)sh[q]);
  }
}

// One block: s_min, s_max, count and the veto threshold veto^2 |diag|^2 into
// stats; clears the bin counts and the mark counters.
__global__ __launch_bounds__(256) void k_amr_range_finish(const double* __restrict__ part, int nparts,
                                                          double diag_re, double diag_im, double veto,
                                                          double* __restrict__ stats,
                                                          unsigned long long* __restrict__ hist,
                                                          unsigned long long* __restrict__ counters) {
  double lo = HUGE_VAL, hi = -HUGE_VAL, cnt = 0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    lo = fmin(lo, part[3 * b + 0]);
    hi = fmax(hi, part[3 * b + 1]);
    cnt += part[3 * b + 2];
  }
  __shared__ double sh[3][4];
  lo = wave_min(lo);
  hi = wave_max(hi);
  cnt = wave_sum(cnt);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = lo;
    sh[1][w] = hi;
    sh[2][w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double c = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
    const double l = fmin(fmin(sh[0][0], sh[0][1]), fmin(sh[0][2], sh[0][3]));
    const double h = fmax(fmax(sh[1][0], sh[1][1]), fmax(sh[1][2], sh[1][3]));
    stats[0] = c > 0 ? sqrt(l) : 0.0;
    stats[1] = c > 0 ? sqrt(h) : 0.0;
    stats[2] = c;
    const double d2 = diag_re * diag_re + diag_im * diag_im;
    stats[3] = (veto * veto) * d2;
    stats[4] = 0;
    stats[5] = 0;
  }
  if (threadIdx.x < kAmrMaxBins) hist[threadIdx.x] = 0;
  if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

// Bin of every persistent vertex (with the residual veto in the top bit; other
// vertices get kNotCand) and the bin counts.
template <int D>
__global__ __launch_bounds__(256) void k_amr_bin(int n, const cpx<double>* __restrict__ u,
                                                 const cpx<double>* __restrict__ r,
                                                 const cpx<double>* __restrict__ dg, double veto2,
                                                 const uint8_t* __restrict__ cls, const double* __restrict__ stats,
                                                 int nb, uint8_t* __restrict__ marks,
                                                 unsigned long long* __restrict__ hist) {
  __shared__ unsigned sh[kAmrMaxBins];
  for (int t = threadIdx.x; t < kAmrMaxBins; t += 256) sh[t] = 0;
  __syncthreads();
  const double smin = stats[0], smax = stats[1], thr = stats[3];
  const bool spread = smax > smin;
  const double range = smax - smin;
  const double dnb = (double)nb;
  unsigned mine = 0;   // lane t < nb counts bin t for its wavefront
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    const bool in_row = row_vertex<D>(row_, x_, n, j, i);
    int b = -1;
    if (in_row) {
      uint8_t m = kNotCand;
      if (cls[i] == kPersistent) {
        const double s = sqrt(amr_s2<D>(u, n, i));
        b = 0;
        if (spread) {
          const double q = floor(((s - smin) / range) * dnb);
          b = q >= dnb - 1 ? nb - 1 : (int)q;
        }
        bool v = false;
        if (r) {
          const cpx<double> rv = r[i];
          double t2 = thr;
          if (dg) {
            const cpx<double> d = dg[i];
            t2 = veto2 * (d.re * d.re + d.im * d.im);
          }
          v = rv.re * rv.re + rv.im * rv.im > t2;
        }
        m = (uint8_t)(b | (v ? kVetoBit : 0));
      }
      marks[i] = m;
    }
    for (int t = 0; t < nb; ++t) {
      const unsigned long long bm = __ballot(b == t);
      if (lane_ == t) mine += (unsigned)__popcll(bm);
    }
  }
  if (lane_ < nb && mine) atomicAdd(&sh[lane_], mine);
  __syncthreads();
  for (int t = threadIdx.x; t < nb; t += 256)
    if (sh[t]) atomicAdd(&hist[t], (unsigned long long)sh[t]);
}

// Numbers of top (k) and bottom (e) bins: |100 count - pct N| least, fewer
// bins on ties; e counts only bins below the top k.
__device__ inline void amr_choose(const unsigned long long* hist, int nb, long long N, int rpct, int epct, int& k,
                                  int& e) {
  long long best = -1, c = 0;
  k = 0;
  for (int t = 0; t <= nb; ++t) {
    if (t > 0) c += (long long)hist[nb - t];
    const long long d = llabs(100 * c - (long long)rpct * N);
    if (best < 0 || d < best) {
      best = d;
      k = t;
    }
  }
  best = -1;
  c = 0;
  e = 0;
  for (int t = 0; t <= nb - k; ++t) {
    if (t > 0) c += (long long)hist[t - 1];
    const long long d = llabs(100 * c - (long long)epct * N);
    if (best < 0 || d < best) {
      best = d;
      e = t;
    }
  }
}

// The decision pass on a 3D level: the criterion march's walk and activity
// map, so that chunks without a candidate are skipped (their mark bytes are
// left as they are: only the candidates' marks are defined, and every reader
// takes them there only).
__global__ __launch_bounds__(256) void k_amr_decide3(int n, uint8_t* __restrict__ marks,
                                                     const uint8_t* __restrict__ cls,
                                                     const uint8_t* __restrict__ act_map,
                                                     const double* __restrict__ stats, int nb, int can_refine,
                                                     int can_erase, unsigned long long* __restrict__ counters) {
  __shared__ double sr[4], se_[4];
  const uint32_t top = (uint32_t)(nb - (int)stats[4]), bot = (uint32_t)(int)stats[5];
  const int lane = threadIdx.x & 63;
  const int nzc = (n + kAmrTz - 1) / kAmrTz, gx = (n + 63) / 64;
  const long long plane = (long long)n * n;
  const int items = gx * n * nzc;
  double nr = 0, ne = 0;
  for (AmrWalk w = amr_walk(gx);; w.q += w.step) {
    const int it = w.item();
    if (it >= items) break;
    if (!act_map[it]) continue;   // no candidate in the chunk
    const int bx = it % gx, t = it / gx;
    const int y = t % n, zs = (t / n) * kAmrTz, ze = min(zs + kAmrTz, n);
    const int x = bx * 64 + lane;
    if (x >= n) continue;
    for (int z = zs; z < ze; ++z) {
      const long long i = (long long)z * plane + (long long)y * n + x;
      const uint32_t m = marks[i];
      uint32_t d = kKeep;
      if (cls[i] == kPersistent && !(m & (kNotCand | kVetoBit))) {
        const uint32_t b = m & kBinMask;
        if (can_refine && b >= top) d = kRefine;
        else if (can_erase && b < bot) d = kErase;
      }
      nr += d == kRefine ? 1 : 0;
      ne += d == kErase ? 1 : 0;
      marks[i] = (uint8_t)d;
    }
  }
  nr = wave_sum(nr);
  ne = wave_sum(ne);
  const int wv = threadIdx.x >> 6;
  if (lane == 0) {
    sr[wv] = nr;
    se_[wv] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = (sr[0] + sr[1]) + (sr[2] + sr[3]), b = (se_[0] + se_[1]) + (se_[2] + se_[3]);
    if (a > 0) atomicAdd(&counters[0], (unsigned long long)a);
    if (b > 0) atomicAdd(&counters[1], (unsigned long long)b);
  }
}

// Marks of a level as the caller sees them: the mark at the candidates, KEEP
// elsewhere.
__global__ __launch_bounds__(256) void k_amr_mask_marks(long long N, const uint8_t* __restrict__ marks,
                                                        const uint8_t* __restrict__ cls, uint8_t* __restrict__ out) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (long long)gridDim.x * 256)
    out[i] = cls[i] == kPersistent ? marks[i] : (uint8_t)kKeep;
}

// One thread: the numbers of top and bottom bins into stats[4], stats[5].
__global__ void k_amr_choose(const unsigned long long* __restrict__ hist, double* __restrict__ stats, int nb,
                             int rpct, int epct) {
  if (threadIdx.x != 0) return;
  unsigned long long h[kAmrMaxBins];
  for (int t = 0; t < nb; ++t) h[t] = hist[t];
  int k, e;
  amr_choose(h, nb, (long long)stats[2], rpct, epct, k, e);
  stats[4] = k;
  stats[5] = e;
}

// Bins to marks, four bytes per lane (with the four class bytes); counts the
// refine and erase marks.
__global__ __launch_bounds__(256) void k_amr_decide(long long nwords, uint32_t* __restrict__ marks,
                                                    const uint32_t* __restrict__ cls,
                                                    const unsigned long long* __restrict__ hist,
                                                    double* __restrict__ stats, int nb, int rpct, int epct,
                                                    int can_refine, int can_erase,
                                                    unsigned long long* __restrict__ counters) {
  __shared__ double sr[4], se_[4];
  const uint32_t top = (uint32_t)(nb - (int)stats[4]), bot = (uint32_t)(int)stats[5];
  double nr = 0, ne = 0;
  for (long long w = blockIdx.x * 256ll + threadIdx.x; w < nwords; w += (long long)gridDim.x * 256) {
    const uint32_t v = marks[w], cw = cls[w];
    uint32_t o = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t m = (v >> (8 * q)) & 0xFFu;
      uint32_t d = kKeep;
      // only candidates carry a bin (other bytes may be left from earlier calls)
      if (((cw >> (8 * q)) & 0xFFu) == kPersistent && !(m & (kNotCand | kVetoBit))) {
        const uint32_t b = m & kBinMask;
        if (can_refine && b >= top) d = kRefine;
        else if (can_erase && b < bot) d = kErase;
      }
      nr += d == kRefine ? 1 : 0;
      ne += d == kErase ? 1 : 0;
      o |= d << (8 * q);
    }
    marks[w] = o;
  }
  nr = wave_sum(nr);
  ne = wave_sum(ne);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sr[wv] = nr;
    se_[wv] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = (sr[0] + sr[1]) + (sr[2] + sr[3]), b = (se_[0] + se_[1]) + (se_[2] + se_[3]);
    if (a > 0) atomicAdd(&counters[0], (unsigned long long)a);
    if (b > 0) atomicAdd(&counters[1], (unsigned long long)b);
  }
}

// Refined-cell update of one level (ncell cells per axis).  parent: the
// coarser level's flags before this step (NULL on the coarsest level); marks:
// this level's vertex marks (NULL: none), read at its candidates (vcls, the
// level's classes); child: the finer level's flags after this step (NULL on
// the last level of cells).
template <int D>
__global__ __launch_bounds__(256) void k_amr_cells(int ncell, uint8_t* __restrict__ cells,
                                                   const uint8_t* __restrict__ parent,
                                                   const uint8_t* __restrict__ marks,
                                                   const uint8_t* __restrict__ vcls,
                                                   const uint8_t* __restrict__ child) {
  MG_ROWS(D, ncell) {
    int c[3];
    long long i;
    if (!row_vertex<D>(row_, x_, ncell, c, i)) continue;
    bool ex = true;
    if (parent) {
      const long long pc = ncell / 3;
      long long pi = c[0] / 3 + pc * (c[1] / 3);
      if (D == 3) pi += pc * pc * (c[2] / 3);
      ex = parent[pi] != 0;
    }
    bool any_r = false, any_e = false;
    if (marks) {
      const long long nv = ncell + 1;
      for (int k = 0; k < (1 << D); ++k) {
        long long vi = (c[0] + (k & 1)) + nv * (c[1] + ((k >> 1) & 1));
        if (D == 3) vi += nv * nv * (c[2] + ((k >> 2) & 1));
        // only the candidates' marks are defined (the 3D decision pass skips chunks without one)
        const uint8_t m = vcls[vi] == kPersistent ? marks[vi] : (uint8_t)kKeep;
        any_r |= m == kRefine;
        any_e |= m == kErase;
      }
    }
    bool ch = false;
    if (child) {
      const long long cn = 3ll * ncell;
      for (int dz = 0; dz < (D == 3 ? 3 : 1); ++dz)
        for (int dy = 0; dy < 3; ++dy) {
          long long ci = 3ll * c[0] + cn * (3ll * c[1] + dy);
          if (D == 3) ci += cn * cn * (3ll * c[2] + dz);
          ch |= (child[ci] | child[ci + 1] | child[ci + 2]) != 0;
        }
    }
    const bool old = cells[i] != 0;
    cells[i] = (ex && (any_r || (old && !(any_e && !ch)))) ? 1 : 0;
  }
}

// Vertex classes of one level from the presence of its cells (parent: the
// coarser level's refined-cell flags; NULL on the coarsest level, where every
// cell is present).
template <int D>
__global__ __launch_bounds__(256) void k_amr_classify(int n, uint8_t* __restrict__ cls,
                                                      const uint8_t* __restrict__ parent) {
  const long long pc = (n - 1) / 3;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    const bool in_row = row_vertex<D>(row_, x_, n, j, i);
    uint8_t v = kAbsent;
    if (in_row) {
      bool inner = true;
      for (int a = 0; a < D; ++a) inner = inner && j[a] >= 1 && j[a] <= n - 2;
      // the 2^d cells around the vertex: loads with clamped indices and no
      // branch, validity applied afterwards, so that they issue together
      int cnt = 0;
#pragma unroll
      for (int k = 0; k < (1 << D); ++k) {
        bool ok = true;
        long long pi = 0, mul = 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const int c = j[a] - ((k >> a) & 1);
          ok = ok && c >= 0 && c <= n - 2;
          pi += mul * (min(max(c, 0), n - 2) / 3);
          mul *= pc;
        }
        const int pv = parent ? (int)parent[pi] : 1;
        cnt += (ok && pv != 0) ? 1 : 0;
      }
      if (inner) v = cnt == (1 << D) ? kPersistent : (cnt > 0 ? kHanging : kAbsent);
      else v = cnt > 0 ? kBoundary : kAbsent;
      cls[i] = v;
    }
  }
}

// The same on a 3D level as a march along z (the grid of the criterion
// march): the parent flags a lane needs for a chunk of kAmrTz planes -- the
// cells x-1 and x, y-1 and y, and z-1 and z for every plane of the chunk lie
// under at most 2 x 2 x 4 parent cells -- are read once per chunk into a bit
// mask, and the activity byte of the chunk is written once (0 or 1), so the
// map needs no clearing.  absent_map holds, per chunk, whether the target
// buffer is known to hold only absent classes there (it travels with the
// buffer): a chunk that stays absent costs its parent flags and no store.
__global__ __launch_bounds__(256) void k_amr_classify3(int n, uint8_t* __restrict__ cls,
                                                       const uint8_t* __restrict__ parent,
                                                       uint8_t* __restrict__ act_map,
                                                       uint8_t* __restrict__ absent_map) {
  const int lane = threadIdx.x & 63;
  const int nzc = (n + kAmrTz - 1) / kAmrTz, gx = (n + 63) / 64;
  const long long plane = (long long)n * n;
  const long long pc = (n - 1) / 3;   // parent cells per axis
  const int items = gx * n * nzc;
  for (AmrWalk w = amr_walk(gx);; w.q += w.step) {
    const int it = w.item();
    if (it >= items) break;
    const int bx = it % gx, t = it / gx;
    const int y = t % n, zs = (t / n) * kAmrTz, ze = min(zs + kAmrTz, n);
    const int x = bx * 64 + lane;
    const bool xin = x < n;
    const int xc = xin ? x : n - 1;
    // x: cell xc-1 (present only if xc >= 1) and cell xc (only if xc <= n-2)
    const bool vx[2] = {xc >= 1, xc <= n - 2};
    const long long px[2] = {(long long)(max(xc - 1, 0) / 3), (long long)(min(xc, n - 2) / 3)};
    const bool vy[2] = {y >= 1, y <= n - 2};
    const long long py[2] = {(long long)(max(y - 1, 0) / 3), (long long)(min(y, n - 2) / 3)};
    // parent planes under the cells zs-1 .. ze-1 (clamped to the grid of cells)
    const int pz0 = max(zs - 1, 0) / 3, pz1 = min(ze - 1, n - 2) / 3;
    unsigned ex = 0xFFFFu;   // bit 4 (pz - pz0) + 2 b + a: parent (px[a], py[b], pz) refined
    if (parent) {
      ex = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pz = min(pz0 + q, pz1);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a)
            if (parent[((long long)pz * pc + py[b]) * pc + px[a]]) ex |= 1u << (4 * q + 2 * b + a);
      }
    }
    // no parent refined around any lane: every vertex of the chunk is absent;
    // when the target buffer already holds zeros there, nothing is written
    const bool present = __ballot(xin && ex != 0u) != 0;
    if (!present && absent_map[it]) {
      if (act_map && lane == 0) act_map[it] = 0;
      continue;
    }
    bool any = false;
    for (int z = zs; z < ze; ++z) {
      const bool vz[2] = {z >= 1, z <= n - 2};
      const int qz[2] = {max(z - 1, 0) / 3 - pz0, min(z, n - 2) / 3 - pz0};
      int cnt = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a)
            cnt += (vz[c] && vy[b] && vx[a] && ((ex >> (4 * qz[c] + 2 * b + a)) & 1u)) ? 1 : 0;
      const bool inner = xc >= 1 && xc <= n - 2 && y >= 1 && y <= n - 2 && z >= 1 && z <= n - 2;
      uint8_t v;
      if (inner) v = cnt == 8 ? kPersistent : (cnt > 0 ? kHanging : kAbsent);
      else v = cnt > 0 ? kBoundary : kAbsent;
      if (xin) cls[(long long)z * plane + (long long)y * n + x] = v;
      any = any || (xin && v == kPersistent);
    }
    const bool act = __ballot(any) != 0;
    if (lane == 0) {
      if (act_map) act_map[it] = act ? 1 : 0;
      absent_map[it] = present ? 0 : 1;
    }
  }
}

// Vertices that became persistent, and hanging vertices, take P u_c;
// vertices that became absent or boundary are set to zero; the others keep
// their values.
template <int D>
__global__ __launch_bounds__(256) void k_amr_interp(int n, const uint8_t* __restrict__ cls_old,
                                                    const uint8_t* __restrict__ cls_new,
                                                    const cpx<double>* __restrict__ uc, cpx<double>* __restrict__ u) {
  const int nc = (n - 1) / 3 + 1;
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const uint8_t a = cls_new[i];
    const uint8_t o = cls_old[i];
    if (a == kHanging || (a == kPersistent && o != kPersistent)) u[i] = prolong_at<double, D>(uc, nc, j);
    else if ((a == kAbsent || a == kBoundary) && a != o) u[i] = czero<double>();
  }
}

// The same on a 3D level as a march along z.  A chunk known to be absent
// before and after the step (the classification's absent maps) is skipped;
// otherwise the class bytes of its kAmrTz planes are read first, and a chunk
// in which no lane has a vertex to write costs nothing more.  Where some lane takes P u_c: P is separable, so a
// lane interpolates its coarse corners in x and y once per coarse plane and
// keeps the two coarse planes that bracket its z in registers.  Corners are
// clamped so that every lane (boundary ones included) computes a bracket
// inside the coarse grid.
__device__ inline cpx<double> amr_xy(const cpx<double>* __restrict__ v, long long base, const long long ci[4],
                                     const double cw[4]) {
  cpx<double> acc = czero<double>();
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = acc + cw[k] * v[base + ci[k]];
  return acc;
}

__global__ __launch_bounds__(256) void k_amr_interp3(int n, const uint8_t* __restrict__ cls_old,
                                                     const uint8_t* __restrict__ cls_new,
                                                     const uint8_t* __restrict__ absent_old,
                                                     const uint8_t* __restrict__ absent_new,
                                                     const cpx<double>* __restrict__ uc,
                                                     cpx<double>* __restrict__ u) {
  const int nc = (n - 1) / 3 + 1;
  const int lane = threadIdx.x & 63;
  const int nzc = (n + kAmrTz - 1) / kAmrTz, gx = (n + 63) / 64;
  const long long pl = (long long)nc * nc;
  const long long plane = (long long)n * n;
  const int items = gx * n * nzc;
  for (AmrWalk w = amr_walk(gx);; w.q += w.step) {
    const int it = w.item();
    if (it >= items) break;
    if (absent_old[it] && absent_new[it]) continue;   // absent before and after: nothing to write
    const int bx = it % gx, t = it / gx;
    const int y = t % n, zs = (t / n) * kAmrTz, ze = min(zs + kAmrTz, n);
    const int x = bx * 64 + lane;
    const bool xin = x < n;
    const int xs = xin ? x : n - 1;
    const int mx = min(xs / 3, nc - 2);
    const double wx1 = (double)(xs - 3 * mx) / 3.0, wx0 = 1.0 - wx1;
    const long long row = (long long)y * n + xs;
    // what each plane of the chunk asks of this lane: 1 take P u_c, 2 set to zero
    unsigned acts = 0;
#pragma unroll
    for (int q = 0; q < kAmrTz; ++q) {
      const long long e = (long long)min(zs + q, ze - 1) * plane + row;
      const uint8_t a = xin ? cls_new[e] : (uint8_t)kAbsent, o = xin ? cls_old[e] : (uint8_t)kAbsent;
      const unsigned act = (a == kHanging || (a == kPersistent && o != kPersistent))
                               ? 1u
                               : (((a == kAbsent || a == kBoundary) && a != o) ? 2u : 0u);
      if (zs + q < ze) acts |= act << (2 * q);
    }
    if (__ballot(acts != 0) == 0) continue;
    const bool take = __ballot((acts & 0x5555u) != 0) != 0;
    long long ci[4] = {0, 0, 0, 0};
    double cw[4] = {0, 0, 0, 0};
    int mz = min(zs / 3, nc - 2);
    cpx<double> s0 = czero<double>(), s1 = czero<double>();
    if (take) {
      const int my = min(y / 3, nc - 2);
      const double wy1 = (double)(y - 3 * my) / 3.0, wy0 = 1.0 - wy1;
      ci[0] = (long long)my * nc + mx;
      ci[1] = ci[0] + 1;
      ci[2] = ci[0] + nc;
      ci[3] = ci[2] + 1;
      cw[0] = wy0 * wx0;
      cw[1] = wy0 * wx1;
      cw[2] = wy1 * wx0;
      cw[3] = wy1 * wx1;
      s0 = amr_xy(uc, mz * pl, ci, cw);
      s1 = amr_xy(uc, (mz + 1) * pl, ci, cw);
    }
    for (int z = zs; z < ze; ++z) {
      const int m = min(z / 3, nc - 2);
      if (take && m != mz) {   // the next coarse interval: shift the bracket by one plane
        mz = m;
        s0 = s1;
        s1 = amr_xy(uc, (mz + 1) * pl, ci, cw);
      }
      const unsigned act = (acts >> (2 * (z - zs))) & 3u;
      if (!xin || act == 0) continue;
      const long long e = (long long)z * plane + row;
      const double wz1 = (double)(z - 3 * m) / 3.0, wz0 = 1.0 - wz1;
      u[e] = csel(act == 1, wz0 * s0 + wz1 * s1, czero<double>());
    }
  }
}

// Counts of the four classes of one level.
template <int D>
__global__ __launch_bounds__(256) void k_amr_count(int n, const uint8_t* __restrict__ cls,
                                                   unsigned long long* __restrict__ out) {
  unsigned c[4] = {0, 0, 0, 0};
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    const uint8_t v = cls[i];
    c[0] += v == 0;
    c[1] += v == 1;
    c[2] += v == 2;
    c[3] += v == 3;
  }
  for (int t = 0; t < 4; ++t) {
    double s = wave_sum((double)c[t]);
    if ((threadIdx.x & 63) == 0 && s > 0) atomicAdd(&out[t], (unsigned long long)s);
  }
}

__global__ void k_amr_zero(unsigned long long* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}


template <class F2, class F3, class... A>
hipError_t amr_launch(int dim, F2 k2, F3 k3, dim3 g, hipStream_t s, A... a) {
  if (dim == 3) hipLaunchKernelGGL(k3, g, dim3(256), 0, s, a...);
  else hipLaunchKernelGGL(k2, g, dim3(256), 0, s, a...);
  return hipGetLastError();
}

struct AmrLevel {
  int n = 0;
  long long N = 0;
  uint8_t* cls = nullptr;
  uint8_t* cls_old = nullptr;
  uint8_t* marks = nullptr;
  uint8_t* cells = nullptr;   // levels below the finest only
  long long ncells = 0;
  uint8_t* act = nullptr;     // 3D: activity map of the criterion march (written whole by the classification)
  long long nact = 0;         // its bytes
  uint8_t* amap = nullptr;    // 3D: chunks of cls known to hold only absent classes
  uint8_t* amap_old = nullptr;   // the same for cls_old
  bool marked = false;
};

}  // namespace
}  // namespace mg

using namespace mg;

struct mg_amr {
  int dim = 0, lmin = 0, lkeep = 0, lmax = 0;
  hipStream_t s = nullptr;
  std::vector<AmrLevel> lv;   // index level - lmin
  double* part = nullptr;
  double* stats = nullptr;
  unsigned long long* hist = nullptr;      // kAmrMaxBins bin counts, 2 mark counters, 4 class counts
  std::vector<void*> owned;

  AmrLevel& at(int l) { return lv[l - lmin]; }

  int alloc(void** p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(MG_ENOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    owned.push_back(*p);
    return MG_OK;
  }

  ~mg_amr() {
    for (void* p : owned) (void)hipFree(p);
  }

  int classify_all() {
    for (int l = lmin; l <= lmax; ++l) {
      AmrLevel& v = at(l);
      std::swap(v.cls, v.cls_old);
      std::swap(v.amap, v.amap_old);
      const uint8_t* par = l > lmin ? at(l - 1).cells : nullptr;
      if (dim == 3) {
        hipLaunchKernelGGL(k_amr_classify3, amr_march_grid(v.n), dim3(256), 0, s, v.n, v.cls, par, v.act, v.amap);
        MG_HIP(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_amr_classify<2>, amr_grid(v.n, dim), dim3(256), 0, s, v.n, v.cls, par);
        MG_HIP(hipGetLastError());
      }
    }
    return MG_OK;
  }

  int sync_old() {
    for (int l = lmin; l <= lmax; ++l) {
      MG_HIP(hipMemcpyAsync(at(l).cls_old, at(l).cls, at(l).N, hipMemcpyDeviceToDevice, s));
      if (at(l).amap)
        MG_HIP(hipMemcpyAsync(at(l).amap_old, at(l).amap, (size_t)at(l).nact, hipMemcpyDeviceToDevice, s));
    }
    return MG_OK;
  }
};

extern "C" {

int mg_amr_setup(int dim, int level_min, int level_keep, int level_max, void* hip_stream, mg_amr** out) {
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(MG_EINVAL, "dim must be 2 or 3");
  if (level_min < 1 || level_keep < level_min || level_max < level_keep)
    return fail(MG_EINVAL, "need 1 <= level_min <= level_keep <= level_max");
  if (level_max > (dim == 3 ? 6 : 9)) return fail(MG_EINVAL, "level_max too large (3D: <= 6, 2D: <= 9)");
  mg_amr* a = new mg_amr();
  a->dim = dim;
  a->lmin = level_min;
  a->lkeep = level_keep;
  a->lmax = level_max;
  a->s = (hipStream_t)hip_stream;
  int rc = MG_OK;
  for (int l = level_min; l <= level_max && rc == MG_OK; ++l) {
    AmrLevel v;
    v.n = (int)ipow(3, l) + 1;
    v.N = ipow(v.n, dim);
    v.ncells = l < level_max ? ipow(ipow(3, l), dim) : 0;
    rc = a->alloc((void**)&v.cls, v.N);
    if (rc == MG_OK) rc = a->alloc((void**)&v.cls_old, v.N);
    if (rc == MG_OK) rc = a->alloc((void**)&v.marks, v.N);
    if (rc == MG_OK) {
      const hipError_t e = hipMemsetAsync(v.marks, 0, v.N, a->s);
      if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    }
    if (rc == MG_OK && v.ncells) rc = a->alloc((void**)&v.cells, v.ncells);
    if (rc == MG_OK && dim == 3) {
      // one byte per (x block of 64, row, chunk of planes), as the classification and the march enumerate them
      const dim3 gc = amr_grid(v.n, dim);
      const long long items = (long long)gc.x * v.n * ((v.n + kAmrTz - 1) / kAmrTz);
      v.nact = items;
      rc = a->alloc((void**)&v.act, (size_t)v.nact);
      // nothing is known of the fresh class buffers: every chunk is written the first time
      if (rc == MG_OK) rc = a->alloc((void**)&v.amap, (size_t)v.nact);
      if (rc == MG_OK) rc = a->alloc((void**)&v.amap_old, (size_t)v.nact);
      for (uint8_t* m : {v.amap, v.amap_old})
        if (rc == MG_OK) {
          const hipError_t e = hipMemsetAsync(m, 0, (size_t)v.nact, a->s);
          if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
        }
    }
    if (rc == MG_OK && v.ncells) {
      const hipError_t e = hipMemsetAsync(v.cells, l < level_keep ? 1 : 0, v.ncells, a->s);
      if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    }
    a->lv.push_back(v);
  }
  if (rc == MG_OK) rc = a->alloc((void**)&a->part, 3 * sizeof(double) * kAmrMaxParts);
  if (rc == MG_OK) rc = a->alloc((void**)&a->stats, 8 * sizeof(double));
  if (rc == MG_OK) rc = a->alloc((void**)&a->hist, (kAmrMaxBins + 8) * sizeof(unsigned long long));
  if (rc == MG_OK) rc = a->classify_all();
  if (rc == MG_OK) rc = a->sync_old();
  if (rc == MG_OK) {
    const hipError_t e = hipStreamSynchronize(a->s);
    if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("adaptivity setup: ") + hipGetErrorString(e));
  }
  if (rc != MG_OK) {
    delete a;
    return rc;
  }
  *out = a;
  return MG_OK;
}

void mg_amr_destroy(mg_amr* a) {
  if (!a) return;
  (void)hipStreamSynchronize(a->s);
  delete a;
}

int mg_amr_mark(mg_amr* a, int level, const mg_c128* u, const mg_c128* r, mg_c128 diag, const mg_c128* diag_field,
                int nbins, int refine_pct,
                int erase_pct, double veto, long long* counts, double* s_range) {
  if (!a || !u) return fail(MG_EINVAL, "NULL argument");
  if (level < a->lmin || level > a->lmax) return fail(MG_EINVAL, "level outside the envelope");
  if (nbins < 1 || nbins > kAmrMaxBins) return fail(MG_EINVAL, "nbins must be in 1..64");
  if (refine_pct < 0 || refine_pct > 100 || erase_pct < 0 || erase_pct > 100 || !(veto >= 0))
    return fail(MG_EINVAL, "percentages in 0..100 and veto >= 0");
  AmrLevel& v = a->at(level);
  if (v.N % 4) return fail(MG_EINVAL, "level size not a multiple of 4 bytes");
  const double veto2 = veto * veto;   // the per-vertex threshold veto^2 |diag_i|^2
  const dim3 g = amr_grid(v.n, a->dim);
  const int nparts = (int)(g.x * g.y);
  unsigned long long* counters = a->hist + kAmrMaxBins;
  const dim3 gm = amr_march_grid(v.n);
  const bool march = a->dim == 3;
  const int nparts_used = march ? (int)(gm.x * gm.y) : nparts;
  if (march) hipLaunchKernelGGL((k_amr_crit3<0, false>), gm, dim3(256), 0, a->s, v.n, (const cpx<double>*)u,
                                (const cpx<double>*)r, (const cpx<double>*)diag_field, veto2, (const uint8_t*)v.cls,
                                (const uint8_t*)v.act, a->part,
                                (const double*)a->stats,
                                nbins, v.marks, a->hist);
  else hipLaunchKernelGGL(k_amr_range<2>, g, dim3(256), 0, a->s, v.n, (const cpx<double>*)u, (const uint8_t*)v.cls,
                          a->part);
  MG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_amr_range_finish, dim3(1), dim3(256), 0, a->s, (const double*)a->part, nparts_used, diag.re,
                     diag.im, veto, a->stats, a->hist, counters);
  MG_HIP(hipGetLastError());
  if (march && diag_field && r)
    hipLaunchKernelGGL((k_amr_crit3<1, true>), gm, dim3(256), 0, a->s, v.n, (const cpx<double>*)u,
                       (const cpx<double>*)r, (const cpx<double>*)diag_field, veto2, (const uint8_t*)v.cls,
                       (const uint8_t*)v.act, a->part, (const double*)a->stats, nbins, v.marks, a->hist);
  else if (march)
    hipLaunchKernelGGL((k_amr_crit3<1, false>), gm, dim3(256), 0, a->s, v.n, (const cpx<double>*)u,
                       (const cpx<double>*)r, (const cpx<double>*)nullptr, veto2, (const uint8_t*)v.cls,
                       (const uint8_t*)v.act, a->part, (const double*)a->stats, nbins, v.marks, a->hist);
  else hipLaunchKernelGGL(k_amr_bin<2>, g, dim3(256), 0, a->s, v.n, (const cpx<double>*)u, (const cpx<double>*)r,
                          (const cpx<double>*)diag_field, veto2,
                          (const uint8_t*)v.cls, (const double*)a->stats, nbins, v.marks, a->hist);
  MG_HIP(hipGetLastError());
  const long long nwords = v.N / 4;
  const unsigned gd = (unsigned)std::min<long long>((nwords + 255) / 256, 8192);
  hipLaunchKernelGGL(k_amr_choose, dim3(1), dim3(64), 0, a->s, (const unsigned long long*)a->hist, a->stats, nbins,
                     refine_pct, erase_pct);
  MG_HIP(hipGetLastError());
  if (march)
    hipLaunchKernelGGL(k_amr_decide3, gm, dim3(256), 0, a->s, v.n, v.marks, (const uint8_t*)v.cls,
                       (const uint8_t*)v.act, (const double*)a->stats, nbins, level < a->lmax ? 1 : 0,
                       level >= a->lkeep ? 1 : 0, counters);
  else
    hipLaunchKernelGGL(k_amr_decide, dim3(gd), dim3(256), 0, a->s, nwords, (uint32_t*)v.marks,
                       (const uint32_t*)v.cls, (const unsigned long long*)a->hist, a->stats, nbins, refine_pct,
                       erase_pct, level < a->lmax ? 1 : 0, level >= a->lkeep ? 1 : 0, counters);
  MG_HIP(hipGetLastError());
  v.marked = true;
  if (counts || s_range) {
    std::vector<unsigned long long> h(kAmrMaxBins + 2);
    double st[8];
    MG_HIP(hipMemcpyAsync(h.data(), a->hist, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, a->s));
    MG_HIP(hipMemcpyAsync(st, a->stats, sizeof(st), hipMemcpyDeviceToHost, a->s));
    MG_HIP(hipStreamSynchronize(a->s));
    if (counts) {
      for (int t = 0; t < nbins; ++t) counts[t] = (long long)h[t];
      counts[nbins + 0] = (long long)st[4];
      counts[nbins + 1] = (long long)st[5];
      counts[nbins + 2] = (long long)st[2];
      counts[nbins + 3] = (long long)h[kAmrMaxBins + 0];
      counts[nbins + 4] = (long long)h[kAmrMaxBins + 1];
    }
    if (s_range) {
      s_range[0] = st[0];
      s_range[1] = st[1];
    }
  }
  return MG_OK;
}

int mg_amr_adapt(mg_amr* a, long long* class_counts) {
  if (!a) return fail(MG_EINVAL, "NULL argument");
  for (int l = a->lmax - 1; l >= a->lmin; --l) {
    AmrLevel& v = a->at(l);
    const int nc = v.n - 1;
    MG_HIP(amr_launch(a->dim, k_amr_cells<2>, k_amr_cells<3>, amr_grid(nc, a->dim), a->s, nc, v.cells,
                      (const uint8_t*)(l > a->lmin ? a->at(l - 1).cells : nullptr),
                      (const uint8_t*)(v.marked ? v.marks : nullptr), (const uint8_t*)v.cls,
                      (const uint8_t*)(l + 1 < a->lmax ? a->at(l + 1).cells : nullptr)));
  }
  for (int l = a->lmin; l <= a->lmax; ++l) a->at(l).marked = false;
  MG_TRY(a->classify_all());
  if (class_counts) {
    const int nl = a->lmax - a->lmin + 1;
    std::vector<unsigned long long> h(4 * (size_t)nl);
    unsigned long long* dc = a->hist + kAmrMaxBins + 2;
    for (int l = a->lmin; l <= a->lmax; ++l) {
      AmrLevel& v = a->at(l);
      hipLaunchKernelGGL(k_amr_zero, dim3(1), dim3(64), 0, a->s, dc, 4);
      MG_HIP(amr_launch(a->dim, k_amr_count<2>, k_amr_count<3>, amr_grid(v.n, a->dim), a->s, v.n,
                        (const uint8_t*)v.cls, dc));
      MG_HIP(hipMemcpyAsync(&h[4 * (size_t)(l - a->lmin)], dc, 4 * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, a->s));
      MG_HIP(hipStreamSynchronize(a->s));
    }
    for (size_t t = 0; t < h.size(); ++t) class_counts[t] = (long long)h[t];
  }
  return MG_OK;
}

int mg_amr_interpolate(mg_amr* a, int level, const mg_c128* u_coarse, mg_c128* u) {
  if (!a || !u_coarse || !u) return fail(MG_EINVAL, "NULL argument");
  if (level <= a->lmin || level > a->lmax) return fail(MG_EINVAL, "level must lie in (level_min, level_max]");
  AmrLevel& v = a->at(level);
  if (a->dim == 3) {
    hipLaunchKernelGGL(k_amr_interp3, amr_march_grid(v.n), dim3(256), 0, a->s, v.n, (const uint8_t*)v.cls_old,
                       (const uint8_t*)v.cls, (const uint8_t*)v.amap_old, (const uint8_t*)v.amap,
                       (const cpx<double>*)u_coarse, (cpx<double>*)u);
    MG_HIP(hipGetLastError());
  } else {
    hipLaunchKernelGGL(k_amr_interp<2>, amr_grid(v.n, a->dim), dim3(256), 0, a->s, v.n, (const uint8_t*)v.cls_old,
                       (const uint8_t*)v.cls, (const cpx<double>*)u_coarse, (cpx<double>*)u);
    MG_HIP(hipGetLastError());
  }
  return MG_OK;
}

int mg_amr_get(mg_amr* a, int level, int what, unsigned char* out) {
  if (!a || !out) return fail(MG_EINVAL, "NULL argument");
  if (level < a->lmin || level > a->lmax) return fail(MG_EINVAL, "level outside the envelope");
  AmrLevel& v = a->at(level);
  const uint8_t* src = nullptr;
  size_t bytes = (size_t)v.N;
  switch (what) {
    case 0: src = v.cls; break;
    case 1: src = v.cls_old; break;
    case 2:
      if (!v.cells) return fail(MG_EINVAL, "the finest level has no refined-cell flags");
      src = v.cells;
      bytes = (size_t)v.ncells;
      break;
    case 3: {
      const unsigned g = (unsigned)std::min<long long>((v.N + 255) / 256, 8192);
      hipLaunchKernelGGL(k_amr_mask_marks, dim3(g), dim3(256), 0, a->s, v.N, (const uint8_t*)v.marks,
                         (const uint8_t*)v.cls, out);
      MG_HIP(hipGetLastError());
      return MG_OK;
    }
    default: return fail(MG_EINVAL, "what must be 0..3");
  }
  MG_HIP(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, a->s));
  return MG_OK;
}

int mg_amr_set_cells(mg_amr* a, int level, const unsigned char* cells) {
  if (!a || !cells) return fail(MG_EINVAL, "NULL argument");
  if (level < a->lmin || level >= a->lmax) return fail(MG_EINVAL, "level must lie in [level_min, level_max)");
  AmrLevel& v = a->at(level);
  MG_HIP(hipMemcpyAsync(v.cells, cells, (size_t)v.ncells, hipMemcpyDeviceToDevice, a->s));
  MG_TRY(a->classify_all());
  return a->sync_old();
}

}  // extern "C"
