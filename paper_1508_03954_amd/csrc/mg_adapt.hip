// Feature-based dynamic adaptivity (Section 5.3) with hanging vertices
// (Section 4) on a dense envelope of levels.
//
// The spacetree is held as one byte per cell and level ("refined into the 3^d
// cells of the next level") over the full regular grid of every level, plus
// one class byte per vertex (absent / persistent / hanging / boundary).  Every
// pass is then a coalesced row sweep over a regular array: no pointer chasing,
// no per-vertex index tables; the cost of a level pass scales with the level's
// envelope, not with the vertices present (the envelope of a 3D level-6
// hierarchy, 389 M vertices, takes 1.2 GB of class and mark bytes).
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
// a vertex that became persistent or hanging takes P u of the coarser level.
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
          v = rv.re * rv.re + rv.im * rv.im > thr;
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

// Bins to marks, four bytes per lane; counts the refine and erase marks.
__global__ __launch_bounds__(256) void k_amr_decide(long long nwords, uint32_t* __restrict__ marks,
                                                    const unsigned long long* __restrict__ hist,
                                                    double* __restrict__ stats, int nb, int rpct, int epct,
                                                    int can_refine, int can_erase,
                                                    unsigned long long* __restrict__ counters) {
  __shared__ int sk, se;
  __shared__ double sr[4], se_[4];
  if (threadIdx.x == 0) {
    int k, e;
    amr_choose(hist, nb, (long long)stats[2], rpct, epct, k, e);
    sk = k;
    se = e;
    if (blockIdx.x == 0) {
      stats[4] = k;
      stats[5] = e;
    }
  }
  __syncthreads();
  const uint32_t top = (uint32_t)(nb - sk), bot = (uint32_t)se;
  double nr = 0, ne = 0;
  for (long long w = blockIdx.x * 256ll + threadIdx.x; w < nwords; w += (long long)gridDim.x * 256) {
    const uint32_t v = marks[w];
    uint32_t o = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t m = (v >> (8 * q)) & 0xFFu;
      uint32_t d = kKeep;
      if (!(m & (kNotCand | kVetoBit))) {
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
// this level's vertex marks (NULL: none); child: the finer level's flags after
// this step (NULL on the last level of cells).
template <int D>
__global__ __launch_bounds__(256) void k_amr_cells(int ncell, uint8_t* __restrict__ cells,
                                                   const uint8_t* __restrict__ parent,
                                                   const uint8_t* __restrict__ marks,
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
        const uint8_t m = marks[vi];
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
  MG_ROWS(D, n) {
    int j[3];
    long long i;
    if (!row_vertex<D>(row_, x_, n, j, i)) continue;
    bool inner = true;
    for (int a = 0; a < D; ++a) inner = inner && j[a] >= 1 && j[a] <= n - 2;
    int cnt = 0;
    const long long pc = (n - 1) / 3;
    for (int k = 0; k < (1 << D); ++k) {
      int c[3] = {j[0] - (k & 1), j[1] - ((k >> 1) & 1), D == 3 ? j[2] - ((k >> 2) & 1) : 0};
      bool ok = true;
      for (int a = 0; a < D; ++a) ok = ok && c[a] >= 0 && c[a] <= n - 2;
      if (!ok) continue;
      if (parent) {
        long long pi = c[0] / 3 + pc * (c[1] / 3);
        if (D == 3) pi += pc * pc * (c[2] / 3);
        if (!parent[pi]) continue;
      }
      ++cnt;
    }
    uint8_t v;
    if (inner) v = cnt == (1 << D) ? kPersistent : (cnt > 0 ? kHanging : kAbsent);
    else v = cnt > 0 ? kBoundary : kAbsent;
    cls[i] = v;
  }
}

// Vertices that became persistent, and hanging vertices, take P u_c; absent
// and boundary vertices hold zero; the others keep their values.
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
    if (a == kHanging || (a == kPersistent && cls_old[i] != kPersistent)) u[i] = prolong_at<double, D>(uc, nc, j);
    else if (a == kAbsent || a == kBoundary) u[i] = czero<double>();
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
      MG_HIP(amr_launch(dim, k_amr_classify<2>, k_amr_classify<3>, amr_grid(v.n, dim), s, v.n, v.cls,
                        (const uint8_t*)(l > lmin ? at(l - 1).cells : nullptr)));
    }
    return MG_OK;
  }

  int sync_old() {
    for (int l = lmin; l <= lmax; ++l)
      MG_HIP(hipMemcpyAsync(at(l).cls_old, at(l).cls, at(l).N, hipMemcpyDeviceToDevice, s));
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
    if (rc == MG_OK && v.ncells) rc = a->alloc((void**)&v.cells, v.ncells);
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

int mg_amr_mark(mg_amr* a, int level, const mg_c128* u, const mg_c128* r, mg_c128 diag, int nbins, int refine_pct,
                int erase_pct, double veto, long long* counts, double* s_range) {
  if (!a || !u) return fail(MG_EINVAL, "NULL argument");
  if (level < a->lmin || level > a->lmax) return fail(MG_EINVAL, "level outside the envelope");
  if (nbins < 1 || nbins > kAmrMaxBins) return fail(MG_EINVAL, "nbins must be in 1..64");
  if (refine_pct < 0 || refine_pct > 100 || erase_pct < 0 || erase_pct > 100 || !(veto >= 0))
    return fail(MG_EINVAL, "percentages in 0..100 and veto >= 0");
  AmrLevel& v = a->at(level);
  if (v.N % 4) return fail(MG_EINVAL, "level size not a multiple of 4 bytes");
  const dim3 g = amr_grid(v.n, a->dim);
  const int nparts = (int)(g.x * g.y);
  unsigned long long* counters = a->hist + kAmrMaxBins;
  MG_HIP(amr_launch(a->dim, k_amr_range<2>, k_amr_range<3>, g, a->s, v.n, (const cpx<double>*)u,
                    (const uint8_t*)v.cls, a->part));
  hipLaunchKernelGGL(k_amr_range_finish, dim3(1), dim3(256), 0, a->s, (const double*)a->part, nparts, diag.re,
                     diag.im, veto, a->stats, a->hist, counters);
  MG_HIP(hipGetLastError());
  MG_HIP(amr_launch(a->dim, k_amr_bin<2>, k_amr_bin<3>, g, a->s, v.n, (const cpx<double>*)u, (const cpx<double>*)r,
                    (const uint8_t*)v.cls, (const double*)a->stats, nbins, v.marks, a->hist));
  const long long nwords = v.N / 4;
  const unsigned gd = (unsigned)std::min<long long>((nwords + 255) / 256, 8192);
  hipLaunchKernelGGL(k_amr_decide, dim3(gd), dim3(256), 0, a->s, nwords, (uint32_t*)v.marks,
                     (const unsigned long long*)a->hist, a->stats, nbins, refine_pct, erase_pct,
                     level < a->lmax ? 1 : 0, level >= a->lkeep ? 1 : 0, counters);
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
                      (const uint8_t*)(v.marked ? v.marks : nullptr),
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
  MG_HIP(amr_launch(a->dim, k_amr_interp<2>, k_amr_interp<3>, amr_grid(v.n, a->dim), a->s, v.n,
                    (const uint8_t*)v.cls_old, (const uint8_t*)v.cls, (const cpx<double>*)u_coarse,
                    (cpx<double>*)u));
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
    case 3: src = v.marks; break;
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
