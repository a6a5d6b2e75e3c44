// Internal declarations shared by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mg {

// Interleaved complex number; 16 B (double) or 8 B (float), naturally aligned
// so that one vertex is one vector load.
template <class T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <class T>
__host__ __device__ inline cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.re = a;
  r.im = b;
  return r;
}

// Per-level operator data, passed by value to kernels.
//   H = alpha * S_K - etad * phi * S_M (constant phi: coef[] by neighbour class),
//   or, cell by cell, H_c = kappa_c K - mu_c M with per-cell coefficients:
//   mass mu_c = phibar_c eta_c^d (phibar_c the mean of the nodal phi over the
//   cell's vertices) and stiffness kappa_c = eta_c^(d-2) (uniform alpha unless
//   cells are rotated individually).
template <class T>
struct OpData {
  int n;                  // vertices per axis
  cpx<T> coef[4];         // constant phi: stencil weight by number of nonzero offsets
  cpx<T> alpha;           // eta^(d-2)
  cpx<T> etad;            // eta^d
  cpx<T> invD;            // constant phi: 1 / diag
  const cpx<T>* cmass;    // per-cell mass coefficients mu_c ((n-1)^d), else nullptr
  const cpx<T>* cstiff;   // per-cell stiffness coefficients kappa_c, or nullptr (alpha)
  const cpx<T>* invDv;    // per-cell path: per-vertex 1 / diag (n^d), else nullptr
};

// Rotation of the cells of one level: the complex grid scaling h -> h
// exp(i theta) of Section 2, with the absorbing layer of Section 7.4 rotating
// the cells near selected faces by their own angle.
struct CellRotation {
  double h;             // real cell side of the level, 3^-l
  double theta;         // angle of the cells outside the layer
  double layer_theta;   // angle of the layer's cells
  double width;         // layer width; 0: no layer
  int faces;            // bit 2a: face x_a = 0, bit 2a + 1: face x_a = 1 (a = 0: x, fastest)
  int conj;             // conjugate mode: every eta_c conjugated
};

// Number of blocks of every kernel that writes reduction partials; the second
// stage sums them in a fixed order, so reductions are deterministic.
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// Launch wrappers (kernels live in mg_kernels.hip).  dim in {2,3}.
template <class T>
hipError_t launch_apply(int dim, const OpData<T>& op, const cpx<T>* x, cpx<T>* y, hipStream_t s);

template <class T>
hipError_t launch_pre(int dim, int n, cpx<T>* u, cpx<T>* sc, const cpx<T>* sf, const cpx<T>* scc,
                      const cpx<T>* sic, int has_coarse, int bpx, hipStream_t s);

template <class T>
hipError_t launch_fine_pre(int dim, int n, const cpx<T>* w, cpx<T>* u, const cpx<T>* scc,
                           const cpx<T>* sic, int has_coarse, int bpx, hipStream_t s);

template <class T>
hipError_t launch_uhat(int dim, int n, const cpx<T>* u, const cpx<T>* uc, cpx<T>* uhat, hipStream_t s);

// r = b - H x; when partials != nullptr also writes per-block (sum |r|^2, max |r|)
// and stores the number of blocks (<= kRedBlocks) in *nparts.  r == nullptr:
// partials only, the residual is not stored (resid_norm_blocks(dim, n) blocks).
template <class T>
hipError_t launch_resid(int dim, const OpData<T>& op, const cpx<T>* b, const cpx<T>* x, cpx<T>* r,
                        double* partials, int* nparts, hipStream_t s);
int resid_norm_blocks(int dim, int n);   // -1 if a level is too wide for kRedBlocks partials

// Coarse post-phase of level l in the Galerkin form (op of level l): restriction
// rho_c = R rho into the coarser b slot plus the pointwise update of level l.
template <class T>
hipError_t launch_post_galerkin(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, int mask_c,
                                cpx<T>* sc, const cpx<T>* sf, cpx<T>* rhoc, cpx<T>* sfc, cpx<T>* sic,
                                hipStream_t s);

// s = omega r / D; sc = s or masked; finest: u += sc in place (sc_out == nullptr),
// coarse: sc_out = sc.  Injection: sfc = sf + sc at c-points (if sfc), sic = s (if sic).
template <class T>
hipError_t launch_update(int dim, const OpData<T>& op, const cpx<T>* r, cpx<T> omega, int mask_c,
                         cpx<T>* u_inplace, cpx<T>* sc_out, const cpx<T>* sf, cpx<T>* sfc, cpx<T>* sic,
                         hipStream_t s);

template <class T>
hipError_t launch_restrict(int dim, int nc, const cpx<T>* vf, cpx<T>* vc, hipStream_t s);

template <class T>
hipError_t launch_inject(int dim, int nc, const cpx<T>* vf, cpx<T>* vc, hipStream_t s);
// vc(m) = vf(stride m) on a level with nc vertices per axis (every vertex).
template <class T>
hipError_t launch_sample(int dim, int nc, int stride, const cpx<T>* vf, cpx<T>* vc, hipStream_t s);
// uf = P uc on the interior of the level with n vertices per axis, 0 on its boundary.
template <class T>
hipError_t launch_prolong(int dim, int n, const cpx<T>* uc, cpx<T>* uf, hipStream_t s);

// Zero-start cycle pieces: z_l = Lop(omega D^-1 rho_l) + P z_(l-1), written
// as z_l = s_l (masked on c-points for hb) + P g with g = z_(l-1), or for BPX
// g = z_(l-1) - I s_l (launch_prec_g).
template <class T>
hipError_t launch_prec_up(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, int mask_c,
                          int is_lmin, const cpx<T>* gc, cpx<T>* z, hipStream_t s);
template <class T>
hipError_t launch_prec_g(int dim, const OpData<T>& op, const cpx<T>* rho, cpx<T> omega, const cpx<T>* zc, cpx<T>* g,
                         hipStream_t s);

// Per-cell coefficients of a level with n vertices per axis from its nodal
// phi: mass mu_c = phibar_c eta_c^d and, when stiff != nullptr, stiffness
// kappa_c = eta_c^(d-2), with eta_c = h exp(i theta_c) from rot (conjugated,
// with phibar, in conjugate mode).
template <class T>
hipError_t launch_cellcoef(int dim, int n, const cpx<T>* phi, cpx<T>* mass, cpx<T>* stiff, CellRotation rot,
                           hipStream_t s);
// v = value on all `count` entries.
template <class T>
hipError_t launch_set_value(size_t count, cpx<T>* v, cpx<double> value, hipStream_t s);
// Lumped load with per-cell rotation: b_j = chi_j 2^-d sum_{c contains j} eta_c^d
// on interior vertices, 0 on the boundary (FP64).
hipError_t launch_rhs_cells(int dim, int n, const cpx<double>* chi, cpx<double>* b, CellRotation rot,
                            hipStream_t s);

template <class T>
hipError_t launch_invdiag(int dim, const OpData<T>& op, cpx<T>* invDv, hipStream_t s);

template <class T>
hipError_t launch_zero_boundary_copy(int dim, int n, const cpx<T>* in, cpx<T>* out, cpx<T> scale,
                                     hipStream_t s);

hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);

template <class S, class D>
hipError_t launch_convert(size_t count, const cpx<S>* in, cpx<D>* out, double scale, hipStream_t s);

// Vector ops for the Krylov driver (interior-only vectors: boundary entries 0).
template <class T>
hipError_t launch_dot(size_t count, const cpx<T>* a, const cpx<T>* b, double* partials, hipStream_t s);
template <class T>
hipError_t launch_norm2(size_t count, const cpx<T>* a, double* partials, hipStream_t s);
// y = a*x + b*y  (complex scalars given in double)
template <class T>
hipError_t launch_axpby(size_t count, cpx<double> a, const cpx<T>* x, cpx<double> b, cpx<T>* y,
                        hipStream_t s);
// p = r + beta (p - w v)
template <class T>
hipError_t launch_bicg_p(size_t count, const cpx<T>* r, const cpx<T>* v, cpx<double> beta,
                         cpx<double> w, cpx<T>* p, hipStream_t s);
// x += a y + w z ; r = s - w t
template <class T>
hipError_t launch_bicg_xr(size_t count, cpx<T>* x, const cpx<T>* y, const cpx<T>* z, cpx<double> a,
                          cpx<double> w, cpx<T>* r, const cpx<T>* sv, const cpx<T>* t, hipStream_t s);

// Fused BiCGStab steps; partials hold N doubles per block (kRedBlocks blocks),
// reduced by launch_finishN:
//   bicg_s   (N = 1): s = r - a v, |s|^2
//   bicg_ts  (N = 3): conj(t).s (re, im), |t|^2
//   bicg_xr2 (N = 3): x += a y + w z, r = s - w t, |r|^2, conj(rh).r (re, im)
template <class T>
hipError_t launch_bicg_s(size_t count, const cpx<T>* r, const cpx<T>* v, cpx<double> a, cpx<T>* sv, double* partials,
                         hipStream_t s);
template <class T>
hipError_t launch_bicg_ts(size_t count, const cpx<T>* t, const cpx<T>* sv, double* partials, hipStream_t s);
template <class T>
hipError_t launch_bicg_xr2(size_t count, cpx<T>* x, const cpx<T>* y, const cpx<T>* z, cpx<double> a, cpx<double> w,
                           cpx<T>* r, const cpx<T>* sv, const cpx<T>* t, const cpx<T>* rh, double* partials,
                           hipStream_t s);
hipError_t launch_finishN(int nvals, const double* partials, int count, double* out, hipStream_t s);

// Residual-refinement helpers: out64 += scale * in32 (in place FP64 accumulate).
hipError_t launch_accum32(size_t count, const cpx<float>* e, double scale, cpx<double>* u, hipStream_t s);

hipError_t launch_grad_potential(int dim, int n, cpx<double> etad, const cpx<double>* u,
                                 const cpx<double>* lam, double* g, hipStream_t s);

// Second reduction stage over `count` block partials [count][2], summed in
// block order: out[0] = sum, out[1] = max (sum_max) or sum of the second
// component (sum2).
hipError_t launch_finish_sum_max(const double* partials, int count, double* out, hipStream_t s);
hipError_t launch_finish_sum2(const double* partials, int count, double* out, hipStream_t s);

// The smallest coarse levels (a few thousand vertices at most) in one
// single-block launch each way: descent of all of them, or Galerkin
// backtracking of all of them plus the coarsest update and the norm's second
// reduction stage.  lv[k] is level l_min + k.
constexpr int kSmallMax = 4;
constexpr int kSmallVertices = 4096;
constexpr int kSmallThreads = 1024;
template <class T>
struct SmallLevel {
  int n;
  cpx<T>*u, *b, *sc, *sf, *si;
  OpData<T> op;
  cpx<T> omega;
};
template <class T>
struct SmallArgs {
  int dim, nl, variant;
  SmallLevel<T> lv[kSmallMax];
  const double* partials;   // post: block partials of the finest sweep, or nullptr
  int nparts;
  double* out;              // post: (sum |r|^2, max |r|)
  int then_pre;             // post: then also the next cycle's pre-phase of these levels
};
template <class T>
hipError_t launch_small_pre(const SmallArgs<T>& a, hipStream_t s);
template <class T>
hipError_t launch_small_post(const SmallArgs<T>& a, hipStream_t s);

// Fused finest-level sweep (GALERKIN form, constant phi); see mg_fused.hip.
template <class T>
struct FusedArgs {
  int n, nc;
  const cpx<T>* w;      // folded iterate in
  cpx<T>* wout;         // folded iterate out
  const cpx<T>* b;      // finest rhs
  const cpx<T>* scc;    // coarse sc (after its pre-phase)
  const cpx<T>* sic;    // coarse si (BPX) or nullptr
  cpx<T>* rhoc;         // coarse b slot <- R r
  cpx<T>* sfc;          // coarse sf <- I sc (ADD) or nullptr
  cpx<T>* sic_out;      // coarse si <- I s (BPX) or nullptr
  cpx<T>* spill;        // 3D: seam rows of R (fused_spill_count(3, n) entries), added by launch_fused_seam
  cpx<T>* zout;         // preconditioner-apply march: z (its wout receives H z); s update: s
  const cpx<T>* w2;     // s update of the restriction march: the vector v of s = b - alpha v
  cpx<double> alpha;    // s update: alpha (the update is formed in double precision)
  cpx<T> coef[4];
  cpx<T> ws;            // omega * (1 / D)
  double* partials;     // per-block (sum |r|^2, max |r|) or nullptr
  int variant;          // 0 add, 1 hb, 2 bpx
  int tile;             // tile variant, 0 .. fused_tile_count(dim) - 1
  int order;            // block-to-tile order (set by the launcher from the tile table)
};
// t0 / t1 (or nullptr): events that receive the sweep kernel's start and end.
template <class T>
hipError_t launch_fused(int dim, const FusedArgs<T>& a, hipStream_t s, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
// Second pass of a 3D sweep: rho_c += the seam rows of R (no-op in 2D).
template <class T>
hipError_t launch_fused_seam(int dim, const FusedArgs<T>& a, hipStream_t s);
// Entries of the seam array a sweep of any tile variant needs (0 in 2D).
size_t fused_spill_count(int dim, int n);
int fused_tile_count(int dim);
// 3D constant-phi operator with the sweep's march: y = H x (apply != 0) or
// r = b - H x with per-block partial norms (when partials != nullptr; their
// count, stencil3_blocks(n), goes to *nparts).  Needs n = 3k + 1 >= 10.
int stencil3_blocks(int n);
template <class T>
hipError_t launch_stencil3(int apply, int n, const cpx<T>* coef, const cpx<T>* b, const cpx<T>* x, cpx<T>* out,
                           double* partials, int* nparts, hipStream_t s);
int fused_partials_blocks(int dim, int n, int tile);  // -1 if unsupported
// rho_c = R x in 3D (nc coarse vertices per axis, 3 (nc - 1) + 1 >= 10 fine)
// with the sweep's march; spill: fused_spill_count(3, n) entries of scratch.
template <class T>
hipError_t launch_restrict3(int nc, const cpx<T>* x, cpx<T>* rhoc, cpx<T>* spill, hipStream_t s);
// Backtracking of a coarse level (level size 3 (nc - 1) + 1, 3D, hb or BPX) in
// the Galerkin form as the restriction march: rhoc = R rho, sc = ws rho (zero
// on c-points), for BPX sic = ws rho at c-points; the seam rows go through
// spill (coarse-level sized) and k_seam3.
template <class T>
hipError_t launch_post3(int nc, int variant, const cpx<T>* rho, cpx<T> ws, cpx<T>* sc, cpx<T>* sic, cpx<T>* rhoc,
                        cpx<T>* spill, hipStream_t s);
// The same for s = r - alpha v, computed in the march: s is stored to sv and
// partials[one per block, restrict3_blocks(nc)] receive |s|^2 over the block.
int restrict3_blocks(int nc);
template <class T>
hipError_t launch_restrict3_s(int nc, const cpx<T>* r, const cpx<T>* v, cpx<double> alpha, cpx<T>* sv, cpx<T>* rhoc,
                              cpx<T>* spill, double* partials, hipStream_t s);
// Finest level of the zero-start cycle and the operator in one 3D pass (n >= 10):
// z = s + P g with s = ws x (zero on c-points if mask_c), y = H z (constant phi).
// dot 1: partials[2 per block] of conj(v2) y; dot 2: partials[3 per block] of
// conj(y) v2 and |y|^2 (prec_apply3_blocks(n) blocks); dot 0: none.
int prec_apply3_blocks(int n);
template <class T>
hipError_t launch_prec_apply3(int n, const cpx<T>* coef, cpx<T> ws, int mask_c, const cpx<T>* x, const cpx<T>* gc,
                              cpx<T>* z, cpx<T>* y, int dot, const cpx<T>* v2, double* partials, hipStream_t s);
// Tile variant with the given shape (3D: coarse rows, rows per thread, coarse
// planes; 2D: coarse rows zc only), or -1.
int fused_tile_index(int dim, int tyc, int rpt, int zc);

}  // namespace mg
