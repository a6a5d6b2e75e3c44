// Context, cycle and solve drivers, and the extern "C" entry points of mg.h.
#include <mutex>

#include "mg_engine.h"

// Scratch of mg_residual_norm_noalloc: the per-block partials of one residual
// pass (a (sum, max) pair for each of at most kRedBlocks blocks) followed by
// the two results of the second reduction stage.  Each device holds its own
// copy until the process ends; every call on a device shares it, so calls
// that overlap on one device race.  Host code never passes `scratch` itself
// (in host code the name is a stand-in, not a device address): mg_setup
// resolves each device's address once with hipGetSymbolAddress and the entry
// point passes that.
constexpr int kNoAllocDoubles = 2 * kRedBlocks + 2;
static __device__ __align__(256) double scratch[kNoAllocDoubles];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;   // per device, nullptr until resolved

// Resolves the scratch address of the current device (once per device) and
// returns that device's index.
static int resolve_scratch(int* device) {
  MG_HIP(hipGetDevice(device));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= *device) g_scratch_ptr.resize(*device + 1, nullptr);
  if (!g_scratch_ptr[*device]) {
    void* p = nullptr;
    MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[*device] = (double*)p;
  }
  return MG_OK;
}

static double* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

static int check_params(const mg_params* p) {
  if (!p) return fail(MG_EINVAL, "params is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(MG_EINVAL, "dim must be 2 or 3");
  if (p->level_min < 1 || p->level_max < p->level_min) return fail(MG_EINVAL, "need 1 <= level_min <= level_max");
  const int maxL = p->dim == 3 ? 6 : 9;   // every vertex index fits 32 bits
  if (p->level_max > maxL) return fail(MG_EINVAL, "level_max too large (3D: <= 6, 2D: <= 9)");
  if (p->variant < MG_ADD || p->variant > MG_BPX) return fail(MG_EINVAL, "bad variant");
  if (p->omega_scheme < MG_OMEGA_CONST || p->omega_scheme > MG_OMEGA_TWO_PHASE) return fail(MG_EINVAL, "bad omega scheme");
  if (p->precision != MG_FP64 && p->precision != MG_FP32_REFINE) return fail(MG_EINVAL, "bad precision");
  if (p->restrict_form < MG_RESTRICT_AUTO || p->restrict_form > MG_RESTRICT_GALERKIN) return fail(MG_EINVAL, "bad restrict_form");
  if (p->sweep < MG_SWEEP_AUTO || p->sweep > MG_SWEEP_FUSED) return fail(MG_EINVAL, "bad sweep");
  if (!(p->layer_width >= 0) || p->layer_width > 1 || !std::isfinite(p->layer_theta))
    return fail(MG_EINVAL, "layer_width must lie in [0, 1] and layer_theta be finite");
  if (p->layer_width > 0 && (p->layer_faces <= 0 || p->layer_faces >= (1 << (2 * p->dim))))
    return fail(MG_EINVAL, "layer_faces must select at least one face of the domain and no other bits");
  return MG_OK;
}

template <class T>
static int sweep_time(Engine<T>& E, double* total_ms, int* count) {
  MG_HIP(hipStreamSynchronize(E.s));
  double tot = 0;
  for (size_t i = 0; i + 1 < E.ev_used; i += 2) {
    float ms = 0;
    MG_HIP(hipEventElapsedTime(&ms, E.ev[i], E.ev[i + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = (int)(E.ev_used / 2);
  return MG_OK;
}

extern "C" {

void mg_params_default(mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 3;
  p->level_min = 1;
  p->level_max = 3;
  p->variant = MG_BPX;
  p->omega_scheme = MG_OMEGA_CONST;
  p->omega.re = 0.6;
  p->omega_L = 1;
  p->precision = MG_FP64;
}

const char* mg_last_error(void) { return g_err.c_str(); }

int mg_setup(const mg_params* p, void* hip_stream, mg_ctx** out) {
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  MG_TRY(check_params(p));
  int device = 0;
  MG_TRY(resolve_scratch(&device));
  mg_ctx* c = new mg_ctx();
  c->p = *p;
  c->p.phi_field = nullptr;
  c->s = (hipStream_t)hip_stream;
  c->device = device;
  const cpx<double>* phi = (const cpx<double>*)p->phi_field;
  int rc;
  if (p->precision == MG_FP64) {
    c->e64 = new Engine<double>();
    rc = c->e64->setup(*p, c->s, phi);
    if (rc == MG_OK) c->op64 = c->e64->lv[p->level_max].op;
  } else {
    c->e32 = new Engine<float>();
    rc = c->e32->setup(*p, c->s, phi);
    if (rc == MG_OK) {
      // FP64 finest operator for the outer refinement loop: a single-level FP64
      // engine holds its data (constant: scalars; nodal phi: cell averages and diagonal).
      mg_params q = *p;
      q.precision = MG_FP64;
      q.sweep = MG_SWEEP_GENERIC;
      q.restrict_form = MG_RESTRICT_AUTO;
      c->e64 = new Engine<double>();
      rc = c->e64->setup(q, c->s, phi, /*op_only=*/true);
      if (rc == MG_OK) c->op64 = c->e64->lv[p->level_max].op;
    }
  }
  if (rc == MG_OK) {
    hipError_t e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) rc = fail(MG_EDEVICE, std::string("setup: ") + hipGetErrorString(e));
  }
  if (rc != MG_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  delete c;
}

int mg_level_size(const mg_ctx* c, int level) {
  if (!c || level < c->p.level_min || level > c->p.level_max) return fail(MG_EINVAL, "bad level");
  return (int)ipow(3, level) + 1;
}

static size_t finest_N(const mg_ctx* c) { return (size_t)ipow(ipow(3, c->p.level_max) + 1, c->p.dim); }

int mg_apply(mg_ctx* c, const mg_c128* x, mg_c128* y) {
  if (!c || !x || !y) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)x == (const void*)y) return fail(MG_EINVAL, "x and y must not alias");
  MG_HIP(launch_apply<double>(c->p.dim, c->op64, (const cpx<double>*)x, (cpx<double>*)y, c->s));
  return MG_OK;
}

int mg_rhs_from_nodal(mg_ctx* c, const mg_c128* chi, mg_c128* b) {
  if (!c || !chi || !b) return fail(MG_EINVAL, "NULL argument");
  if (c->p.layer_width > 0) {
    mg_params q = c->p;
    q.conjugate = 0;   // the load weight is that of the forward problem
    MG_HIP(launch_rhs_cells(c->p.dim, (int)ipow(3, c->p.level_max) + 1, (const cpx<double>*)chi, (cpx<double>*)b,
                            rotation(q, c->p.level_max), c->s));
    return MG_OK;
  }
  const LevelScalars ls = level_scalars(c->p.dim, c->p.level_max, c->p.theta, false);
  MG_HIP(launch_zero_boundary_copy<double>(c->p.dim, (int)ipow(3, c->p.level_max) + 1, (const cpx<double>*)chi,
                                           (cpx<double>*)b, to_c<double>(ls.etad), c->s));
  return MG_OK;
}

// Engine-precision staging of a c128 argument (FP32 contexts convert).
static int stage_in(mg_ctx* c, const mg_c128* src, cpx<float>** out) {
  if (!c->r32) {
    void* q;
    MG_HIP(hipMalloc(&q, finest_N(c) * sizeof(cpx<float>)));
    c->owned.push_back(q);
    c->r32 = (cpx<float>*)q;
  }
  MG_HIP((launch_convert<double, float>(finest_N(c), (const cpx<double>*)src, c->r32, 1.0, c->s)));
  *out = c->r32;
  return MG_OK;
}

static int stage_e32(mg_ctx* c) {
  if (!c->e32v) {
    void* q;
    MG_HIP(hipMalloc(&q, finest_N(c) * sizeof(cpx<float>)));
    c->owned.push_back(q);
    c->e32v = (cpx<float>*)q;
  }
  return MG_OK;
}

int mg_set_rhs(mg_ctx* c, const mg_c128* b) {
  if (!c || !b) return fail(MG_EINVAL, "NULL argument");
  if (c->p.precision == MG_FP64) return c->e64->set_rhs((const cpx<double>*)b);
  cpx<float>* t;
  MG_TRY(stage_in(c, b, &t));
  return c->e32->set_rhs(t);
}

int mg_set_solution(mg_ctx* c, const mg_c128* u) {
  if (!c || !u) return fail(MG_EINVAL, "NULL argument");
  if (c->p.precision == MG_FP64) return c->e64->set_solution((const cpx<double>*)u);
  cpx<float>* t;
  MG_TRY(stage_in(c, u, &t));
  return c->e32->set_solution(t);
}

int mg_cycle(mg_ctx* c, int ncycles, double* res_h, double* res_max) {
  if (!c || ncycles < 0) return fail(MG_EINVAL, "bad argument");
  if (ncycles == 0) return MG_OK;
  if (c->p.precision == MG_FP64) return c->e64->cycles(ncycles, res_h, res_max);
  return c->e32->cycles(ncycles, res_h, res_max);
}

int mg_flush(mg_ctx* c, mg_c128* u_out) {
  if (!c) return fail(MG_EINVAL, "NULL ctx");
  if (c->p.precision == MG_FP64) return c->e64->flush((cpx<double>*)u_out);
  MG_TRY(c->e32->flush(nullptr));
  if (u_out)
    MG_HIP((launch_convert<float, double>(finest_N(c), c->e32->w[c->e32->cur], (cpx<double>*)u_out, 1.0, c->s)));
  return MG_OK;
}

int mg_get_level(mg_ctx* c, int level, int field, mg_c128* out) {
  if (!c || !out) return fail(MG_EINVAL, "NULL argument");
  if (level < c->p.level_min || level > c->p.level_max) return fail(MG_EINVAL, "bad level");
  if (field < MG_FIELD_U || field > MG_FIELD_SI) return fail(MG_EINVAL, "bad field");
  const size_t N = (size_t)ipow(ipow(3, level) + 1, c->p.dim);
  if (c->p.precision == MG_FP64) {
    const cpx<double>* f = c->e64->field(level, field);
    if (!f) MG_HIP(launch_fill(out, N * sizeof(cpx<double>), c->s));
    else MG_HIP(hipMemcpyAsync(out, f, N * sizeof(cpx<double>), hipMemcpyDeviceToDevice, c->s));
  } else {
    const cpx<float>* f = c->e32->field(level, field);
    if (!f) MG_HIP(launch_fill(out, N * sizeof(cpx<double>), c->s));
    else MG_HIP((launch_convert<float, double>(N, f, (cpx<double>*)out, 1.0, c->s)));
  }
  return MG_OK;
}

int mg_precondition(mg_ctx* c, const mg_c128* v, mg_c128* z) {
  if (!c || !v || !z) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)v == (const void*)z) return fail(MG_EINVAL, "v and z must not alias");
  if (c->p.precision == MG_FP64) return c->e64->precondition((const cpx<double>*)v, (cpx<double>*)z);
  cpx<float>* t;
  MG_TRY(stage_in(c, v, &t));
  MG_TRY(stage_e32(c));
  MG_TRY(c->e32->precondition(t, c->e32v));
  MG_HIP((launch_convert<float, double>(finest_N(c), c->e32v, (cpx<double>*)z, 1.0, c->s)));
  return MG_OK;
}

int mg_precondition_apply(mg_ctx* c, const mg_c128* v, mg_c128* z, mg_c128* y) {
  if (!c || !v || !z || !y) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)v == (const void*)z || (const void*)v == (const void*)y || (const void*)z == (const void*)y)
    return fail(MG_EINVAL, "v, z and y must not alias");
  if (c->p.precision != MG_FP64) return fail(MG_EINVAL, "mg_precondition_apply: complex128 contexts only");
  return c->e64->precondition_apply_any((const cpx<double>*)v, (cpx<double>*)z, (cpx<double>*)y);
}

int mg_residual_norm(mg_ctx* c, const mg_c128* u, const mg_c128* b, double* res_h) {
  if (!c || !u || !b || !res_h) return fail(MG_EINVAL, "NULL argument");
  return c->e64->resid_norm((const cpx<double>*)u, (const cpx<double>*)b, res_h, nullptr);
}

int mg_residual_norm_noalloc(mg_ctx* c, const mg_c128* u, const mg_c128* b, double* res_h, double* res_max) {
  if (!c || !u || !b || (!res_h && !res_max)) return fail(MG_EINVAL, "NULL argument");
  const int n = (int)ipow(3, c->p.level_max) + 1;
  const int blocks = resid_norm_blocks(c->p.dim, n);
  if (blocks < 1 || 2 * blocks + 2 > kNoAllocDoubles)
    return fail(MG_EINVAL, "level too wide for the fixed scratch of mg_residual_norm_noalloc (" +
                               std::to_string(kNoAllocDoubles) + " doubles)");
  double* sp = scratch_of(c->device);
  if (!sp) return fail(MG_EDEVICE, "scratch address of the context's device was not resolved");
  int np = 0;
  MG_HIP(launch_resid<double>(c->p.dim, c->op64, (const cpx<double>*)b, (const cpx<double>*)u, nullptr, sp, &np,
                              c->s));
  if (np != blocks) return fail(MG_EDEVICE, "residual pass used an unexpected block count");
  MG_HIP(launch_finish_sum_max(sp, np, sp + 2 * kRedBlocks, c->s));
  double h[2];
  MG_HIP(hipMemcpyAsync(h, sp + 2 * kRedBlocks, sizeof(h), hipMemcpyDeviceToHost, c->s));
  MG_HIP(hipStreamSynchronize(c->s));
  if (res_h) *res_h = std::sqrt(std::pow(3.0, -c->p.dim * c->p.level_max) * h[0]);
  if (res_max) *res_max = h[1];
  return MG_OK;
}

// FP64 residual refinement with complex64 inner corrections:
//   r = b - H u (FP64), rho = |r|, e = inner solve of H e = r / rho in complex64,
//   u += rho e (FP64), until |r| / |b| <= rtol.
static int refine_solve(mg_ctx* c, const cpx<double>* b, cpx<double>* u, double rtol, int maxit, int driver,
                        int* iters_out, double* relres_out) {
  Engine<double>& E = *c->e64;
  Engine<float>& F = *c->e32;
  const size_t N = finest_N(c);
  const int dim = c->p.dim, n = (int)ipow(3, c->p.level_max) + 1;
  MG_TRY(E.ensure_scratch());
  MG_TRY(stage_e32(c));
  if (!c->r32) {
    void* q;
    MG_HIP(hipMalloc(&q, N * sizeof(cpx<float>)));
    c->owned.push_back(q);
    c->r32 = (cpx<float>*)q;
  }
  cpx<double>* r = E.tR;
  MG_HIP(launch_zero_boundary_copy<double>(dim, n, u, u, mk(1.0, 0.0), c->s));
  double bn;
  MG_HIP(launch_zero_boundary_copy<double>(dim, n, b, E.tRh, mk(1.0, 0.0), c->s));
  MG_TRY(E.norm2(E.tRh, &bn));
  if (bn == 0.0) {
    MG_HIP(launch_fill(u, N * sizeof(cpx<double>), c->s));
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    return MG_OK;
  }
  const double inner_tol = c->p.inner_rtol > 0 ? c->p.inner_rtol : kInnerRtolDefault;
  int total_inner = 0, status = MG_ENOTCONV;
  double rel = 1.0, rel0 = -1.0;
  for (int outer = 0; outer < 100; ++outer) {
    MG_HIP(launch_resid<double>(dim, c->op64, E.tRh, u, r, nullptr, nullptr, c->s));
    double rn;
    MG_TRY(E.norm2(r, &rn));
    rel = rn / bn;
    if (rel0 < 0) rel0 = rel;
    if (!std::isfinite(rel) || rel > 1e8 * std::max(rel0, 1e-300)) {
      status = MG_EDIVERGED;
      break;
    }
    if (rel <= rtol) {
      status = MG_OK;
      break;
    }
    if (total_inner >= maxit) break;
    MG_HIP((launch_convert<double, float>(N, r, c->r32, 1.0 / rn, c->s)));
    MG_HIP(launch_fill(c->e32v, N * sizeof(cpx<float>), c->s));
    int its = 0;
    double inner_rel = 0;
    const int budget = std::max(1, maxit - total_inner);
    int irc;
    if (driver == MG_BICGSTAB) {
      irc = F.bicgstab(c->r32, c->e32v, inner_tol, budget, &its, &inner_rel);
    } else {
      irc = F.stationary(c->r32, c->e32v, inner_tol, std::min(budget, 50), &its, &inner_rel);
    }
    if (irc != MG_OK && irc != MG_ENOTCONV && irc != MG_EDIVERGED) return irc;
    total_inner += std::max(its, 1);
    if (irc == MG_EDIVERGED) {
      status = MG_EDIVERGED;
      break;
    }
    MG_HIP(launch_accum32(N, c->e32v, rn, u, c->s));
  }
  if (iters_out) *iters_out = total_inner;
  if (relres_out) *relres_out = rel;
  return status;
}

int mg_solve(mg_ctx* c, const mg_c128* b, mg_c128* u, double rtol, int maxit, int driver, int* iters_out,
             double* relres_out) {
  if (!c || !b || !u) return fail(MG_EINVAL, "NULL argument");
  if (!(rtol > 0) || maxit < 1) return fail(MG_EINVAL, "need rtol > 0 and maxit >= 1");
  if (driver != MG_STATIONARY && driver != MG_BICGSTAB) return fail(MG_EINVAL, "bad driver");
  if (c->p.precision == MG_FP32_REFINE)
    return refine_solve(c, (const cpx<double>*)b, (cpx<double>*)u, rtol, maxit, driver, iters_out, relres_out);
  Engine<double>& E = *c->e64;
  if (driver == MG_BICGSTAB) return E.bicgstab((const cpx<double>*)b, (cpx<double>*)u, rtol, maxit, iters_out, relres_out);
  return E.stationary((const cpx<double>*)b, (cpx<double>*)u, rtol, maxit, iters_out, relres_out);
}

int mg_prolong(mg_ctx* c, int level, const mg_c128* uc, mg_c128* uf) {
  if (!c || !uc || !uf) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)uc == (const void*)uf) return fail(MG_EINVAL, "uc and uf must not alias");
  if (level < 2 || level > c->p.level_max) return fail(MG_EINVAL, "need 2 <= level <= level_max");
  MG_HIP(launch_prolong<double>(c->p.dim, (int)ipow(3, level) + 1, (const cpx<double>*)uc, (cpx<double>*)uf, c->s));
  return MG_OK;
}

mg_ctx::~mg_ctx() {
  for (Nested& q : nested) mg_destroy(q.ctx);
  delete e64;
  delete e32;
  for (void* q : owned) (void)hipFree(q);
}

static int alloc_c128(mg_ctx* c, mg_c128** out, size_t count) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, count * sizeof(mg_c128));
  if (e != hipSuccess) return fail(MG_ENOMEM, std::string("nested solve: ") + hipGetErrorString(e));
  c->owned.push_back(q);
  *out = (mg_c128*)q;
  return MG_OK;
}

int mg_solve_nested(mg_ctx* c, const mg_c128* chi, mg_c128* u, int level_start, double coarse_rtol, double rtol,
                    int maxit, int driver, int* iters_out, double* relres_out) {
  if (!c || !chi || !u) return fail(MG_EINVAL, "NULL argument");
  if ((const void*)chi == (const void*)u) return fail(MG_EINVAL, "chi and u must not alias");
  const int L = c->p.level_max, dim = c->p.dim;
  if (level_start < c->p.level_min || level_start > L) return fail(MG_EINVAL, "need level_min <= level_start <= level_max");
  if (!(coarse_rtol > 0) || !(rtol > 0) || maxit < 1) return fail(MG_EINVAL, "need rtol, coarse_rtol > 0 and maxit >= 1");
  if (driver != MG_STATIONARY && driver != MG_BICGSTAB) return fail(MG_EINVAL, "bad driver");
  const bool varying = c->p.precision == MG_FP64 ? c->e64->varying : c->e32->varying;
  if (varying) return fail(MG_EINVAL, "nested solves need a constant phi");
  if (c->nested.size() < (size_t)L) c->nested.resize(L);
  const mg_c128* uprev = nullptr;
  // levels level_start .. L-1: solve with the load sampled there, from the
  // prolonged solution of the level below (zero on the first)
  for (int l = level_start; l < L; ++l) {
    mg_ctx::Nested& q = c->nested[l];
    const size_t Nl = (size_t)ipow(ipow(3, l) + 1, dim);
    if (!q.ctx) {
      mg_params pl = c->p;
      pl.level_max = l;
      pl.phi_field = nullptr;
      MG_TRY(mg_setup(&pl, c->s, &q.ctx));
      MG_TRY(alloc_c128(c, &q.chi, Nl));
      MG_TRY(alloc_c128(c, &q.b, Nl));
      MG_TRY(alloc_c128(c, &q.u, Nl));
    }
    MG_HIP(launch_sample<double>(dim, (int)ipow(3, l) + 1, (int)ipow(3, L - l), (const cpx<double>*)chi,
                                 (cpx<double>*)q.chi, c->s));
    MG_TRY(mg_rhs_from_nodal(q.ctx, q.chi, q.b));
    if (uprev) MG_TRY(mg_prolong(q.ctx, l, uprev, q.u));
    else MG_HIP(launch_fill(q.u, Nl * sizeof(mg_c128), c->s));
    int its = 0;
    double rel = 0;
    const int rc = mg_solve(q.ctx, q.b, q.u, coarse_rtol, maxit, driver, &its, &rel);
    if (rc != MG_OK && rc != MG_ENOTCONV) return rc;
    uprev = q.u;
  }
  if (!c->nested_b) MG_TRY(alloc_c128(c, &c->nested_b, finest_N(c)));
  MG_TRY(mg_rhs_from_nodal(c, chi, c->nested_b));
  if (uprev) MG_TRY(mg_prolong(c, L, uprev, u));
  else MG_HIP(launch_fill(u, finest_N(c) * sizeof(mg_c128), c->s));
  return mg_solve(c, c->nested_b, u, rtol, maxit, driver, iters_out, relres_out);
}

int mg_tiles(const mg_ctx* c, int* current, int* count) {
  if (!c) return fail(MG_EINVAL, "NULL ctx");
  const bool f = c->p.precision == MG_FP64 ? c->e64->fused : c->e32->fused;
  if (current) *current = f ? (c->p.precision == MG_FP64 ? c->e64->tile : c->e32->tile) : -1;
  if (count) *count = f ? fused_tile_count(c->p.dim) : 0;
  return MG_OK;
}

int mg_set_tile(mg_ctx* c, int tile) {
  if (!c) return fail(MG_EINVAL, "NULL ctx");
  const bool f = c->p.precision == MG_FP64 ? c->e64->fused : c->e32->fused;
  if (!f) return fail(MG_EINVAL, "the context has no fused sweep");
  if (tile < 0 || tile >= fused_tile_count(c->p.dim)) return fail(MG_EINVAL, "tile out of range");
  if (c->p.precision == MG_FP64) c->e64->set_tile(tile);
  else c->e32->set_tile(tile);
  return MG_OK;
}

int mg_autotune(mg_ctx* c, int reps, int* best_tile, double* best_us, double* times_us) {
  if (!c || reps < 1) return fail(MG_EINVAL, "bad argument");
  if (c->p.precision == MG_FP64) return c->e64->autotune(reps, best_tile, best_us, times_us);
  return c->e32->autotune(reps, best_tile, best_us, times_us);
}

int mg_time_sweeps(mg_ctx* c, int enable) {
  if (!c) return fail(MG_EINVAL, "NULL ctx");
  if (c->p.precision == MG_FP64) {
    c->e64->timing = enable != 0;
    if (enable) c->e64->ev_used = 0;
  } else {
    c->e32->timing = enable != 0;
    if (enable) c->e32->ev_used = 0;
  }
  return MG_OK;
}

int mg_sweep_time(mg_ctx* c, double* total_ms, int* count) {
  if (!c) return fail(MG_EINVAL, "NULL ctx");
  if (c->p.precision == MG_FP64) return sweep_time(*c->e64, total_ms, count);
  return sweep_time(*c->e32, total_ms, count);
}

int mg_grad_potential(mg_ctx* c, const mg_c128* u, const mg_c128* lam, double* dJdV) {
  if (!c || !u || !lam || !dJdV) return fail(MG_EINVAL, "NULL argument");
  if (c->p.layer_width > 0) return fail(MG_EINVAL, "the potential gradient needs a uniform rotation (no absorbing layer)");
  const LevelScalars ls = level_scalars(c->p.dim, c->p.level_max, c->p.theta, false);
  MG_HIP(launch_grad_potential(c->p.dim, (int)ipow(3, c->p.level_max) + 1, to_c<double>(ls.etad),
                               (const cpx<double>*)u, (const cpx<double>*)lam, dJdV, c->s));
  return MG_OK;
}

}  // extern "C"
