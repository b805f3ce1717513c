// C ABI of the IFGF library: argument checks, status codes, plan lifetime,
// statistics and test hooks.  Nothing throws across this boundary.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include <memory>

#include "internal.h"

namespace ifgf {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      throw Error{IFGF_ENOMEM, std::string(what) + ": " + hipGetErrorString(e)};
    throw Error{IFGF_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

void DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) nbytes = 16;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{IFGF_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed"};
  }
  bytes = nbytes;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

DevBuf::~DevBuf() { release(); }

StageTimer::StageTimer(ifgf_plan_s* pp, hipStream_t ss, int stage) : p(pp), s(ss) {
  if (p->ev.empty() || 2 * (p->ev_used + 1) > (int)p->ev.size()) return;
  slot = p->ev_used++;
  p->ev_stage[slot] = stage;
  (void)hipEventRecord(p->ev[2 * slot], s);
}

StageTimer::~StageTimer() {
  if (slot >= 0) (void)hipEventRecord(p->ev[2 * slot + 1], s);
}

static void free_events(ifgf_plan_s* p) {
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->ev_stage.clear();
  p->ev_used = 0;
}

}  // namespace ifgf

using namespace ifgf;

template <typename F> static ifgf_status guarded(F&& f) {
  try {
    f();
    set_last_error("");
    return IFGF_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return IFGF_ENOMEM;
  } catch (...) {
    set_last_error("unexpected exception");
    return IFGF_EINTERNAL;
  }
}

struct BusyGuard {
  std::atomic<int>* busy;
  bool ok;
  template <typename H> explicit BusyGuard(H* h) : busy(&h->busy) {
    int expect = 0;
    ok = busy->compare_exchange_strong(expect, 1);
  }
  ~BusyGuard() {
    if (ok) busy->store(0);
  }
};

extern "C" {

void ifgf_options_default(ifgf_options* o) {
  if (!o) return;
  o->p_s = 4;
  o->p_ang = 6;
  o->ns0 = 2;
  o->nc0 = 4;
  o->depth = 0;
  o->leaf_h_lambda = 0.5;
  o->precision = IFGF_PREC_FP32_INTERP;
  o->max_rhs = 1;
  o->kernel = IFGF_KERNEL_COMBINED;
  o->prop_kernel = IFGF_PROP_AUTO;
  o->target_kernel = IFGF_TARGET_AUTO;
  o->far_field = 0;
}

const char* ifgf_status_string(ifgf_status st) {
  switch (st) {
    case IFGF_OK: return "ok";
    case IFGF_EINVAL: return "invalid argument";
    case IFGF_EDUPLICATE: return "duplicate points";
    case IFGF_ENOMEM: return "out of memory";
    case IFGF_EHIP: return "HIP error";
    case IFGF_EUNSUPPORTED: return "unsupported option";
    case IFGF_EBUSY: return "plan busy";
    case IFGF_EINTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ifgf_last_error(void) { return g_last_error.c_str(); }

// Plan creation shared by ifgf_plan_create and ifgf_plan_create_targets: the
// first n_src of the n points carry densities, the others are targets only.
static void create_plan(ifgf_plan_s*& p, int64_t n, int64_t n_src, const double* points, const double* normals,
                        const double* weights, double k, double eta, const ifgf_options* opt, hipStream_t stream) {
  if (n < 1 || n > (int64_t)0x7fffffff) throw Error{IFGF_EINVAL, "n out of range"};
  if (!(k > 0.0) || !std::isfinite(k) || !std::isfinite(eta)) throw Error{IFGF_EINVAL, "k must be finite and > 0"};
  ifgf_options o;
  ifgf_options_default(&o);
  if (opt) o = *opt;
  if (o.p_s < 1 || o.p_ang < 1 || o.p_s > IFGF_MAXP || o.p_ang > IFGF_MAXP) throw Error{IFGF_EINVAL, "bad p_s/p_ang"};
  if (o.ns0 < 1 || o.nc0 < 1) throw Error{IFGF_EINVAL, "bad ns0/nc0"};
  if (o.depth < 0 || o.depth > 11) throw Error{IFGF_EINVAL, "depth must be in 0..11"};
  if (o.depth == 0 && !(o.leaf_h_lambda > 0.0)) throw Error{IFGF_EINVAL, "leaf_h_lambda must be > 0"};
  if (o.precision != IFGF_PREC_FP64 && o.precision != IFGF_PREC_FP32_INTERP) throw Error{IFGF_EINVAL, "bad precision"};
  if (o.max_rhs < 1) throw Error{IFGF_EINVAL, "max_rhs must be >= 1"};
  if (o.prop_kernel < IFGF_PROP_AUTO || o.prop_kernel > IFGF_PROP_PAIRS) throw Error{IFGF_EINVAL, "bad prop_kernel"};
  if (o.target_kernel < IFGF_TARGET_AUTO || o.target_kernel > IFGF_TARGET_PAIRS)
    throw Error{IFGF_EINVAL, "bad target_kernel"};
  if (o.kernel != IFGF_KERNEL_COMBINED && o.kernel != IFGF_KERNEL_CONSTANT) throw Error{IFGF_EINVAL, "bad kernel"};
  if (o.far_field != 0 && o.far_field != 1) throw Error{IFGF_EINVAL, "far_field must be 0 or 1"};
  if (!supported_order(o.p_s, o.p_ang, o.precision))
    throw Error{IFGF_EUNSUPPORTED, "p_s/p_ang pair not compiled in for this precision"};
  p = new ifgf_plan_s();
  p->n = n;
  p->n_src = n_src;
  p->k = k;
  p->eta = eta;
  p->opt = o;
  p->P = o.p_s * o.p_ang * o.p_ang;
  build_plan(p, points, normals, weights, stream);
  if (n_src < n) p->uext.alloc(sizeof(double) * 2 * (size_t)n * o.max_rhs);
}

ifgf_status ifgf_plan_create(ifgf_plan* out, int64_t n, const double* points, const double* normals,
                             const double* weights, double k, double eta, const ifgf_options* opt, void* stream) {
  if (out) *out = nullptr;
  ifgf_plan_s* p = nullptr;
  ifgf_status st = guarded([&] {
    if (!out || !points || !normals || !weights) throw Error{IFGF_EINVAL, "null pointer argument"};
    create_plan(p, n, n, points, normals, weights, k, eta, opt, (hipStream_t)stream);
    *out = p;
  });
  if (st != IFGF_OK) {
    delete p;
  }
  return st;
}

ifgf_status ifgf_plan_create_targets(ifgf_plan* out, int64_t n, const double* points, const double* normals,
                                     const double* weights, int64_t nt, const double* targets, double k, double eta,
                                     const ifgf_options* opt, void* stream) {
  if (out) *out = nullptr;
  ifgf_plan_s* p = nullptr;
  ifgf_status st = guarded([&] {
    if (!out || !points || !normals || !weights || !targets) throw Error{IFGF_EINVAL, "null pointer argument"};
    if (n < 1 || nt < 1 || n + nt > (int64_t)0x7fffffff) throw Error{IFGF_EINVAL, "n or nt out of range"};
    const hipStream_t s = (hipStream_t)stream;
    // one point set: the sources, then the targets with zero weight and normal
    const int64_t m = n + nt;
    DevBuf up, un, uw;
    up.alloc(sizeof(double) * 3 * m);
    un.alloc(sizeof(double) * 3 * m);
    uw.alloc(sizeof(double) * m);
    HIPCHK(hipMemcpyAsync(up.p, points, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(up.as<double>() + 3 * n, targets, sizeof(double) * 3 * nt, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(un.p, normals, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(un.as<double>() + 3 * n, 0, sizeof(double) * 3 * nt, s));
    HIPCHK(hipMemcpyAsync(uw.p, weights, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(uw.as<double>() + n, 0, sizeof(double) * nt, s));
    create_plan(p, m, n, up.as<double>(), un.as<double>(), uw.as<double>(), k, eta, opt, s);
    HIPCHK(hipStreamSynchronize(s));   // the union arrays are freed on return
    *out = p;
  });
  if (st != IFGF_OK) {
    delete p;
  }
  return st;
}

static void check_apply_args(ifgf_plan p, const void* in, void* outp, int32_t nrhs, int32_t dtype) {
  if (!p || !in || !outp) throw Error{IFGF_EINVAL, "null pointer argument"};
  if (in == outp) throw Error{IFGF_EINVAL, "input and output alias"};
  if (nrhs < 1 || nrhs > p->opt.max_rhs) throw Error{IFGF_EINVAL, "nrhs out of range (1..max_rhs)"};
  if (dtype != IFGF_C64 && dtype != IFGF_C128) throw Error{IFGF_EINVAL, "bad dtype"};
}

ifgf_status ifgf_apply(ifgf_plan p, const void* sigma, void* u, int32_t nrhs, int32_t dtype, void* stream) {
  return ifgf_apply_stages(p, sigma, u, nrhs, dtype, 3, 0, 1 << 20, stream);
}

ifgf_status ifgf_apply_stages(ifgf_plan p, const void* sigma, void* u, int32_t nrhs, int32_t dtype, int32_t stage_mask,
                              int32_t level_lo, int32_t level_hi, void* stream) {
  return guarded([&] {
    check_apply_args(p, sigma, u, nrhs, dtype);
    BusyGuard g(p);
    if (!g.ok) throw Error{IFGF_EBUSY, "another apply on this plan is being enqueued"};
    run_apply(p, sigma, u, nrhs, dtype, stage_mask, level_lo, level_hi, (hipStream_t)stream);
  });
}

ifgf_status ifgf_apply_adjoint(ifgf_plan p, const void* v, void* out, int32_t nrhs, int32_t dtype, int32_t conjugate,
                               void* stream) {
  return guarded([&] {
    check_apply_args(p, v, out, nrhs, dtype);
    if (p->n_src < p->n) throw Error{IFGF_EUNSUPPORTED, "no transposed apply for a plan with separate targets"};
    BusyGuard g(p);
    if (!g.ok) throw Error{IFGF_EBUSY, "another apply on this plan is being enqueued"};
    run_adjoint(p, v, out, nrhs, dtype, conjugate ? 1 : 0, (hipStream_t)stream);
  });
}

ifgf_status ifgf_plan_autotune(ifgf_plan p, int32_t reps, ifgf_tune_report* report, void* stream) {
  return guarded([&] {
    if (!p) throw Error{IFGF_EINVAL, "null plan"};
    if (reps < 1) throw Error{IFGF_EINVAL, "reps must be >= 1"};
    if (p->batch_refs.load() > 0) throw Error{IFGF_EBUSY, "a batch is built over this plan"};
    BusyGuard g(p);
    if (!g.ok) throw Error{IFGF_EBUSY, "another apply on this plan is being enqueued"};
    ifgf_tune_report r;
    run_autotune(p, reps, &r, (hipStream_t)stream);
    if (report) *report = r;
  });
}

ifgf_status ifgf_far_field(ifgf_plan p, const void* sigma, int64_t ndir, const double* dirs, void* uinf,
                           int32_t dtype, void* stream) {
  return guarded([&] {
    if (!p || !sigma || !dirs || !uinf) throw Error{IFGF_EINVAL, "null pointer argument"};
    if (ndir < 1 || ndir > ((int64_t)1 << 31) / 64) throw Error{IFGF_EINVAL, "ndir out of range"};
    if (dtype != IFGF_C64 && dtype != IFGF_C128) throw Error{IFGF_EINVAL, "bad dtype"};
    if (p->opt.kernel != IFGF_KERNEL_COMBINED) throw Error{IFGF_EINVAL, "the far field needs the combined kernel"};
    if (p->D >= 3 && !p->opt.far_field) throw Error{IFGF_EINVAL, "plan created without far_field = 1"};
    BusyGuard g(p);
    if (!g.ok) throw Error{IFGF_EBUSY, "another apply on this plan is being enqueued"};
    run_far_field(p, sigma, ndir, dirs, uinf, dtype, (hipStream_t)stream);
  });
}

void ifgf_gmres_options_default(ifgf_gmres_options* o) {
  if (!o) return;
  o->restart = 30;
  o->max_iter = 300;
  o->tol = 1e-4;
  o->alpha_re = 0.5;
  o->alpha_im = 0.0;
  o->use_guess = 0;
}

ifgf_status ifgf_gmres_solve(ifgf_plan p, const void* f, void* sigma, const ifgf_gmres_options* opt, int32_t* iters,
                             double* rel_res, double* history, void* stream) {
  return guarded([&] {
    if (!p || !f || !sigma || !iters || !rel_res) throw Error{IFGF_EINVAL, "null pointer argument"};
    if (f == sigma) throw Error{IFGF_EINVAL, "f and sigma alias"};
    if (p->n_src < p->n) throw Error{IFGF_EINVAL, "a plan with separate targets is not a square operator"};
    ifgf_gmres_options o;
    ifgf_gmres_options_default(&o);
    if (opt) o = *opt;
    if (o.restart < 1 || o.restart > 1000) throw Error{IFGF_EINVAL, "restart out of range (1..1000)"};
    if (o.max_iter < 1) throw Error{IFGF_EINVAL, "max_iter must be >= 1"};
    if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) throw Error{IFGF_EINVAL, "tol must be finite and >= 0"};
    if (!std::isfinite(o.alpha_re) || !std::isfinite(o.alpha_im)) throw Error{IFGF_EINVAL, "alpha must be finite"};
    BusyGuard g(p);
    if (!g.ok) throw Error{IFGF_EBUSY, "another apply on this plan is being enqueued"};
    run_gmres(p, f, sigma, o, iters, rel_res, history, (hipStream_t)stream);
    p->last_rhs = 1;
  });
}

ifgf_status ifgf_plan_get_stats(ifgf_plan p, ifgf_plan_stats* st) {
  return guarded([&] {
    if (!p || !st) throw Error{IFGF_EINVAL, "null pointer argument"};
    std::memset(st, 0, sizeof(*st));
    st->depth = p->D;
    st->n = p->n;
    st->root_side = p->L;
    for (int a = 0; a < 3; ++a) st->root_corner[a] = p->corner[a];
    st->p_s = p->opt.p_s;
    st->p_ang = p->opt.p_ang;
    st->precision = p->opt.precision;
    int64_t bytes = 0;
    auto add = [&](const DevBuf& b) { bytes += (int64_t)b.bytes; };
    add(p->perm); add(p->keys); add(p->pts); add(p->nrm); add(p->w); add(p->a); add(p->uacc); add(p->err);
    add(p->tpart);
    add(p->Ms); add(p->Ma); add(p->Msf); add(p->Maf);
    for (int d = 1; d <= p->D; ++d) {
      const LevelPlan& l = p->lev[d];
      st->boxes[d] = l.nb;
      st->ns[d] = l.geom.ns;
      st->nc[d] = l.geom.nc;
      st->cones[d] = l.nrel;
      st->cousin_pairs[d] = l.cousin_pairs;
      st->prop_evals[d] = l.prop_evals;
      st->pair_rows[d] = l.pair_rows;
      st->pair_row_cones[d] = l.pair_row_cones;
      add(l.start); add(l.coords); add(l.centre); add(l.parent); add(l.child_lo); add(l.nbr_off); add(l.nbr);
      add(l.cou_off); add(l.cou); add(l.pbox); add(l.slot); add(l.slot_off); add(l.rel_box); add(l.rel_cone);
      add(l.Fn); add(l.Fc); add(l.work); add(l.ti_slot); add(l.ti_tile); add(l.ti_child); add(l.ti_geo); add(l.near_work); add(l.leaf_work);
      add(l.ti_qlist); add(l.ti_rec); add(l.adj_tiles); add(l.adj_slots); add(l.adj_gref); add(l.adj_gref_off);
      add(l.pr_slot); add(l.pr_loc); add(l.pr_fim); add(l.pr_val); add(l.pr_off); add(l.pr_pos);
      add(l.pr_tgt); add(l.pr_run);
      add(l.up_slot); add(l.up_loc); add(l.up_fim); add(l.up_val); add(l.up_base); add(l.up_pos);
      add(l.up_node); add(l.up_run);
      add(p->adj_g[d]);
      if (d >= 4 && p->lev[d - 1].nrel > 0)
        st->prop_kernel[d] = p->lev[d - 1].up_use ? IFGF_PROP_PAIRS
                             : p->lev[d - 1].ntile > 0 ? IFGF_PROP_CONE : IFGF_PROP_NODE;
    }
    st->near_pairs = p->near_pairs;
    st->device_bytes = bytes;
  });
}

static void sync_copy(void* dst, const void* src, size_t bytes) {
  HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice));
}

ifgf_status ifgf_plan_export_order(ifgf_plan p, int32_t* perm, uint32_t* keys) {
  return guarded([&] {
    if (!p) throw Error{IFGF_EINVAL, "null plan"};
    if (perm) sync_copy(perm, p->perm.p, sizeof(int) * p->n);
    if (keys) sync_copy(keys, p->keys.p, sizeof(uint32_t) * p->n);
  });
}

ifgf_status ifgf_plan_export_boxes(ifgf_plan p, int32_t d, int32_t* start, int32_t* coords) {
  return guarded([&] {
    if (!p || d < 1 || d > p->D) throw Error{IFGF_EINVAL, "bad plan or level"};
    const LevelPlan& l = p->lev[d];
    if (start) sync_copy(start, l.start.p, sizeof(int) * (l.nb + 1));
    if (coords) sync_copy(coords, l.coords.p, sizeof(int) * 3 * l.nb);
  });
}

ifgf_status ifgf_plan_export_lists(ifgf_plan p, int32_t d, int32_t kind, int32_t* off, int32_t* idx, int64_t* len) {
  return guarded([&] {
    if (!p || d < 1 || d > p->D) throw Error{IFGF_EINVAL, "bad plan or level"};
    if (kind == 1 && d < 3) throw Error{IFGF_EINVAL, "cousin lists exist for d >= 3"};
    const LevelPlan& l = p->lev[d];
    const DevBuf& o = kind == 0 ? l.nbr_off : l.cou_off;
    const DevBuf& x = kind == 0 ? l.nbr : l.cou;
    int64_t cnt = kind == 0 ? l.nnbr : l.ncou;
    if (len) *len = cnt;
    if (off) sync_copy(off, o.p, sizeof(int) * (l.nb + 1));
    if (idx && cnt > 0) sync_copy(idx, x.p, sizeof(int) * cnt);
  });
}

ifgf_status ifgf_plan_export_cones(ifgf_plan p, int32_t d, int32_t* box, int32_t* cone) {
  return guarded([&] {
    if (!p || d < 3 || d > p->D) throw Error{IFGF_EINVAL, "bad plan or level"};
    const LevelPlan& l = p->lev[d];
    if (l.nrel == 0) return;
    if (box) sync_copy(box, l.rel_box.p, sizeof(int) * l.nrel);
    if (cone) sync_copy(cone, l.rel_cone.p, sizeof(int) * l.nrel);
  });
}

ifgf_status ifgf_plan_export_field(ifgf_plan p, int32_t d, int32_t what, void* dst) {
  return guarded([&] {
    if (!p || !dst || d < 3 || d > p->D) throw Error{IFGF_EINVAL, "bad plan, level or pointer"};
    const LevelPlan& l = p->lev[d];
    if (what == 0 && d != p->D) throw Error{IFGF_EINVAL, "node values are kept for the finest level only"};
    size_t csz = p->opt.precision == IFGF_PREC_FP32_INTERP ? 8 : 16;
    size_t bytes = csz * (size_t)l.nrel * p->P * std::max(1, p->last_rhs);
    if (!bytes) return;
    if (what == 0)
      run_export_nodes(p, dst, nullptr);   // the default stream, as the copies here
    else
      sync_copy(dst, l.Fc.p, bytes);
  });
}

ifgf_status ifgf_plan_check(ifgf_plan p, int32_t* flags) {
  return guarded([&] {
    if (!p || !flags) throw Error{IFGF_EINVAL, "null pointer argument"};
    HIPCHK(hipMemcpy(flags, p->err.p, sizeof(int), hipMemcpyDeviceToHost));
  });
}

ifgf_status ifgf_plan_set_profiling(ifgf_plan p, int32_t max_launches) {
  return guarded([&] {
    if (!p || max_launches < 0) throw Error{IFGF_EINVAL, "bad plan or count"};
    HIPCHK(hipDeviceSynchronize());
    free_events(p);
    if (max_launches == 0) return;
    p->ev.resize(2 * (size_t)max_launches, nullptr);
    p->ev_stage.assign(max_launches, 0);
    for (auto& e : p->ev) HIPCHK(hipEventCreate(&e));
  });
}

ifgf_status ifgf_plan_read_profile(ifgf_plan p, double* ms, int64_t* launches) {
  return guarded([&] {
    if (!p || !ms || !launches) throw Error{IFGF_EINVAL, "null pointer argument"};
    for (int i = 0; i < IFGF_NSTAGES; ++i) {
      ms[i] = 0;
      launches[i] = 0;
    }
    for (int i = 0; i < p->ev_used; ++i) {
      HIPCHK(hipEventSynchronize(p->ev[2 * i + 1]));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, p->ev[2 * i], p->ev[2 * i + 1]));
      ms[p->ev_stage[i]] += t;
      launches[p->ev_stage[i]] += 1;
    }
    p->ev_used = 0;
  });
}

void ifgf_plan_destroy(ifgf_plan p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  free_events(p);
  delete p;
}

ifgf_status ifgf_batch_create(ifgf_batch* out, int32_t nplans, const ifgf_plan* plans) {
  if (out) *out = nullptr;
  std::unique_ptr<ifgf_batch_s> b;
  ifgf_status st = guarded([&] {
    if (!out || !plans) throw Error{IFGF_EINVAL, "null pointer argument"};
    if (nplans < 1 || nplans > IFGF_BATCH_MAX) throw Error{IFGF_EINVAL, "nplans out of range (1..IFGF_BATCH_MAX)"};
    b.reset(new ifgf_batch_s);
    for (int g = 0; g < nplans; ++g) {
      ifgf_plan_s* p = plans[g];
      if (!p) throw Error{IFGF_EINVAL, "null plan in batch"};
      if (p->n_src < p->n) throw Error{IFGF_EINVAL, "a plan with separate targets cannot join a batch"};
      for (auto* q : b->plans)
        if (q == p) throw Error{IFGF_EINVAL, "a plan appears twice in the batch"};
      const ifgf_plan_s* p0 = plans[0];
      if (p->opt.precision != p0->opt.precision || p->opt.p_s != p0->opt.p_s || p->opt.p_ang != p0->opt.p_ang)
        throw Error{IFGF_EINVAL, "batch plans must share precision, p_s and p_ang"};
      b->plans.push_back(p);
    }
    HIPCHK(hipGetDevice(&b->device));
    HIPCHK(hipDeviceSynchronize());
    run_batch_prepare(b.get());
    HIPCHK(hipDeviceSynchronize());
  });
  if (st == IFGF_OK) {
    for (auto* p : b->plans) p->batch_refs.fetch_add(1);
    *out = b.release();
  }
  return st;
}

// Argument checks shared by the two batch applies.
static void check_batch_args(ifgf_batch b, const void* const* sigma, void* const* u, int32_t dtype) {
  if (!b || !sigma || !u) throw Error{IFGF_EINVAL, "null pointer argument"};
  if (dtype != IFGF_C64 && dtype != IFGF_C128) throw Error{IFGF_EINVAL, "bad dtype"};
  const int ng = (int)b->plans.size();
  for (int g = 0; g < ng; ++g) {
    if (!sigma[g] || !u[g]) throw Error{IFGF_EINVAL, "null sigma or u pointer"};
    for (int h = 0; h < ng; ++h)
      if ((const void*)u[g] == sigma[h]) throw Error{IFGF_EINVAL, "an output aliases an input"};
  }
}

// Busy flags of the batch and of each of its plans, taken together (fixed
// storage: no allocation) and released on scope exit.
struct BatchGuard {
  std::atomic<int>* held[IFGF_BATCH_MAX + 1];
  int n = 0;
  bool take(std::atomic<int>* busy) {
    int expect = 0;
    if (!busy->compare_exchange_strong(expect, 1)) return false;
    held[n++] = busy;
    return true;
  }
  ~BatchGuard() {
    for (int i = 0; i < n; ++i) held[i]->store(0);
  }
};

static void batch_apply_common(ifgf_batch b, const void* const* sigma, void* const* u, int32_t dtype, int* ctr,
                               void* stream) {
  BatchGuard g;
  if (!g.take(&b->busy)) throw Error{IFGF_EBUSY, "another apply of this batch is being enqueued"};
  for (auto* p : b->plans)
    if (!g.take(&p->busy)) throw Error{IFGF_EBUSY, "an apply on a plan of the batch is being enqueued"};
  run_batch_apply(b, sigma, u, dtype, ctr, (hipStream_t)stream);
  for (auto* p : b->plans) p->last_rhs = 1;
}

ifgf_status ifgf_batch_apply(ifgf_batch b, const void* const* sigma, void* const* u, int32_t dtype, void* stream) {
  return guarded([&] {
    check_batch_args(b, sigma, u, dtype);
    batch_apply_common(b, sigma, u, dtype, nullptr, stream);
  });
}

ifgf_status ifgf_batch_apply_noalloc(ifgf_batch b, const void* const* sigma, void* const* u, int32_t dtype,
                                     void* stream) {
  return guarded([&] {
    check_batch_args(b, sigma, u, dtype);
    if (b->nctr > BATCH_STATIC_COUNTERS)
      throw Error{IFGF_EINVAL, "the batch needs more completion counters than the static array holds"};
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != b->device) throw Error{IFGF_EINVAL, "the batch's device is not the current device"};
    batch_apply_common(b, sigma, u, dtype, batch_static_counters(dev), stream);
  });
}

ifgf_status ifgf_batch_check(ifgf_batch b, int32_t* flags) {
  return guarded([&] {
    if (!b || !flags) throw Error{IFGF_EINVAL, "null pointer argument"};
    int f = 0;
    HIPCHK(hipMemcpy(&f, b->err.p, sizeof(int), hipMemcpyDeviceToHost));
    for (auto* p : b->plans) {
      int pf = 0;
      HIPCHK(hipMemcpy(&pf, p->err.p, sizeof(int), hipMemcpyDeviceToHost));
      f |= pf;
    }
    *flags = f;
  });
}

ifgf_status ifgf_batch_set_spin_limit(ifgf_batch b, int32_t limit) {
  return guarded([&] {
    if (!b || limit < 0) throw Error{IFGF_EINVAL, "bad batch or limit"};
    b->spin_limit = limit;
  });
}

ifgf_status ifgf_batch_get_info(ifgf_batch b, int64_t* items, int32_t* segments, int32_t* grid, int32_t* block) {
  return guarded([&] {
    if (!b) throw Error{IFGF_EINVAL, "null batch"};
    if (items) *items = b->total;
    if (segments) *segments = b->nseg;
    if (grid) *grid = b->grid;
    if (block) *block = b->block;
  });
}

void ifgf_batch_destroy(ifgf_batch b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  for (auto* p : b->plans) p->batch_refs.fetch_sub(1);
  delete b;
}

}  // extern "C"
