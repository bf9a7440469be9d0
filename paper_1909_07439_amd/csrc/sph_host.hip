// sph_host.hip -- the C ABI (include/sph.h): context, validation, phase
// orchestration on the library stream, inspection copies and event timing.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sph_ctx.h"

namespace sph {
hipError_t launch_node_boxes(sph_ctx* c, const sph_particles* s);
hipError_t launch_reset_counters(sph_ctx* c);
hipError_t launch_step_begin(sph_ctx* c, double dt_host);
hipError_t launch_pack_xyzm(sph_ctx* c, const sph_particles* s);
hipError_t launch_force_reset(sph_ctx* c);
hipError_t launch_leaf_state(sph_ctx* c, int v);
}  // namespace sph

namespace {

constexpr int kRing = 1024;  // timed launches kept per phase
enum Phase {
  kPhSort = 0,
  kPhPermute,
  kPhTree,
  kPhDensity,
  kPhForce,
  kPhIntegrate,
  kPhStep,
  kPhLists,
  kPhDensityFb,
  kPhForceFb,
  kPhAdjoint,
  kPhAdjForce,
  kNPh
};

}  // namespace

// Event rings of the phase timings, owned by the context.
struct sph_timing {
  hipEvent_t start[kNPh][kRing];
  hipEvent_t stop[kNPh][kRing];
  int count[kNPh];
  bool ready = false;
};

namespace {

// Reason of the last failed sph_create on this thread (no context exists to
// hold it); returned by sph_last_error(NULL).
thread_local std::string g_create_err;

sph_status fail(sph_ctx* c, sph_status st, const char* what) {
  if (c) c->err = what;
  return st;
}

sph_status hip_fail(sph_ctx* c, hipError_t e, const char* where) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString(e));
  if (c) c->err = buf;
  return SPH_E_HIP;
}

#define HIPCHK(c, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
  } while (0)

void ph_begin(sph_ctx* c, int ph) {
  sph_timing* x = c->tm;
  if (!x || !x->ready || !c->timing) return;
  const int k = x->count[ph];
  if (k < kRing) (void)hipEventRecord(x->start[ph][k], c->stream);
}
void ph_end(sph_ctx* c, int ph) {
  sph_timing* x = c->tm;
  if (!x || !x->ready || !c->timing) return;
  const int k = x->count[ph];
  if (k < kRing) {
    (void)hipEventRecord(x->stop[ph][k], c->stream);
    x->count[ph] = k + 1;
  }
}

sph_status check_parts(sph_ctx* c, const sph_particles* p, bool need_state_out,
                       bool need_dens_out) {
  if (!p) return fail(c, SPH_E_ARG, "particles is NULL");
  if (p->n < 1 || p->n > c->n_max) return fail(c, SPH_E_ARG, "n must be in [1, n_max]");
  if (!p->x || !p->y || !p->z || !p->m || !p->h)
    return fail(c, SPH_E_ARG, "x, y, z, m and h are required");
  if (need_state_out && (!p->vx || !p->vy || !p->vz || !p->u || !p->ax || !p->ay || !p->az ||
                         !p->dudt))
    return fail(c, SPH_E_ARG, "vx, vy, vz, u, ax, ay, az and dudt are required");
  if (need_dens_out && (!p->u || !p->rho || !p->omega || !p->P || !p->cs || !p->vsig_dt))
    return fail(c, SPH_E_ARG, "u, rho, omega, P, cs and vsig_dt are required");
  return SPH_OK;
}

sph_status status_of_err(sph_ctx* c, uint32_t e) {
  using namespace sph;
  if (e == 0) return SPH_OK;
  std::string s = "device error:";
  if (e & kErrNonFinite) s += " non-finite value;";
  if (e & kErrDomain) s += " 2h reaches half a periodic box length;";
  if (e & kErrNoConv) s += " smoothing length did not converge;";
  if (e & kErrNodes) s += " tree node capacity exceeded;";
  if (e & kErrFrontier) s += " walk frontier capacity exceeded (density);";
  if (e & kErrFrontierForce) s += " walk frontier capacity exceeded (force);";
  if (e & kErrPairs) s += " pair list capacity exceeded;";
  if (e & kErrIds) s += " particle id outside [0, n) in the adjoint;";
  if (e & kErrSort) s += " radix-sort look-back did not complete;";
  c->err = s;
  if (e & kErrIds) return SPH_E_ARG;
  if (e & kErrNonFinite) return SPH_E_NONFINITE;
  if (e & kErrDomain) return SPH_E_DOMAIN;
  if (e & kErrNoConv) return SPH_E_NOCONV;
  return SPH_E_OVERFLOW;
}

// Read the device state (synchronising) and report its error word.
sph_status sync_state(sph_ctx* c, bool clear_err) {
  HIPCHK(c, hipMemcpyAsync(c->hs, c->ds, sizeof(sph::DevState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint32_t e = c->hs->err;
  if (e && clear_err) {
    const uint32_t z = 0;
    HIPCHK(c, hipMemcpyAsync(&c->ds->err, &z, sizeof(z), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return status_of_err(c, e);
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, sizeof(T) * (count ? count : 1));
}

}  // namespace

extern "C" {

sph_status sph_create(const sph_params* prm, int64_t n_max, void* stream, sph_ctx** out) {
  auto reject = [](const char* why) {
    g_create_err = std::string("sph_create: ") + why;
    return SPH_E_ARG;
  };
  if (!out) return reject("out is NULL");
  *out = nullptr;
  if (!prm) return reject("params is NULL");
  if (n_max < 1 || n_max > (int64_t)0x3fffffff) return reject("n_max outside [1, 2^30)");
  const sph_params& P = *prm;
  for (int a = 0; a < 3; ++a)
    if (!(P.box_len[a] > 0.0) || !isfinite(P.box_lo[a])) return reject("bad box");
  if (!(P.hfact > 0.0) || !(P.gamma > 0.0) || !(P.gamma_minus_1 > 0.0) || !(P.c_cour > 0.0))
    return reject("hfact, gamma, gamma_minus_1 and c_cour must be > 0");
  if (P.alpha_av < 0 || P.beta_av < 0 || P.alpha_u < 0)
    return reject("alpha_av, beta_av and alpha_u must be >= 0");
  if (P.kernel < 0 || P.kernel > 2) return reject("unknown kernel (0 M4, 1 M6, 2 Wendland C6)");
  if (P.n_leaf < 1 || P.n_leaf > 64) return reject("n_leaf outside [1, 64]");
  if (!(P.n_group == 4 || P.n_group == 8 || P.n_group == 16 || P.n_group == 32))
    return reject("n_group must be 4, 8, 16 or 32");
  if (P.precision != SPH_PREC_FP64 && P.precision != SPH_PREC_MIXED)
    return reject("unknown precision");

  sph_ctx* c = new (std::nothrow) sph_ctx();
  if (!c) {
    g_create_err = "sph_create: out of host memory";
    return SPH_E_NOMEM;
  }
  c->prm = P;
  c->n_max = n_max;
  c->stream = (hipStream_t)stream;
  sph::KParams& k = c->kp;
  double lmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    k.lo[a] = P.box_lo[a];
    k.len[a] = P.box_len[a];
    k.half[a] = 0.5 * P.box_len[a];
    k.inv_len[a] = 1.0 / P.box_len[a];
    k.periodic[a] = P.periodic[a] ? 1 : 0;
    lmax = std::max(lmax, P.box_len[a]);
  }
  k.key_scale = 2097152.0 / lmax;
  k.gamma = P.gamma;
  k.gm1 = P.gamma_minus_1;
  k.hfact = P.hfact;
  k.alpha = P.alpha_av;
  k.beta = P.beta_av;
  k.alpha_u = P.alpha_u;
  k.c_cour = P.c_cour;
  k.fixed_passes = P.h_tol < 0.0 ? 1 : 0;
  k.h_tol = (P.h_tol > 0.0) ? P.h_tol : (P.precision == SPH_PREC_MIXED ? 2e-7 : 1e-14);
  k.max_iter = P.max_h_iter > 0 ? P.max_h_iter : 30;
  k.h_margin = P.h_margin > 1.0 ? P.h_margin : 1.1;
  k.n = 0;
  k.n_leaf = P.n_leaf;
  k.n_group = P.n_group;
  k.precision = P.precision;
  // smoothing kernel of Sect. 2.3: support in units of h and 3D normalisation
  k.kernel = P.kernel;
  k.support = (P.kernel == 1) ? 3.0 : 2.0;
  k.knorm = (P.kernel == 1) ? 1.0 / (120.0 * M_PI)
                            : (P.kernel == 2 ? 1365.0 / (512.0 * M_PI) : 1.0 / M_PI);
  // list rows: entries within support * h_margin * h of a uniform density
  // (4/3 pi (support hfact margin)^3 particles) with 40% room; 128 or 256
  {
    const double reach = k.support * P.hfact * k.h_margin;
    const double expect = 4.0 / 3.0 * M_PI * reach * reach * reach;
    k.nl_cap = (1.4 * expect <= 128.0) ? 128 : sph::kNLCapMax;
  }

  auto bail = [&](hipError_t e, const char* where) {
    sph_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SPH_E_NOMEM
                                                                                : SPH_E_HIP;
    char buf[512];
    snprintf(buf, sizeof(buf), "sph_create: %s: %s", where, hipGetErrorString(e));
    g_create_err = buf;
    sph_destroy(c);
    return st;
  };
#define ALLOC(ptr, cnt)                          \
  do {                                           \
    hipError_t e_ = dalloc(&(ptr), (size_t)(cnt)); \
    if (e_ != hipSuccess) return bail(e_, #ptr); \
  } while (0)

  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return bail(e, "hipGetDevice");
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) return bail(e, "attribute");
  c->n_cu = ncu > 0 ? ncu : 256;
  c->walk_blocks = ((c->n_cu * 16 + 7) / 8) * 8;

  const int64_t N = n_max;
  const int64_t nblk_sort = (N + sph::kSortTile - 1) / sph::kSortTile;
  const int64_t nblk_tree = (N + sph::kTreeTile - 1) / sph::kTreeTile;
  const int64_t scan_max = std::max<int64_t>(256 * nblk_sort, sph::kLevels * nblk_tree);
  ALLOC(c->keys[0], N);
  ALLOC(c->keys[1], N);
  ALLOC(c->vals[0], N);
  ALLOC(c->vals[1], N);
  c->n_max_sort_blocks = nblk_sort;
  ALLOC(c->radix_cnt, 8 * 256 * nblk_sort + 8 * 256 + 64);
  ALLOC(c->scan_part, scan_max / sph::kScanTile + 16);
  ALLOC(c->scan_total, 16);
  ALLOC(c->gtmp, (int64_t)sph::kMaxFields * N);
  ALLOC(c->gtmp_id, N);
  if (P.precision == SPH_PREC_MIXED)
    ALLOC(c->qxyzm, N);
  else
    ALLOC(c->xyzm, N);
  ALLOC(c->dlev, N);
  ALLOC(c->lleaf, N);
  ALLOC(c->gsize, N);
  ALLOC(c->gstart, N);
  ALLOC(c->tree_cnt, sph::kLevels * nblk_tree);
  ALLOC(c->grp_cnt, nblk_tree);
  c->node_cap = 2 * N + 1024;
  ALLOC(c->node_level, c->node_cap);
  ALLOC(c->node_first, c->node_cap);
  ALLOC(c->node_count, c->node_cap);
  ALLOC(c->node_parent, c->node_cap);
  ALLOC(c->node_child, c->node_cap);
  ALLOC(c->node_nchild, c->node_cap);
  ALLOC(c->wnode, c->node_cap);
  ALLOC(c->chunk_box, 8 * ((N + sph::kChunk - 1) / sph::kChunk));
  ALLOC(c->grp_first, N);
  ALLOC(c->grp_count, N);
  ALLOC(c->ginfo, N);
  c->pool_cap = std::min<int64_t>(16 * N + 256 * (int64_t)c->walk_blocks, 0x7fffffff);
  ALLOC(c->leaf_pool, c->pool_cap);
  ALLOC(c->gl_off, N);
  ALLOC(c->gl_cnt, N);
  ALLOC(c->nl_idx, (int64_t)k.nl_cap * N);
  ALLOC(c->nl_len, N);
  ALLOC(c->gflag, N);
  ALLOC(c->flag_list, N);
  ALLOC(c->walk_spill, (int64_t)2 * sph::kSpill * c->walk_blocks);
  ALLOC(c->grp_of, N);
  if (P.precision == SPH_PREC_MIXED) ALLOC(c->qrec, N);
  {
    const size_t rec = (P.precision == SPH_PREC_MIXED) ? sizeof(sph::FRec32) : sizeof(sph::FRec64);
    e = hipMalloc(&c->frec, rec * (size_t)N);
    if (e != hipSuccess) return bail(e, "frec");
  }
  ALLOC(c->a1, 4 * N);
  ALLOC(c->nb_cnt, N);
  ALLOC(c->nb_off, N + 1);
  ALLOC(c->red_part, 512 * 12);
  ALLOC(c->red_out, 16);
  ALLOC(c->ds, 1);
  e = hipHostMalloc((void**)&c->hs, sizeof(sph::DevState), hipHostMallocDefault);
  if (e != hipSuccess) return bail(e, "hipHostMalloc");
  memset(c->hs, 0, sizeof(sph::DevState));
  c->hs->dt_min_enc = sph::enc_f64(__builtin_huge_val());
  e = hipMemcpyAsync(c->ds, c->hs, sizeof(sph::DevState), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return bail(e, "init state");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(e, "sync");
#undef ALLOC
  sph_timing* x = new (std::nothrow) sph_timing();
  if (!x) {
    g_create_err = "sph_create: out of host memory";
    sph_destroy(c);
    return SPH_E_NOMEM;
  }
  c->tm = x;
  bool ok = true;
  // timing-only events: no system-scope fence when one is recorded (the
  // cache write-back and invalidation would idle the GPU for microseconds at
  // every phase boundary); sph_timings reads them after a stream synchronise
  const unsigned evf = hipEventDisableSystemFence;
  for (int ph = 0; ph < kNPh && ok; ++ph) {
    x->count[ph] = 0;
    for (int r = 0; r < kRing && ok; ++r) {
      ok = hipEventCreateWithFlags(&x->start[ph][r], evf) == hipSuccess &&
           hipEventCreateWithFlags(&x->stop[ph][r], evf) == hipSuccess;
    }
  }
  x->ready = ok;
  g_create_err.clear();
  *out = c;
  return SPH_OK;
}

void sph_destroy(sph_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (sph_timing* x = c->tm) {
    // events that were created are destroyed; a failed creation left the rest null
    for (int ph = 0; ph < kNPh; ++ph)
      for (int r = 0; r < kRing; ++r) {
        if (x->start[ph][r]) (void)hipEventDestroy(x->start[ph][r]);
        if (x->stop[ph][r]) (void)hipEventDestroy(x->stop[ph][r]);
      }
    delete x;
    c->tm = nullptr;
  }
  void* ptrs[] = {c->keys[0],   c->keys[1],     c->vals[0],      c->vals[1],     c->radix_cnt,
                  c->scan_part, c->scan_total,  c->gtmp,         c->gtmp_id,     c->dlev,
                  c->lleaf,     c->gsize,        c->gstart,       c->tree_cnt,    c->grp_cnt,
                  c->node_level, c->node_first, c->node_count,   c->node_parent, c->node_child,
                  c->node_nchild, c->chunk_box, c->wnode,       c->grp_first,
                  c->grp_count, c->ginfo,       c->frec,         c->a1,          c->nb_cnt,
                  c->nb_off,    c->red_part,    c->red_out,      c->ds,
                  c->leaf_pool, c->gl_off,      c->gl_cnt,       c->nl_idx,      c->nl_len,
                  c->gflag,     c->flag_list,   c->walk_spill,   c->grp_of,    c->qrec,
                  c->adj_abar,  c->adj_raw,     c->adj_ab,       c->xyzm,
                  c->qxyzm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->hs) (void)hipHostFree(c->hs);
  delete c;
}

static sph_status do_build(sph_ctx* c, sph_particles* p, bool outputs_too, bool predict) {
  c->n = (int32_t)p->n;
  c->kp.n = c->n;
  c->densities_on_tree = 0;
  ph_begin(c, kPhSort);
  HIPCHK(c, sph::launch_predict_keys(c, p, predict, 0.0));
  HIPCHK(c, sph::launch_sort(c));
  ph_end(c, kPhSort);
  ph_begin(c, kPhPermute);
  HIPCHK(c, sph::launch_permute(c, p, outputs_too));
  ph_end(c, kPhPermute);
  ph_begin(c, kPhTree);
  HIPCHK(c, sph::launch_tree(c));
  HIPCHK(c, sph::launch_node_boxes(c, p));
  ph_end(c, kPhTree);
  return SPH_OK;
}

sph_status sph_build_tree(sph_ctx* c, sph_particles* p) {
  if (!c) return SPH_E_ARG;
  sph_status st = check_parts(c, p, false, false);
  if (st != SPH_OK) return st;
  HIPCHK(c, sph::launch_reset_counters(c));
  return do_build(c, p, true, false);
}

// Density of the current tree: neighbour lists, the list density and the
// walking kernel for flagged groups; or the walking kernel for all groups.
static sph_status run_density(sph_ctx* c, sph_particles* p) {
  if (sph::lists_mode(c)) {
    ph_begin(c, kPhLists);
    HIPCHK(c, sph::launch_lists(c, p));
    ph_end(c, kPhLists);
    ++c->lists_launches;
    ph_begin(c, kPhDensity);
    HIPCHK(c, sph::launch_density_lists(c, p));
    ph_end(c, kPhDensity);
    ph_begin(c, kPhDensityFb);
    HIPCHK(c, sph::launch_density(c, p, true));
    ph_end(c, kPhDensityFb);
  } else {
    ph_begin(c, kPhDensity);
    HIPCHK(c, sph::launch_density(c, p, false));
    ph_end(c, kPhDensity);
  }
  ++c->density_launches;
  ++c->densities_on_tree;
  return SPH_OK;
}

// Force: from the lists while they hold every pair, the walking kernel for
// the rest (or for all groups).
static sph_status run_force(sph_ctx* c, sph_particles* p, bool step_mode) {
  if (sph::lists_mode(c)) {
    ph_begin(c, kPhForce);
    HIPCHK(c, sph::launch_force_lists(c, p, step_mode));
    ph_end(c, kPhForce);
    ph_begin(c, kPhForceFb);
    HIPCHK(c, sph::launch_force(c, p, step_mode, true));
    ph_end(c, kPhForceFb);
  } else {
    ph_begin(c, kPhForce);
    HIPCHK(c, sph::launch_force(c, p, step_mode, false));
    ph_end(c, kPhForce);
  }
  ++c->force_launches;
  return SPH_OK;
}

sph_status sph_density(sph_ctx* c, sph_particles* p, int32_t* iters_out) {
  if (!c) return SPH_E_ARG;
  sph_status st = check_parts(c, p, false, true);
  if (st != SPH_OK) return st;
  if (p->n != c->n) return fail(c, SPH_E_ARG, "n differs from the last sph_build_tree");
  // the packed positions and masses the list and density kernels gather are
  // taken from the arrays as they are now (m may have changed since the build;
  // the mixed code records are packed with the h_max refresh below)
  HIPCHK(c, sph::launch_pack_xyzm(c, p));
  // the node and group h_max are brought up to the h in p->h first (the
  // caller may have changed h since the build, and a later pass on the same
  // tree starts from the h the last one converged to), or the list walk
  // could leave out a neighbour whose h grew past its node's h_max
  HIPCHK(c, sph::launch_node_h(c, p, true));
  HIPCHK(c, sph::launch_leaf_state(c, 1));
  st = run_density(c, p);
  if (st != SPH_OK) return st;
  if (iters_out) {
    st = sync_state(c, true);
    *iters_out = c->hs->max_iter;
    return st;
  }
  return SPH_OK;
}

sph_status sph_force(sph_ctx* c, sph_particles* p, double* dt_next_out) {
  if (!c) return SPH_E_ARG;
  sph_status st = check_parts(c, p, true, true);
  if (st != SPH_OK) return st;
  if (p->n != c->n) return fail(c, SPH_E_ARG, "n differs from the last sph_build_tree");
  HIPCHK(c, sph::launch_node_h(c, p, false));
  HIPCHK(c, sph::launch_force_reset(c));
  st = run_force(c, p, false);
  if (st != SPH_OK) return st;
  if (dt_next_out) {
    st = sync_state(c, true);
    *dt_next_out = sph::dec_f64(c->hs->dt_min_enc);
    return st;
  }
  return SPH_OK;
}

sph_status sph_step(sph_ctx* c, sph_particles* p, double dt, double* dt_next_out) {
  if (!c) return SPH_E_ARG;
  sph_status st = check_parts(c, p, true, true);
  if (st != SPH_OK) return st;
  if (!isfinite(dt)) return fail(c, SPH_E_ARG, "dt is not finite");
  // phase events on one call in timing_every; other entry points always record
  struct TimingScope {
    sph_ctx* c;
    ~TimingScope() { c->timing = c->timing_every > 0; }
  } scope{c};
  c->timing = c->timing_every > 0 && (c->step_calls++ % c->timing_every) == 0;
  ph_begin(c, kPhStep);
  HIPCHK(c, sph::launch_step_begin(c, dt));
  st = do_build(c, p, false, true);
  if (st != SPH_OK) return st;
  st = run_density(c, p);
  if (st != SPH_OK) return st;
  HIPCHK(c, sph::launch_node_h(c, p, false));
  st = run_force(c, p, true);
  if (st != SPH_OK) return st;
  ph_begin(c, kPhIntegrate);
  HIPCHK(c, sph::launch_correct(c, p));
  ph_end(c, kPhIntegrate);
  ph_end(c, kPhStep);
  if (dt_next_out) {
    st = sync_state(c, true);
    *dt_next_out = sph::dec_f64(c->hs->dt_min_enc);
    return st;
  }
  return SPH_OK;
}

// ---- adjoint ----------------------------------------------------------------

static sph_status adj_check(sph_ctx* c, const sph_particles* p, const sph_cotangents* g) {
  sph_status st = check_parts(c, p, true, true);
  if (st != SPH_OK) return st;
  if (!p->id) return fail(c, SPH_E_ARG, "the adjoint needs particle ids (p->id)");
  if (!g || !g->x || !g->y || !g->z || !g->vx || !g->vy || !g->vz || !g->u || !g->ax || !g->ay ||
      !g->az || !g->dudt)
    return fail(c, SPH_E_ARG, "every cotangent array is required");
  if (!sph::lists_mode(c)) return fail(c, SPH_E_ARG, "the adjoint needs n_group 4 or 8");
  if (c->kp.fixed_passes)
    return fail(c, SPH_E_ARG, "the adjoint differentiates the iterated density (h_tol >= 0)");
  if (!c->adj_raw) {
    const int64_t N = c->n_max;
    hipError_t e = hipMalloc(&c->adj_abar, 32 * (size_t)N);
    if (e == hipSuccess) e = hipMalloc((void**)&c->adj_raw, 7 * sizeof(double) * (size_t)N);
    if (e == hipSuccess) e = hipMalloc((void**)&c->adj_ab, sizeof(double2) * (size_t)N);
    if (e != hipSuccess) {
      (void)hipFree(c->adj_abar);
      (void)hipFree(c->adj_raw);
      (void)hipFree(c->adj_ab);
      c->adj_abar = nullptr;
      c->adj_raw = nullptr;
      c->adj_ab = nullptr;
      return hip_fail(c, e, "adjoint workspace");
    }
  }
  return SPH_OK;
}

// The adjoint kernels read the neighbour-list rows of the forward pass.  They
// hold every density and force pair unless a group was flagged (its row
// overflowed or some h outgrew it); then the rows are rebuilt at the current
// h and must be complete.
static sph_status adj_launch(sph_ctx* c, const sph_particles* p, sph_cotangents* g, double dt,
                             bool step_mode) {
  ph_begin(c, kPhAdjoint);
  HIPCHK(c, sph::launch_adjoint(c, p, g, dt, step_mode, 0));
  ph_begin(c, kPhAdjForce);
  HIPCHK(c, sph::launch_adjoint(c, p, g, dt, step_mode, 1));
  ph_end(c, kPhAdjForce);
  HIPCHK(c, sph::launch_adjoint(c, p, g, dt, step_mode, 2));
  ph_end(c, kPhAdjoint);
  return SPH_OK;
}

static sph_status adj_rows(sph_ctx* c, const sph_particles* p) {
  sph_status st = sync_state(c, true);
  if (st != SPH_OK) return st;
  if (c->hs->n_flagged == 0) return SPH_OK;
  HIPCHK(c, sph::launch_node_h(c, p, true));
  HIPCHK(c, sph::launch_leaf_state(c, 1));
  HIPCHK(c, sph::launch_lists(c, p));
  ++c->lists_launches;
  st = sync_state(c, true);
  if (st != SPH_OK) return st;
  if (c->hs->n_flagged != 0)
    return fail(c, SPH_E_OVERFLOW, "adjoint: a neighbour-list row cannot hold all neighbours");
  return SPH_OK;
}

sph_status sph_eval_adjoint(sph_ctx* c, const sph_particles* p, sph_cotangents* g) {
  if (!c) return SPH_E_ARG;
  sph_status st = adj_check(c, p, g);
  if (st != SPH_OK) return st;
  if (p->n != c->n) return fail(c, SPH_E_ARG, "n differs from the last sph_build_tree");
  st = adj_rows(c, p);
  if (st != SPH_OK) return st;
  return adj_launch(c, p, g, 0.0, false);
}

sph_status sph_step_adjoint(sph_ctx* c, sph_particles* p, double dt, sph_cotangents* g) {
  if (!c) return SPH_E_ARG;
  sph_status st = adj_check(c, p, g);
  if (st != SPH_OK) return st;
  if (!(dt > 0.0) || !isfinite(dt)) return fail(c, SPH_E_ARG, "the step adjoint needs dt > 0");
  // the forward step up to the corrector (as sph_step)
  ph_begin(c, kPhStep);
  HIPCHK(c, sph::launch_step_begin(c, dt));
  st = do_build(c, p, false, true);
  if (st != SPH_OK) return st;
  st = run_density(c, p);
  if (st != SPH_OK) return st;
  HIPCHK(c, sph::launch_node_h(c, p, false));
  st = run_force(c, p, true);
  if (st != SPH_OK) return st;
  ph_end(c, kPhStep);
  // reverse sweep at the predicted state (x1, v_p, u_p, new a in scratch)
  st = adj_rows(c, p);
  if (st != SPH_OK) return st;
  st = adj_launch(c, p, g, dt, true);
  if (st != SPH_OK) return st;
  ph_begin(c, kPhIntegrate);
  HIPCHK(c, sph::launch_correct(c, p));
  ph_end(c, kPhIntegrate);
  return SPH_OK;
}

sph_status sph_reduce(sph_ctx* c, const sph_particles* p, double out[12]) {
  if (!c || !out) return SPH_E_ARG;
  sph_status st = check_parts(c, p, true, false);
  if (st != SPH_OK) return st;
  HIPCHK(c, sph::launch_reduce(c, p, c->red_out));
  HIPCHK(c, hipMemcpyAsync(out, c->red_out, 12 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SPH_OK;
}

sph_status sph_reduce_noalloc(const sph_particles* p, void* stream, double out[12]) {
  auto reject = [](const char* why) {
    g_create_err = std::string("sph_reduce_noalloc: ") + why;
    return SPH_E_ARG;
  };
  if (!p || !out) return reject("particles or out is NULL");
  if (p->n < 1 || p->n > (int64_t)0x7fffffff) return reject("n must be in [1, 2^31 - 1]");
  if (!p->m || !p->vx || !p->vy || !p->vz || !p->u || !p->ax || !p->ay || !p->az || !p->dudt)
    return reject("m, vx, vy, vz, u, ax, ay, az and dudt are required");
  const hipError_t e = sph::reduce_noalloc(p, (hipStream_t)stream, out);
  if (e != hipSuccess) {
    g_create_err = std::string("sph_reduce_noalloc: ") + hipGetErrorString(e);
    return SPH_E_HIP;
  }
  return SPH_OK;
}

sph_status sph_check(sph_ctx* c) {
  if (!c) return SPH_E_ARG;
  return sync_state(c, true);
}

sph_status sph_get_keys(sph_ctx* c, uint64_t* keys, int64_t* perm) {
  if (!c || c->n < 1) return SPH_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (keys) HIPCHK(c, hipMemcpy(keys, c->keys[0], sizeof(uint64_t) * c->n, hipMemcpyDeviceToHost));
  if (perm) {
    std::vector<uint32_t> v(c->n);
    HIPCHK(c, hipMemcpy(v.data(), c->vals[0], sizeof(uint32_t) * c->n, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n; ++i) perm[i] = v[i];
  }
  return SPH_OK;
}

sph_status sph_get_tree(sph_ctx* c, int64_t* n_nodes, int32_t* level, uint64_t* prefix,
                        int64_t* first, int64_t* count, int64_t* child_first, int32_t* n_child) {
  if (!c || !n_nodes || c->n < 1) return SPH_E_ARG;
  sph_status st = sync_state(c, false);
  if (st != SPH_OK) return st;
  const int64_t nn = c->hs->n_nodes;
  const int64_t cap = *n_nodes;
  *n_nodes = nn;
  if (!level && !prefix && !first && !count && !child_first && !n_child) return SPH_OK;
  if (cap < nn) return fail(c, SPH_E_ARG, "node arrays too small");
  std::vector<int32_t> lv(nn), fi(nn), co(nn), ch(nn), nc(nn);
  std::vector<uint64_t> keys(c->n);
  HIPCHK(c, hipMemcpy(lv.data(), c->node_level, 4 * nn, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(fi.data(), c->node_first, 4 * nn, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(co.data(), c->node_count, 4 * nn, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(ch.data(), c->node_child, 4 * nn, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(nc.data(), c->node_nchild, 4 * nn, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(keys.data(), c->keys[0], 8 * (size_t)c->n, hipMemcpyDeviceToHost));
  // inner-node counts: sums of the (contiguous) children, deepest first
  std::vector<int64_t> cnt64(nn);
  for (int64_t k = nn - 1; k >= 0; --k) {
    if (nc[k] == 0) {
      cnt64[k] = co[k];
    } else {
      int64_t t = 0;
      for (int q = 0; q < nc[k]; ++q) t += cnt64[ch[k] + q];
      cnt64[k] = t;
    }
  }
  for (int64_t k = 0; k < nn; ++k) {
    if (level) level[k] = lv[k];
    if (first) first[k] = fi[k];
    if (count) count[k] = cnt64[k];
    if (child_first) child_first[k] = nc[k] ? ch[k] : -1;
    if (n_child) n_child[k] = nc[k];
    if (prefix) {
      const int l = lv[k];
      prefix[k] = (l == 0) ? 0ull : (keys[fi[k]] >> (3 * (sph::kKeyLevels - l)));
    }
  }
  return SPH_OK;
}

sph_status sph_get_groups(sph_ctx* c, int64_t* n_groups, int64_t* first, int64_t* count) {
  if (!c || !n_groups || c->n < 1) return SPH_E_ARG;
  sph_status st = sync_state(c, false);
  if (st != SPH_OK) return st;
  const int64_t ng = c->hs->n_groups;
  const int64_t cap = *n_groups;
  *n_groups = ng;
  if (!first && !count) return SPH_OK;
  if (cap < ng) return fail(c, SPH_E_ARG, "group arrays too small");
  std::vector<int32_t> fi(ng), co(ng);
  HIPCHK(c, hipMemcpy(fi.data(), c->grp_first, 4 * ng, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(co.data(), c->grp_count, 4 * ng, hipMemcpyDeviceToHost));
  for (int64_t g = 0; g < ng; ++g) {
    if (first) first[g] = fi[g];
    if (count) count[g] = co[g];
  }
  return SPH_OK;
}

// CSR of exact neighbour sets at the current h on the host, from the group
// walk (source 0) or from the list rows (source 1).
static sph_status export_sets(sph_ctx* c, const sph_particles* p, int mode, int source,
                              int64_t* offsets, int32_t* idx, int64_t cap, const char* who) {
  if (source == 0) {
    HIPCHK(c, sph::launch_node_h(c, p, true));  // the current h, whatever the force used
    HIPCHK(c, sph::launch_neighbours(c, p, mode, c->nb_cnt, nullptr, nullptr));
  } else {
    HIPCHK(c, sph::launch_row_sets(c, p, mode, c->nb_cnt, nullptr, nullptr));
  }
  std::vector<int32_t> cnt(c->n);
  HIPCHK(c, hipMemcpyAsync(cnt.data(), c->nb_cnt, 4 * (size_t)c->n, hipMemcpyDeviceToHost,
                           c->stream));
  sph_status st = sync_state(c, true);
  if (st != SPH_OK) return st;
  offsets[0] = 0;
  for (int i = 0; i < c->n; ++i) {
    if (cnt[i] < 0) return fail(c, SPH_E_OVERFLOW, "a particle's list row is incomplete");
    offsets[i + 1] = offsets[i] + cnt[i];
  }
  const int64_t total = offsets[c->n];
  if (!idx) return SPH_OK;
  if (cap < total) return fail(c, SPH_E_ARG, "idx capacity too small");
  int32_t* didx = nullptr;
  HIPCHK(c, hipMalloc((void**)&didx, sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1)));
  hipError_t e = hipMemcpyAsync(c->nb_off, offsets, 8 * ((size_t)c->n + 1), hipMemcpyHostToDevice,
                                c->stream);
  if (e == hipSuccess)
    e = source == 0 ? sph::launch_neighbours(c, p, mode, nullptr, c->nb_off, didx)
                    : sph::launch_row_sets(c, p, mode, c->nb_cnt, didx, c->nb_off);
  if (e == hipSuccess)
    e = hipMemcpyAsync(idx, didx, 4 * (size_t)total, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(didx);
  if (e != hipSuccess) return hip_fail(c, e, who);
  for (int i = 0; i < c->n; ++i) std::sort(idx + offsets[i], idx + offsets[i + 1]);
  return sync_state(c, true);
}

sph_status sph_neighbours(sph_ctx* c, const sph_particles* p, int32_t mode, int64_t* offsets,
                          int32_t* idx, int64_t cap) {
  if (!c || !offsets || (mode != 0 && mode != 1)) return SPH_E_ARG;
  sph_status st = check_parts(c, p, false, false);
  if (st != SPH_OK) return st;
  if (p->n != c->n) return fail(c, SPH_E_ARG, "n differs from the last sph_build_tree");
  return export_sets(c, p, mode, 0, offsets, idx, cap, "sph_neighbours");
}

sph_status sph_list_pairs(sph_ctx* c, const sph_particles* p, int32_t mode, int64_t* offsets,
                          int32_t* idx, int64_t cap) {
  if (!c || !offsets || (mode != 0 && mode != 1)) return SPH_E_ARG;
  sph_status st = check_parts(c, p, false, false);
  if (st != SPH_OK) return st;
  if (p->n != c->n) return fail(c, SPH_E_ARG, "n differs from the last sph_build_tree");
  if (!sph::lists_mode(c)) return fail(c, SPH_E_ARG, "the list rows need n_group 4 or 8");
  if (c->lists_launches == 0 || c->densities_on_tree == 0)
    return fail(c, SPH_E_ARG, "no density pass on this tree has built the list rows");
  // rows of flagged groups are incomplete: rebuilt at the current h once;
  // particles still flagged went through the walking kernels, whose sets the
  // group walk with the same exact predicate gives
  st = sync_state(c, true);
  if (st != SPH_OK) return st;
  if (c->hs->n_flagged != 0) {
    HIPCHK(c, sph::launch_node_h(c, p, true));
    HIPCHK(c, sph::launch_leaf_state(c, 1));
    HIPCHK(c, sph::launch_lists(c, p));
    ++c->lists_launches;
    st = sync_state(c, true);
    if (st != SPH_OK) return st;
  }
  const int source = c->hs->n_flagged == 0 ? 1 : 0;
  return export_sets(c, p, mode, source, offsets, idx, cap, "sph_list_pairs");
}

sph_status sph_set_timing(sph_ctx* c, int32_t every) {
  if (!c || every < 0) return SPH_E_ARG;
  c->timing_every = every;
  c->timing = every > 0;
  c->step_calls = 0;
  return SPH_OK;
}

sph_status sph_timings(sph_ctx* c, double out[12]) {
  if (!c || !out) return SPH_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 12; ++k) out[k] = 0.0;
  sph_timing* x = c->tm;
  if (!x || !x->ready) return SPH_OK;
  const int map[kNPh] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
  for (int ph = 0; ph < kNPh; ++ph) {
    double s = 0.0;
    const int n = x->count[ph];
    for (int r = 0; r < n; ++r) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, x->start[ph][r], x->stop[ph][r]) == hipSuccess) s += ms;
    }
    out[map[ph]] = n ? s / n : 0.0;
    x->count[ph] = 0;
  }
  return SPH_OK;
}

sph_status sph_stats(sph_ctx* c, int64_t out[18]) {
  if (!c || !out) return SPH_E_ARG;
  HIPCHK(c, hipMemcpyAsync(c->hs, c->ds, sizeof(sph::DevState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const sph::DevState& s = *c->hs;
  out[0] = s.n_nodes;
  out[1] = s.n_groups;
  out[2] = s.max_iter;
  out[3] = (int64_t)s.n_pairs_density;
  out[4] = (int64_t)s.n_pairs_force;
  out[5] = (int64_t)s.n_sums_density;
  out[6] = (int64_t)s.n_cand_density;
  out[7] = (int64_t)s.n_cand_force;
  out[8] = s.n_rewalk;
  out[9] = s.err;
  out[10] = (int64_t)s.tot_sums_density;
  out[11] = (int64_t)s.tot_pairs_force;
  out[12] = c->density_launches;
  out[13] = c->force_launches;
  out[14] = s.n_flag_rows;
  out[15] = s.n_flag_grew;
  out[16] = (int64_t)s.tot_cand_lists;
  out[17] = c->lists_launches;
  return SPH_OK;
}

const char* sph_last_error(const sph_ctx* c) {
  if (!c) return g_create_err.empty() ? "null context" : g_create_err.c_str();
  return c->err.c_str();
}

}  // extern "C"
