/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH hydrodynamics library.
 *
 * The library computes the per-step hydrodynamics of Bonsai-SPH (Bedorf &
 * Portegies Zwart, arXiv:1909.07439): space-filling-curve keys and sort, the
 * octree and particle groups (Sect. 3.1), the group tree walk for neighbours
 * (Sect. 3.2), the variable-h density (Sect. 2.2; iterated as in Sect.
 * 3.2.1), the hydrodynamic force with artificial viscosity and conductivity
 * (Sect. 2.4-2.6, eq:acc, eq:energy, eq:vsig, eq:viscosity_shock) and the
 * leapfrog step with a global Courant time step (Sect. 2.4, eq:predict_pos,
 * eq:predict_vel, eq:correct_vel, eq:timestep; Sect. 3.3).
 *
 * Conventions for every entry point:
 *   - Particle fields are caller-owned DEVICE arrays (length n, contiguous,
 *     float64 unless stated).  The library never allocates, frees or keeps
 *     them beyond a call.  sph_build_tree and sph_step reorder them in place.
 *   - All scratch memory is allocated once by sph_create (sized for n_max);
 *     the compute calls allocate nothing.
 *   - Work is enqueued on the HIP stream given to sph_create.  Calls that
 *     return host values (iters_out, dt_next_out, sph_reduce, sph_get_*,
 *     sph_neighbours) synchronise that stream; with NULL out-pointers
 *     sph_density / sph_force / sph_step do not synchronise.
 *   - No exception crosses the ABI.  Every call returns a status; on failure
 *     sph_last_error() describes it.  Device-side failures (an overflowing
 *     walk list, a non-converging smoothing length, a non-finite result) are
 *     latched in a device error word and reported by the next call that
 *     synchronises, and by sph_check().
 *   - One context must not be used from two host threads at once.
 */
#ifndef SPH_H
#define SPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx; /* opaque; owns all scratch */

typedef enum {
  SPH_OK = 0,
  SPH_E_ARG = -1,       /* bad argument (NULL pointer, n > n_max, bad parameter) */
  SPH_E_NOMEM = -2,     /* device allocation failed in sph_create */
  SPH_E_HIP = -3,       /* a HIP runtime call failed */
  SPH_E_NOCONV = -4,    /* smoothing-length iteration did not converge */
  SPH_E_OVERFLOW = -5,  /* a fixed-capacity list (tree nodes, walk lists) overflowed */
  SPH_E_DOMAIN = -6,    /* the kernel support S h reaches half a periodic box length */
  SPH_E_NONFINITE = -7  /* a NaN/Inf appeared in an input or a result */
} sph_status;

typedef enum { SPH_PREC_FP64 = 0, SPH_PREC_MIXED = 1 } sph_precision;

/* Run parameters (copied by sph_create). */
typedef struct {
  double box_lo[3];     /* box corner */
  double box_len[3];    /* box side lengths; keys use cubic cells of side max(box_len) */
  int32_t periodic[3];  /* 1: periodic axis (minimum image); 0: open */
  double gamma;         /* adiabatic index */
  double gamma_minus_1; /* gamma - 1, given separately so that it is exact */
  double hfact;         /* h = hfact (m/rho)^(1/3) (Sect. 2.2); 1.2 */
  double alpha_av;      /* artificial viscosity alpha (Sect. 2.5); 1 */
  double beta_av;       /* artificial viscosity beta; 2 */
  double alpha_u;       /* artificial conductivity alpha_u (Sect. 2.6); 1 */
  double c_cour;        /* Courant factor (eq:timestep); 0.3 */
  int32_t kernel;       /* smoothing kernel (Sect. 2.3): 0 = M4 cubic spline (support 2h),
                           1 = M6 quintic spline (support 3h), 2 = Wendland C6 (support 2h) */
  int32_t n_leaf;       /* max particles per tree leaf (Sect. 3.1); 1..64 */
  int32_t n_group;      /* max particles per walk group (Sect. 3.1); one of 4,8,16,32 */
  int32_t precision;    /* sph_precision: pair arithmetic in FP64, or in FP32 on separations
                           formed from 32-bit fixed-point position codes (2^32 per periodic
                           length; 2^31 over the tree's root box on an open axis) with
                           positions, h, the integration and the reductions in FP64 */
  double h_tol;         /* h is converged when |S0(h) - m (hfact/h)^3| <= 3 h_tol m (hfact/h)^3,
                           i.e. a Newton step would move it by <= ~h_tol*h; 0 selects the
                           default (1e-14 FP64, 2e-7 mixed); < 0: three fixed passes */
  int32_t max_h_iter;   /* iteration limit before SPH_E_NOCONV (default 30 if <= 0) */
  int32_t reserved0;
  double h_margin;      /* neighbour lists cover r < S h h_margin (S the kernel support in
                           units of h) so h may grow by that
                           factor without a new walk (default 1.1 if <= 1) */
} sph_params;

/* Particle set: SoA device pointers, all of length n.  "in" fields are read,
   "out" fields written; sph_build_tree / sph_step permute every non-NULL
   field into curve order.  Optional outputs may be NULL where stated. */
typedef struct {
  int64_t n;
  int64_t* id;  /* in/out: caller's particle ids, permuted with the particles (may be NULL) */
  double *x, *y, *z;       /* in: positions, inside the box on periodic axes */
  double *vx, *vy, *vz;    /* in: velocities */
  double* m;               /* in: masses (> 0) */
  double* u;               /* in: specific internal energy */
  double* h;               /* in: smoothing-length start value; out: converged h */
  double *ax, *ay, *az;    /* out (sph_force); in+out (sph_step: previous acceleration) */
  double* dudt;            /* out (sph_force); in+out (sph_step) */
  double* rho;             /* out (sph_density) */
  double* omega;           /* out (sph_density): grad-h term Omega */
  double* P;               /* out (sph_density): pressure */
  double* cs;              /* out (sph_density): sound speed */
  double* vsig_dt;         /* out (sph_force): max signal speed for the time step */
} sph_particles;

/* Create a context for up to n_max particles on the current HIP device.
   stream: a hipStream_t (NULL = default stream).  Allocates all scratch.
   Errors: SPH_E_ARG (bad parameter), SPH_E_NOMEM, SPH_E_HIP. */
sph_status sph_create(const sph_params* params, int64_t n_max, void* stream, sph_ctx** out);

/* Destroy a context and free its scratch.  NULL is ignored. */
void sph_destroy(sph_ctx* ctx);

/* Keys, sort and tree (Sect. 3.1): computes 63-bit Morton keys of the
   positions (21 bits per axis, x in the top bit of each triple), sorts the
   particles stably by key, permutes every non-NULL field of *p in place into
   that order, then builds the octree (a cell holding more than n_leaf
   particles above level 21 is split into its non-empty children), the
   particle groups (maximal cells with at most n_group particles; oversized
   level-21 cells cut into chunks) and the tight bounding boxes of both.
   Errors: SPH_E_ARG, SPH_E_OVERFLOW (node capacity), SPH_E_HIP. */
sph_status sph_build_tree(sph_ctx* ctx, sph_particles* p);

/* Density (Sect. 2.2, Sect. 3.2.1) on the tree of the last sph_build_tree:
   for every particle the smoothing length is iterated to the root of
   sum_j m_j W(r_ij, h) = m (hfact/h)^3 (j within the support S h: S = 2
   for M4 and Wendland C6, 3 for M6; self included), with a
   wavefront-wide convergence vote per group; then rho, Omega = 1 + h S1/(3
   rho), P = (gamma-1) rho u and cs = sqrt(gamma (gamma-1) u) are written.
   iters_out (may be NULL; if given, the call synchronises): the largest
   number of density sums any group needed.  The positions must be those the
   tree was built from (in its order); m, h, u and v may have changed since:
   the call takes them as they are, and first brings the tree's node and group
   h_max up to the h in p->h (a later call on the same tree starts from the h
   the previous one converged to).
   Errors: SPH_E_NOCONV, SPH_E_OVERFLOW, SPH_E_DOMAIN, SPH_E_NONFINITE. */
sph_status sph_density(sph_ctx* ctx, sph_particles* p, int32_t* iters_out);

/* Hydrodynamic force (Sect. 2.4-2.6): for every pair with r < S max(h_i,h_j)
   the pressure, artificial-viscosity and conductivity terms; writes ax, ay,
   az, dudt and vsig_dt.  Needs rho, omega, P, cs from sph_density on the
   same tree; the neighbours' x, m, h, v and u are those of that call (the
   density pass packs them into per-particle records the force gathers), so
   a change to v or u takes effect through another sph_density.  dt_next_out (may be NULL; if given the call synchronises):
   c_cour * min_i h_i / vsig_dt_i.  The same value is also kept on the device
   for sph_step.
   Errors: SPH_E_OVERFLOW, SPH_E_NONFINITE, SPH_E_HIP. */
sph_status sph_force(sph_ctx* ctx, sph_particles* p, double* dt_next_out);

/* One leapfrog step (Sect. 2.4, Sect. 3.3): predict r, v, u with the
   previous ax, ay, az, dudt; wrap positions into periodic boxes; rebuild the
   tree; density; force; correct v and u; store the new accelerations.
   dt > 0: that step; dt <= 0: the Courant step left on the device by the last
   sph_force / sph_step (no host round trip).  dt_next_out as in sph_force.
   Particles are left in the new curve order. */
sph_status sph_step(sph_ctx* ctx, sph_particles* p, double dt, double* dt_next_out);

/* Global FP64 sums in a fixed order (deterministic): out[12] = {E, E_kin,
   E_th, p_x, p_y, p_z, sum m a_x, sum m a_y, sum m a_z, dE/dt = sum m (v.a +
   du/dt), sum m |a|, sum m (|v.a| + |du/dt|)}.  E is the total energy whose
   relative change the paper uses as its conservation measure (Sect. 4.5,
   eq:energy_error); the momentum and energy-rate sums test the
   conservation of the pair forms of eq:acc and eq:energy.  Synchronises. */
sph_status sph_reduce(sph_ctx* ctx, const sph_particles* p, double out[12]);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the sums
   of sph_reduce without a context.  The per-block partial sums and the
   results live in one file-scope device array of the library (49,280 bytes
   on each GPU it runs on, held until the process ends); the call allocates
   nothing.  Every call on a GPU uses that GPU's array, so calls that overlap
   on one GPU (several host threads or streams) race; calls in sequence do
   not (each writes every partial before reading it).  p: n in [1, 2^31 - 1],
   and m, vx, vy, vz, u, ax, ay, az, dudt (device arrays of the current
   device).  stream: a hipStream_t of the current device (NULL = default).
   out: HOST array of 12 doubles, the values of sph_reduce bit for bit.
   Synchronises the stream.  Errors: SPH_E_ARG (NULL pointers, n out of
   range, a missing field), SPH_E_HIP; sph_last_error(NULL) describes them. */
sph_status sph_reduce_noalloc(const sph_particles* p, void* stream, double out[12]);

/* Device error word of the last calls, as a status (SPH_OK if clean); clears
   it.  Synchronises. */
sph_status sph_check(sph_ctx* ctx);

/* ---- inspection (host copies; synchronising; for tests and tools) ---- */

/* Sorted keys of the last sph_build_tree (the space-filling-curve keys of
   Sect. 3.1) and perm[k] = pre-sort index of the particle now at position k.
   Host arrays of n entries (either may be NULL). */
sph_status sph_get_keys(sph_ctx* ctx, uint64_t* keys, int64_t* perm);

/* Octree of the last sph_build_tree (Sect. 3.1: the sorted curve chopped
   into sections of at most n_leaf particles) in canonical order (by level,
   then key).
   *n_nodes: in = capacity of the arrays, out = node count.  With all arrays
   NULL only the count is returned.  child_first is -1 for leaves.
   Errors: SPH_E_ARG if the capacity is too small. */
sph_status sph_get_tree(sph_ctx* ctx, int64_t* n_nodes, int32_t* level, uint64_t* prefix,
                        int64_t* first, int64_t* count, int64_t* child_first,
                        int32_t* n_child);

/* Particle groups of the last sph_build_tree (Sect. 3.1: sections of the
   sorted curve with at most n_group particles, which walk the tree
   together), ordered by first particle.  *n_groups: in = capacity of the
   host arrays first, count; out = group count (NULL arrays: count only). */
sph_status sph_get_groups(sph_ctx* ctx, int64_t* n_groups, int64_t* first, int64_t* count);

/* Neighbour sets found by the group tree walk (Sect. 3.2: a node is opened
   while it lies within the group's search radius; the density set uses the
   particle's own smoothing range, the force set the larger of the pair's),
   as CSR over the current particle order with ascending indices: mode 0 =
   density set (r < S h_i, self included), mode 1 = force set (j != i,
   r < S max(h_i, h_j)), using the h currently in p->h and the FP64
   predicate of both precision modes.  This is an inspection walk of its
   own; sph_list_pairs gives the sets of the hot path.
   offsets: host array of n+1 entries (always filled); idx: host array of
   cap entries (may be NULL to query the total in offsets[n]).
   Errors: SPH_E_ARG (cap too small: offsets are still filled). */
sph_status sph_neighbours(sph_ctx* ctx, const sph_particles* p, int32_t mode, int64_t* offsets,
                          int32_t* idx, int64_t cap);

/* The pairs the hot path's density (mode 0) and force (mode 1) list
   kernels accept (Sect. 3.2, 3.2.1): each particle's neighbour-list row
   written by the last density pass's list walk, filtered with the exact
   FP64 predicate at the h currently in p->h (density: r < S h_i, self
   included; force: j != i, r < S max(h_i, h_j)).  The mixed mode's FP32
   test is settled in FP64 near the boundary, so both precisions accept the
   FP64 sets.  CSR over the current particle order with ascending indices;
   offsets, idx and cap as in sph_neighbours.  If some group was flagged in
   that pass (a row overflowed or an h outgrew it) the rows are first
   rebuilt at the current h; particles still flagged went through the walking
   kernels, and the sets then come from the group walk with the same exact
   predicate (as sph_neighbours).  Needs n_group 4 or 8 and a density pass on
   the current tree.  Errors: SPH_E_ARG, SPH_E_HIP. */
sph_status sph_list_pairs(sph_ctx* ctx, const sph_particles* p, int32_t mode, int64_t* offsets,
                          int32_t* idx, int64_t cap);

/* Mean duration of the launches of each phase since the previous call, in
   milliseconds, from HIP events recorded on the library stream around each
   phase (at most 1024 launches per phase are kept): out[0..11] = {keys+sort,
   permute, tree, density, force, integrate, total step, neighbour lists,
   density of flagged groups, force of flagged groups, adjoint kernels of
   sph_eval_adjoint / sph_step_adjoint, the force-adjoint kernel alone}.
   The density, force, integrate, neighbour-list, flagged-group and
   force-adjoint phases each bracket exactly one kernel.  Clears the kept
   events.  Synchronises. */
sph_status sph_timings(sph_ctx* ctx, double out[12]);

/* Which calls record the phase events of sph_timings: sph_step records them
   on one call in `every` (the first after this call, then every every-th),
   0 records none; every other entry point records them whenever every > 0.
   The default is 1 (every call).  Each recorded phase boundary leaves the
   GPU idle for a few microseconds, so a throughput run samples (e.g. every =
   8) and sph_timings averages over the sampled launches.  Returns SPH_E_ARG
   for every < 0.  Host-only; no GPU work. */
sph_status sph_set_timing(sph_ctx* ctx, int32_t every);

/* Counters of the work done (for throughput accounting).  out[0..9] refer
   to the last sph_build_tree / sph_step: {tree nodes, groups, most density
   sums any group needed, true density neighbours (r < S h, self included) at
   the converged h, force pairs, density pair terms summed over all passes,
   density candidate tests, force candidate tests, walks done by the density
   pass, device error word}.  out[10..13] are running totals since
   sph_create: {density pair terms, force pairs, density launches, force
   launches}; differences of two calls give the work of the launches in
   between.  out[14..15] refer to the last density pass: {groups whose
   neighbour-list rows overflowed, groups in which some h outgrew the rows};
   both went through the walking kernels.  out[16..17] are running totals:
   {candidate tests of the neighbour-list kernel, its launches}.
   Synchronises. */
sph_status sph_stats(sph_ctx* ctx, int64_t out[18]);

/* ---- adjoint (reverse-mode derivative) ---------------------------------

   The derivative of the equations of Sect. 2.2-2.6 (density sums, the root
   h of sum_j m_j W(r_ij, h) = m (hfact/h)^3, Omega, P, cs, the momentum and
   energy equations with viscosity and conductivity) and of the leapfrog
   (Sect. 2.4), with three things held fixed: the neighbour sets of the
   forward evaluation, the viscosity switches (approaching pairs) and dt.
   The root h enters through its implicit derivative -(dS0/dx)/(dS0/dh -
   d[m (hfact/h)^3]/dh).  The conductivity's signal speed sqrt|P_i - P_j| has
   no derivative where P_i = P_j; its derivative there is taken as zero.

   Cotangent arrays: eleven caller-owned DEVICE float64 arrays of n entries,
   indexed by the particle's id, not by its current position: the particles'
   order changes with every tree build, the cotangents keep theirs.  p->id
   must be non-NULL and hold a permutation of 0..n-1. */
typedef struct {
  double *x, *y, *z;     /* positions */
  double *vx, *vy, *vz;  /* velocities */
  double* u;             /* specific internal energy */
  double *ax, *ay, *az;  /* accelerations */
  double* dudt;          /* du/dt */
} sph_cotangents;

/* Adjoint of the evaluation last done by sph_density + sph_force on p (no
   sph_build_tree or sph_step in between; p unchanged).  Reads g->ax, ay, az,
   dudt (the cotangents of that evaluation's outputs) and ADDS the cotangents
   of its inputs x, y, z, vx, vy, vz, u to g->x ... g->u; g->ax ... g->dudt
   are left unchanged.  Asynchronous unless the neighbour rows of the forward
   pass were incomplete (a group overflowed its row or some h outgrew it):
   then the call synchronises and rebuilds the rows at the current h.
   Needs n_group 4 or 8 and the iterated density (h_tol >= 0).  The first
   adjoint call on a context allocates its adjoint workspace (about 100 bytes
   per particle of n_max); later calls allocate nothing.
   Errors: SPH_E_ARG, SPH_E_NOMEM (workspace), SPH_E_OVERFLOW (a neighbour row
   cannot hold all neighbours), SPH_E_HIP. */
sph_status sph_eval_adjoint(sph_ctx* ctx, const sph_particles* p, sph_cotangents* g);

/* Adjoint of one leapfrog step.  p must hold the state at the START of the
   step being differentiated, exactly as it was passed to sph_step (x, v, u,
   the previous a and dudt, h, m, id; any order).  The call performs that
   step (p ends as sph_step would leave it; dt > 0 is required, the step is
   frozen at that value), then replaces the cotangents of the step's outputs
   held in g (x, v, u, a, dudt at the step's end) by those of its inputs
   (x, v, u, a, dudt at its start).  Chaining K calls backwards over saved
   step-start states, then one sph_eval_adjoint of the initial evaluation,
   gives the gradient of a K-step rollout.  Synchronises like
   sph_eval_adjoint.  Errors as sph_step and sph_eval_adjoint. */
sph_status sph_step_adjoint(sph_ctx* ctx, sph_particles* p, double dt, sph_cotangents* g);

/* Human-readable description of the last failure of this context; with
   ctx == NULL, of the last failed sph_create on the calling thread. */
const char* sph_last_error(const sph_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
