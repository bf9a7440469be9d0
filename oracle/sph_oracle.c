/*
 * sph_oracle.c -- plain FP64 CPU oracle for the SPH hydrodynamics step of
 * Bedorf & Portegies Zwart, "Bonsai-SPH: A GPU accelerated astrophysical
 * Smoothed Particle Hydrodynamics code" (arXiv:1909.07439).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source, header, table or helper with the HIP library.
 *
 * Everything is IEEE double, built with -ffp-contract=off; where a fused
 * multiply-add is part of a definition it is written as fma() explicitly.
 * Loops over particles are independent and parallelised with OpenMP; every
 * particle's sums run in a fixed order (ascending neighbour index).
 *
 * Definitions followed (paper sections / equations):
 *   density sum .................... Sect. 2.2, density equation
 *   h <-> rho relation ............. Sect. 2.2, smoothing-length equation
 *   Omega (grad-h term) ............ Sect. 2.2, Omega definition
 *   smoothing kernels .............. Sect. 2.3 (kernel list: M4 cubic, M6
 *                                    quintic, Wendland C6); the polynomials,
 *                                    supports and 3D normalisations are the
 *                                    standard ones (not printed in the paper)
 *   leapfrog predict / correct ..... Sect. 2.4, eq:predict_pos, eq:predict_vel,
 *                                    eq:correct_vel
 *   Courant step ................... Sect. 2.4, eq:timestep
 *   acceleration ................... Sect. 2.4, eq:acc (without gravity)
 *   internal energy rate ........... Sect. 2.4, eq:energy
 *   artificial viscosity ........... Sect. 2.5, q_ij and eq:vsig
 *   artificial conductivity ........ Sect. 2.6, eq:viscosity_shock, F_ij and
 *                                    v^u_sig definitions
 *   space-filling-curve keys, sort,
 *   tree and groups by chopping .... Sect. 3.1 (Tree Construction)
 *   neighbour criteria ............. Sect. 3.2 (density: the particle's own
 *                                    smoothing range; force: the larger of the
 *                                    two smoothing ranges)
 * Readings where the paper is silent or garbled are listed in the design
 * notes of the repository and restated at the function that uses them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_NOCONV (-4)
#define ORC_E_OVERFLOW (-5)

#define ORC_KEY_LEVELS 21 /* 21 bits per axis, 63-bit keys */

typedef struct {
  double box_lo[3];
  double box_len[3];
  int periodic[3];
  double gamma;
  double gamma_minus_1; /* passed separately so gamma=1.0001 keeps an exact gamma-1 */
  double hfact;
  double alpha_av;
  double beta_av;
  double alpha_u;
  double c_cour;
  int n_leaf;
  int n_group;
  double h_tol;   /* NR stop: |dh| <= h_tol*h.  h_tol < 0: three fixed NR passes */
  int max_h_iter; /* NR iterations before the bracketing fallback */
  int kernel;     /* 0: M4 cubic spline, 1: M6 quintic spline, 2: Wendland C6 */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Smoothing kernels in 3D (Sect. 2.3 names them; the forms below are the    */
/* standard ones).  W(r,h) = C f(q) / h^3 with q = r/h and support S h:       */
/*                                                                          */
/* M4 cubic spline, S = 2, C = 1/pi:                                         */
/*   f(q) = 1 - 3/2 q^2 + 3/4 q^3       0 <= q < 1                           */
/*        = 1/4 (2 - q)^3               1 <= q < 2                           */
/* M6 quintic spline, S = 3, C = 1/(120 pi):                                 */
/*   f(q) = (3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5    0 <= q < 1                   */
/*        = (3-q)^5 - 6 (2-q)^5                 1 <= q < 2                   */
/*        = (3-q)^5                             2 <= q < 3                   */
/* Wendland C6 with compact support H = 2h, S = 2, C = 1365/(512 pi):        */
/*   f(q) = (1 - q/2)^8 (4 q^3 + 25/4 q^2 + 4 q + 1)    0 <= q < 2           */
/* (the 3D C6 function (1-x)^8 (32 x^3 + 25 x^2 + 8 x + 1) of x = r/H).      */
/* f = 0 beyond the support.  Derived quantities:                           */
/*   F(r,h) = dW/dr = C f'(q) / h^4          (the F_ij of Sect. 2.6)          */
/*   dW/dh  = -C (3 f(q) + q f'(q)) / h^4                                    */
/* ------------------------------------------------------------------------ */
static double ipow(double t, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= t;
  return r;
}

double orc_kernel_support(int kind) { return kind == 1 ? 3.0 : 2.0; }

static double kern_norm(int kind) {
  if (kind == 1) return 1.0 / (120.0 * M_PI);
  if (kind == 2) return 1365.0 / (512.0 * M_PI);
  return 1.0 / M_PI;
}

static double kern_f(int kind, double q) {
  if (kind == 1) {
    if (q >= 3.0) return 0.0;
    double f = ipow(3.0 - q, 5);
    if (q < 2.0) f -= 6.0 * ipow(2.0 - q, 5);
    if (q < 1.0) f += 15.0 * ipow(1.0 - q, 5);
    return f;
  }
  if (kind == 2) {
    if (q >= 2.0) return 0.0;
    return ipow(1.0 - 0.5 * q, 8) * (((4.0 * q + 6.25) * q + 4.0) * q + 1.0);
  }
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) return 0.25 * ipow(2.0 - q, 3);
  return 0.0;
}

static double kern_df(int kind, double q) {
  if (kind == 1) {
    if (q >= 3.0) return 0.0;
    double d = -5.0 * ipow(3.0 - q, 4);
    if (q < 2.0) d += 30.0 * ipow(2.0 - q, 4);
    if (q < 1.0) d -= 75.0 * ipow(1.0 - q, 4);
    return d;
  }
  if (kind == 2) {
    /* d/dq of (1 - q/2)^8 g(q): (1 - q/2)^7 [-4 g(q) + (1 - q/2) g'(q)],
       which collapses to -(11/4) q (8 q^2 + 7 q + 2) (1 - q/2)^7 */
    if (q >= 2.0) return 0.0;
    return -2.75 * q * ((8.0 * q + 7.0) * q + 2.0) * ipow(1.0 - 0.5 * q, 7);
  }
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) return -0.75 * ipow(2.0 - q, 2);
  return 0.0;
}

static double kern_w(int kind, double r, double h) {
  return kern_norm(kind) * kern_f(kind, r / h) / (h * h * h);
}

static double kern_F(int kind, double r, double h) {
  return kern_norm(kind) * kern_df(kind, r / h) / (h * h * h * h);
}

static double kern_dwdh(int kind, double r, double h) {
  double q = r / h;
  return -kern_norm(kind) * (3.0 * kern_f(kind, q) + q * kern_df(kind, q)) / (h * h * h * h);
}

/* Vectorised access to the kernels for the self-tests. */
void orc_kernel(int kind, int64_t n, const double* r, const double* h, double* w, double* F,
                double* dwdh) {
  for (int64_t i = 0; i < n; ++i) {
    w[i] = kern_w(kind, r[i], h[i]);
    F[i] = kern_F(kind, r[i], h[i]);
    dwdh[i] = kern_dwdh(kind, r[i], h[i]);
  }
}

void orc_kernel_m4(int64_t n, const double* r, const double* h, double* w, double* F,
                   double* dwdh) {
  orc_kernel(0, n, r, h, w, F, dwdh);
}

/* ------------------------------------------------------------------------ */
/* Space-filling-curve keys (Sect. 3.1): Morton order, 21 bits per axis.     */
/*   q_d  = (x_d - lo_d) * (2^21 / L_max)       (one subtract, one multiply)  */
/*   i_d  = clamp(floor(q_d), 0, 2^21 - 1)                                   */
/*   key  = bits interleaved x,y,z from the most significant level down:     */
/*          bit b of i_x -> key bit 3b+2, of i_y -> 3b+1, of i_z -> 3b.      */
/* ------------------------------------------------------------------------ */
static uint64_t quantise(double x, double lo, double scale) {
  double q = (x - lo) * scale;
  double top = 2097151.0; /* 2^21 - 1 */
  if (!(q >= 0.0)) return 0; /* also maps NaN to 0 */
  q = floor(q);
  if (q > top) q = top;
  return (uint64_t)q;
}

static uint64_t interleave3(uint64_t ix, uint64_t iy, uint64_t iz) {
  uint64_t key = 0;
  for (int b = ORC_KEY_LEVELS - 1; b >= 0; --b) {
    key |= ((ix >> b) & 1ull) << (3 * b + 2);
    key |= ((iy >> b) & 1ull) << (3 * b + 1);
    key |= ((iz >> b) & 1ull) << (3 * b);
  }
  return key;
}

static double key_scale(const orc_params* p) {
  double lmax = p->box_len[0];
  if (p->box_len[1] > lmax) lmax = p->box_len[1];
  if (p->box_len[2] > lmax) lmax = p->box_len[2];
  return 2097152.0 / lmax;
}

void orc_keys(int64_t n, const double* x, const double* y, const double* z,
              const orc_params* p, uint64_t* keys) {
  double s = key_scale(p);
  for (int64_t i = 0; i < n; ++i) {
    keys[i] = interleave3(quantise(x[i], p->box_lo[0], s),
                          quantise(y[i], p->box_lo[1], s),
                          quantise(z[i], p->box_lo[2], s));
  }
}

/* Stable ascending sort by key: ties keep the input order.  perm[k] is the  */
/* input index of the k-th particle in key order.                            */
static const uint64_t* g_sort_keys; /* qsort has no context argument */
static int cmp_key_then_index(const void* a, const void* b) {
  int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
  uint64_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
  if (ka < kb) return -1;
  if (ka > kb) return 1;
  return (ia > ib) - (ia < ib);
}

void orc_sort(int64_t n, const uint64_t* keys, int64_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  g_sort_keys = keys;
  qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_then_index);
  g_sort_keys = NULL;
}

/* ------------------------------------------------------------------------ */
/* Octree by chopping the sorted curve (Sect. 3.1).                           */
/* A cell at level l holds the particles whose key shares its top 3l bits.   */
/* The root (level 0) holds all particles.  A cell with more than n_leaf     */
/* particles below level 21 is split into its non-empty children.  Nodes    */
/* are emitted level by level, and within a level in key order.              */
/* ------------------------------------------------------------------------ */
static int digit_at(uint64_t key, int level) { /* 3-bit child digit, level>=1 */
  return (int)((key >> (3 * (ORC_KEY_LEVELS - level))) & 7ull);
}

static uint64_t prefix_at(uint64_t key, int level) {
  if (level == 0) return 0;
  return key >> (3 * (ORC_KEY_LEVELS - level));
}

int64_t orc_tree(int64_t n, const uint64_t* skeys, int n_leaf, int64_t cap,
                 int32_t* level, uint64_t* prefix, int64_t* first,
                 int64_t* count, int64_t* child_first, int32_t* n_child) {
  if (n <= 0 || n_leaf < 1) return ORC_E_ARG;
  int64_t nn = 0;
  if (cap < 1) return ORC_E_OVERFLOW;
  level[0] = 0;
  prefix[0] = 0;
  first[0] = 0;
  count[0] = n;
  child_first[0] = -1;
  n_child[0] = 0;
  nn = 1;
  int64_t lev_begin = 0, lev_end = 1;
  for (int l = 0; l < ORC_KEY_LEVELS && lev_begin < lev_end; ++l) {
    for (int64_t k = lev_begin; k < lev_end; ++k) {
      if (count[k] <= n_leaf) continue; /* leaf */
      child_first[k] = nn;
      int64_t a = first[k], e = first[k] + count[k];
      while (a < e) {
        int d = digit_at(skeys[a], l + 1);
        int64_t b = a;
        while (b < e && digit_at(skeys[b], l + 1) == d) ++b;
        if (nn >= cap) return ORC_E_OVERFLOW;
        level[nn] = l + 1;
        prefix[nn] = prefix_at(skeys[a], l + 1);
        first[nn] = a;
        count[nn] = b - a;
        child_first[nn] = -1;
        n_child[nn] = 0;
        ++nn;
        ++n_child[k];
        a = b;
      }
    }
    lev_begin = lev_end;
    lev_end = nn;
  }
  return nn;
}

/* Particle groups (Sect. 3.1): chop the curve until each section holds at   */
/* most n_group particles.  The chopped cells with <= n_group particles are  */
/* the group cells; consecutive group cells that are children of the same    */
/* parent are then packed, in curve order and greedily, into sections of at  */
/* most n_group particles (a child that is chopped further ends a pack).  A   */
/* level-21 cell that is still larger (identical keys) is cut into            */
/* consecutive chunks of n_group.  Emitted in key order.                     */
static int64_t emit_group(int64_t a, int64_t c, int64_t cap, int64_t nn, int64_t* first,
                          int64_t* count) {
  if (nn < 0) return nn;
  if (nn >= cap) return ORC_E_OVERFLOW;
  first[nn] = a;
  count[nn] = c;
  return nn + 1;
}

static int64_t groups_rec(const uint64_t* skeys, int64_t a, int64_t c, int l,
                          int n_group, int64_t cap, int64_t nn, int64_t* first,
                          int64_t* count) {
  if (nn < 0) return nn;
  if (c <= n_group) return emit_group(a, c, cap, nn, first, count);
  if (l == ORC_KEY_LEVELS) {
    for (int64_t s = a; s < a + c; s += n_group)
      nn = emit_group(s, (a + c - s < n_group) ? (a + c - s) : n_group, cap, nn, first, count);
    return nn;
  }
  int64_t e = a + c;
  int64_t pa = a, pc = 0; /* the open pack of group cells (pc == 0: none) */
  while (a < e) {
    int d = digit_at(skeys[a], l + 1);
    int64_t b = a;
    while (b < e && digit_at(skeys[b], l + 1) == d) ++b;
    if (b - a <= n_group) {
      if (pc > 0 && pc + (b - a) <= n_group) {
        pc += b - a;
      } else {
        if (pc > 0) nn = emit_group(pa, pc, cap, nn, first, count);
        pa = a;
        pc = b - a;
      }
    } else {
      if (pc > 0) nn = emit_group(pa, pc, cap, nn, first, count);
      pc = 0;
      nn = groups_rec(skeys, a, b - a, l + 1, n_group, cap, nn, first, count);
    }
    if (nn < 0) return nn;
    a = b;
  }
  if (pc > 0) nn = emit_group(pa, pc, cap, nn, first, count);
  return nn;
}

int64_t orc_groups(int64_t n, const uint64_t* skeys, int n_group, int64_t cap,
                   int64_t* first, int64_t* count) {
  if (n <= 0 || n_group < 1) return ORC_E_ARG;
  return groups_rec(skeys, 0, n, 0, n_group, cap, 0, first, count);
}

/* ------------------------------------------------------------------------ */
/* Pair geometry.  dx = x_i - x_j, folded once to the nearest periodic image */
/* on periodic axes; r^2 = fma(dz,dz, fma(dy,dy, dx*dx)).                     */
/* ------------------------------------------------------------------------ */
static double fold(double d, double len, int periodic) {
  if (periodic) {
    double half = 0.5 * len;
    if (d > half)
      d -= len;
    else if (d < -half)
      d += len;
  }
  return d;
}

static double pair_r2(const double* x, const double* y, const double* z,
                      int64_t i, int64_t j, const orc_params* p, double* dx,
                      double* dy, double* dz) {
  double ax = fold(x[i] - x[j], p->box_len[0], p->periodic[0]);
  double ay = fold(y[i] - y[j], p->box_len[1], p->periodic[1]);
  double az = fold(z[i] - z[j], p->box_len[2], p->periodic[2]);
  if (dx) {
    *dx = ax;
    *dy = ay;
    *dz = az;
  }
  return fma(az, az, fma(ay, ay, ax * ax));
}

/* density criterion: j within the support S h_i (self included)            */
static int in_density(double r2, double hi, double S) {
  double s = S * hi;
  return r2 < s * s;
}
/* force criterion: j != i within the support of the larger of h_i, h_j     */
static int in_force(double r2, double hi, double hj, double S) {
  double s = S * (hi > hj ? hi : hj);
  return r2 < s * s;
}

/* ------------------------------------------------------------------------ */
/* Search tree for the oracle's own neighbour queries: the same chopped     */
/* octree, built over a key-sorted copy of the positions, with tight boxes   */
/* and the largest h of each node.  Queries descend recursively.             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n, nn;
  int64_t* perm; /* sorted slot -> input index */
  int64_t* first;
  int64_t* count;
  int64_t* child_first;
  int32_t* n_child;
  double* lo; /* 3 per node */
  double* hi;
  double* hmax;
  int32_t* level;
  uint64_t* prefix;
} orc_stree;

static void stree_free(orc_stree* t) {
  free(t->perm);
  free(t->first);
  free(t->count);
  free(t->child_first);
  free(t->n_child);
  free(t->lo);
  free(t->hi);
  free(t->hmax);
  free(t->level);
  free(t->prefix);
  memset(t, 0, sizeof(*t));
}

static int stree_build(orc_stree* t, int64_t n, const double* x,
                       const double* y, const double* z, const double* h,
                       const orc_params* p) {
  memset(t, 0, sizeof(*t));
  t->n = n;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t* skeys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  t->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t cap = 2 * n + 64;
  t->first = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
  t->count = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
  t->child_first = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
  t->n_child = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  t->level = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  t->prefix = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
  if (!keys || !skeys || !t->perm || !t->first || !t->count ||
      !t->child_first || !t->n_child || !t->level || !t->prefix) {
    free(keys);
    free(skeys);
    stree_free(t);
    return ORC_E_NOMEM;
  }
  orc_keys(n, x, y, z, p, keys);
  orc_sort(n, keys, t->perm);
  for (int64_t k = 0; k < n; ++k) skeys[k] = keys[t->perm[k]];
  int nl = p->n_leaf > 0 ? p->n_leaf : 16;
  int64_t nn = orc_tree(n, skeys, nl, cap, t->level, t->prefix, t->first,
                        t->count, t->child_first, t->n_child);
  free(keys);
  free(skeys);
  if (nn < 0) {
    stree_free(t);
    return (int)nn;
  }
  t->nn = nn;
  t->lo = (double*)malloc(sizeof(double) * 3 * (size_t)nn);
  t->hi = (double*)malloc(sizeof(double) * 3 * (size_t)nn);
  t->hmax = (double*)malloc(sizeof(double) * (size_t)nn);
  if (!t->lo || !t->hi || !t->hmax) {
    stree_free(t);
    return ORC_E_NOMEM;
  }
  /* tight boxes and largest h: plain loop over each node's members */
  for (int64_t k = 0; k < nn; ++k) {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hm = 0.0;
    for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; ++s) {
      int64_t j = t->perm[s];
      double c[3] = {x[j], y[j], z[j]};
      for (int d = 0; d < 3; ++d) {
        if (c[d] < lo[d]) lo[d] = c[d];
        if (c[d] > hi[d]) hi[d] = c[d];
      }
      if (h && h[j] > hm) hm = h[j];
    }
    for (int d = 0; d < 3; ++d) {
      t->lo[3 * k + d] = lo[d];
      t->hi[3 * k + d] = hi[d];
    }
    t->hmax[k] = hm;
  }
  return ORC_OK;
}

/* squared distance from a point to a node box, nearest periodic image per  */
/* axis; only used to prune, so it is made slightly conservative by caller. */
static double point_box_d2(const orc_stree* t, int64_t k, const double c[3],
                           const orc_params* p) {
  double d2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double lo = t->lo[3 * k + d], hi = t->hi[3 * k + d];
    double best = INFINITY;
    int nimg = p->periodic[d] ? 3 : 1;
    for (int s = 0; s < nimg; ++s) {
      double shift = (s == 0) ? 0.0 : (s == 1 ? p->box_len[d] : -p->box_len[d]);
      double v = c[d] + shift;
      double g = 0.0;
      if (v < lo)
        g = lo - v;
      else if (v > hi)
        g = v - hi;
      if (g < best) best = g;
    }
    d2 += best * best;
  }
  return d2;
}

typedef struct {
  int64_t* idx;
  int64_t n, cap;
} orc_list;

static int list_push(orc_list* l, int64_t v) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 128;
    int64_t* ni = (int64_t*)realloc(l->idx, sizeof(int64_t) * (size_t)nc);
    if (!ni) return ORC_E_NOMEM;
    l->idx = ni;
    l->cap = nc;
  }
  l->idx[l->n++] = v;
  return ORC_OK;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* mode 0: density set of particle i at smoothing length hi (self included)  */
/* mode 1: force set (j != i, r < 2 max(h_i, h_j)); uses the tree's hmax.    */
static void stree_query(const orc_stree* t, int64_t k, int64_t i, double hi,
                        int mode, const double* x, const double* y,
                        const double* z, const double* h, const orc_params* p,
                        orc_list* out, int* err) {
  if (*err) return;
  double c[3] = {x[i], y[i], z[i]};
  double reach = orc_kernel_support(p->kernel) * ((mode == 1 && t->hmax[k] > hi) ? t->hmax[k] : hi);
  double d2 = point_box_d2(t, k, c, p);
  if (!(d2 <= reach * reach * (1.0 + 1e-9))) return;
  if (t->child_first[k] < 0) {
    for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; ++s) {
      int64_t j = t->perm[s];
      double r2 = pair_r2(x, y, z, i, j, p, NULL, NULL, NULL);
      const double S = orc_kernel_support(p->kernel);
      int take = (mode == 0) ? in_density(r2, hi, S)
                             : (j != i && in_force(r2, hi, h[j], S));
      if (take && list_push(out, j) != ORC_OK) {
        *err = ORC_E_NOMEM;
        return;
      }
    }
    return;
  }
  for (int32_t c2 = 0; c2 < t->n_child[k]; ++c2)
    stree_query(t, t->child_first[k] + c2, i, hi, mode, x, y, z, h, p, out,
                err);
}

static int neighbours_of(const orc_stree* t, int64_t i, double hi, int mode,
                         const double* x, const double* y, const double* z,
                         const double* h, const orc_params* p, orc_list* out) {
  int err = 0;
  out->n = 0;
  stree_query(t, 0, i, hi, mode, x, y, z, h, p, out, &err);
  if (err) return err;
  qsort(out->idx, (size_t)out->n, sizeof(int64_t), cmp_i64);
  return ORC_OK;
}

/* Neighbour sets as CSR with ascending indices.  offsets has n+1 entries.   */
/* brute = 1: test every pair (O(N^2)); brute = 0: via the search tree.       */
/* Returns the total number of entries, or a negative status.  If the total */
/* exceeds cap, offsets are still filled and ORC_E_OVERFLOW is returned.    */
/* As orc_neighbours, for the particles sel[0..nsel) only (all if sel is   */
/* NULL); offsets has nsel+1 entries and row k belongs to particle sel[k].   */
int64_t orc_neighbours_sel(int64_t n, const double* x, const double* y,
                           const double* z, const double* h, const orc_params* p,
                           int mode, int brute, const int64_t* sel, int64_t nsel,
                           int64_t* offsets, int64_t* idx, int64_t cap) {
  if (n <= 0) return ORC_E_ARG;
  if (!sel) nsel = n;
  const double S = orc_kernel_support(p->kernel);
  int64_t* cnt = (int64_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int64_t));
  if (!cnt) return ORC_E_NOMEM;
  orc_stree t;
  int st = ORC_OK;
  if (!brute) {
    st = stree_build(&t, n, x, y, z, h, p);
    if (st != ORC_OK) {
      free(cnt);
      return st;
    }
  }
  /* pass 1: counts */
#pragma omp parallel
  {
    orc_list l = {0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < nsel; ++k) {
      const int64_t i = sel ? sel[k] : k;
      if (brute) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
          double r2 = pair_r2(x, y, z, i, j, p, NULL, NULL, NULL);
          if (mode == 0 ? in_density(r2, h[i], S) : (j != i && in_force(r2, h[i], h[j], S))) ++c;
        }
        cnt[k] = c;
      } else {
        if (neighbours_of(&t, i, h[i], mode, x, y, z, h, p, &l) != ORC_OK) {
#pragma omp atomic write
          st = ORC_E_NOMEM;
        }
        cnt[k] = l.n;
      }
    }
    free(l.idx);
  }
  offsets[0] = 0;
  for (int64_t k = 0; k < nsel; ++k) offsets[k + 1] = offsets[k] + cnt[k];
  int64_t total = offsets[nsel];
  if (st == ORC_OK && total <= cap && idx) {
#pragma omp parallel
    {
      orc_list l = {0};
#pragma omp for schedule(dynamic, 64)
      for (int64_t k = 0; k < nsel; ++k) {
        const int64_t i = sel ? sel[k] : k;
        int64_t o = offsets[k];
        if (brute) {
          for (int64_t j = 0; j < n; ++j) {
            double r2 = pair_r2(x, y, z, i, j, p, NULL, NULL, NULL);
            if (mode == 0 ? in_density(r2, h[i], S) : (j != i && in_force(r2, h[i], h[j], S))) idx[o++] = j;
          }
        } else {
          if (neighbours_of(&t, i, h[i], mode, x, y, z, h, p, &l) != ORC_OK) {
#pragma omp atomic write
            st = ORC_E_NOMEM;
          }
          for (int64_t q = 0; q < l.n; ++q) idx[o + q] = l.idx[q];
        }
      }
      free(l.idx);
    }
  }
  if (!brute) stree_free(&t);
  free(cnt);
  if (st != ORC_OK) return st;
  if (total > cap) return ORC_E_OVERFLOW;
  return total;
}

int64_t orc_neighbours(int64_t n, const double* x, const double* y,
                       const double* z, const double* h, const orc_params* p,
                       int mode, int brute, int64_t* offsets, int64_t* idx,
                       int64_t cap) {
  return orc_neighbours_sel(n, x, y, z, h, p, mode, brute, NULL, n, offsets, idx, cap);
}

/* ------------------------------------------------------------------------ */
/* Density with variable smoothing length (Sect. 2.2, Sect. 3.2.1).          */
/* For particle i the density at smoothing length h is the gather sum        */
/*   S0(h) = sum_{j: r_ij < 2h} m_j W(r_ij, h)       (self included)          */
/* and h must satisfy the h-rho relation with rho = S0(h), i.e. the root of  */
/*   f(h) = S0(h) - m_i (hfact/h)^3.                                          */
/* With S1(h) = sum m_j dW/dh, f'(h) = S1 + 3 m_i (hfact/h)^3 / h, and        */
/*   Omega = 1 - (dh/drho) S1 = 1 + h S1 / (3 rho),  dh/drho = -h/(3 rho).     */
/* Newton-Raphson from the input h; a step that is not downhill or leaves   */
/* [0.8h, 1.2h], or too many steps, hands over to bracketing + bisection.   */
/* The result is the root; rho and Omega are then evaluated at it.          */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_stree* t;
  const double *x, *y, *z, *m;
  const orc_params* p;
  orc_list* l;
} dens_ctx;

static int dens_sums(const dens_ctx* c, int64_t i, double h, double* S0,
                     double* S1, int64_t* nn) {
  int st = neighbours_of(c->t, i, h, 0, c->x, c->y, c->z, NULL, c->p, c->l);
  if (st != ORC_OK) return st;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t k = 0; k < c->l->n; ++k) {
    int64_t j = c->l->idx[k];
    double r = sqrt(pair_r2(c->x, c->y, c->z, i, j, c->p, NULL, NULL, NULL));
    s0 += c->m[j] * kern_w(c->p->kernel, r, h);
    s1 += c->m[j] * kern_dwdh(c->p->kernel, r, h);
  }
  *S0 = s0;
  *S1 = s1;
  if (nn) *nn = c->l->n;
  return ORC_OK;
}

static double rho_of_h(double m, double hfact, double h) {
  double t = hfact / h;
  return m * (t * t * t);
}

static int dens_f(const dens_ctx* c, int64_t i, double h, double* f) {
  double S0, S1;
  int st = dens_sums(c, i, h, &S0, &S1, NULL);
  if (st != ORC_OK) return st;
  *f = S0 - rho_of_h(c->m[i], c->p->hfact, h);
  return ORC_OK;
}

static int dens_bisect(const dens_ctx* c, int64_t i, double h0, double tol,
                       double* hout, int* iters) {
  double f0;
  int st = dens_f(c, i, h0, &f0);
  if (st != ORC_OK) return st;
  double lo = h0, hi = h0, flo = f0, fhi = f0;
  int k = 0;
  if (f0 == 0.0) {
    *hout = h0;
    return ORC_OK;
  }
  if (f0 < 0.0) { /* h too small: grow the upper end */
    while (fhi < 0.0) {
      lo = hi;
      flo = fhi;
      hi = hi * 1.2;
      if ((st = dens_f(c, i, hi, &fhi)) != ORC_OK) return st;
      if (++k > 200) return ORC_E_NOCONV;
    }
  } else {
    while (flo > 0.0) {
      hi = lo;
      fhi = flo;
      lo = lo / 1.2;
      if ((st = dens_f(c, i, lo, &flo)) != ORC_OK) return st;
      if (++k > 200) return ORC_E_NOCONV;
    }
  }
  (void)flo;
  (void)fhi;
  while (hi - lo > tol * lo) {
    double mid = 0.5 * (lo + hi), fm;
    if ((st = dens_f(c, i, mid, &fm)) != ORC_OK) return st;
    if (fm == 0.0) {
      lo = hi = mid;
      break;
    }
    if (fm < 0.0)
      lo = mid;
    else
      hi = mid;
    if (++k > 400) return ORC_E_NOCONV;
  }
  *hout = 0.5 * (lo + hi);
  *iters += k;
  return ORC_OK;
}

/* Density of the particles sel[0..nsel) (all particles if sel is NULL, then */
/* nsel = n); outputs are packed: entry k belongs to particle sel[k].        */
int orc_density_sel(int64_t n, const double* x, const double* y, const double* z,
                    const double* m, const double* h_in, const orc_params* p,
                    const int64_t* sel, int64_t nsel, double* h_out, double* rho,
                    double* omega, int64_t* nneigh, int32_t* iters) {
  if (n <= 0) return ORC_E_ARG;
  if (!sel) nsel = n;
  orc_stree t;
  int st = stree_build(&t, n, x, y, z, NULL, p);
  if (st != ORC_OK) return st;
  int status = ORC_OK;
  int fixed = p->h_tol < 0.0;
  double tol = fixed ? 0.0 : p->h_tol;
  int max_it = p->max_h_iter > 0 ? p->max_h_iter : 30;
#pragma omp parallel
  {
    orc_list l = {0};
    dens_ctx c = {&t, x, y, z, m, p, &l};
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < nsel; ++k) {
      const int64_t i = sel ? sel[k] : k;
      double h = h_in[i];
      int it = 0, done = 0, need_bisect = 0, s = ORC_OK;
      if (!(h > 0.0) || !(m[i] > 0.0)) s = ORC_E_ARG;
      /* fixed passes (Sect. 3.2.1: the density is computed three times):   */
      /* two clamped Newton updates from the sums at h0 and h1, then the    */
      /* third sum at h2 below gives rho and Omega                          */
      int passes = fixed ? 2 : max_it;
      for (it = 0; it < passes && s == ORC_OK; ++it) {
        double S0, S1;
        s = dens_sums(&c, i, h, &S0, &S1, NULL);
        if (s != ORC_OK) break;
        double rh = rho_of_h(m[i], p->hfact, h);
        double f = S0 - rh;
        double fp = S1 + 3.0 * rh / h;
        double hn = h - f / fp;
        if (!(fp > 0.0) || !(hn >= 0.8 * h) || !(hn <= 1.2 * h)) {
          if (fixed) { /* fixed passes: clamp the step instead of bracketing */
            if (!(fp > 0.0))
              hn = h;
            else if (hn > 1.2 * h)
              hn = 1.2 * h;
            else
              hn = 0.8 * h;
          } else {
            need_bisect = 1;
            break;
          }
        }
        if (!fixed && fabs(hn - h) <= tol * h) {
          h = hn;
          done = 1;
          ++it;
          break;
        }
        h = hn;
      }
      if (!fixed && !done && s == ORC_OK) need_bisect = 1;
      /* the fallback brackets the root and bisects down to a relative     */
      /* width of 1e-15, so its result is as sharp as a converged NR root  */
      if (need_bisect && s == ORC_OK) s = dens_bisect(&c, i, h, 1e-15, &h, &it);
      double S0 = 0.0, S1 = 0.0;
      int64_t nnb = 0;
      if (s == ORC_OK) s = dens_sums(&c, i, h, &S0, &S1, &nnb);
      if (s != ORC_OK) {
#pragma omp atomic write
        status = s;
      }
      h_out[k] = h;
      rho[k] = S0;
      omega[k] = 1.0 + h * S1 / (3.0 * S0);
      if (nneigh) nneigh[k] = nnb;
      if (iters) iters[k] = it;
    }
    free(l.idx);
  }
  stree_free(&t);
  return status;
}

int orc_density(int64_t n, const double* x, const double* y, const double* z,
                const double* m, const double* h_in, const orc_params* p,
                double* h_out, double* rho, double* omega, int64_t* nneigh,
                int32_t* iters) {
  return orc_density_sel(n, x, y, z, m, h_in, p, NULL, n, h_out, rho, omega, nneigh, iters);
}

/* Equation of state.  The paper names only the adiabatic index (Sect. 4),  */
/* so the ideal-gas law is taken: P = (gamma-1) rho u, c = sqrt(gamma P/rho) */
/* written as sqrt(gamma (gamma-1) u).                                       */
void orc_eos(int64_t n, const double* rho, const double* u, const orc_params* p,
             double* P, double* cs) {
  for (int64_t i = 0; i < n; ++i) {
    P[i] = p->gamma_minus_1 * rho[i] * u[i];
    cs[i] = sqrt(p->gamma * p->gamma_minus_1 * u[i]);
  }
}

/* ------------------------------------------------------------------------ */
/* Hydrodynamic force (Sect. 2.4 - 2.6).  For every j != i with              */
/* r_ij < 2 max(h_i, h_j), with rhat = (r_i - r_j)/r, w = (v_i - v_j).rhat,  */
/* F_i = F(r, h_i), F_j = F(r, h_j):                                          */
/*   approaching pairs (w < 0):  vs_i = alpha c_i + beta |w|,                 */
/*                               vs_j = alpha c_j + beta |w|,                 */
/*                               q_i = -1/2 rho_i vs_i w, q_j likewise;       */
/*   otherwise q_i = q_j = 0 and no viscous heating.                          */
/*   a_i    = - sum m_j [ (P_i+q_i)/(rho_i^2 Om_i) F_i                         */
/*                       + (P_j+q_j)/(rho_j^2 Om_j) F_j ] rhat                 */
/*   du_i/dt=  P_i/(rho_i^2 Om_i) sum m_j w F_i                               */
/*           - 1/(Om_i rho_i) sum_{w<0} m_j vs_i (1/2) w^2 F_i                */
/*           + sum m_j alpha_u v^u_ij (u_i - u_j) (1/2)[F_i/(Om_i rho_i)      */
/*                                                  + F_j/(Om_j rho_j)]       */
/*   v^u_ij = sqrt(|P_i - P_j| / rhobar),  rhobar = (rho_i + rho_j)/2          */
/*   vsig_dt_i = max(alpha c_i, max_j (alpha c_i + beta |w|))                 */
/* The viscous heating carries 1/rho_i and acts only where q_i acts: that is */
/* the reading under which viscosity conserves total energy exactly.  The    */
/* conductivity sum carries the symmetric factor (1/2)[...] of the garbled   */
/* printed term.  anorm_i / unorm_i are sums of pair-term magnitudes, used   */
/* to normalise errors of a_i and du_i/dt.                                    */
/* ------------------------------------------------------------------------ */
/* Force on the particles sel[0..nsel) (all if sel is NULL); outputs packed. */
int orc_force_sel(int64_t n, const double* x, const double* y, const double* z,
                  const double* vx, const double* vy, const double* vz,
                  const double* m, const double* u, const double* h,
                  const double* rho, const double* omega, const double* P,
                  const double* cs, const orc_params* p, const int64_t* sel,
                  int64_t nsel, double* ax, double* ay, double* az, double* dudt,
                  double* vsig_dt, double* anorm, double* unorm, int64_t* nneigh) {
  if (n <= 0) return ORC_E_ARG;
  if (!sel) nsel = n;
  orc_stree t;
  int st = stree_build(&t, n, x, y, z, h, p);
  if (st != ORC_OK) return st;
  int status = ORC_OK;
  const double al = p->alpha_av, be = p->beta_av, au = p->alpha_u;
#pragma omp parallel
  {
    orc_list l = {0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t k = 0; k < nsel; ++k) {
      const int64_t i = sel ? sel[k] : k;
      int s = neighbours_of(&t, i, h[i], 1, x, y, z, h, p, &l);
      if (s != ORC_OK) {
#pragma omp atomic write
        status = s;
        continue;
      }
      double gi = P[i] / (rho[i] * rho[i] * omega[i]);
      double ki = 1.0 / (omega[i] * rho[i]);
      double sx = 0.0, sy = 0.0, sz = 0.0, an = 0.0;
      double du_p = 0.0, du_v = 0.0, du_c = 0.0, un = 0.0;
      double vmax = al * cs[i];
      if (al == 0.0) vmax = cs[i];
      for (int64_t k = 0; k < l.n; ++k) {
        int64_t j = l.idx[k];
        double dx, dy, dz;
        double r2 = pair_r2(x, y, z, i, j, p, &dx, &dy, &dz);
        double r = sqrt(r2);
        double ex = dx / r, ey = dy / r, ez = dz / r;
        double w = (vx[i] - vx[j]) * ex + (vy[i] - vy[j]) * ey +
                   (vz[i] - vz[j]) * ez;
        double Fi = kern_F(p->kernel, r, h[i]);
        double Fj = kern_F(p->kernel, r, h[j]);
        double qi = 0.0, qj = 0.0, vsi = 0.0;
        if (w < 0.0) {
          vsi = al * cs[i] + be * fabs(w);
          double vsj = al * cs[j] + be * fabs(w);
          qi = -0.5 * rho[i] * vsi * w;
          qj = -0.5 * rho[j] * vsj * w;
        }
        double vdt = al * cs[i] + be * fabs(w);
        if (vdt > vmax) vmax = vdt;
        double ti = (P[i] + qi) / (rho[i] * rho[i] * omega[i]) * Fi;
        double tj = (P[j] + qj) / (rho[j] * rho[j] * omega[j]) * Fj;
        double pa = m[j] * (ti + tj);
        sx -= pa * ex;
        sy -= pa * ey;
        sz -= pa * ez;
        an += fabs(pa);
        double e1 = gi * m[j] * w * Fi;
        double e2 = -ki * m[j] * vsi * 0.5 * w * w * Fi;
        double rbar = 0.5 * (rho[i] + rho[j]);
        double vu = sqrt(fabs(P[i] - P[j]) / rbar);
        double kj = 1.0 / (omega[j] * rho[j]);
        double e3 = m[j] * au * vu * (u[i] - u[j]) * 0.5 * (Fi * ki + Fj * kj);
        du_p += e1;
        du_v += e2;
        du_c += e3;
        un += fabs(e1) + fabs(e2) + fabs(e3);
      }
      ax[k] = sx;
      ay[k] = sy;
      az[k] = sz;
      dudt[k] = du_p + du_v + du_c;
      vsig_dt[k] = vmax;
      if (anorm) anorm[k] = an;
      if (unorm) unorm[k] = un;
      if (nneigh) nneigh[k] = l.n;
    }
    free(l.idx);
  }
  stree_free(&t);
  return status;
}

int orc_force(int64_t n, const double* x, const double* y, const double* z,
              const double* vx, const double* vy, const double* vz,
              const double* m, const double* u, const double* h,
              const double* rho, const double* omega, const double* P,
              const double* cs, const orc_params* p, double* ax, double* ay,
              double* az, double* dudt, double* vsig_dt, double* anorm,
              double* unorm, int64_t* nneigh) {
  return orc_force_sel(n, x, y, z, vx, vy, vz, m, u, h, rho, omega, P, cs, p, NULL, n, ax, ay,
                       az, dudt, vsig_dt, anorm, unorm, nneigh);
}

/* Courant step (Sect. 2.4, eq:timestep): dt = C_cour min_i h_i / vsig_i.   */
double orc_courant_dt(int64_t n, const double* h, const double* vsig_dt,
                      const orc_params* p) {
  double best = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    double d = p->c_cour * h[i] / vsig_dt[i];
    if (d < best) best = d;
  }
  return best;
}

/* Wrap a coordinate into [lo, lo+L) on a periodic axis (one fold).          */
static double wrap(double v, double lo, double len, int periodic) {
  if (!periodic) return v;
  if (v >= lo + len)
    v -= len;
  else if (v < lo)
    v += len;
  return v;
}

/* Leapfrog predictor (Sect. 2.4, eq:predict_pos and eq:predict_vel); the   */
/* internal energy is predicted the same way (the paper states only r, v):  */
/*   r1 = r0 + v0 dt + (1/2) a0 dt^2,  v_p = v0 + a0 dt,  u_p = u0 + du0 dt. */
/* r1 is evaluated as r0 + (v0*dt + (0.5*dt*dt)*a0).                          */
void orc_predict(int64_t n, double* x, double* y, double* z, double* vx,
                 double* vy, double* vz, double* u, const double* ax,
                 const double* ay, const double* az, const double* dudt,
                 double dt, const orc_params* p) {
  double hdt2 = 0.5 * dt * dt;
  for (int64_t i = 0; i < n; ++i) {
    x[i] = wrap(x[i] + (vx[i] * dt + hdt2 * ax[i]), p->box_lo[0], p->box_len[0], p->periodic[0]);
    y[i] = wrap(y[i] + (vy[i] * dt + hdt2 * ay[i]), p->box_lo[1], p->box_len[1], p->periodic[1]);
    z[i] = wrap(z[i] + (vz[i] * dt + hdt2 * az[i]), p->box_lo[2], p->box_len[2], p->periodic[2]);
    vx[i] = vx[i] + ax[i] * dt;
    vy[i] = vy[i] + ay[i] * dt;
    vz[i] = vz[i] + az[i] * dt;
    u[i] = u[i] + dudt[i] * dt;
  }
}

/* Leapfrog corrector (Sect. 2.4, eq:correct_vel): v1 = v_p + (1/2)(a1-a0)dt */
/* and u1 = u_p + (1/2)(du1-du0)dt; a0, du0 are then replaced by a1, du1.    */
void orc_correct(int64_t n, double* vx, double* vy, double* vz, double* u,
                 double* ax0, double* ay0, double* az0, double* dudt0,
                 const double* ax1, const double* ay1, const double* az1,
                 const double* dudt1, double dt) {
  double hdt = 0.5 * dt;
  for (int64_t i = 0; i < n; ++i) {
    vx[i] = vx[i] + (ax1[i] - ax0[i]) * hdt;
    vy[i] = vy[i] + (ay1[i] - ay0[i]) * hdt;
    vz[i] = vz[i] + (az1[i] - az0[i]) * hdt;
    u[i] = u[i] + (dudt1[i] - dudt0[i]) * hdt;
    ax0[i] = ax1[i];
    ay0[i] = ay1[i];
    az0[i] = az1[i];
    dudt0[i] = dudt1[i];
  }
}

/* Global sums: out = {E, E_kin, E_th, p_x, p_y, p_z, sum m a_x, sum m a_y,  */
/* sum m a_z, dE/dt = sum m (v.a + du/dt), sum m |a|, sum m (|v.a|+|du/dt|)} */
void orc_reduce(int64_t n, const double* vx, const double* vy, const double* vz,
                const double* m, const double* u, const double* ax,
                const double* ay, const double* az, const double* dudt,
                double out[12]) {
  for (int k = 0; k < 12; ++k) out[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    double ek = 0.5 * m[i] * v2, et = m[i] * u[i];
    double va = vx[i] * ax[i] + vy[i] * ay[i] + vz[i] * az[i];
    out[1] += ek;
    out[2] += et;
    out[3] += m[i] * vx[i];
    out[4] += m[i] * vy[i];
    out[5] += m[i] * vz[i];
    out[6] += m[i] * ax[i];
    out[7] += m[i] * ay[i];
    out[8] += m[i] * az[i];
    out[9] += m[i] * (va + dudt[i]);
    out[10] += m[i] * sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
    out[11] += m[i] * (fabs(va) + fabs(dudt[i]));
  }
  out[0] = out[1] + out[2];
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel loops (k <= 0: leave unchanged). */
void orc_set_num_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}
