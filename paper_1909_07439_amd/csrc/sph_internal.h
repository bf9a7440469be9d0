// sph_internal.h -- device-side building blocks and the context layout of
// the gfx950 SPH library.  Not part of the public ABI (include/sph.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

namespace sph {

constexpr int kKeyLevels = 21;  // 21 bits per axis -> levels 1..21
constexpr int kLevels = 22;     // tree levels 0..21
constexpr int kWave = 64;

// ---- device error word bits ------------------------------------------------
enum : uint32_t {
  kErrNoConv = 1u,
  kErrNodes = 2u,      // tree node capacity
  kErrFrontier = 4u,   // walk frontier capacity
  kErrPairs = 8u,      // per-particle pair list capacity
  kErrDomain = 16u,    // 2h >= L/2 on a periodic axis
  kErrNonFinite = 32u,
  kErrLeaves = 64u,
  kErrFrontierForce = 128u,  // walk frontier capacity in the force pass
  kErrIds = 256u,            // a particle id outside [0, n) (adjoint cotangent index)
  kErrSort = 512u,           // a radix-sort look-back wait ran out (should not happen)
};

// Fixed-point frame of the positions in the mixed-precision force records.
// Axis a maps x to the code floor((x - o[a]) inv[a]): on a periodic axis inv
// = 2^32 / L and the code is kept modulo 2^32, so the wrapped 32-bit
// difference of two codes is the nearest periodic image; on an open axis the
// frame spans the root node's box with 2^31 codes (clamped), so a difference
// never wraps.  Code difference times step[a] is the separation to within one
// step (L 2^-32 on a periodic axis), with no FP64 arithmetic and no fold.
struct QFrame {
  double o[3];
  double inv[3];
  float step[3];
  int32_t pad;
};

__device__ __forceinline__ int32_t qcode(double x, const QFrame& f, int a, int periodic) {
  const double t = floor((x - f.o[a]) * f.inv[a]);
  if (periodic) return (int32_t)(uint32_t)(uint64_t)(int64_t)t;  // modulo 2^32
  return (int32_t)fmin(fmax(t, 0.0), 2147483647.0);
}

// Separation a - b of two codes of one axis (wrapped 32-bit difference).
__device__ __forceinline__ float qsep(int32_t a, int32_t b, float step) {
  return (float)(int32_t)((uint32_t)a - (uint32_t)b) * step;
}

// Device-resident scalars of one context.
// Every wavefront of the walk kernels adds its counts once; the counters
// that all of them update sit 256 bytes apart (separate cache lines and L2
// channels), so those atomics do not queue behind each other.
struct DevState {
  int32_t n_nodes;
  int32_t n_groups;
  int32_t leaf_state;     // 0: no stored leaf lists, 1: valid for the force, 2: some h outgrew them
  int32_t lists_missing;  // some group needs the walking kernels (h refresh needed)
  int32_t n_flag_rows;    // groups whose neighbour-list rows overflowed (walking kernels)
  int32_t n_flag_grew;    // groups in which some h outgrew the rows (walking kernels)
  int32_t n_flagged;      // entries of the flagged-group list (both kinds)
  int32_t pad1;
  double dt_cur;          // step used by the running sph_step
  alignas(256) uint32_t err;
  alignas(256) int32_t max_iter;                  // most density sums any group needed
  alignas(256) unsigned long long dt_min_enc;     // ordered encoding of min_i c_cour h_i / vsig_i
  alignas(256) unsigned long long n_pairs_density;  // true neighbours (r < 2h) at the final pass
  alignas(256) unsigned long long n_pairs_force;    // force pairs
  alignas(256) unsigned long long n_sums_density;   // sum over groups of (density passes * pairs)
  alignas(256) unsigned long long n_cand_density;   // candidate tests in the density walks
  alignas(256) unsigned long long n_cand_force;     // candidate tests in the force walks
  alignas(256) int32_t n_rewalk;
  alignas(256) unsigned long long tot_sums_density;  // n_sums_density over every launch so far
  alignas(256) unsigned long long tot_pairs_force;   // n_pairs_force over every launch so far
  alignas(256) unsigned long long tot_cand_lists;    // candidate tests of the list kernel so far
  alignas(256) QFrame qf;  // frame of the mixed force records (set with each tree's node boxes)
};

// Walk view of a tree node: centre, conservative half-widths, largest h.
struct alignas(16) WalkNode {
  double c[3];
  float w[3];    // half-widths rounded up
  float hmax;    // largest smoothing length, rounded up
  int32_t first;
  int32_t count;
  int32_t child;   // first child (children are contiguous); -1 for leaves
  int32_t nchild;  // 0 for leaves
};
static_assert(sizeof(WalkNode) == 56 || sizeof(WalkNode) == 64, "WalkNode layout");

struct alignas(16) GroupInfo {
  double c[3];
  double w[3];
  double hmax;
  int32_t first;
  int32_t count;
};

// Parameters as the kernels see them.
struct KParams {
  double lo[3];
  double len[3];
  double half[3];  // 0.5 * len (exact)
  double inv_len[3];
  int32_t periodic[3];
  double key_scale;  // 2^21 / max(len)
  double gamma, gm1, hfact, alpha, beta, alpha_u, c_cour;
  double h_tol;
  int32_t max_iter;
  int32_t fixed_passes;  // 1: three fixed passes (h_tol < 0)
  double h_margin;
  int32_t n;
  int32_t n_leaf;
  int32_t n_group;
  int32_t precision;
  int32_t kernel;   // 0 M4 cubic, 1 M6 quintic, 2 Wendland C6
  double support;   // kernel support in units of h (2, 3, 2)
  double knorm;     // 3D normalisation C of W = C f(r/h) / h^3
  int32_t nl_cap;   // entries per neighbour-list row (128 or 256)
};

// ---- small device helpers ---------------------------------------------------
__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return (l == 0) ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Order-preserving map of doubles to unsigned 64-bit integers, so that
// atomicMin / atomicMax on the integers implement min / max on the doubles.
__host__ __device__ __forceinline__ unsigned long long enc_f64(double x) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double dec_f64(unsigned long long e) {
  unsigned long long b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
  return __builtin_bit_cast(double, b);
}

}  // namespace sph

// Host-side launchers implemented in sph_kernels.hip.
struct sph_ctx;
namespace sph {
hipError_t launch_predict_keys(sph_ctx* c, const sph_particles* p, bool predict, double dt_host);
hipError_t launch_sort(sph_ctx* c);
hipError_t launch_permute(sph_ctx* c, const sph_particles* p, bool outputs_too);
hipError_t launch_tree(sph_ctx* c);
hipError_t launch_node_h(sph_ctx* c, const sph_particles* p, bool always);
bool lists_mode(const sph_ctx* c);
hipError_t launch_lists(sph_ctx* c, const sph_particles* p);
hipError_t launch_density_lists(sph_ctx* c, const sph_particles* p);
hipError_t launch_density(sph_ctx* c, const sph_particles* p, bool flagged_only);
hipError_t launch_force_lists(sph_ctx* c, const sph_particles* p, bool step_mode);
hipError_t launch_row_sets(sph_ctx* c, const sph_particles* p, int mode, int32_t* counts,
                           int32_t* idx, const int64_t* offsets);
hipError_t launch_force(sph_ctx* c, const sph_particles* p, bool step_mode, bool flagged_only);
hipError_t launch_correct(sph_ctx* c, const sph_particles* p);
hipError_t launch_reduce(sph_ctx* c, const sph_particles* p, double* dev_out);
hipError_t reduce_noalloc(const sph_particles* p, hipStream_t stream, double* out);
hipError_t launch_neighbours(sph_ctx* c, const sph_particles* p, int mode, int32_t* counts,
                             const int64_t* offsets, int32_t* idx);
// implemented in sph_adjoint.hip
// part 0: seed, 1: force adjoint, 2: density adjoint and final combination
hipError_t launch_adjoint(sph_ctx* c, const sph_particles* p, const sph_cotangents* g, double dt,
                          bool step_mode, int part);
}  // namespace sph
