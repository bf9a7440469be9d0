// sph_ctx.h -- the library context: run parameters, device scratch, events.
#pragma once

#include <string>

#include "sph_internal.h"

namespace sph {
constexpr int kMaxFields = 20;
constexpr int kSortTile = 2048;  // keys per radix-sort block (256 threads x 8)
constexpr int kTreeTile = 256;   // particles per tree block
constexpr int kScanTile = 2048;  // elements per scan block
constexpr int kNLCapMax = 256;  // largest neighbour-list row (entries)
constexpr int kChunk = 256;     // particles per chunk box (inner-node boxes of small trees)
constexpr int kSmallTree = 1 << 21;  // particles up to which inner nodes take one launch
constexpr int kSpill = 4096;    // walk frontier entries per level beyond LDS, per wavefront

// Per-particle data the force loop reads for a neighbour j (written by the
// density pass once h, rho, Omega are final).
struct alignas(16) FRec64 {
  double x, y, z, m;
  double vx, vy, vz, u;
  double hinv, hinv4pi, g, k;  // g = P/(rho^2 Omega), k = 1/(rho Omega)
  double c, P, rho, h;
};
struct alignas(16) FRec32 {
  int32_t qx, qy, qz;  // position codes in the frame DevState::qf
  float m;
  float h, vx, vy, vz;
  float u, hinv, hinv4pi, g;
  float k, c, P, rho;
};
static_assert(sizeof(FRec64) == 128, "FRec64");
static_assert(sizeof(FRec32) == 64, "FRec32");

// Raw pointers of an sph_particles, as kernels take them.
struct Parts {
  int64_t* id;
  double *x, *y, *z, *vx, *vy, *vz, *m, *u, *h, *ax, *ay, *az, *dudt, *rho, *omega, *P, *cs,
      *vsig;
};
}  // namespace sph

struct sph_ctx {
  sph_params prm;
  sph::KParams kp;
  int64_t n_max = 0;
  int32_t n = 0;  // particles of the current tree
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  int walk_blocks = 0;

  // sort
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* radix_cnt = nullptr;  // look-back status (8 passes x 256 x blocks), histograms, tickets
  int64_t n_max_sort_blocks = 0;
  uint32_t* scan_part = nullptr;  // block partials of the scans
  uint32_t* scan_total = nullptr; // scratch totals (several slots)
  // permute
  double* gtmp = nullptr;  // kMaxFields * n_max
  double4* xyzm = nullptr; // FP64: packed x, y, z, m in key order (written by the permute)
  int4* qxyzm = nullptr;    // mixed: position codes (DevState::qf) and m as FP32, key order
  int64_t* gtmp_id = nullptr;
  // tree
  uint8_t* dlev = nullptr;
  uint8_t* lleaf = nullptr;
  uint8_t* gsize = nullptr;  // particles of the group starting at each particle (0 elsewhere)
  uint8_t* gstart = nullptr;
  uint32_t* tree_cnt = nullptr;  // kLevels * blocks (level-major), scanned in place
  uint32_t* grp_cnt = nullptr;   // blocks
  int64_t node_cap = 0;
  int32_t* node_level = nullptr;
  int32_t* node_first = nullptr;
  int32_t* node_count = nullptr;
  int32_t* node_parent = nullptr;
  int32_t* node_child = nullptr;
  int32_t* node_nchild = nullptr;
  double* chunk_box = nullptr;  // 8 per chunk of kChunk sorted particles: lo xyz, hi xyz, h_max
  sph::WalkNode* wnode = nullptr;
  int32_t* grp_first = nullptr;
  int32_t* grp_count = nullptr;
  sph::GroupInfo* ginfo = nullptr;
  int2* leaf_pool = nullptr;   // leaf lists stored by the density walk (per-wave regions)
  int64_t pool_cap = 0;
  int32_t* gl_off = nullptr;   // per group: first pool entry
  int32_t* gl_cnt = nullptr;   // per group: entries, -1 if not stored
  int32_t* nl_idx = nullptr;   // neighbour-list rows, kp.nl_cap entries per particle
  int32_t* nl_len = nullptr;   // entries found per particle (may exceed kp.nl_cap)
  int32_t* gflag = nullptr;    // per group: 0 lists complete, 1 row overflow, 2 h outgrew rows
  int32_t* flag_list = nullptr;  // indices of the flagged groups (DevState::n_flagged of them)
  int32_t* walk_spill = nullptr; // 2 * kSpill frontier entries per walk wavefront
  int32_t* grp_of = nullptr;     // group of each particle (neighbour-list kernel)
  int4* qrec = nullptr;          // mixed: position codes (DevState::qf) and h as FP32, key order
  // density / force
  void* frec = nullptr;        // FRec64 or FRec32 per particle
  double* a1 = nullptr;        // 4 * n_max: new ax, ay, az, dudt inside sph_step
  // adjoint workspace (allocated by the first adjoint call)
  void* adj_abar = nullptr;    // cotangents of a, du/dt in key order (double4 or float4)
  double* adj_raw = nullptr;   // 7 * n_max: cotangents of x, v and u from the force adjoint
  double2* adj_ab = nullptr;   // alpha, beta of the density adjoint
  int32_t* nb_cnt = nullptr;   // neighbour-export counts
  int64_t* nb_off = nullptr;   // neighbour-export offsets (device)
  double* red_part = nullptr;  // reduction partials
  double* red_out = nullptr;   // 12 results
  sph::DevState* ds = nullptr;
  sph::DevState* hs = nullptr;  // pinned host mirror
  struct sph_timing* tm = nullptr;  // phase event rings (host code)
  bool timing = true;      // record phase events for the current call
  int timing_every = 1;    // sph_step records them on one call in this many (0: never)
  int64_t step_calls = 0;  // sph_step calls since sph_set_timing
  int64_t density_launches = 0;  // launches of the density kernel so far
  int32_t densities_on_tree = 0; // density passes since the last tree build
  int64_t force_launches = 0;    // launches of the force kernel so far
  int64_t lists_launches = 0;    // launches of the neighbour-list kernel so far
  std::string err;
};
