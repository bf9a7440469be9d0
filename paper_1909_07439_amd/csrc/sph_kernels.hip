// sph_kernels.hip -- gfx950 kernels of the SPH hydrodynamics step.
//
//   keys + sort + permute ....... Sect. 3.1 (space-filling curve, sort)
//   tree + groups ............... Sect. 3.1 (chopping the curve)
//   group tree walk ............. Sect. 3.2 (breadth-first, one wave per group)
//   density + h iteration ....... Sect. 2.2 and Sect. 3.2.1
//   hydro force ................. Sect. 2.4 (eq:acc, eq:energy), 2.5, 2.6
//   leapfrog + Courant step ..... Sect. 2.4 (eq:predict_pos, eq:predict_vel,
//                                 eq:correct_vel, eq:timestep), Sect. 3.3
//
// Built with -ffp-contract=off: every fused multiply-add is an explicit fma().
#include <math.h>

#include <mutex>

#include <type_traits>

#include "sph_ctx.h"

namespace sph {

#define SPH_INF (__builtin_huge_val())

// ============================================================================
// Wave / block primitives (wave64)
// ============================================================================
// v moved across lanes by a DPP control (row_shr:n = 0x110 + n, row_bcast:15
// = 0x142, row_bcast:31 = 0x143); lanes without a source, or outside the
// enabled rows, read 0.  Called with every lane of the wavefront active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes: Hillis-Steele within each row of
// 16 lanes, then the row totals carried by the two row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += dpp_u32<0x111, 0xf>(v);
  v += dpp_u32<0x112, 0xf>(v);
  v += dpp_u32<0x114, 0xf>(v);
  v += dpp_u32<0x118, 0xf>(v);
  v += dpp_u32<0x142, 0xa>(v);
  v += dpp_u32<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
  return v;
}

__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, kWave));
  return v;
}

// Sum over the LPI consecutive lanes of a particle slot (aligned segments).
template <int LPI>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int d = LPI / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}
template <int LPI>
__device__ __forceinline__ double seg_max(double v) {
#pragma unroll
  for (int d = LPI / 2; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
  return v;
}
template <int LPI>
__device__ __forceinline__ uint32_t seg_sum_u32(uint32_t v) {
#pragma unroll
  for (int d = LPI / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over a 256-thread block; lds must hold 4 words.
__device__ __forceinline__ uint32_t block256_excl_scan(uint32_t v, uint32_t* lds,
                                                       uint32_t* total) {
  const uint32_t inc = wave_incl_scan_u32(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t s = lds[k];
    off += (k < w) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// ============================================================================
// Device-wide exclusive scan of uint32 (three launches).  Tiles of 2048.
// ============================================================================
__global__ __launch_bounds__(256) void k_scan_partials(const uint32_t* __restrict__ in, int64_t n,
                                                        uint32_t* __restrict__ part) {
  __shared__ uint32_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += (base + k < n) ? in[base + k] : 0u;
  uint32_t tot;
  block256_excl_scan(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block of 1024 threads scans nb partials in chunks; writes the total.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ part, int nb,
                                                    uint32_t* __restrict__ total_out,
                                                    int32_t* __restrict__ total_i32) {
  __shared__ uint32_t lds[16];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t v = (i < nb) ? part[i] : 0u;
    const uint32_t inc = wave_incl_scan_u32(v);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      uint32_t s = lds[k];
      off += (k < w) ? s : 0u;
      tot += s;
    }
    const uint32_t c0 = carry;
    if (i < nb) part[i] = c0 + off + inc - v;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (total_out) *total_out = carry;
    if (total_i32) *total_i32 = (int32_t)carry;
  }
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                     const uint32_t* __restrict__ part) {
  __shared__ uint32_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  uint32_t v[8];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t off = block256_excl_scan(s, lds, &tot) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (base + k < n) out[base + k] = off;
    off += v[k];
  }
}

// Exclusive scan of up to kScanSingleMax uint32 (n a multiple of 4, data
// 16-byte aligned) by one block of 1024 threads in one launch: every thread
// owns a contiguous run of at most 16 uint4, loaded all at once.
constexpr int kScanSingleMax = 1024 * 64;

__global__ __launch_bounds__(1024) void k_scan_single(uint32_t* __restrict__ data, int n,
                                                       uint32_t* __restrict__ total_out,
                                                       int32_t* __restrict__ total_i32) {
  __shared__ uint32_t lds[16];
  const int t = threadIdx.x;
  const int q = (n + 4095) / 4096;  // uint4 per thread, <= 16
  const int nq = n >> 2;
  uint4* d4 = reinterpret_cast<uint4*>(data);
  uint4 v[16];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int idx = t * q + k;
    v[k] = (k < q && idx < nq) ? d4[idx] : make_uint4(0u, 0u, 0u, 0u);
    s += v[k].x + v[k].y + v[k].z + v[k].w;
  }
  const uint32_t inc = wave_incl_scan_u32(s);
  const int w = t >> 6, lane = t & 63;
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t x = lds[k];
    off += (k < w) ? x : 0u;
    tot += x;
  }
  off += inc - s;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int idx = t * q + k;
    if (k < q && idx < nq) {
      uint4 o;
      o.x = off;
      off += v[k].x;
      o.y = off;
      off += v[k].y;
      o.z = off;
      off += v[k].z;
      o.w = off;
      off += v[k].w;
      d4[idx] = o;
    }
  }
  if (t == 0) {
    if (total_out) *total_out = tot;
    if (total_i32) *total_i32 = (int32_t)tot;
  }
}

static hipError_t scan_u32(sph_ctx* c, uint32_t* data, int64_t n, uint32_t* total,
                           int32_t* total_i32) {
  if (n > 0 && n <= kScanSingleMax && (n & 3) == 0 && (reinterpret_cast<uintptr_t>(data) & 15) == 0) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, c->stream, data, (int)n, total,
                       total_i32);
    return hipGetLastError();
  }
  const int nb = (int)((n + kScanTile - 1) / kScanTile);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(256), 0, c->stream, data, n, c->scan_part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, c->stream, c->scan_part, nb, total,
                     total_i32);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, c->stream, data, data, n,
                     c->scan_part);
  return hipGetLastError();
}

// ============================================================================
// Predict (optional) + Morton keys
// ============================================================================
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// (x - lo) * scale, floored and clamped to [0, 2^21 - 1]; NaN -> 0.
__device__ __forceinline__ uint64_t quantise(double x, double lo, double scale) {
  double q = (x - lo) * scale;
  if (!(q >= 0.0)) return 0ull;
  q = floor(q);
  return (q > 2097151.0) ? 2097151ull : (uint64_t)q;
}

__device__ __forceinline__ double wrap_coord(double v, double lo, double len, int periodic) {
  if (periodic) {
    if (v >= lo + len)
      v -= len;
    else if (v < lo)
      v += len;
  }
  return v;
}

// Block 0 also clears the radix sort's digit histograms and tile tickets
// (the sort follows at once).
__global__ __launch_bounds__(256) void k_predict_keys(KParams kp, Parts p, int predict,
                                                       const DevState* __restrict__ ds,
                                                       uint64_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals,
                                                       uint32_t* __restrict__ ghist,
                                                       uint32_t* __restrict__ tickets,
                                                       uint32_t* __restrict__ err) {
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < 8 * 256; k += blockDim.x) ghist[k] = 0u;
    if (threadIdx.x < 8) tickets[threadIdx.x] = 0u;
  }
  const int n = kp.n;
  const double dt = predict ? ds->dt_cur : 0.0;
  const double hdt2 = 0.5 * dt * dt;
  bool bad = false;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double x = p.x[i], y = p.y[i], z = p.z[i];
    if (predict) {
      const double vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
      const double ax = p.ax[i], ay = p.ay[i], az = p.az[i];
      x = wrap_coord(x + (vx * dt + hdt2 * ax), kp.lo[0], kp.len[0], kp.periodic[0]);
      y = wrap_coord(y + (vy * dt + hdt2 * ay), kp.lo[1], kp.len[1], kp.periodic[1]);
      z = wrap_coord(z + (vz * dt + hdt2 * az), kp.lo[2], kp.len[2], kp.periodic[2]);
      p.x[i] = x;
      p.y[i] = y;
      p.z[i] = z;
      p.vx[i] = vx + ax * dt;
      p.vy[i] = vy + ay * dt;
      p.vz[i] = vz + az * dt;
      p.u[i] = p.u[i] + p.dudt[i] * dt;
    }
    bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
    const uint64_t ix = quantise(x, kp.lo[0], kp.key_scale);
    const uint64_t iy = quantise(y, kp.lo[1], kp.key_scale);
    const uint64_t iz = quantise(z, kp.lo[2], kp.key_scale);
    keys[i] = (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
    vals[i] = (uint32_t)i;
  }
  if (bad) atomicOr(err, kErrNonFinite);
}

// ============================================================================
// LSD radix sort of (key, index), 8 bits per pass, stable.
// ============================================================================
// Lanes (among `active`) whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t active) {
  uint64_t m = active;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = ballot64(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// Wave-aggregated increment of an LDS digit counter: when every active lane
// of the wavefront holds the same digit (the high digits of a curve-ordered
// tile) one lane adds the whole count.
__device__ __forceinline__ void lds_count_digit(uint32_t* cnt, uint32_t d, bool valid) {
  const uint64_t act = ballot64(valid);
  if (act == 0ull) return;
  const int lead = __builtin_ctzll(act);
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, lead);  // lead is uniform
  const uint64_t same = ballot64(valid && d == d0);
  if (same == act) {
    if (lane_id() == lead) atomicAdd(&cnt[d0], (uint32_t)popc64(act));
  } else if (valid) {
    atomicAdd(&cnt[d], 1u);
  }
}

// One-sweep radix sort.  k_radix_prep counts the digits of all eight passes
// in one read of the keys (global histograms) and clears the look-back
// status of every pass; k_radix_pass then sorts one 8-bit digit per launch:
// each block takes the next tile (an atomic ticket, so every earlier tile
// belongs to a block that already runs), publishes its digit counts, and
// looks back over the earlier tiles' published counts or inclusive prefixes
// for its exclusive prefix (decoupled look-back), then scatters stably.
// Status words: flag in the top two bits (1 count only, 2 inclusive prefix),
// the count in the low 30 (n < 2^30).  A word carries nothing but itself, so
// relaxed device-scope atomics suffice (no acquire/release cache maintenance).
constexpr uint32_t kStAgg = 1u << 30, kStPre = 2u << 30, kStMask = (1u << 30) - 1u;
constexpr int kLookbackSpin = 1 << 22;  // bounded wait; the predecessors always publish
constexpr int kLookW = 16;               // earlier tiles read per look-back round

__global__ __launch_bounds__(256) void k_radix_prep(const uint64_t* __restrict__ keys, int n,
                                                     int nblk, uint32_t* __restrict__ status,
                                                     uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[8][256];
  const int tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < 8; ++p) h[p][tid] = 0u;
  __syncthreads();
  for (int t = blockIdx.x; t < nblk; t += gridDim.x) {
#pragma unroll
    for (int p = 0; p < 8; ++p) status[((int64_t)p * nblk + t) * 256 + tid] = 0u;
    const int base = t * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortTile / 256; ++k) {
      const int i = base + k * 256 + tid;
      const bool valid = i < n;
      const uint64_t key = valid ? keys[i] : 0ull;
#pragma unroll
      for (int p = 0; p < 8; ++p) lds_count_digit(h[p], (uint32_t)((key >> (8 * p)) & 255ull), valid);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 8; ++p)
    if (h[p][tid]) atomicAdd(&ghist[p * 256 + tid], h[p][tid]);
}

__global__ __launch_bounds__(256) void k_radix_pass(const uint64_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout,
                                                     uint32_t* __restrict__ vout, int n,
                                                     int pass, int nblk,
                                                     uint32_t* __restrict__ status,
                                                     const uint32_t* __restrict__ ghist,
                                                     uint32_t* __restrict__ tickets,
                                                     uint32_t* __restrict__ err) {
  constexpr int PER = kSortTile / 256;
  constexpr int NS = PER * 4;  // (key slice, wavefront) sets of 64 keys, in key order
  // wc[d * NS + s]: keys of digit d in set s, then the tile's keys of digit d
  // before set s (at most kSortTile: 16 bits suffice)
  // the digit counts (16 KB), then the tile in digit order (24 KB)
  __shared__ alignas(16) unsigned char s_buf[kSortTile * 12];
  static_assert(256 * NS * 2 <= kSortTile * 12, "digit counts fit the tile buffer");
  uint16_t* wc = reinterpret_cast<uint16_t*>(s_buf);
  uint64_t* s_key = reinterpret_cast<uint64_t*>(s_buf);
  uint32_t* s_val = reinterpret_cast<uint32_t*>(s_buf + kSortTile * 8);
  __shared__ uint32_t run[256];
  __shared__ uint32_t lst[256];
  __shared__ uint32_t lds4[4];
  __shared__ int s_tile;
  static_assert(kSortTile <= 65535, "16-bit tile offsets");
  const int tid = threadIdx.x, w = tid >> 6;
  const int shift = 8 * pass;
  const uint32_t gh = ghist[pass * 256 + tid];  // in flight from the start
  {
    uint32_t* z = reinterpret_cast<uint32_t*>(wc);
#pragma unroll
    for (int q = 0; q < NS / 2; ++q) z[q * 256 + tid] = 0u;
  }
  if (tid == 0) s_tile = (int)atomicAdd(&tickets[pass], 1u);
  __syncthreads();
  const int tile = s_tile;
  const int base = tile * kSortTile;
  uint64_t key[PER];
  uint32_t val[PER], rank[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = base + k * 256 + tid;
    key[k] = i < n ? kin[i] : 0ull;
    val[k] = i < n ? vin[i] : 0u;
  }
  // rank of each key among the equal digits of its set (wave ballots), and
  // the count of every digit in every set
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const bool valid = base + k * 256 + tid < n;
    const uint32_t d = (uint32_t)((key[k] >> shift) & 255ull);
    const uint64_t m = match_digit8(d, ballot64(valid));
    rank[k] = (uint32_t)popc64(m & lanemask_lt());
    if (valid && rank[k] == 0) wc[d * NS + k * 4 + w] = (uint16_t)popc64(m);
  }
  __syncthreads();
  // thread d: exclusive offsets of digit d over the sets, and the tile's count
  uint32_t mine = 0u;
  {
    uint16_t c[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) c[q] = wc[tid * NS + q];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const uint32_t v = c[q];
      c[q] = (uint16_t)mine;
      mine += v;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) wc[tid * NS + q] = c[q];
  }
  // publish this tile's counts; scan the global digit counts while earlier
  // tiles publish theirs; then the exclusive prefix over earlier tiles
  uint32_t* st = status + (int64_t)pass * nblk * 256;
  __hip_atomic_store(&st[(int64_t)tile * 256 + tid], (tile == 0 ? kStPre : kStAgg) | mine,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // start of every digit: keys with a smaller digit anywhere
  uint32_t all;
  const uint32_t gofs = block256_excl_scan(gh, lds4, &all);
  uint32_t excl = 0u;
  if (tile > 0) {
    // a window of kLookW earlier tiles per round: their loads are in flight
    // together, so a long chain of published counts costs one latency per
    // window rather than one per tile
    int t = tile - 1, spins = 0;
    while (t >= 0) {
      uint32_t v[kLookW];
#pragma unroll
      for (int q = 0; q < kLookW; ++q)
        v[q] = (t - q >= 0) ? __hip_atomic_load(&st[(int64_t)(t - q) * 256 + tid], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : kStPre;  // before tile 0: prefix 0
      int used = 0;
      bool done = false;
#pragma unroll
      for (int q = 0; q < kLookW; ++q) {
        if (done || used < q) continue;  // stopped at an earlier entry
        const uint32_t f = v[q] & ~kStMask;
        if (f == 0u) continue;  // not published yet: poll again from here
        excl += v[q] & kStMask;
        used = q + 1;
        done = f == kStPre;
      }
      if (done) break;
      t -= used;
      if (used == 0 && ++spins > kLookbackSpin) {
        atomicOr(err, kErrSort);
        break;
      }
    }
    __hip_atomic_store(&st[(int64_t)tile * 256 + tid], kStPre | (excl + mine), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  // the tile's keys in digit order in LDS first, so that each digit's run is
  // stored by consecutive lanes to consecutive addresses
  uint32_t tot2;
  const uint32_t ls = block256_excl_scan(mine, lds4, &tot2);  // tile-local start of digit tid
  lst[tid] = ls;
  run[tid] = gofs + excl - ls;  // global position of local position 0, for digit tid
  __syncthreads();
  uint32_t lp[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const uint32_t d = (uint32_t)((key[k] >> shift) & 255ull);
    lp[k] = lst[d] + (uint32_t)wc[d * NS + k * 4 + w] + rank[k];
  }
  __syncthreads();  // the counts are overwritten by the sorted tile
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (base + k * 256 + tid < n) {
      s_key[lp[k]] = key[k];
      s_val[lp[k]] = val[k];
    }
  }
  __syncthreads();
  const int cnt = min(kSortTile, n - base);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = k * 256 + tid;
    if (q < cnt) {
      const uint64_t kk = s_key[q];
      const uint32_t d = (uint32_t)((kk >> shift) & 255ull);
      const uint32_t pos = run[d] + (uint32_t)q;
      kout[pos] = kk;
      vout[pos] = s_val[q];
    }
  }
}

// ============================================================================
// Permute the particle fields into key order (gather, then copy back).
// ============================================================================
struct FieldSet {
  double* f[kMaxFields];
  int64_t* id;
  int nf;
  int im;           // index of m in f (x, y, z are f[0..2])
  double4* xyzm;    // packed x, y, z, m in the new order (FP64 density gathers), or null
};

__global__ __launch_bounds__(256) void k_gather(FieldSet fs, const uint32_t* __restrict__ perm,
                                                 double* __restrict__ tmp,
                                                 int64_t* __restrict__ tmp_id, int n,
                                                 int64_t stride) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const uint32_t j = perm[k];
    for (int f = 0; f < fs.nf; ++f) tmp[f * stride + k] = fs.f[f][j];
    if (fs.id) tmp_id[k] = fs.id[j];
  }
}

__global__ __launch_bounds__(256) void k_copy_back(FieldSet fs, const double* __restrict__ tmp,
                                                    const int64_t* __restrict__ tmp_id, int n,
                                                    int64_t stride) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    for (int f = 0; f < fs.nf; ++f) fs.f[f][k] = tmp[f * stride + k];
    if (fs.id) fs.id[k] = tmp_id[k];
    if (fs.xyzm)
      fs.xyzm[k] =
          make_double4(tmp[k], tmp[stride + k], tmp[2 * stride + k], tmp[fs.im * stride + k]);
  }
}

// Packed x, y, z, m from the particle arrays (the density entry point: the
// caller may have changed m, or x with it, since the permute wrote them).
__global__ __launch_bounds__(256) void k_pack_xyzm(Parts p, int n, double4* __restrict__ xyzm) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    xyzm[k] = make_double4(p.x[k], p.y[k], p.z[k], p.m[k]);
}

// Node h_max refresh modes: 1 a new tree (boxes too), 2 always, 0 only while
// the neighbour lists of the tree are not valid for the force.
__device__ __forceinline__ bool h_refresh_needed(const DevState* ds, int mode) {
  return mode != 0 || ds->leaf_state != 1 || ds->lists_missing != 0;
}

// The mixed kernels' 16-byte gather records: position codes in the tree's
// frame (DevState::qf, set with the node boxes) and m (the density gather)
// or h (the list kernel's candidates) in FP32.  Rewritten with every refresh
// of the nodes' h_max (mode as there), so that a list pass sees the h the
// walk's radii were sized for.
__global__ __launch_bounds__(256) void k_pack_q(KParams kp, Parts p, int n,
                                                const DevState* __restrict__ ds, int mode,
                                                int4* __restrict__ qm, int4* __restrict__ qh) {
  if (!h_refresh_needed(ds, mode)) return;
  const QFrame f = ds->qf;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t qx = qcode(p.x[k], f, 0, kp.periodic[0]);
    const int32_t qy = qcode(p.y[k], f, 1, kp.periodic[1]);
    const int32_t qz = qcode(p.z[k], f, 2, kp.periodic[2]);
    qm[k] = make_int4(qx, qy, qz, __float_as_int((float)p.m[k]));
    qh[k] = make_int4(qx, qy, qz, __float_as_int((float)p.h[k]));
  }
}

// ============================================================================
// Tree and groups from the sorted keys, in three launches.
//
// d(s): level at which keys s-1 and s first differ (1..21; 22 if equal),
// d(0) = d(n) = 0.  The level-l cell containing s spans [a, b) with a the
// last index <= s and b the first index > s where d <= l.  A cell at level
// l is a node iff its parent holds more than n_leaf particles, i.e. iff the
// smallest level L(s) at which the cell containing s holds <= n_leaf
// particles is >= l.  So the nodes starting at s are the levels
// d(s)..L(s), and L(s) is found in a window of n_leaf keys on each side:
//   L(s) = min over s < b <= s+T, b-T <= a <= s of max(d(a), d(b)).
// ============================================================================
constexpr int kHalo = 64;  // n_leaf, n_group <= 64

__device__ __forceinline__ int diff_level(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0ull) return 22;
  return (__clzll((long long)x) + 2) / 3;
}

__device__ __forceinline__ int window_level(const uint8_t* d, int idx, int s, int n, int T) {
  int run = d[idx];
  int best = 22;
  for (int k = 0; k < T; ++k) {
    if (k > 0 && s - k >= 0) run = min(run, (int)d[idx - k]);
    const int b = s + T - k;
    if (b <= n) best = min(best, max((int)d[idx + T - k], run));
  }
  return best;
}

// First index > s whose key leaves the level-l cell of s (galloping search).
__device__ __forceinline__ int cell_end(const uint64_t* __restrict__ keys, int n, int s, int l) {
  if (l == 0) return n;
  const int sh = 3 * (kKeyLevels - l);
  const uint64_t pre = keys[s] >> sh;
  int lo = s, step = 1;
  while (lo + step < n && (keys[lo + step] >> sh) == pre) {
    lo += step;
    step <<= 1;
  }
  int hi = min(lo + step, n);
  while (hi - lo > 1) {
    const int mid = lo + ((hi - lo) >> 1);
    if ((keys[mid] >> sh) == pre)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

// Groups (Sect. 3.1): the group cells are the chopped cells of at most
// n_group particles (level lg >= 1, so their parent P holds more).
// Consecutive children of P that are group cells are packed, in curve order
// and greedily, into groups of at most n_group particles; a child that is
// chopped further ends a pack.  For the group cell starting at s: whether a
// group starts there, and its particle count.  D(j) is the level at which
// keys j-1 and j first differ (0 at j <= 0 and j >= n), so j begins a new
// level-l cell iff D(j) <= l.  The run of group-cell siblings around s is
// found from s outwards (at most eight children, each of at most n_group
// particles), then packed from its first cell.
template <typename DFn>
__device__ void group_pack(DFn D, int n, int s, int lg, int n_group, bool& start, int& count) {
  int rs = s;  // first particle of the run
  for (int k = 0; k < 7 && D(rs) > lg - 1; ++k) {
    int j = rs - 1;  // the previous sibling starts at the last boundary before rs
    while (j > rs - n_group && D(j) > lg) --j;
    if (D(j) > lg) break;  // that sibling holds more than n_group particles
    rs = j;
  }
  int acc = 0;      // particles of the open pack
  int pstart = -1;  // its first particle
  start = false;
  count = 0;
  for (int c0 = rs;;) {
    int c1 = c0 + 1;
    while (c1 < n && c1 <= c0 + n_group && D(c1) > lg) ++c1;
    if (c1 > c0 + n_group) break;  // a chopped sibling ends the run
    const int cc = c1 - c0;
    const bool joins = acc > 0 && acc + cc <= n_group;
    if (pstart == s && !joins) break;  // the pack that starts at s is complete
    if (joins) {
      acc += cc;
    } else {
      acc = cc;
      pstart = c0;
    }
    if (c0 == s && pstart != s) return;  // s's cell joined an earlier pack
    c0 = c1;
    if (c0 >= n || D(c0) <= lg - 1) break;  // P ends
  }
  start = pstart == s;
  count = start ? acc : 0;
}

// The same packing from 192-bit boundary masks over particles [w0, w0 + 192)
// (bit p: particle w0 + p begins a cell at the group level, bc, or at the
// parent level, bp); s sits at bit ps.  For n_group <= 8 every cell the
// packing of s inspects lies within 64 particles of s.
__device__ __forceinline__ bool bit3(const uint64_t (&m)[3], int p) {
  return (m[p >> 6] >> (p & 63)) & 1ull;
}
__device__ __forceinline__ int hi_below(const uint64_t (&m)[3], int p) {  // or -1
  for (int w = p >> 6; w >= 0; --w) {
    uint64_t v = m[w];
    if (w == (p >> 6)) v &= (p & 63) ? (~0ull >> (64 - (p & 63))) : 0ull;
    if (v != 0ull) return w * 64 + 63 - __builtin_clzll(v);
  }
  return -1;
}
__device__ __forceinline__ int lo_above(const uint64_t (&m)[3], int p) {  // or 192
  for (int w = (p + 1) >> 6; w < 3; ++w) {
    uint64_t v = m[w];
    if (w == ((p + 1) >> 6)) v &= ~0ull << ((p + 1) & 63);
    if (v != 0ull) return w * 64 + __builtin_ctzll(v);
  }
  return 192;
}
__device__ void group_pack_masks(const uint64_t (&bc)[3], const uint64_t (&bp)[3], int ps,
                                 int n_group, bool& start, int& count) {
  int rs = ps;
  for (int k = 0; k < 7 && !bit3(bp, rs); ++k) {
    const int pb = hi_below(bc, rs);
    if (pb < rs - n_group) break;  // that sibling holds more than n_group particles
    rs = pb;
  }
  int acc = 0, pstart = -1;
  start = false;
  count = 0;
  for (int c0 = rs;;) {
    const int c1 = lo_above(bc, c0);
    if (c1 - c0 > n_group) break;  // a chopped sibling ends the run
    const int cc = c1 - c0;
    const bool joins = acc > 0 && acc + cc <= n_group;
    if (pstart == ps && !joins) break;
    if (joins) {
      acc += cc;
    } else {
      acc = cc;
      pstart = c0;
    }
    if (c0 == ps && pstart != ps) return;
    c0 = c1;
    if (bit3(bp, c0)) break;  // P ends
  }
  start = pstart == ps;
  count = start ? acc : 0;
}

__global__ __launch_bounds__(256) void k_tree_levels(const uint64_t* __restrict__ keys, int n,
                                                      int n_leaf, int n_group,
                                                      uint8_t* __restrict__ dlev,
                                                      uint8_t* __restrict__ lleaf,
                                                      uint8_t* __restrict__ gsize,
                                                      uint8_t* __restrict__ gstart,
                                                      uint32_t* __restrict__ tree_cnt,
                                                      uint32_t* __restrict__ grp_cnt, int nblk,
                                                      int32_t* __restrict__ nnchild,
                                                      int64_t node_cap) {
  __shared__ uint8_t d[kTreeTile + 2 * kHalo + 1];
  // child counts of every node slot cleared for k_tree_emit's increments
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < node_cap;
       k += (int64_t)gridDim.x * blockDim.x)
    nnchild[k] = 0;
  __shared__ uint32_t lc[kLevels];
  __shared__ uint32_t gc;
  const int base = blockIdx.x * kTreeTile;
  for (int t = threadIdx.x; t < kTreeTile + 2 * kHalo + 1; t += blockDim.x) {
    const int j = base - kHalo + t;
    d[t] = (j <= 0 || j >= n) ? (uint8_t)0 : (uint8_t)diff_level(keys[j - 1], keys[j]);
  }
  if (threadIdx.x < kLevels) lc[threadIdx.x] = 0;
  if (threadIdx.x == 0) gc = 0;
  __syncthreads();
  const int s = base + threadIdx.x;
  const bool valid = s < n;
  const int idx = kHalo + threadIdx.x;
  int ds = 0, ll = 0, lg_raw = kLevels;
  if (valid) {
    ds = d[idx];
    ll = min(window_level(d, idx, s, n, n_leaf), kKeyLevels);
    lg_raw = window_level(d, idx, s, n, n_group);
  }
  bool start = false;
  int gcount = 0;
  const bool cell = valid && lg_raw <= kKeyLevels && ds <= lg_raw;  // s begins its group cell
  if (cell && lg_raw == 0) {
    start = true;
    gcount = n;  // the whole set is one group
  }
  if (n_group <= 8) {
    // per wavefront and group level L: boundary masks over the 192
    // particles around the wavefront's 64, from the LDS window
    const int lane = threadIdx.x & (kWave - 1);
    const int t0 = threadIdx.x - lane;  // window index of particle s - lane - 64
    uint64_t todo = ballot64(cell && lg_raw >= 1);
    while (todo != 0ull) {
      const int L = __builtin_amdgcn_readlane(lg_raw, __builtin_ctzll(todo));
      uint64_t bc[3], bp[3];
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        const int dj = d[t0 + kWave * w + lane];
        bc[w] = ballot64(dj <= L);
        bp[w] = ballot64(dj <= L - 1);
      }
      const bool mine = cell && lg_raw == L;
      if (mine) group_pack_masks(bc, bp, lane + kWave, n_group, start, gcount);
      todo &= ~ballot64(mine);
    }
  } else if (cell && lg_raw >= 1) {
    // diff levels from the block's LDS window (it reaches kHalo particles
    // past the tile on both sides), else from the keys
    auto D = [&](int j) -> int {
      const int t = j - base + kHalo;
      if (t >= 0 && t < kTreeTile + 2 * kHalo + 1) return d[t];
      return (j <= 0 || j >= n) ? 0 : diff_level(keys[j - 1], keys[j]);
    };
    group_pack(D, n, s, lg_raw, n_group, start, gcount);
  }
  if (valid && lg_raw > kKeyLevels) {
    // level-21 cell with more than n_group identical keys: cut in chunks
    int a = s;
    while (a > 0 && keys[a - 1] == keys[a]) --a;
    start = ((s - a) % n_group) == 0;
    if (start) gcount = min(n_group, cell_end(keys, n, s, kKeyLevels) - s);
  }
  if (valid) {
    dlev[s] = (uint8_t)ds;
    lleaf[s] = (uint8_t)ll;
    gsize[s] = (uint8_t)gcount;
    gstart[s] = start ? 1 : 0;
    for (int l = ds; l <= ll; ++l) atomicAdd(&lc[l], 1u);
    if (start) atomicAdd(&gc, 1u);
  }
  __syncthreads();
  if (threadIdx.x < kLevels) tree_cnt[threadIdx.x * nblk + blockIdx.x] = lc[threadIdx.x];
  if (threadIdx.x == 0) grp_cnt[blockIdx.x] = gc;
}

__global__ __launch_bounds__(256) void k_tree_emit(
    const uint64_t* __restrict__ keys, int n, int n_group, const uint8_t* __restrict__ dlev,
    const uint8_t* __restrict__ lleaf, const uint8_t* __restrict__ gsize,
    const uint8_t* __restrict__ gstart, const uint32_t* __restrict__ tree_off,
    const uint32_t* __restrict__ grp_off, int nblk, int64_t node_cap,
    int32_t* __restrict__ nlevel, int32_t* __restrict__ nfirst, int32_t* __restrict__ ncount,
    int32_t* __restrict__ nparent, int32_t* __restrict__ nchild, int32_t* __restrict__ nnchild,
    int32_t* __restrict__ gfirst, int32_t* __restrict__ gcount, DevState* __restrict__ ds) {
  __shared__ uint32_t wc[4][kLevels];
  __shared__ uint32_t gw[4];
  if ((int64_t)ds->n_nodes > node_cap || ds->n_nodes < 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ds->err, kErrNodes);
    return;
  }
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int s = blockIdx.x * kTreeTile + tid;
  const bool valid = s < n;
  const int dsv = valid ? dlev[s] : 99;
  const int ll = valid ? lleaf[s] : -1;
  const bool gs = valid && gstart[s];
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = ballot64(valid && dsv <= l && l <= ll);
    if (lane == 0) wc[w][l] = (uint32_t)popc64(b);
  }
  const uint64_t bg = ballot64(gs);
  if (lane == 0) gw[w] = (uint32_t)popc64(bg);
  __syncthreads();
  int prev = -1, par_at_d = -1;
  for (int l = 0; l < kLevels; ++l) {
    const bool mem = valid && dsv <= l && l <= ll;
    const uint64_t b = ballot64(mem);
    uint32_t r = (uint32_t)popc64(b & lanemask_lt());
    for (int q = 0; q < w; ++q) r += wc[q][l];
    const int idx = (int)(tree_off[l * nblk + blockIdx.x] + r);
    if (valid && l == dsv - 1) par_at_d = idx - 1;  // last level-(d-1) node before s
    if (mem) {
      nlevel[idx] = l;
      nfirst[idx] = s;
      // only leaves need their particle count (the walk reads particles of
      // leaves only); inner counts are derived on the host for inspection
      ncount[idx] = (l == ll) ? cell_end(keys, n, s, l) - s : 0;
      const int parent = (l == 0) ? -1 : (l == dsv ? par_at_d : prev);
      nparent[idx] = parent;
      nchild[idx] = -1;
      if (l > dsv) nchild[prev] = idx;  // first child of (l-1, s) is (l, s)
      if (parent >= 0) atomicAdd(&nnchild[parent], 1);
      prev = idx;
    }
  }
  uint32_t rg = (uint32_t)popc64(bg & lanemask_lt());
  for (int q = 0; q < w; ++q) rg += gw[q];
  if (gs) {
    const int g = (int)(grp_off[blockIdx.x] + rg);
    gfirst[g] = s;
    gcount[g] = gsize[s];
  }
}

// If the tree outgrew the node arrays, report it and leave an empty tree so
// that no later launch reads or writes past the arrays (one thread, after
// k_tree_emit; repeating it changes nothing).
__device__ __forceinline__ void tree_guard(DevState* ds, int64_t node_cap) {
  if ((int64_t)ds->n_nodes > node_cap || ds->n_nodes < 0) {
    atomicOr(&ds->err, kErrNodes);
    ds->n_nodes = 0;
    ds->n_groups = 0;
  }
}

// ---- node and group boxes and largest h -----------------------------------
// Every leaf and group covers a contiguous range of the sorted particles:
// k_range_boxes reduces each one's particles (four per wavefront, 16 lanes
// each, so the particle loads coalesce).  Inner nodes then take the union of
// their children's boxes and the largest of their h_max, one launch per
// level from the deepest up (k_level_boxes).  No atomics.  A leaf's or
// group's box is exactly the range's; an inner node's holds its children's
// conservative (rounded-up) boxes, so every box contains its particles.
// mode 1: boxes and h_max of a new tree; 0: h_max only, skipped on the device
// while the neighbour lists of the tree are valid; 2: h_max only, always.
struct Box7 {
  double lo[3], hi[3], hm;
};

__device__ __forceinline__ void box_empty(Box7& b) {
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = SPH_INF;
    b.hi[a] = -SPH_INF;
  }
  b.hm = 0.0;
}

__device__ __forceinline__ float f32_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, SPH_INF);
  return f;
}

__device__ __forceinline__ void write_node_box(const Box7& b, int it, int f, int e, int nc,
                                               const int32_t* __restrict__ nchild,
                                               WalkNode* __restrict__ wn, int do_bb) {
  if (do_bb) {
    WalkNode w;
    for (int a = 0; a < 3; ++a) {
      const double c = 0.5 * (b.lo[a] + b.hi[a]);
      w.c[a] = c;
      w.w[a] = f32_up(fmax(b.hi[a] - c, c - b.lo[a]));
    }
    w.hmax = f32_up(b.hm);
    w.first = f;
    w.count = e - f;
    w.child = nc ? nchild[it] : -1;
    w.nchild = nc;
    wn[it] = w;
  } else {
    wn[it].hmax = f32_up(b.hm);
  }
}

__device__ __forceinline__ void write_group_box(const Box7& b, int g, int f, int e,
                                                GroupInfo* __restrict__ gi, int do_bb) {
  if (do_bb) {
    GroupInfo G;
    for (int a = 0; a < 3; ++a) {
      G.c[a] = 0.5 * (b.lo[a] + b.hi[a]);
      G.w[a] = fmax(b.hi[a] - G.c[a], G.c[a] - b.lo[a]);
    }
    G.hmax = b.hm;
    G.first = f;
    G.count = e - f;
    gi[g] = G;
  } else {
    gi[g].hmax = b.hm;
  }
}

__global__ void k_tree_guard(DevState* __restrict__ ds, int64_t node_cap) {
  if (blockIdx.x == 0 && threadIdx.x == 0) tree_guard(ds, node_cap);
}

// Small trees: every inner node by one wavefront, in the launch of the leaves
// and groups, from the particles of its range and the boxes of the whole
// kChunk-particle chunks inside it (k_chunk_boxes); its range ends where its
// next sibling starts, or, for a last child, where its parent's range ends.
// One launch instead of one per level; on large trees the chunks' particles
// are read by many nodes of the lower levels, and the per-level launches win.
__device__ __forceinline__ void wave_box(Box7& b, int do_bb) {
  if (do_bb)
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = wave_min_f64(b.lo[a]);
      b.hi[a] = wave_max_f64(b.hi[a]);
    }
  b.hm = wave_max_f64(b.hm);
}

// Lane-partial box of particles [a, e), lanes striding by 64.
__device__ __forceinline__ void add_particles(Box7& b, int a, int e, const double* __restrict__ x,
                                              const double* __restrict__ y,
                                              const double* __restrict__ z,
                                              const double* __restrict__ h, int do_bb) {
#pragma unroll 4
  for (int s = a + lane_id(); s < e; s += kWave) {
    if (do_bb) {
      const double px = x[s], py = y[s], pz = z[s];
      b.lo[0] = fmin(b.lo[0], px);
      b.hi[0] = fmax(b.hi[0], px);
      b.lo[1] = fmin(b.lo[1], py);
      b.hi[1] = fmax(b.hi[1], py);
      b.lo[2] = fmin(b.lo[2], pz);
      b.hi[2] = fmax(b.hi[2], pz);
    }
    b.hm = fmax(b.hm, h[s]);
  }
}

// cb: 8 doubles per chunk (lo xyz, hi xyz, h_max, unused).
__global__ __launch_bounds__(256) void k_chunk_boxes(const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ h, int n,
                                                      double* __restrict__ cb,
                                                      DevState* __restrict__ ds, int mode,
                                                      int64_t node_cap) {
  // boxes of a new tree: its node count is checked before k_range_boxes reads it
  if (mode == 1 && blockIdx.x == 0 && threadIdx.x == 0) tree_guard(ds, node_cap);
  if (!h_refresh_needed(ds, mode)) return;
  const int do_bb = mode == 1 ? 1 : 0;
  const int nch = (n + kChunk - 1) / kChunk;
  const int wpb = blockDim.x / kWave;
  for (int c = blockIdx.x * wpb + (int)(threadIdx.x / kWave); c < nch; c += gridDim.x * wpb) {
    Box7 b;
    box_empty(b);
    add_particles(b, c * kChunk, min(n, (c + 1) * kChunk), x, y, z, h, do_bb);
    wave_box(b, do_bb);
    if (lane_id() == 0) {
      double* o = cb + 8 * (int64_t)c;
      if (do_bb)
        for (int a = 0; a < 3; ++a) {
          o[a] = b.lo[a];
          o[3 + a] = b.hi[a];
        }
      o[6] = b.hm;
    }
  }
}

__device__ void inner_ranges(int blk, int nblocks, const double* __restrict__ x,
                             const double* __restrict__ y, const double* __restrict__ z,
                             const double* __restrict__ h, int n, const double* __restrict__ cb,
                             const int32_t* __restrict__ nfirst,
                             const int32_t* __restrict__ nparent,
                             const int32_t* __restrict__ nchild,
                             const int32_t* __restrict__ nnchild, WalkNode* __restrict__ wn,
                             int nn, int do_bb) {
  const int wpb = blockDim.x / kWave;
  const int nw = nblocks * wpb;
  for (int it = blk * wpb + (int)(threadIdx.x / kWave); it < nn; it += nw) {
    const int nc = nnchild[it];
    if (nc == 0) continue;
    const int f = nfirst[it];
    int e = n;
    int k = it;
    while (k > 0) {
      const int p = nparent[k];
      if (p < 0) break;
      if (k + 1 < nchild[p] + nnchild[p]) {
        e = nfirst[k + 1];
        break;
      }
      k = p;
    }
    Box7 b;
    box_empty(b);
    const int c0 = (f + kChunk - 1) / kChunk, c1 = e / kChunk;
    if (c1 > c0) {
      add_particles(b, f, c0 * kChunk, x, y, z, h, do_bb);
      for (int c = c0 + lane_id(); c < c1; c += kWave) {
        const double* q = cb + 8 * (int64_t)c;
        if (do_bb)
          for (int a = 0; a < 3; ++a) {
            b.lo[a] = fmin(b.lo[a], q[a]);
            b.hi[a] = fmax(b.hi[a], q[3 + a]);
          }
        b.hm = fmax(b.hm, q[6]);
      }
      add_particles(b, c1 * kChunk, e, x, y, z, h, do_bb);
    } else {
      add_particles(b, f, e, x, y, z, h, do_bb);
    }
    wave_box(b, do_bb);
    if (lane_id() == 0) write_node_box(b, it, f, e, nc, nchild, wn, do_bb);
  }
}

__global__ __launch_bounds__(256) void k_range_boxes(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ h, const int32_t* __restrict__ nfirst,
    const int32_t* __restrict__ ncount, const int32_t* __restrict__ nchild,
    const int32_t* __restrict__ nnchild, WalkNode* __restrict__ wn,
    const int32_t* __restrict__ gfirst, const int32_t* __restrict__ gcount,
    GroupInfo* __restrict__ gi, const DevState* __restrict__ ds, int mode, int nb_items, int n,
    const double* __restrict__ cb, const int32_t* __restrict__ nparent) {
  if (!h_refresh_needed(ds, mode)) return;
  const int do_bb = mode == 1 ? 1 : 0;
  const int nn = ds->n_nodes, ng = ds->n_groups;
  if ((int)blockIdx.x >= nb_items) {  // small trees: the inner nodes
    inner_ranges((int)blockIdx.x - nb_items, (int)gridDim.x - nb_items, x, y, z, h, n, cb,
                 nfirst, nparent, nchild, nnchild, wn, nn, do_bb);
    return;
  }
  // items 0..nn-1 are nodes (inner ones are left to k_level_boxes), the rest
  // groups; the trip count is uniform over the wavefront (its shuffles)
  const int seg = lane_id() >> 4, sub = lane_id() & 15;
  const int wpb = blockDim.x / kWave;
  const int nwv = nb_items * wpb;
  for (int base = (blockIdx.x * wpb + (int)(threadIdx.x / kWave)) * 4; base < nn + ng;
       base += nwv * 4) {
    const int it = base + seg;
    const bool is_node = it < nn;
    const bool item = it < nn + ng && !(is_node && nnchild[it] != 0);
    int f = 0, e = 0;
    if (item) {
      f = is_node ? nfirst[it] : gfirst[it - nn];
      e = f + (is_node ? ncount[it] : gcount[it - nn]);
    }
    Box7 b;
    box_empty(b);
    for (int s = f + sub; s < e; s += 16) {
      if (do_bb) {
        const double px = x[s], py = y[s], pz = z[s];
        b.lo[0] = fmin(b.lo[0], px);
        b.hi[0] = fmax(b.hi[0], px);
        b.lo[1] = fmin(b.lo[1], py);
        b.hi[1] = fmax(b.hi[1], py);
        b.lo[2] = fmin(b.lo[2], pz);
        b.hi[2] = fmax(b.hi[2], pz);
      }
      b.hm = fmax(b.hm, h[s]);
    }
    for (int d = 8; d > 0; d >>= 1) {
      if (do_bb)
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = fmin(b.lo[a], __shfl_xor(b.lo[a], d, 16));
          b.hi[a] = fmax(b.hi[a], __shfl_xor(b.hi[a], d, 16));
        }
      b.hm = fmax(b.hm, __shfl_xor(b.hm, d, 16));
    }
    if (item && sub == 0) {
      if (is_node)
        write_node_box(b, it, f, e, 0, nchild, wn, do_bb);
      else
        write_group_box(b, it - nn, f, e, gi, do_bb);
    }
  }
}

// An inner node from its children (already final): the union of their boxes
// and the largest of their h_max; its range ends where its last child's ends.
__device__ __forceinline__ void inner_node(int it, const int32_t* __restrict__ nfirst,
                                           const int32_t* __restrict__ nchild,
                                           const int32_t* __restrict__ nnchild,
                                           WalkNode* __restrict__ wn, int mode) {
  const int nc = nnchild[it];
  if (nc == 0) return;
  const int c0 = nchild[it];
  double lo[3] = {SPH_INF, SPH_INF, SPH_INF}, hi[3] = {-SPH_INF, -SPH_INF, -SPH_INF};
  float hm = 0.f;
  int last_end = 0;
  for (int q = 0; q < nc; ++q) {
    const WalkNode w = wn[c0 + q];
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], w.c[a] - (double)w.w[a]);
      hi[a] = fmax(hi[a], w.c[a] + (double)w.w[a]);
    }
    hm = fmaxf(hm, w.hmax);
    last_end = w.first + w.count;
  }
  if (mode == 1) {
    WalkNode w;
    for (int a = 0; a < 3; ++a) {
      const double c = 0.5 * (lo[a] + hi[a]);
      w.c[a] = c;
      w.w[a] = f32_up(fmax(hi[a] - c, c - lo[a]));
    }
    w.hmax = hm;
    w.first = nfirst[it];
    w.count = last_end - w.first;
    w.child = c0;
    w.nchild = nc;
    wn[it] = w;
  } else {
    wn[it].hmax = hm;
  }
}

// Nodes are numbered level by level: level l is [off[l nblk], off[(l+1) nblk]).
__device__ __forceinline__ void level_range(int level, const uint32_t* __restrict__ off, int nblk,
                                            int nn, int& beg, int& end) {
  beg = (int)off[level * nblk];
  end = min(level + 1 < kLevels ? (int)off[(level + 1) * nblk] : nn, nn);
}

// The inner nodes of one level (large trees: one launch per level).
__global__ __launch_bounds__(256) void k_level_boxes(int level, const uint32_t* __restrict__ level_off,
                                                      int nblk, const int32_t* __restrict__ nfirst,
                                                      const int32_t* __restrict__ nchild,
                                                      const int32_t* __restrict__ nnchild,
                                                      WalkNode* __restrict__ wn,
                                                      const DevState* __restrict__ ds, int mode) {
  if (!h_refresh_needed(ds, mode)) return;
  int beg, end;
  level_range(level, level_off, nblk, ds->n_nodes, beg, end);
  for (int it = beg + blockIdx.x * blockDim.x + threadIdx.x; it < end;
       it += gridDim.x * blockDim.x)
    inner_node(it, nfirst, nchild, nnchild, wn, mode);
}

// Fixed-point frame of the mixed force records (QFrame) for the positions of
// the current tree: the box on periodic axes, the root node's box (a
// conservative one: its half-widths are rounded up) on open axes.
__global__ void k_qframe(KParams kp, const WalkNode* __restrict__ nodes,
                         DevState* __restrict__ ds) {
  if (threadIdx.x >= 3) return;
  const int a = threadIdx.x;
  QFrame& f = ds->qf;
  if (kp.periodic[a]) {
    f.o[a] = kp.lo[a];
    f.inv[a] = 4294967296.0 / kp.len[a];
    f.step[a] = (float)(kp.len[a] / 4294967296.0);
  } else {
    const bool any = ds->n_nodes > 0;
    const double c = any ? nodes[0].c[a] : 0.0;
    const double w = any ? (double)nodes[0].w[a] : 0.0;
    const double ext = w > 0.0 ? 2.0 * w : 1.0;
    f.o[a] = c - 0.5 * ext;
    f.inv[a] = 2147483648.0 / ext;
    f.step[a] = (float)(ext / 2147483648.0);
  }
}

// ============================================================================
// Group tree walk (Sect. 3.2): one wavefront per group, breadth-first.  The
// frontier lives in LDS; nodes are tested 64 at a time, opened inner nodes
// push their (contiguous) children, opened leaves append (first, count) to an
// LDS leaf list that is flushed through a candidate loop when it fills.  An
// inner node that lies wholly within the opening radius is appended whole
// (its particle range), which keeps the frontier to the nodes that straddle
// the edge of the search region.
// The opening test is conservative (a superset); the exact pair predicate is
// applied in the candidate loop.
// ============================================================================
constexpr int kFCap = 512;  // frontier entries per level in LDS
constexpr int kLCap = 128;  // leaves per flush
constexpr int kPMax = 128;  // pairs per particle slot
constexpr int kTile = 256;  // candidates staged in LDS at a time
constexpr int kSG = 8;      // groups sharing one super-group walk
constexpr int kSLCap = 256; // leaves a super-group walk may collect

// Nearest periodic image of a separation d (|d| < 1.5 len for positions in
// the box).  Branch-free: the two selects compile to conditional moves, so a
// wavefront does not split over the sign of d.
__device__ __forceinline__ double fold(double d, double len, double half, int periodic) {
  const double lp = periodic ? len : 0.0;
  double t = d > half ? d - lp : d;
  t = d < -half ? d + lp : t;
  return t;
}

// Largest squared distance between a point of the group box and a point of
// the node box, along the nearest periodic image of the centres (an upper
// bound of the minimum-image distance of every such pair).
__device__ __forceinline__ double box_far2(const WalkNode& nd, const GroupInfo& G,
                                           const KParams& kp) {
  double d2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double dc = nd.c[a] - G.c[a];
    if (kp.periodic[a]) dc = dc - kp.len[a] * rint(dc * kp.inv_len[a]);
    const double far = fabs(dc) + (double)nd.w[a] + G.w[a];
    d2 = d2 + far * far;
  }
  return d2;
}

// min-image squared distance between a node box and the group box
__device__ __forceinline__ double box_gap2(const WalkNode& nd, const GroupInfo& G,
                                           const KParams& kp) {
  double d2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double dc = nd.c[a] - G.c[a];
    if (kp.periodic[a]) dc = dc - kp.len[a] * rint(dc * kp.inv_len[a]);
    double gap = fabs(dc) - (double)nd.w[a] - G.w[a];
    gap = gap > 0.0 ? gap : 0.0;
    d2 = d2 + gap * gap;
  }
  return d2;
}

struct WalkLds {
  int lfirst[kLCap];
  int lcnt[kLCap];
  int lnode[kLCap];
  int loff[kLCap + 1];
};

// Candidate tile: up to kTile candidates of the flushed leaves.  FP64 path:
// absolute positions; FP32 path: positions relative to the group centre,
// folded to the nearest periodic image once, when staged.  `a` carries one
// more per-particle value (m_j for the density, h_j for the force), `j` the
// particle index.
template <typename T>
struct TileOf {
  T x[kTile];
  T y[kTile];
  T z[kTile];
  T a[kTile];
  int j[kTile];
};

// Breadth-first walk.  open_r(node) returns the opening radius for a node;
// flush(nleaf) consumes the leaf list (loff filled).  A level's frontier
// holds kFCap entries in LDS and continues in this wavefront's region of
// global memory (`spill`, kSpill entries per level; search regions much
// larger than the local particle spacing need it).  Returns false on
// frontier overflow.
template <bool WHOLE = true, typename RadiusFn, typename FlushFn>
__device__ bool group_walk(const WalkNode* __restrict__ nodes, const GroupInfo& G,
                           const KParams& kp, WalkLds& L, int (&front)[2][kFCap],
                           int* __restrict__ spill, RadiusFn open_r, FlushFn flush) {
  const int lane = threadIdx.x;
  const int cap = kFCap + kSpill;
  auto fget = [&](int lvl, int k) -> int {
    return k < kFCap ? front[lvl][k]
                     : __hip_atomic_load(&spill[lvl * kSpill + (k - kFCap)], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  };
  auto fput = [&](int lvl, int k, int v) {
    if (k < kFCap)
      front[lvl][k] = v;
    else
      __hip_atomic_store(&spill[lvl * kSpill + (k - kFCap)], v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  };
  int nf = 1, cur = 0, nleaf = 0;
  if (lane == 0) front[0][0] = 0;
  __syncthreads();
  bool ok = true;
  while (nf > 0) {
    int nn = 0;
    for (int base = 0; base < nf; base += kWave) {
      const int k = base + lane;
      const bool act = k < nf;
      WalkNode nd;
      bool open = false, inside = false;
      int id = 0;
      if (act) {
        id = fget(cur, k);
        nd = nodes[id];
        const double R = open_r(nd);
        open = box_gap2(nd, G, kp) < R * R;
        // an inner node wholly within the radius of every point of the group
        // box is taken whole, like a leaf, all of its leaves being opened
        // (unless WHOLE is false: then only true leaves are listed)
        inside = WHOLE && open && nd.nchild > 0 && box_far2(nd, G, kp) < R * R;
      }
      const bool leaf = open && (nd.nchild == 0 || inside);
      const bool inner = open && nd.nchild > 0 && !inside;
      const uint64_t lb = ballot64(leaf);
      const int nl = popc64(lb);
      if (nleaf + nl > kLCap) {
        flush(nleaf);
        nleaf = 0;
      }
      if (leaf) {
        const int pos = nleaf + popc64(lb & lanemask_lt());
        L.lfirst[pos] = nd.first;
        L.lcnt[pos] = nd.count;
        L.lnode[pos] = id;
      }
      nleaf += nl;
      const uint32_t nc = inner ? (uint32_t)nd.nchild : 0u;
      const uint32_t inc = wave_incl_scan_u32(nc);
      const uint32_t tot = __shfl(inc, kWave - 1, kWave);
      if (nn + (int)tot > cap) {
        ok = false;
      } else {
        const int o = nn + (int)(inc - nc);
        for (uint32_t q = 0; q < nc; ++q) fput(cur ^ 1, o + q, nd.child + (int)q);
        nn += (int)tot;
      }
      __syncthreads();
    }
    if (!ok) break;
    nf = nn;
    cur ^= 1;
  }
  if (nleaf > 0) flush(nleaf);
  return ok;
}

// The same leaf collection as group_walk, but over a list of leaves that a
// walk for an enclosing region already found (super-group walk): every listed
// leaf is tested against this group's box.
template <typename RadiusFn, typename FlushFn>
__device__ void list_walk(const WalkNode* __restrict__ nodes, const int* sl, int nsl,
                          const GroupInfo& G, const KParams& kp, WalkLds& L, RadiusFn open_r,
                          FlushFn flush) {
  const int lane = threadIdx.x;
  int nleaf = 0;
  for (int base = 0; base < nsl; base += kWave) {
    const int k = base + lane;
    WalkNode nd;
    bool open = false;
    if (k < nsl) {
      nd = nodes[sl[k]];
      const double R = open_r(nd);
      open = box_gap2(nd, G, kp) < R * R;
    }
    const uint64_t lb = ballot64(open);
    const int nl = popc64(lb);
    if (nleaf + nl > kLCap) {
      flush(nleaf);
      nleaf = 0;
    }
    if (open) {
      const int pos = nleaf + popc64(lb & lanemask_lt());
      L.lfirst[pos] = nd.first;
      L.lcnt[pos] = nd.count;
      L.lnode[pos] = sl[k];
    }
    nleaf += nl;
    __syncthreads();
  }
  if (nleaf > 0) flush(nleaf);
}

// Exclusive scan of the leaf counts into L.loff[0..nleaf].
__device__ __forceinline__ int leaf_offsets(WalkLds& L, int nleaf) {
  const int lane = threadIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < nleaf; base += kWave) {
    const int k = base + lane;
    const uint32_t v = (k < nleaf) ? (uint32_t)L.lcnt[k] : 0u;
    const uint32_t inc = wave_incl_scan_u32(v);
    if (k < nleaf) L.loff[k] = (int)(carry + inc - v);
    carry += __shfl(inc, kWave - 1, kWave);
  }
  if (lane == 0) L.loff[nleaf] = (int)carry;
  __syncthreads();
  return (int)carry;
}

// Stage candidates [c0, c0+cnt) of the flushed leaves into the LDS tile.
// Every lane resolves its candidates' particle indices first and then issues
// all their loads before storing any, so a whole tile costs about one
// memory latency instead of one per candidate step.
template <typename T>
__device__ __forceinline__ void stage_tile(const WalkLds& L, int nleaf, int c0, int cnt,
                                           const double* __restrict__ px,
                                           const double* __restrict__ py,
                                           const double* __restrict__ pz,
                                           const double* __restrict__ pa, TileOf<T>& S,
                                           const GroupInfo& G, const KParams& kp) {
  constexpr int PER = kTile / kWave;
  const int lane = threadIdx.x;
  int jj[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = lane + q * kWave;
    jj[q] = -1;
    if (t < cnt) {
      const int c = c0 + t;
      int lo = 0, hi = nleaf;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.loff[mid] <= c)
          lo = mid;
        else
          hi = mid;
      }
      jj[q] = L.lfirst[lo] + (c - L.loff[lo]);
    }
  }
  double vx[PER], vy[PER], vz[PER], va[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = jj[q] >= 0 ? jj[q] : 0;
    vx[q] = px[j];
    vy[q] = py[j];
    vz[q] = pz[j];
    va[q] = pa[j];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = lane + q * kWave;
    if (jj[q] >= 0) {
      if constexpr (std::is_same<T, float>::value) {
        S.x[t] = (float)fold(vx[q] - G.c[0], kp.len[0], kp.half[0], kp.periodic[0]);
        S.y[t] = (float)fold(vy[q] - G.c[1], kp.len[1], kp.half[1], kp.periodic[1]);
        S.z[t] = (float)fold(vz[q] - G.c[2], kp.len[2], kp.half[2], kp.periodic[2]);
        S.a[t] = (float)va[q];
      } else {
        S.x[t] = vx[q];
        S.y[t] = vy[q];
        S.z[t] = vz[q];
        S.a[t] = va[q];
      }
      S.j[t] = jj[q];
    }
  }
  __syncthreads();
}

// Candidate loop over the flushed leaves, one staged tile at a time: lane
// `sub` of every slot visits tile entries sub, sub+LPI, ...;
// body(valid, c) is called by all lanes with c the tile index.
template <int LPI, typename T, typename Body>
__device__ __forceinline__ void for_tiles(const WalkLds& L, int nleaf, int total, int sub,
                                          const double* __restrict__ px,
                                          const double* __restrict__ py,
                                          const double* __restrict__ pz,
                                          const double* __restrict__ pa, TileOf<T>& S,
                                          const GroupInfo& G, const KParams& kp, Body body) {
  for (int c0 = 0; c0 < total; c0 += kTile) {
    const int cnt = min(kTile, total - c0);
    stage_tile<T>(L, nleaf, c0, cnt, px, py, pz, pa, S, G, kp);
    for (int cb = 0; cb < cnt; cb += LPI) {
      const int c = cb + sub;
      body(c < cnt, c);
    }
    __syncthreads();
  }
}

// Load entries [b, b+nl) of a stored leaf list into the LDS leaf list.
__device__ __forceinline__ void load_leaves(WalkLds& L, const int2* __restrict__ pool, int off,
                                            int b, int nl) {
  for (int k = threadIdx.x; k < nl; k += kWave) {
    const int2 e = pool[off + b + k];
    L.lfirst[k] = e.x;
    L.lcnt[k] = e.y;
  }
  __syncthreads();
}

// ---- smoothing kernels of Sect. 2.3: W = C f(q) / h^3, q = r / h ----------
// M4 cubic spline (support 2, C = 1/pi), M6 quintic spline (support 3,
// C = 1/(120 pi)), Wendland C6 on the support H = 2h (C = 1365/(512 pi)).
// f(q) and f'(q); the kind is uniform over a launch.
template <typename T>
__device__ __forceinline__ void kern_f_df(int kind, T q, T& f, T& df) {
  if (kind == 1) {
    const T a = T(3) - q, b = T(2) - q, c = T(1) - q;
    const T t3 = a > T(0) ? a : T(0), t2 = b > T(0) ? b : T(0), t1 = c > T(0) ? c : T(0);
    const T s3 = t3 * t3, s2 = t2 * t2, s1 = t1 * t1;
    const T q3 = s3 * s3, q2 = s2 * s2, q1 = s1 * s1;  // fourth powers
    f = q3 * t3 - T(6) * q2 * t2 + T(15) * q1 * t1;
    df = T(-5) * q3 + T(30) * q2 - T(75) * q1;
  } else if (kind == 2) {
    const T u = T(1) - T(0.5) * q;
    const T s = u > T(0) ? u : T(0);
    const T s2 = s * s, s4 = s2 * s2, s7 = s4 * s2 * s;
    f = s7 * s * (((T(4) * q + T(6.25)) * q + T(4)) * q + T(1));
    df = T(-2.75) * q * ((T(8) * q + T(7)) * q + T(2)) * s7;
  } else {
    const T t = T(2) - q;
    const T tp = t > T(0) ? t : T(0);
    // inner branch (q < 1): 1 - 1.5 q^2 + 0.75 q^3 and -3q + 2.25 q^2
    const T fi = T(1) + q * q * (T(0.75) * q - T(1.5));
    const T dfi = q * (T(2.25) * q - T(3));
    // outer branch (1 <= q < 2): 0.25 (2-q)^3 and -0.75 (2-q)^2
    const T fo = T(0.25) * tp * tp * tp;
    const T dfo = T(-0.75) * tp * tp;
    const bool in = q < T(1);
    f = in ? fi : fo;
    df = in ? dfi : dfo;
  }
}

template <typename T>
__device__ __forceinline__ T kern_df(int kind, T q) {
  if (kind == 1) {
    const T a = T(3) - q, b = T(2) - q, c = T(1) - q;
    const T t3 = a > T(0) ? a : T(0), t2 = b > T(0) ? b : T(0), t1 = c > T(0) ? c : T(0);
    const T s3 = t3 * t3, s2 = t2 * t2, s1 = t1 * t1;
    return T(-5) * s3 * s3 + T(30) * s2 * s2 - T(75) * s1 * s1;
  }
  if (kind == 2) {
    const T u = T(1) - T(0.5) * q;
    const T s = u > T(0) ? u : T(0);
    const T s2 = s * s, s4 = s2 * s2;
    return T(-2.75) * q * ((T(8) * q + T(7)) * q + T(2)) * (s4 * s2 * s);
  }
  const T t = T(2) - q;
  const T tp = t > T(0) ? t : T(0);
  const T dfi = q * (T(2.25) * q - T(3));
  const T dfo = T(-0.75) * tp * tp;
  return q < T(1) ? dfi : dfo;
}

__device__ __forceinline__ float fast_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float fast_rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// The same shapes with the kind fixed at compile time (the list kernels are
// instantiated per kind, so their pair loops carry no branch on it) and the
// polynomials in fused multiply-adds.  M4 in one expression for both
// branches: f = t^3/4 - s^3, f' = 3 s^2 - 3 t^2/4, s = max(1-q, 0),
// t = max(2-q, 0).
template <int KIND, typename T>
__device__ __forceinline__ void kf_df(T q, T& f, T& df) {
  if constexpr (KIND == 1) {
    const T a = T(3) - q, b = T(2) - q, c = T(1) - q;
    const T t3 = a > T(0) ? a : T(0), t2 = b > T(0) ? b : T(0), t1 = c > T(0) ? c : T(0);
    const T s3 = t3 * t3, s2 = t2 * t2, s1 = t1 * t1;
    const T q3 = s3 * s3, q2 = s2 * s2, q1 = s1 * s1;  // fourth powers
    f = fma(T(15) * q1, t1, fma(T(-6) * q2, t2, q3 * t3));
    df = fma(T(-75), q1, fma(T(30), q2, T(-5) * q3));
  } else if constexpr (KIND == 2) {
    const T u = fma(T(-0.5), q, T(1));
    const T s = u > T(0) ? u : T(0);
    const T s2 = s * s, s4 = s2 * s2, s7 = s4 * s2 * s;
    f = (s7 * s) * fma(fma(fma(T(4), q, T(6.25)), q, T(4)), q, T(1));
    df = (T(-2.75) * q) * fma(fma(T(8), q, T(7)), q, T(2)) * s7;
  } else {
    const T a = T(2) - q, b = T(1) - q;
    const T t = a > T(0) ? a : T(0), s = b > T(0) ? b : T(0);
    const T t2 = t * t, s2 = s * s;
    f = fma(T(0.25) * t2, t, -(s2 * s));
    df = fma(T(3) * s, s, T(-0.75) * t2);
  }
}

template <int KIND, typename T>
__device__ __forceinline__ T kdf(T q) {
  if constexpr (KIND == 1) {
    const T a = T(3) - q, b = T(2) - q, c = T(1) - q;
    const T t3 = a > T(0) ? a : T(0), t2 = b > T(0) ? b : T(0), t1 = c > T(0) ? c : T(0);
    const T s3 = t3 * t3, s2 = t2 * t2, s1 = t1 * t1;
    return fma(T(-75) * s1, s1, fma(T(30) * s2, s2, T(-5) * s3 * s3));
  } else if constexpr (KIND == 2) {
    const T u = fma(T(-0.5), q, T(1));
    const T s = u > T(0) ? u : T(0);
    const T s2 = s * s, s4 = s2 * s2;
    return (T(-2.75) * q) * fma(fma(T(8), q, T(7)), q, T(2)) * (s4 * s2 * s);
  } else {
    const T a = T(2) - q, b = T(1) - q;
    const T t = a > T(0) ? a : T(0), s = b > T(0) ? b : T(0);
    return fma(T(3) * s, s, T(-0.75) * (t * t));
  }
}

// Nearest periodic image of a separation d (|d| < L) of the mixed-precision
// pair loops, in three FP64 operations: d - L rint(d / L) (lp = L, ilp = 1/L
// on periodic axes, 0 on open ones).  It agrees with fold() except within a
// rounding of |d| = L/2, far outside any support (S h < L/2).
__device__ __forceinline__ double fold_r(double d, double lp, double ilp) {
  return fma(-lp, rint(d * ilp), d);
}

// The exact FP64 pair predicate of both precisions: r^2 = fma(dz, dz,
// fma(dy, dy, dx dx)) of the nearest-image separation against
// (S max(h_i, h_j))^2 (force set, `force`) or (S h_i)^2 (density set).
__device__ __forceinline__ bool exact_pair(const KParams& kp, const double* __restrict__ x,
                                           const double* __restrict__ y,
                                           const double* __restrict__ z,
                                           const double* __restrict__ h, int i, int j,
                                           bool force) {
  const double dx = fold(x[i] - x[j], kp.len[0], kp.half[0], kp.periodic[0]);
  const double dy = fold(y[i] - y[j], kp.len[1], kp.half[1], kp.periodic[1]);
  const double dz = fold(z[i] - z[j], kp.len[2], kp.half[2], kp.periodic[2]);
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double hi = h[i], hj = h[j];
  const double sr = kp.support * ((force && hj > hi) ? hj : hi);
  return r2 < sr * sr;
}

// FP32 pair tests of the mixed mode lie within about 1e-6 (relative) of the
// FP64 ones; a test this close to the boundary is settled by exact_pair.
constexpr float kBorder = 4e-5f;

// ============================================================================
// Density: one wave per group (GS = 64/LPI particle slots of LPI lanes).
// Pair lists (r, m_j) for r < 2 h_i * margin are built once by the walk and
// kept in LDS while h is iterated; the walk is redone only if some h grows
// past its list radius.  Newton-Raphson on f(h) = S0(h) - m (hfact/h)^3 with
// a bracket; the group leaves the loop when a ballot shows every slot
// converged, after one more sum at the converged h.  A group whose lists
// would overflow sums on the fly during a walk at the current h instead.
// The first walk opens nodes with the force criterion widened by the margin
// and stores the group's leaf list, so that the force pass can replay it.
// ============================================================================

// Global Courant minimum: the atomic is skipped when the stored value is
// already smaller (most wavefronts once the first ones have finished).
__device__ __forceinline__ void dt_min_update(DevState* ds, double dm) {
  const unsigned long long e = enc_f64(dm);
  const unsigned long long cur =
      __hip_atomic_load(&ds->dt_min_enc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (e < cur) atomicMin(&ds->dt_min_enc, e);
}

// rho, Omega, P, c_s of particle i at its converged h (Sect. 2.2 and the
// ideal-gas closure), and the record the force loop reads for it; stored by
// the lane with `write`.
template <bool MIXED>
__device__ __forceinline__ void density_outputs(const KParams& kp, const Parts& p,
                                                void* __restrict__ frec_out, int i, double xi,
                                                double yi, double zi, double mi, double h,
                                                double S0, double S1, double minhalf,
                                                uint32_t& err, bool write,
                                                const DevState* __restrict__ ds) {
  const double rho = S0;
  const double omega = 1.0 + h * S1 / (3.0 * rho);
  const double u = p.u[i];
  const double P = kp.gm1 * rho * u;
  const double cs = sqrt(kp.gamma * kp.gm1 * u);
  if (!(isfinite(rho) && isfinite(omega) && isfinite(P) && isfinite(cs))) err |= kErrNonFinite;
  if (kp.support * h >= minhalf) err |= kErrDomain;
  if (!write) return;
  p.h[i] = h;
  p.rho[i] = rho;
  p.omega[i] = omega;
  p.P[i] = P;
  p.cs[i] = cs;
  const double hinv = 1.0 / h;
  const double g = P / (rho * rho * omega);
  const double kk = 1.0 / (rho * omega);
  const double hinv4pi = hinv * hinv * hinv * hinv * kp.knorm;
  if constexpr (MIXED) {
    FRec32 r;
    const QFrame& f = ds->qf;
    r.qx = qcode(xi, f, 0, kp.periodic[0]);
    r.qy = qcode(yi, f, 1, kp.periodic[1]);
    r.qz = qcode(zi, f, 2, kp.periodic[2]);
    r.m = (float)mi;
    r.h = (float)h;
    r.vx = (float)p.vx[i];
    r.vy = (float)p.vy[i];
    r.vz = (float)p.vz[i];
    r.u = (float)u;
    r.hinv = (float)hinv;
    r.hinv4pi = (float)hinv4pi;
    r.g = (float)g;
    r.k = (float)kk;
    r.c = (float)cs;
    r.P = (float)P;
    r.rho = (float)rho;
    reinterpret_cast<FRec32*>(frec_out)[i] = r;
  } else {
    FRec64 r;
    r.x = xi;
    r.y = yi;
    r.z = zi;
    r.m = mi;
    r.vx = p.vx[i];
    r.vy = p.vy[i];
    r.vz = p.vz[i];
    r.u = u;
    r.hinv = hinv;
    r.hinv4pi = hinv4pi;
    r.g = g;
    r.k = kk;
    r.c = cs;
    r.P = P;
    r.rho = rho;
    r.h = h;
    reinterpret_cast<FRec64*>(frec_out)[i] = r;
  }
}

template <bool MIXED, int LPI>
__global__ __launch_bounds__(64) void k_density(KParams kp, Parts p,
                                                const WalkNode* __restrict__ nodes,
                                                const GroupInfo* __restrict__ groups,
                                                void* __restrict__ frec_out,
                                                int2* __restrict__ pool, int64_t pool_cap,
                                                int32_t* __restrict__ gl_off,
                                                int32_t* __restrict__ gl_cnt,
                                                const int32_t* __restrict__ flag_list,
                                                int32_t* __restrict__ walk_spill,
    DevState* __restrict__ ds) {
  int* __restrict__ spill = walk_spill + (int64_t)blockIdx.x * 2 * kSpill;
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int GS = kWave / LPI;
  // flag_list != nullptr: only the groups the neighbour-list kernels
  // flagged, each with its own walk and without storing leaf lists
  const bool fb = flag_list != nullptr;
  __shared__ WalkLds L;
  __shared__ int s_front[2][kFCap];
  __shared__ TileOf<R> T;
  __shared__ R s_r[kPMax * GS];
  __shared__ R s_m[kPMax * GS];
  __shared__ int s_sl[kSLCap];  // leaves found by the super-group walk

  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  const int ng = ds->n_groups;
  // waves take super-groups of kSG consecutive groups; each XCD a contiguous
  // range of them, so that neighbouring groups share that XCD's L2
  // flagged groups are spread one per wavefront (they are few, and heavy)
  // (striped over all wavefronts of all XCDs)
  const int sgs = fb ? 1 : kSG;
  const int nsg = fb ? ds->n_flagged : (ng + sgs - 1) / sgs;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int chunk = (nsg + 7) >> 3;
  const int sbeg = fb ? (int)blockIdx.x : xcd * chunk;
  const int send = fb ? nsg : min(sbeg + chunk, nsg);
  const int sstep = fb ? (int)gridDim.x : nloc;
  const double margin = kp.h_margin;
  double minhalf = SPH_INF;
  for (int a = 0; a < 3; ++a)
    if (kp.periodic[a]) minhalf = fmin(minhalf, kp.half[a]);
  // this wave's region of the leaf-list pool
  const int64_t rsize = pool_cap / gridDim.x;
  const int64_t rbase = (int64_t)blockIdx.x * rsize;
  int64_t rpos = 0;

  uint32_t err = 0;
  int it_max = 0;
  unsigned long long pairs_final = 0, sums = 0, cands = 0;
  int walks = 0;
  bool grew = false;

  for (int sg = fb ? sbeg : sbeg + local; sg < send; sg += sstep) {
   const int g0 = fb ? flag_list[sg] : sg * sgs, g1 = fb ? g0 + 1 : min(g0 + sgs, ng);
   // ---- super-group box (union of the group boxes) and largest start h
   GroupInfo SG;
   {
     const bool v = !fb && lane < g1 - g0;
     GroupInfo Gk;
     if (v) Gk = groups[g0 + lane];
     for (int a = 0; a < 3; ++a) {
       const double lo = wave_min_f64(v ? Gk.c[a] - Gk.w[a] : SPH_INF);
       const double hi = wave_max_f64(v ? Gk.c[a] + Gk.w[a] : -SPH_INF);
       SG.c[a] = 0.5 * (lo + hi);
       SG.w[a] = fmax(hi - SG.c[a], SG.c[a] - lo);
     }
     SG.hmax = wave_max_f64(v ? Gk.hmax : 0.0);
     SG.first = 0;
     SG.count = 0;
   }
   // ---- one walk for the super-group: every leaf any of its groups can need
   int nsl = 0;
   bool sok = true;
   {
     const double hs = margin * SG.hmax;
     auto sradius = [&](const WalkNode& nd) {
       return kp.support * fmax(hs, margin * (double)nd.hmax) * (1.0 + 4e-9);
     };
     auto sflush = [&](int nleaf) {
       if (nsl + nleaf <= kSLCap) {
         for (int q = lane; q < nleaf; q += kWave) s_sl[nsl + q] = L.lnode[q];
       } else {
         sok = false;
       }
       nsl += nleaf;
       __syncthreads();
     };
     if (fb) {
       sok = false;  // flagged groups walk on their own
     } else {
       if (!group_walk(nodes, SG, kp, L, s_front, spill, sradius, sflush)) sok = false;
       ++walks;
     }
   }
   for (int g = g0; g < g1; ++g) {
    if (fb && lane == 0) gl_cnt[g] = -1;  // its force pass walks
    const GroupInfo G = groups[g];
    const bool act = slot < G.count;
    const int i = G.first + (act ? slot : 0);
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i], mi = p.m[i];
    double h = p.h[i];
    if (!(h > 0.0) || !isfinite(h)) {
      err |= kErrNonFinite;
      h = 1.0;
    }
    const double h0 = h;
    float xr = 0.f, yr = 0.f, zr = 0.f;  // FP32 path: position relative to the group centre
    if constexpr (MIXED) {
      xr = (float)fold(xi - G.c[0], kp.len[0], kp.half[0], kp.periodic[0]);
      yr = (float)fold(yi - G.c[1], kp.len[1], kp.half[1], kp.periodic[1]);
      zr = (float)fold(zi - G.c[2], kp.len[2], kp.half[2], kp.periodic[2]);
    }
    double hlim = h * margin;
    double hlo = 0.0, hhi = SPH_INF;
    bool conv = !act;
    bool need = true;
    bool store = !fb;  // the first walk stores the leaf list
    const int64_t gstart = rpos;
    bool gover = false;
    int npair = 0;
    int nit = 0;
    double S0 = 0.0, S1 = 0.0;
    uint32_t nnb = 0;
    bool failed = false;
    bool stream = false;  // group-wide: a pair list overflowed, sum on the fly instead
    while (true) {
      if (!stream && ballot64(act && need) != 0ull) {
        // ---- walk and fill the pair lists (r < 2 hlim_i)
        const double hm = wave_max_f64(act ? hlim : 0.0);
        const double rl = kp.support * hlim, rl2 = rl * rl;
        const float rl2f = (float)rl2 * 1.00001f;
        npair = 0;
        auto radius = [&](const WalkNode& nd) {
          const double r = store ? fmax(hm, margin * (double)nd.hmax) : hm;
          return kp.support * r * (1.0 + 4e-9);
        };
        auto flush = [&](int nleaf) {
          const int total = leaf_offsets(L, nleaf);
          if (store) {
            if (!gover && rpos + nleaf <= rsize) {
              for (int k = lane; k < nleaf; k += kWave)
                pool[rbase + rpos + k] = make_int2(L.lfirst[k], L.lcnt[k]);
              rpos += nleaf;
            } else {
              gover = true;
            }
          }
          cands += (unsigned long long)total * ((act && sub == 0) ? 1u : 0u);
          for_tiles<LPI, R>(L, nleaf, total, sub, p.x, p.y, p.z, p.m, T, G, kp,
                            [&](bool valid, int c) {
            bool pred = false;
            R rv = R(0), mj = R(0);
            if (valid && act) {
              if constexpr (MIXED) {
                const float dx = xr - T.x[c], dy = yr - T.y[c], dz = zr - T.z[c];
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                pred = r2 < rl2f;
                rv = fast_sqrt(r2);
              } else {
                const double dx = fold(xi - T.x[c], kp.len[0], kp.half[0], kp.periodic[0]);
                const double dy = fold(yi - T.y[c], kp.len[1], kp.half[1], kp.periodic[1]);
                const double dz = fold(zi - T.z[c], kp.len[2], kp.half[2], kp.periodic[2]);
                const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                pred = r2 < rl2;
                if (pred) rv = sqrt(r2);
              }
              mj = T.a[c];
            }
            const uint64_t b = ballot64(pred);
            const uint32_t seg = (uint32_t)((b >> (slot * LPI)) & ((LPI == 64) ? ~0ull : ((1ull << LPI) - 1ull)));
            const int pos = npair + __popc(seg & ((1u << sub) - 1u));
            if (pred && pos < kPMax) {
              s_r[pos * GS + slot] = rv;
              s_m[pos * GS + slot] = mj;
            }
            npair += __popc(seg);
          });
          __syncthreads();
        };
        bool wok;
        if (store && sok)
          wok = true, list_walk(nodes, s_sl, nsl, G, kp, L, radius, flush);
        else
          wok = group_walk(nodes, G, kp, L, s_front, spill, radius, flush);
        if (!wok) {
          err |= kErrFrontier;
          failed = true;
        }
        if (store) {
          if (lane == 0) {
            gl_off[g] = (int32_t)(rbase + gstart);
            gl_cnt[g] = (gover || failed) ? -1 : (int32_t)(rpos - gstart);
            if (gover || failed) atomicOr(&ds->lists_missing, 1);
          }
          store = false;
        }
        if (ballot64(failed) != 0ull) {
          failed = true;
          break;
        }
        if (ballot64(npair > kPMax) != 0ull) stream = true;
        need = false;
        ++walks;
      }
      // ---- one density sum at the current h
      const double hinv = 1.0 / h;
      double a0 = 0.0, a1 = 0.0;
      uint32_t cnt = 0;
      if (stream) {
        // walk at the current h and accumulate the candidates directly
        const double Rg = kp.support * wave_max_f64(act ? h : 0.0) * (1.0 + 4e-9);
        const double twoh = kp.support * h, rl2 = twoh * twoh;
        const float rl2f = (float)rl2;
        const float hinvf = (float)hinv;
        auto radius = [&](const WalkNode&) { return Rg; };
        auto flush = [&](int nleaf) {
          const int total = leaf_offsets(L, nleaf);
          for_tiles<LPI, R>(L, nleaf, total, sub, p.x, p.y, p.z, p.m, T, G, kp,
                            [&](bool valid, int c) {
            if (valid && act) {
              if constexpr (MIXED) {
                const float dx = xr - T.x[c], dy = yr - T.y[c], dz = zr - T.z[c];
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                if (r2 < rl2f) {
                  const float m = T.a[c];
                  const float q = fast_sqrt(r2) * hinvf;
                  float f, df;
                  kern_f_df<float>(kp.kernel, q, f, df);
                  a0 += (double)(m * f);
                  a1 += (double)(m * (3.0f * f + q * df));
                  ++cnt;
                }
              } else {
                const double dx = fold(xi - T.x[c], kp.len[0], kp.half[0], kp.periodic[0]);
                const double dy = fold(yi - T.y[c], kp.len[1], kp.half[1], kp.periodic[1]);
                const double dz = fold(zi - T.z[c], kp.len[2], kp.half[2], kp.periodic[2]);
                const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (r2 < rl2) {
                  const double mj = T.a[c];
                  const double q = sqrt(r2) * hinv;
                  double f, df;
                  kern_f_df<double>(kp.kernel, q, f, df);
                  a0 += mj * f;
                  a1 += mj * (3.0 * f + q * df);
                  ++cnt;
                }
              }
            }
          });
          __syncthreads();
        };
        if (!group_walk(nodes, G, kp, L, s_front, spill, radius, flush)) {
          err |= kErrFrontier;
          failed = true;
        }
        if (ballot64(failed) != 0ull) {
          failed = true;
          break;
        }
        ++walks;
      } else if (MIXED) {
        // each lane sums its few terms in FP32; lanes are combined in FP64
        const float hinvf = (float)hinv;
        const float twohf = (float)(kp.support * h);
        float s0 = 0.f, s1 = 0.f;
        for (int k = sub; k < npair; k += LPI) {
          const float r = (float)s_r[k * GS + slot], m = (float)s_m[k * GS + slot];
          const float q = r * hinvf;
          float f, df;
          kern_f_df<float>(kp.kernel, q, f, df);
          s0 = fmaf(m, f, s0);
          s1 = fmaf(m, fmaf(q, df, 3.0f * f), s1);
          cnt += (r < twohf) ? 1u : 0u;
        }
        a0 = (double)s0;
        a1 = (double)s1;
      } else {
        const double twoh = kp.support * h;
        for (int k = sub; k < npair; k += LPI) {
          const double r = (double)s_r[k * GS + slot], m = (double)s_m[k * GS + slot];
          const double q = r * hinv;
          double f, df;
          kern_f_df<double>(kp.kernel, q, f, df);
          a0 += m * f;
          a1 += m * (3.0 * f + q * df);
          cnt += (r < twoh) ? 1u : 0u;
        }
      }
      a0 = seg_sum<LPI>(a0);
      a1 = seg_sum<LPI>(a1);
      cnt = seg_sum_u32<LPI>(cnt);
      const double h3 = hinv * hinv * hinv;
      S0 = a0 * h3 * kp.knorm;
      S1 = -a1 * h3 * hinv * kp.knorm;
      nnb = cnt;
      sums += (act && sub == 0) ? (unsigned long long)cnt : 0ull;
      // ---- decide: a slot is done when the h-rho relation holds at its
      // current h to the tolerance (then S0, S1 above are its final sums);
      // otherwise it takes a safeguarded Newton step and is summed again
      bool moved = false;
      if (!conv) {
        const double t = kp.hfact * hinv;
        const double rh = mi * (t * t * t);
        const double f = S0 - rh;
        const double fp = S1 + 3.0 * rh * hinv;
        double hn = h;
        if (kp.fixed_passes) {
          hn = h - f / fp;
          if (!(fp > 0.0))
            hn = h;
          else if (hn > 1.2 * h)
            hn = 1.2 * h;
          else if (hn < 0.8 * h)
            hn = 0.8 * h;
          // three density computations (Sect. 3.2.1): two updates, then
          // rho and Omega from the third sum at the h it used
          conv = (nit + 1) >= 2;
          moved = true;
        } else if (fabs(f) <= 3.0 * kp.h_tol * rh) {
          // |f| / f' <= tol h (f' = 3 rho_h Omega / h): converged at this h
          conv = true;
        } else {
          if (f < 0.0)
            hlo = fmax(hlo, h);
          else
            hhi = fmin(hhi, h);
          hn = h - f / fp;
          const bool bad = !(fp > 0.0) || !(hn >= 0.8 * h) || !(hn <= 1.2 * h) ||
                           !(hn > hlo) || !(hn < hhi);
          if (bad) {
            if (hlo > 0.0 && hhi < SPH_INF)
              hn = 0.5 * (hlo + hhi);
            else
              hn = (f < 0.0) ? 1.2 * h : h / 1.2;
          }
          // a step at the rounding level of h: sum once more there and stop
          conv = fabs(hn - h) <= 4e-16 * h;
          moved = true;
        }
        if (moved) {
          h = hn;
          if (h > hlim) {
            hlim = h * margin;
            need = true;
          }
          ++nit;
          if (nit > kp.max_iter) {
            err |= kErrNoConv;
            conv = true;
          }
        }
      }
      if (ballot64(!conv || moved) == 0ull) break;  // every slot summed at its final h
    }
    it_max = max(it_max, nit + 1);
    if (act && !failed && h > h0 * margin) grew = true;
    if (act && !failed) {
      density_outputs<MIXED>(kp, p, frec_out, i, xi, yi, zi, mi, h, S0, S1, minhalf, err,
                             sub == 0, ds);
      if (sub == 0) {
        pairs_final += nnb;
      }
    }
   }
  }
  // one set of atomics per wave
  const bool ballot_any = ballot64(grew) != 0ull;
  const uint64_t b = ballot64(err != 0);
  uint32_t eall = err;
  for (int d = 32; d > 0; d >>= 1) eall |= __shfl_xor(eall, d, kWave);
  unsigned long long pf = pairs_final;
  for (int d = 32; d > 0; d >>= 1) pf += __shfl_xor(pf, d, kWave);
  unsigned long long cd = cands, sm = sums;
  for (int d = 32; d > 0; d >>= 1) {
    cd += __shfl_xor(cd, d, kWave);
    sm += __shfl_xor(sm, d, kWave);
  }
  sums = sm;
  if (lane == 0) {
    if (b) atomicOr(&ds->err, eall);
    if (it_max > 0) atomicMax(&ds->max_iter, it_max);
    if (pf) atomicAdd(&ds->n_pairs_density, pf);
    if (sums) atomicAdd(&ds->n_sums_density, sums);
    if (sums && !fb) atomicAdd(&ds->tot_sums_density, sums);
    if (cd) atomicAdd(&ds->n_cand_density, cd);
    if (walks) atomicAdd(&ds->n_rewalk, walks);
    if (ballot_any) atomicMax(&ds->leaf_state, 2);
  }
}

// ============================================================================
// Force: one wave per group.  The walk opens a node if the group box comes
// within 2 max(h_max,group, h_max,node) of it; candidates j != i with
// r < 2 max(h_i, h_j) go to a per-slot LDS list of indices; the pair loop
// then reads each neighbour's record.
// ============================================================================
template <bool MIXED>
struct FRecOf {
  using T = FRec64;
};
template <>
struct FRecOf<true> {
  using T = FRec32;
};

template <bool MIXED, int LPI>
__global__ __launch_bounds__(64) void k_force(KParams kp, Parts p,
                                              const WalkNode* __restrict__ nodes,
                                              const GroupInfo* __restrict__ groups,
                                              const void* __restrict__ frec_in,
                                              const int2* __restrict__ pool,
                                              const int32_t* __restrict__ gl_off,
                                              const int32_t* __restrict__ gl_cnt,
                                              double* __restrict__ out_ax,
                                              double* __restrict__ out_ay,
                                              double* __restrict__ out_az,
                                              double* __restrict__ out_du,
                                              const int32_t* __restrict__ flag_list,
                                              int32_t* __restrict__ walk_spill,
    DevState* __restrict__ ds) {
  int* __restrict__ spill = walk_spill + (int64_t)blockIdx.x * 2 * kSpill;
  using Rec = typename FRecOf<MIXED>::T;
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int GS = kWave / LPI;
  __shared__ WalkLds L;
  __shared__ int s_front[2][kFCap];
  __shared__ TileOf<R> T;
  __shared__ int s_j[kPMax * GS];
  const bool use_lists = ds->leaf_state == 1;
  const Rec* __restrict__ rec = reinterpret_cast<const Rec*>(frec_in);

  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  const int ng = ds->n_groups;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int chunk = (ng + 7) >> 3;
  const int gbeg = xcd * chunk, gend = min(gbeg + chunk, ng);
  uint32_t err = 0;
  unsigned long long pairs = 0, cands = 0;
  double dtmin = SPH_INF;

  // flag_list != nullptr while the neighbour lists hold every pair (leaf_state
  // 1): the list kernel does the unflagged groups, and the few flagged ones
  // are striped over all wavefronts
  const bool only_flagged = flag_list != nullptr && use_lists;
  const int g_first = only_flagged ? (int)blockIdx.x : gbeg + local;
  const int g_end = only_flagged ? ds->n_flagged : gend;
  const int g_step = only_flagged ? (int)gridDim.x : nloc;
  for (int gk = g_first; gk < g_end; gk += g_step) {
    const int g = only_flagged ? flag_list[gk] : gk;
    const GroupInfo G = groups[g];
    const bool act = slot < G.count;
    const int i = G.first + (act ? slot : 0);
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i], hi = p.h[i];
    const Rec ri = rec[i];
    float xr = 0.f, yr = 0.f, zr = 0.f;  // FP32 path: position relative to the group centre
    const float hif = (float)hi;
    if constexpr (MIXED) {
      xr = (float)fold(xi - G.c[0], kp.len[0], kp.half[0], kp.periodic[0]);
      yr = (float)fold(yi - G.c[1], kp.len[1], kp.half[1], kp.periodic[1]);
      zr = (float)fold(zi - G.c[2], kp.len[2], kp.half[2], kp.periodic[2]);
    }
    double ax = 0.0, ay = 0.0, az = 0.0, du = 0.0, vmax = 0.0;
    int npair = 0;
    // ---- pair loop over the pending list entries of each slot
    auto compute = [&]() {
      if constexpr (MIXED) {
        const float al = (float)kp.alpha, be = (float)kp.beta, au = (float)kp.alpha_u;
        const float vxi = ri.vx, vyi = ri.vy, vzi = ri.vz;
        const float hinvi = ri.hinv, h4i = ri.hinv4pi, gi = ri.g, ki = ri.k, ci = ri.c;
        const float Pi = ri.P, rhoi = ri.rho, ui = ri.u;
        const float qsx = ds->qf.step[0], qsy = ds->qf.step[1], qsz = ds->qf.step[2];
        auto pair = [&](const Rec& rj) {
          const float dx = qsep(ri.qx, rj.qx, qsx);
          const float dy = qsep(ri.qy, rj.qy, qsy);
          const float dz = qsep(ri.qz, rj.qz, qsz);
          const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          const float rinv = __builtin_amdgcn_rsqf(r2);
          const float r = r2 * rinv;
          const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
          const float w = fmaf(vzi - rj.vz, ez, fmaf(vyi - rj.vy, ey, (vxi - rj.vx) * ex));
          const float Fi = kern_df<float>(kp.kernel, r * hinvi) * h4i;
          const float Fj = kern_df<float>(kp.kernel, r * rj.hinv) * rj.hinv4pi;
          const float aw = fabsf(w);
          const bool app = w < 0.0f;
          const float vsi = fmaf(be, aw, al * ci);
          const float vsj = fmaf(be, aw, al * rj.c);
          const float ti = app ? fmaf(-0.5f * vsi * w, ki, gi) : gi;
          const float tj = app ? fmaf(-0.5f * vsj * w, rj.k, rj.g) : rj.g;
          const float pa = rj.m * fmaf(ti, Fi, tj * Fj);
          ax -= (double)(pa * ex);
          ay -= (double)(pa * ey);
          az -= (double)(pa * ez);
          const float mwF = rj.m * w * Fi;
          float e = gi * mwF;
          if (app) e = fmaf(-0.5f * ki * vsi * w, mwF, e);
          const float dP = fabsf(Pi - rj.P);
          const float vu = fast_sqrt(dP * fast_rcp(0.5f * (rhoi + rj.rho)));
          e = fmaf(rj.m * au * vu * (ui - rj.u), 0.5f * fmaf(Fi, ki, Fj * rj.k), e);
          du += (double)e;
          vmax = fmax(vmax, (double)vsi);
        };
        for (int k = sub; k < npair; k += 2 * LPI) {
          const int k2 = k + LPI;
          const bool two = k2 < npair;
          const int j1 = s_j[k * GS + slot];
          const int j2 = two ? s_j[k2 * GS + slot] : j1;
          const Rec r1 = rec[j1];
          const Rec r2 = rec[j2];
          pair(r1);
          if (two) pair(r2);
        }
      } else {
        const double al = kp.alpha, be = kp.beta, au = kp.alpha_u;
        const double vxi = ri.vx, vyi = ri.vy, vzi = ri.vz;
        const double hinvi = ri.hinv, h4i = ri.hinv4pi, gi = ri.g, ki = ri.k, ci = ri.c;
        const double Pi = ri.P, rhoi = ri.rho, ui = ri.u;
        auto pair = [&](const Rec& rj) {
          const double dx = fold(xi - rj.x, kp.len[0], kp.half[0], kp.periodic[0]);
          const double dy = fold(yi - rj.y, kp.len[1], kp.half[1], kp.periodic[1]);
          const double dz = fold(zi - rj.z, kp.len[2], kp.half[2], kp.periodic[2]);
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double r = sqrt(r2);
          const double rinv = 1.0 / r;
          const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
          const double w = fma(vzi - rj.vz, ez, fma(vyi - rj.vy, ey, (vxi - rj.vx) * ex));
          const double Fi = kern_df<double>(kp.kernel, r * hinvi) * h4i;
          const double Fj = kern_df<double>(kp.kernel, r * rj.hinv) * rj.hinv4pi;
          const double aw = fabs(w);
          const bool app = w < 0.0;
          const double vsi = fma(be, aw, al * ci);
          const double vsj = fma(be, aw, al * rj.c);
          const double ti = app ? fma(-0.5 * vsi * w, ki, gi) : gi;
          const double tj = app ? fma(-0.5 * vsj * w, rj.k, rj.g) : rj.g;
          const double pa = rj.m * fma(ti, Fi, tj * Fj);
          ax -= pa * ex;
          ay -= pa * ey;
          az -= pa * ez;
          const double mwF = rj.m * w * Fi;
          double e = gi * mwF;
          if (app) e = fma(-0.5 * ki * vsi * w, mwF, e);
          const double vu = sqrt(fabs(Pi - rj.P) / (0.5 * (rhoi + rj.rho)));
          e = fma(rj.m * au * vu * (ui - rj.u), 0.5 * fma(Fi, ki, Fj * rj.k), e);
          du += e;
          vmax = fmax(vmax, vsi);
        };
        for (int k = sub; k < npair; k += 2 * LPI) {
          const int k2 = k + LPI;
          const bool two = k2 < npair;
          const int j1 = s_j[k * GS + slot];
          const int j2 = two ? s_j[k2 * GS + slot] : j1;
          const Rec r1 = rec[j1];
          const Rec r2 = rec[j2];
          pair(r1);
          if (two) pair(r2);
        }
      }
      pairs += (act && sub == 0) ? (unsigned long long)npair : 0ull;
      npair = 0;
    };
    const double hg = G.hmax;
    auto radius = [&](const WalkNode& nd) {
      return kp.support * fmax(hg, (double)nd.hmax) * (1.0 + 4e-9);
    };
    auto flush = [&](int nleaf) {
      const int total = leaf_offsets(L, nleaf);
      cands += (unsigned long long)total * ((act && sub == 0) ? 1u : 0u);
      for_tiles<LPI, R>(L, nleaf, total, sub, p.x, p.y, p.z, p.h, T, G, kp,
                        [&](bool valid, int c) {
        // one candidate step adds at most LPI entries per slot: empty the
        // lists through the pair loop before they can overflow
        if (ballot64(npair > kPMax - LPI) != 0ull) {
          __syncthreads();
          compute();
          __syncthreads();
        }
        bool pred = false;
        const int j = valid ? T.j[c] : -1;
        if (valid && act && j != i) {
          if constexpr (MIXED) {
            const float dx = xr - T.x[c], dy = yr - T.y[c], dz = zr - T.z[c];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float hj = T.a[c];
            const float sr = (float)kp.support * fmaxf(hif, hj);
            pred = r2 < sr * sr * 1.00001f;
          } else {
            const double dx = fold(xi - T.x[c], kp.len[0], kp.half[0], kp.periodic[0]);
            const double dy = fold(yi - T.y[c], kp.len[1], kp.half[1], kp.periodic[1]);
            const double dz = fold(zi - T.z[c], kp.len[2], kp.half[2], kp.periodic[2]);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const double hj = T.a[c];
            const double sr = kp.support * (hi > hj ? hi : hj);
            pred = r2 < sr * sr;
          }
        }
        const uint64_t b = ballot64(pred);
        const uint32_t seg = (uint32_t)((b >> (slot * LPI)) & ((LPI == 64) ? ~0ull : ((1ull << LPI) - 1ull)));
        const int pos = npair + __popc(seg & ((1u << sub) - 1u));
        if (pred) s_j[pos * GS + slot] = j;
        npair += __popc(seg);
      });
      __syncthreads();
    };
    const int lcount = use_lists ? gl_cnt[g] : -1;
    if (lcount >= 0) {
      // replay the leaf list the density walk stored for this group
      const int off = gl_off[g];
      for (int b = 0; b < lcount; b += kLCap) {
        const int nl = min(kLCap, lcount - b);
        load_leaves(L, pool, off, b, nl);
        flush(nl);
      }
    } else if (!group_walk(nodes, G, kp, L, s_front, spill, radius, flush)) {
      err |= kErrFrontierForce;
    }
    __syncthreads();
    compute();
    ax = seg_sum<LPI>(ax);
    ay = seg_sum<LPI>(ay);
    az = seg_sum<LPI>(az);
    du = seg_sum<LPI>(du);
    vmax = seg_max<LPI>(vmax);
    if (act) {
      const double v0 = (kp.alpha == 0.0) ? (double)ri.c : kp.alpha * (double)ri.c;
      const double vs = fmax(vmax, v0);
      if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(du))) err |= kErrNonFinite;
      if (sub == 0) {
        out_ax[i] = ax;
        out_ay[i] = ay;
        out_az[i] = az;
        out_du[i] = du;
        p.vsig[i] = vs;
      }
      dtmin = fmin(dtmin, kp.c_cour * hi / vs);
    }
  }
  const uint64_t b = ballot64(err != 0);
  uint32_t eall = err;
  for (int d = 32; d > 0; d >>= 1) eall |= __shfl_xor(eall, d, kWave);
  unsigned long long pf = pairs, cd = cands;
  for (int d = 32; d > 0; d >>= 1) {
    pf += __shfl_xor(pf, d, kWave);
    cd += __shfl_xor(cd, d, kWave);
  }
  const double dm = wave_min_f64(dtmin);
  if (lane == 0) {
    if (b) atomicOr(&ds->err, eall);
    if (pf) atomicAdd(&ds->n_pairs_force, pf);
    if (pf && flag_list == nullptr) atomicAdd(&ds->tot_pairs_force, pf);
    if (cd) atomicAdd(&ds->n_cand_force, cd);
    if (dm < SPH_INF) dt_min_update(ds, dm);
  }
}

// ============================================================================
// Neighbour lists (Sect. 3.2).  k_lists: one wavefront per super-group of
// kSGL consecutive groups (aligned runs of the curve, hence compact).  Each
// XCD's super-groups go round its wavefronts; those left over after the last
// full round are cut into aligned units of 4, 2 or 1 groups, the largest size
// that still gives every wavefront at most one unit, so that the last round
// costs a fraction of a super-group.  The super-group's particles are loaded
// once, one per lane.  The super-group walk collects every leaf any of its
// groups can need; one pass over that list then tests each leaf against the
// box of every group of the super-group (one bit per group), so a node is
// read once per super-group.  Each group then loads the particles of its
// leaves, one candidate per lane, and for each of its particles i in turn
// appends the indices j of every candidate with
//     r_ij < 2 max(hl_i, hl_j),   hl = h_margin * (h at the start),
// to the fixed-capacity row i of nl_idx (self included): one ballot and one
// coalesced store per particle and 64 candidates, in candidate order.  As
// long as no h grows past its hl, a row is a superset of the density
// neighbours (r < 2 h_i) and of the force pairs (r < 2 max(h_i, h_j)); the
// density and force list kernels apply the exact predicates.  A group with
// an overflowing row or a failed walk is flagged (gflag = 1) and left to the
// walking kernels.  The group of every particle is kept (grp_of) for the list
// kernels, which work on chunks of consecutive particles instead of groups.
// ============================================================================

constexpr int kSGL = 8;       // groups per super-group of the list kernel
constexpr int kSLCapL = 512;  // leaves a list-kernel super-group walk may collect
constexpr int kListPer = 4;   // candidates each lane loads per list-kernel tile

// The value a wave-uniform lane `l` holds, as a wave-uniform scalar.
__device__ __forceinline__ float lane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// base + the number of set bits of m below this lane (mbcnt: two VALU ops)
__device__ __forceinline__ int rank_below(uint64_t m, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
}

// Squared search radius (support * x)^2 of the list predicate, with a
// relative slack of 1e-5 in FP32.  Every step rounds monotonically, so the
// value at max(a, b) is the larger of the values at a and at b: the pair test
// compares r^2 with the larger of the particle's and the candidate's value.
__device__ __forceinline__ float list_thr(float support, float x) {
  const float s = support * x;
  return s * s * 1.00001f;
}
__device__ __forceinline__ double list_thr(double support, double x) {
  const double s = support * x;
  return s * s;
}

template <bool MIXED, int LPI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void k_lists(KParams kp, Parts p, const WalkNode* __restrict__ nodes,
             const GroupInfo* __restrict__ groups, int32_t* __restrict__ nl_idx,
             int32_t* __restrict__ nl_len, int32_t* __restrict__ gflag,
             int32_t* __restrict__ flag_list, int32_t* __restrict__ grp_of,
             const int4* __restrict__ qrec, int32_t* __restrict__ walk_spill,
             DevState* __restrict__ ds) {
  int* __restrict__ spill = walk_spill + (int64_t)blockIdx.x * 2 * kSpill;
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int GS = kWave / LPI;  // particles per group at most
  constexpr int PER = kListPer;  // candidates per lane per tile
  static_assert(kSGL * GS <= kWave, "one lane per particle of a super-group");
  __shared__ WalkLds L;
  // the frontier is live only during walks, the leaf ranges of the
  // super-group only after its walk; a group that walks on its own (the
  // super-group's list overflowed) takes the node ids instead
  __shared__ union {
    int front[2][kFCap];
    struct {
      int first[kSLCapL];
      int cntbits[kSLCapL];  // particle count | (one bit per group) << 24
    } sl;
  } U;
  __shared__ int s_sl[kSLCapL];  // leaf node ids of the walk
  __shared__ double s_hm[kSGL];  // largest hl of each group
  // one flag per candidate of a tile: a flushed leaf's range starts there
  __shared__ alignas(4) uint8_t s_start[PER * kWave];
  const int lane = threadIdx.x;
  const int ng = ds->n_groups;
  const int nsg = (ng + kSGL - 1) / kSGL;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int chunk = (nsg + 7) >> 3;
  const int sbeg = xcd * chunk, send = min(sbeg + chunk, nsg);
  // full rounds of super-groups, then the tail [gt0, gx1) in units of tsz groups
  const int nfull = (max(send - sbeg, 0) / nloc) * nloc;
  const int gt0 = min((sbeg + nfull) * kSGL, ng), gx1 = min(send * kSGL, ng);
  int tsz = 1;
  while (tsz < kSGL && (gx1 - gt0 + tsz - 1) / tsz > nloc) tsz *= 2;
  const int nunits = nfull + (gx1 - gt0 + tsz - 1) / tsz;
  const double margin = kp.h_margin;
  const R supr = (R)kp.support, marginr = (R)margin;
  const int cap = kp.nl_cap;
  float lpf[3], ilpf[3];  // periodic lengths and their inverses in FP32 (0 on open axes)
  for (int a = 0; a < 3; ++a) {
    lpf[a] = kp.periodic[a] ? (float)kp.len[a] : 0.f;
    ilpf[a] = kp.periodic[a] ? (float)kp.inv_len[a] : 0.f;
  }
  // FP32 path: positions are code differences (the tree's fixed-point frame)
  // from the group's centre; reach bounds the list radius of every pair
  const QFrame& qf = ds->qf;
  const double reach =
      kp.support * margin * (ds->n_nodes > 0 ? (double)nodes[0].hmax : 0.0) * (1.0 + 1e-4);
  bool flagged = false;
  int nflag = 0;
  unsigned long long cands = 0;
  int walks = 0;

  for (int u = local; u < nunits; u += nloc) {
    int g0, g1;
    if (u < nfull) {
      g0 = (sbeg + u) * kSGL;
      g1 = min(g0 + kSGL, ng);
    } else {
      g0 = gt0 + (u - nfull) * tsz;
      g1 = min(g0 + tsz, gx1);
    }
    const int ngs = g1 - g0;
    GroupInfo SG;
    {
      const bool v = lane < ngs;
      GroupInfo Gk;
      if (v) Gk = groups[g0 + lane];
      for (int a = 0; a < 3; ++a) {
        const double lo = wave_min_f64(v ? Gk.c[a] - Gk.w[a] : SPH_INF);
        const double hi = wave_max_f64(v ? Gk.c[a] + Gk.w[a] : -SPH_INF);
        SG.c[a] = 0.5 * (lo + hi);
        SG.w[a] = fmax(hi - SG.c[a], SG.c[a] - lo);
      }
      SG.hmax = wave_max_f64(v ? Gk.hmax : 0.0);
      SG.first = 0;
      SG.count = 0;
    }
    // one particle per lane for the whole super-group (lane = group * GS +
    // slot): position (FP32 path: relative to its group's centre, folded) and
    // squared search radius, read as scalars by the pair loop; the largest
    // hl of each group
    const int pgk = lane / GS, psl = lane % GS;
    bool pact = false;
    int pi = 0;
    R xq = R(0), yq = R(0), zq = R(0), tq = R(0);
    {
      double hl = 0.0;
      if (pgk < ngs) {
        const GroupInfo& Gp = groups[g0 + pgk];
        pact = psl < Gp.count;
        pi = Gp.first + (pact ? psl : 0);
        const double xi = p.x[pi], yi = p.y[pi], zi = p.z[pi], hi = p.h[pi];
        if constexpr (MIXED) {
          xq = qsep(qcode(xi, qf, 0, kp.periodic[0]), qcode(Gp.c[0], qf, 0, kp.periodic[0]),
                    qf.step[0]);
          yq = qsep(qcode(yi, qf, 1, kp.periodic[1]), qcode(Gp.c[1], qf, 1, kp.periodic[1]),
                    qf.step[1]);
          zq = qsep(qcode(zi, qf, 2, kp.periodic[2]), qcode(Gp.c[2], qf, 2, kp.periodic[2]),
                    qf.step[2]);
        } else {
          xq = xi;
          yq = yi;
          zq = zi;
        }
        tq = list_thr(supr, (R)(margin * hi));
        if (pact) hl = margin * hi;
      }
      hl = seg_max<GS>(hl);
      if (psl == 0 && pgk < ngs) s_hm[pgk] = hl;
    }
    __syncthreads();
    int npv = 0;  // entries appended to this lane's particle's row so far
    int nsl = 0;
    bool sok = true;
    {
      const double hs = margin * SG.hmax;
      auto sradius = [&](const WalkNode& nd) {
        return kp.support * fmax(hs, margin * (double)nd.hmax) * (1.0 + 4e-9);
      };
      auto sflush = [&](int nleaf) {
        if (nsl + nleaf <= kSLCapL) {
          for (int q = lane; q < nleaf; q += kWave) s_sl[nsl + q] = L.lnode[q];
        } else {
          sok = false;
        }
        nsl += nleaf;
        __syncthreads();
      };
      if (!group_walk<!MIXED>(nodes, SG, kp, L, U.front, spill, sradius, sflush)) sok = false;
      __syncthreads();  // the frontier's LDS becomes the leaf ranges
      ++walks;
    }
    if (sok) {
      // each leaf against every group's box, with that group's radius; a
      // range of 2^24 particles or more (coincident keys, or a whole inner
      // node) does not fit beside the bits: the groups then walk on their own
      // two leaves per lane per trip, their node loads in flight together
      for (int base = 0; base < nsl; base += 2 * kWave) {
        const int ka = base + lane, kb = base + kWave + lane;
        const WalkNode na = nodes[s_sl[ka < nsl ? ka : 0]];
        const WalkNode nb = nodes[s_sl[kb < nsl ? kb : 0]];
        bool big = false;
        auto leaf_bits = [&](const WalkNode& nd, int k) {
          int bits = 0;
          for (int gk = 0; gk < ngs; ++gk) {
            const double rg = kp.support * fmax(s_hm[gk], margin * (double)nd.hmax) * (1.0 + 4e-9);
            if (box_gap2(nd, groups[g0 + gk], kp) < rg * rg) bits |= 1 << gk;
          }
          big = big || nd.count >= (1 << 24);
          U.sl.first[k] = nd.first;
          U.sl.cntbits[k] = (nd.count & 0xffffff) | (bits << 24);
        };
        if (ka < nsl) leaf_bits(na, ka);
        if (kb < nsl) leaf_bits(nb, kb);
        if (ballot64(big) != 0ull) sok = false;
      }
      __syncthreads();
    }
    for (int g = g0; g < g1; ++g) {
      const int gk = g - g0;
      const GroupInfo G = groups[g];
      const int cnt = G.count;
      const int l0 = gk * GS;  // lane of the group's first particle
      const double hm = s_hm[gk];
      auto radius = [&](const WalkNode& nd) {
        return kp.support * fmax(hm, margin * (double)nd.hmax) * (1.0 + 4e-9);
      };
      // FP32 path: the group centre's codes; a candidate's offset from the
      // centre is the wrapped code difference, its nearest image.  A pair's
      // difference of offsets is then the pair's nearest image whenever it
      // lies within reach, unless the group's half-width and the reach
      // together come to half a periodic length on some axis (tiny periodic
      // boxes): that group folds every pair separation instead.
      int32_t qgx = 0, qgy = 0, qgz = 0;
      bool amb = false;
      if constexpr (MIXED) {
        qgx = qcode(G.c[0], qf, 0, kp.periodic[0]);
        qgy = qcode(G.c[1], qf, 1, kp.periodic[1]);
        qgz = qcode(G.c[2], qf, 2, kp.periodic[2]);
        for (int a = 0; a < 3; ++a)
          if (kp.periodic[a] && G.w[a] + reach >= kp.half[a]) amb = true;
      }
      auto flush = [&](int nleaf) {
        const int total = leaf_offsets(L, nleaf);
        if (lane == 0) cands += (unsigned long long)total * (unsigned)cnt;
        // leaves hold at least one particle each (tree cells are cut from
        // the sorted keys), so the leaf of candidate c is the number of leaf
        // ranges starting at or before c, less one
        int lt = -1;  // leaf of the candidate before the tile
        for (int c0 = 0; c0 < total; c0 += PER * kWave) {
          const int cn = min(PER * kWave, total - c0);
          // flag the starts of the leaf ranges within the tile
          static_assert(PER * kWave % (4 * kWave) == 0, "whole dwords per lane");
#pragma unroll
          for (int w = 0; w < PER / 4; ++w) reinterpret_cast<int*>(s_start)[lane + w * kWave] = 0;
          __syncthreads();
          for (int l = lt + 1 + lane;; l += kWave) {
            const int o = l < nleaf ? L.loff[l] - c0 : cn;
            const bool in = o < cn;
            if (in && o >= 0) s_start[o] = 1;
            if (ballot64(in) != ~0ull) break;
          }
          __syncthreads();
          // resolve this lane's candidates, then issue all their loads
          int jj[PER];
#pragma unroll
          for (int q = 0; q < PER; ++q) {
            const int t = lane + q * kWave;
            const int st = t < cn ? (int)s_start[t] : 0;
            const uint64_t b = ballot64(st != 0);
            const int lo = rank_below(b, lt + st);
            lt += popc64(b);
            jj[q] = t < cn ? L.lfirst[lo] + (c0 + t - L.loff[lo]) : -1;
          }
          R cx[PER], cy[PER], cz[PER], ct[PER];
          if constexpr (MIXED) {
            // one 16-byte load per candidate: its position codes and its h
            int4 v[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) v[q] = qrec[jj[q] >= 0 ? jj[q] : 0];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
              cx[q] = qsep(v[q].x, qgx, qf.step[0]);
              cy[q] = qsep(v[q].y, qgy, qf.step[1]);
              cz[q] = qsep(v[q].z, qgz, qf.step[2]);
              ct[q] = list_thr(supr, marginr * __int_as_float(v[q].w));
            }
          } else {
            double vx[PER], vy[PER], vz[PER], vh[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
              const int j = jj[q] >= 0 ? jj[q] : 0;
              vx[q] = p.x[j];
              vy[q] = p.y[j];
              vz[q] = p.z[j];
              vh[q] = p.h[j];
            }
#pragma unroll
            for (int q = 0; q < PER; ++q) {
              cx[q] = vx[q];
              cy[q] = vy[q];
              cz[q] = vz[q];
              ct[q] = list_thr(supr, marginr * (R)vh[q]);
            }
          }
          uint64_t vm[PER];  // lanes holding a candidate, per quarter of the tile
#pragma unroll
          for (int q = 0; q < PER; ++q) vm[q] = ballot64(jj[q] >= 0);
          // particle-major: each particle's values are read from its lane once
          // per tile; its row gets the tile's candidates in order
          auto particles = [&](auto fold_pairs) {
            constexpr bool FOLD = decltype(fold_pairs)::value;
            for (int s = 0; s < cnt; ++s) {
              const int ls = l0 + s;
              const R px = lane_val(xq, ls), py = lane_val(yq, ls), pz = lane_val(zq, ls);
              const R pt = lane_val(tq, ls);
              int32_t* __restrict__ row = nl_idx + (int64_t)(G.first + s) * cap;
              int n = __builtin_amdgcn_readlane(npv, ls);
#pragma unroll
              for (int q = 0; q < PER; ++q) {
                if (q * kWave < cn) {
                  // one compare per ballot; candidates past the tile's end
                  // are masked out afterwards (scalar AND)
                  bool hit;
                  if constexpr (MIXED) {
                    float dx = px - cx[q], dy = py - cy[q], dz = pz - cz[q];
                    if constexpr (FOLD) {
                      dx = fmaf(-lpf[0], rintf(dx * ilpf[0]), dx);
                      dy = fmaf(-lpf[1], rintf(dy * ilpf[1]), dy);
                      dz = fmaf(-lpf[2], rintf(dz * ilpf[2]), dz);
                    }
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    // r2 and the radii are >= 0: their bit patterns order
                    // like their values (an integer max needs no NaN care)
                    hit = __float_as_int(r2) < max(__float_as_int(pt), __float_as_int(ct[q]));
                  } else {
                    const double dx = fold(px - cx[q], kp.len[0], kp.half[0], kp.periodic[0]);
                    const double dy = fold(py - cy[q], kp.len[1], kp.half[1], kp.periodic[1]);
                    const double dz = fold(pz - cz[q], kp.len[2], kp.half[2], kp.periodic[2]);
                    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    hit = r2 < fmax(pt, ct[q]);
                  }
                  const bool pred = hit & (jj[q] >= 0);
                  const uint64_t b = ballot64(hit) & vm[q];
                  const int pos = rank_below(b, n);
                  if (pred & (pos < cap)) row[(unsigned)pos] = jj[q];
                  n += popc64(b);
                }
              }
              npv = lane == ls ? n : npv;
            }
          };
          if (MIXED && amb)
            particles(std::true_type{});
          else
            particles(std::false_type{});
        }
        __syncthreads();  // L is refilled next
      };
      bool gok = sok;
      if (sok) {
        int nleaf = 0;
        for (int base = 0; base < nsl; base += kWave) {
          const int k = base + lane;
          const bool open = k < nsl && ((U.sl.cntbits[k] >> (24 + gk)) & 1);
          const uint64_t lb = ballot64(open);
          const int nl = popc64(lb);
          if (nleaf + nl > kLCap) {
            flush(nleaf);
            nleaf = 0;
          }
          if (open) {
            const int pos = nleaf + popc64(lb & lanemask_lt());
            L.lfirst[pos] = U.sl.first[k];
            L.lcnt[pos] = U.sl.cntbits[k] & 0xffffff;
            L.lnode[pos] = s_sl[k];
          }
          nleaf += nl;
          __syncthreads();
        }
        if (nleaf > 0) flush(nleaf);
      } else {
        // the super-group's leaf list overflowed: the group walks for its
        // own leaf list; a group whose list overflows too is left to the
        // walking kernels
        int ngl = 0;
        gok = true;
        auto gflush = [&](int nleaf) {
          if (ngl + nleaf <= kSLCapL) {
            for (int q = lane; q < nleaf; q += kWave) s_sl[ngl + q] = L.lnode[q];
          } else {
            gok = false;
          }
          ngl += nleaf;
          __syncthreads();
        };
        if (!group_walk<!MIXED>(nodes, G, kp, L, U.front, spill, radius, gflush)) gok = false;
        __syncthreads();
        ++walks;
        if (gok) list_walk(nodes, s_sl, ngl, G, kp, L, radius, flush);
      }
      const bool mine = lane >= l0 && lane < l0 + cnt;
      const bool bad = !gok || ballot64(mine && npv > cap) != 0ull;
      if (lane == 0) {
        gflag[g] = bad ? 1 : 0;
        if (bad) flag_list[atomicAdd(&ds->n_flagged, 1)] = g;
      }
      flagged |= bad;
      nflag += bad ? 1 : 0;
    }
    if (pact) {
      nl_len[pi] = npv;
      grp_of[pi] = g0 + pgk;
    }
  }
  unsigned long long cd = cands;
  for (int d = 32; d > 0; d >>= 1) cd += __shfl_xor(cd, d, kWave);
  if (lane == 0) {
    if (cd) atomicAdd(&ds->n_cand_density, cd);
    if (cd) atomicAdd(&ds->tot_cand_lists, cd);
    if (walks) atomicAdd(&ds->n_rewalk, walks);
    if (flagged) {
      atomicOr(&ds->lists_missing, 1);
      atomicAdd(&ds->n_flag_rows, nflag);
    }
  }
}

// Groups of this wave under the XCD-aware static schedule: block b works on
// the contiguous eighth of the groups that belongs to XCD b mod 8.
struct GroupRange {
  int beg, end, step;
};
__device__ __forceinline__ GroupRange xcd_groups(int ng) {
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int chunk = (ng + 7) >> 3;
  const int gbeg = xcd * chunk;
  return GroupRange{gbeg + local, min(gbeg + chunk, ng), nloc};
}

// ============================================================================
// Density from the neighbour lists (Sect. 2.2, Sect. 3.2.1): one wavefront
// per group, LPI lanes per particle.  Each lane gathers the separations and
// masses of its share of the row once (registers), then the h iteration
// re-sums them: Newton-Raphson on f(h) = S0(h) - m (hfact/h)^3 with the same
// safeguards as the walking kernel, a wavefront ballot deciding when the
// group is done.  A group in which some h passes hl (its rows may then miss
// neighbours) is flagged (gflag = 2) for the walking kernel, and the force
// pass then walks for every group (leaf_state 2).
// ============================================================================
// LDS slot of row entry k of particle slot s in the list density kernel's
// entry arrays (GS slots per entry).  A lane reads entries k = sub + LPI t, so
// the 32 lanes of a half-wavefront span 32 / GS consecutive values of sub;
// flipping the slot's top bit on every other run of 32 / GS entries puts
// them in 32 distinct banks.
template <int GS>
__device__ __forceinline__ int ent_idx(int k, int s) {
  return k * GS + (s ^ ((GS / 2) * ((k * GS / 32) & 1)));
}

template <bool MIXED, int LPI, int CAP, int KIND>
__global__ __launch_bounds__(64) void k_density_lists(KParams kp, Parts p,
                                                      const GroupInfo* __restrict__ groups,
                                                      const int32_t* __restrict__ nl_idx,
                                                      const int32_t* __restrict__ nl_len,
                                                      int32_t* __restrict__ gflag,
                                                      int32_t* __restrict__ flag_list,
                                                      const int32_t* __restrict__ grp_of,
                                                      const void* __restrict__ pos,
                                                      void* __restrict__ frec_out,
                                                      DevState* __restrict__ ds) {
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int E = CAP / LPI;  // row entries per lane (CAP = kp.nl_cap)
  constexpr int GS = kWave / LPI;
  __shared__ R s_r[CAP * GS];  // separation and mass of row entry k of slot s at ent_idx(k, s)
  __shared__ R s_m[CAP * GS];
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  constexpr int CS = kWave / LPI;  // particles per chunk
  const int nch = (kp.n + CS - 1) / CS;
  const GroupRange gr = xcd_groups(nch);
  const double margin = kp.h_margin;
  double minhalf = SPH_INF;
  for (int a = 0; a < 3; ++a)
    if (kp.periodic[a]) minhalf = fmin(minhalf, kp.half[a]);
  uint32_t err = 0;
  int it_max = 0;
  unsigned long long pairs_final = 0, sums = 0;
  bool outgrew_any = false;
  int ngrew = 0;
  // gathered per row entry: x, y, z, m (FP64), or position codes and m (mixed)
  const double4* __restrict__ xyzm = reinterpret_cast<const double4*>(pos);
  const int4* __restrict__ qpos = reinterpret_cast<const int4*>(pos);
  const QFrame& qf = ds->qf;

  for (int g = gr.beg; g < gr.end; g += gr.step) {
    const int first = g * CS, count = min(CS, kp.n - first);
    const bool inr = slot < count;
    const int i = first + (inr ? slot : 0);
    // particles of groups the list kernel flagged are left to the walking kernel
    const int gi = grp_of[i];
    const bool act = inr && gflag[gi] == 0;
    if (ballot64(act) == 0ull) continue;
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i], mi = p.m[i];
    int32_t qxi = 0, qyi = 0, qzi = 0;  // mixed: i's position codes
    if constexpr (MIXED) {
      qxi = qcode(xi, qf, 0, kp.periodic[0]);
      qyi = qcode(yi, qf, 1, kp.periodic[1]);
      qzi = qcode(zi, qf, 2, kp.periodic[2]);
    }
    double h = p.h[i];
    if (!(h > 0.0) || !isfinite(h)) {
      err |= kErrNonFinite;
      h = 1.0;
    }
    const double hl = margin * h;
    const int len = act ? nl_len[i] : 0;
    const int32_t* __restrict__ row = nl_idx + (int64_t)i * CAP;
    int lmax = len;
    for (int d = 32; d > 0; d >>= 1) lmax = max(lmax, __shfl_xor(lmax, d, kWave));
    // ---- gather: separation and mass of every row entry into LDS, four
    // entries per lane at a time (their loads in flight together)
    for (int t0 = 0; t0 < E; t0 += 4) {
      if (__builtin_amdgcn_readfirstlane(t0 * LPI) >= lmax) break;
      int jj[4];
      bool vv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = sub + LPI * (t0 + q);
        vv[q] = k < len;
        jj[q] = vv[q] ? row[k] : i;
      }
      // every slot is computed and stored (entries past the row's length sit
      // below CAP and are never read): a conditional use would let the
      // compiler sink each load into it and serialise the four gathers
      if constexpr (MIXED) {
        int4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = qpos[jj[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = sub + LPI * (t0 + q);
          const float fx = qsep(qxi, v[q].x, qf.step[0]);
          const float fy = qsep(qyi, v[q].y, qf.step[1]);
          const float fz = qsep(qzi, v[q].z, qf.step[2]);
          s_r[ent_idx<GS>(k, slot)] = fast_sqrt(fmaf(fz, fz, fmaf(fy, fy, fx * fx)));
          s_m[ent_idx<GS>(k, slot)] = __int_as_float(v[q].w);
        }
      } else {
        double gx[4], gy[4], gz[4], gm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double4 v = xyzm[jj[q]];
          gx[q] = v.x;
          gy[q] = v.y;
          gz[q] = v.z;
          gm[q] = v.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = sub + LPI * (t0 + q);
          const double dx = fold(xi - gx[q], kp.len[0], kp.half[0], kp.periodic[0]);
          const double dy = fold(yi - gy[q], kp.len[1], kp.half[1], kp.periodic[1]);
          const double dz = fold(zi - gz[q], kp.len[2], kp.half[2], kp.periodic[2]);
          s_r[ent_idx<GS>(k, slot)] = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
          s_m[ent_idx<GS>(k, slot)] = gm[q];
        }
      }
    }
    // ---- h iteration over the gathered entries
    double hlo = 0.0, hhi = SPH_INF;
    bool conv = !act, outgrew = false;
    int nit = 0;
    double S0 = 0.0, S1 = 0.0;
    uint32_t nnb = 0;
    while (true) {
      const double hinv = 1.0 / h;
      double a0 = 0.0, a1 = 0.0;
      uint32_t cnt = 0;
      if constexpr (MIXED) {
        // each lane sums its few terms in FP32; lanes are combined in FP64
        const float hinvf = (float)hinv, twohf = (float)(kp.support * h);
        float s0 = 0.f, s1 = 0.f;
        for (int k = sub; k < len; k += LPI) {
          const float r = s_r[ent_idx<GS>(k, slot)], m = s_m[ent_idx<GS>(k, slot)];
          const float q = r * hinvf;
          float f, df;
          kf_df<KIND, float>(q, f, df);
          s0 = fmaf(m, f, s0);
          s1 = fmaf(m, fmaf(q, df, 3.0f * f), s1);
          cnt += (r < twohf) ? 1u : 0u;
        }
        a0 = (double)s0;
        a1 = (double)s1;
      } else {
        const double twoh = kp.support * h;
        for (int k = sub; k < len; k += LPI) {
          const double r = s_r[ent_idx<GS>(k, slot)], m = s_m[ent_idx<GS>(k, slot)];
          const double q = r * hinv;
          double f, df;
          kf_df<KIND, double>(q, f, df);
          a0 = fma(m, f, a0);
          a1 = fma(m, fma(q, df, 3.0 * f), a1);
          cnt += (r < twoh) ? 1u : 0u;
        }
      }
      a0 = seg_sum<LPI>(a0);
      a1 = seg_sum<LPI>(a1);
      cnt = seg_sum_u32<LPI>(cnt);
      const double h3 = hinv * hinv * hinv;
      S0 = a0 * h3 * kp.knorm;
      S1 = -a1 * h3 * hinv * kp.knorm;
      nnb = cnt;
      sums += (act && sub == 0) ? (unsigned long long)cnt : 0ull;
      bool moved = false;
      if (!conv) {
        const double t = kp.hfact * hinv;
        const double rh = mi * (t * t * t);
        const double f = S0 - rh;
        const double fp = S1 + 3.0 * rh * hinv;
        double hn = h;
        if (kp.fixed_passes) {
          hn = h - f / fp;
          if (!(fp > 0.0))
            hn = h;
          else if (hn > 1.2 * h)
            hn = 1.2 * h;
          else if (hn < 0.8 * h)
            hn = 0.8 * h;
          // three density computations (Sect. 3.2.1): two updates, then
          // rho and Omega from the third sum at the h it used
          conv = (nit + 1) >= 2;
          moved = true;
        } else if (fabs(f) <= 3.0 * kp.h_tol * rh) {
          conv = true;
        } else {
          if (f < 0.0)
            hlo = fmax(hlo, h);
          else
            hhi = fmin(hhi, h);
          hn = h - f / fp;
          const bool bad = !(fp > 0.0) || !(hn >= 0.8 * h) || !(hn <= 1.2 * h) ||
                           !(hn > hlo) || !(hn < hhi);
          if (bad) {
            if (hlo > 0.0 && hhi < SPH_INF)
              hn = 0.5 * (hlo + hhi);
            else
              hn = (f < 0.0) ? 1.2 * h : h / 1.2;
          }
          conv = fabs(hn - h) <= 4e-16 * h;
          moved = true;
        }
        if (moved) {
          h = hn;
          if (h > hl) outgrew = true;
          ++nit;
          if (nit > kp.max_iter) {
            err |= kErrNoConv;
            conv = true;
          }
        }
      }
      if (ballot64(outgrew) != 0ull) break;  // rows too short: the walking kernel redoes it
      if (ballot64(!conv || moved) == 0ull) break;
    }
    if (ballot64(outgrew) != 0ull) {
      // the groups of every particle of this chunk go to the walking kernel
      if (act && sub == 0 && atomicCAS(&gflag[gi], 0, 2) == 0) {
        flag_list[atomicAdd(&ds->n_flagged, 1)] = gi;
        ++ngrew;
      }
      outgrew_any = true;
      continue;
    }
    it_max = max(it_max, nit + 1);
    if (act) {
      density_outputs<MIXED>(kp, p, frec_out, i, xi, yi, zi, mi, h, S0, S1, minhalf, err,
                             sub == 0, ds);
      if (sub == 0) pairs_final += nnb;
    }
  }
  const uint64_t b = ballot64(err != 0);
  uint32_t eall = err;
  for (int d = 32; d > 0; d >>= 1) eall |= __shfl_xor(eall, d, kWave);
  unsigned long long pf = pairs_final, sm = sums;
  for (int d = 32; d > 0; d >>= 1) {
    pf += __shfl_xor(pf, d, kWave);
    sm += __shfl_xor(sm, d, kWave);
    ngrew += __shfl_xor(ngrew, d, kWave);
  }
  outgrew_any = ballot64(outgrew_any) != 0ull;
  if (lane == 0) {
    if (b) atomicOr(&ds->err, eall);
    if (it_max > 0) atomicMax(&ds->max_iter, it_max);
    if (pf) atomicAdd(&ds->n_pairs_density, pf);
    if (sm) atomicAdd(&ds->n_sums_density, sm);
    if (sm) atomicAdd(&ds->tot_sums_density, sm);
    if (outgrew_any) {
      atomicMax(&ds->leaf_state, 2);
      atomicOr(&ds->lists_missing, 1);
      atomicAdd(&ds->n_flag_grew, ngrew);
    }
  }
}

// ============================================================================
// Force from the neighbour lists (Sect. 2.4-2.6): one wavefront per group,
// LPI lanes per particle, each lane walking its share of row i.  The exact
// pair predicate (j != i, r < 2 max(h_i, h_j) with the converged h) is applied
// to every entry; accepted pairs add the pressure, viscosity and conductivity
// terms.  Runs only while every row is complete (leaf_state 1); flagged
// groups are left to the walking kernel.
// ============================================================================
template <bool MIXED, int LPI, int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void k_force_lists(KParams kp, Parts p,
                                                    const GroupInfo* __restrict__ groups,
                                                    const void* __restrict__ frec_in,
                                                    const int32_t* __restrict__ nl_idx,
                                                    const int32_t* __restrict__ nl_len,
                                                    const int32_t* __restrict__ gflag,
                                                    const int32_t* __restrict__ grp_of,
                                                    double* __restrict__ out_ax,
                                                    double* __restrict__ out_ay,
                                                    double* __restrict__ out_az,
                                                    double* __restrict__ out_du,
                                                    DevState* __restrict__ ds) {
  if (ds->leaf_state != 1) return;
  using Rec = typename FRecOf<MIXED>::T;
  const Rec* __restrict__ rec = reinterpret_cast<const Rec*>(frec_in);
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  constexpr int CS = kWave / LPI;  // particles per chunk
  const int nch = (kp.n + CS - 1) / CS;
  const GroupRange gr = xcd_groups(nch);
  uint32_t err = 0;
  unsigned long long pairs = 0, cands = 0;
  double dtmin = SPH_INF;

  for (int g = gr.beg; g < gr.end; g += gr.step) {
    const int first = g * CS, count = min(CS, kp.n - first);
    const bool inr = slot < count;
    const int i = first + (inr ? slot : 0);
    // particles of flagged groups are left to the walking kernel
    const bool act = inr && gflag[grp_of[i]] == 0;
    if (ballot64(act) == 0ull) continue;
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i], hi = p.h[i];
    const Rec ri = rec[i];
    const int len = act ? nl_len[i] : 0;
    const int32_t* __restrict__ row = nl_idx + (int64_t)i * kp.nl_cap;
    int lmax = len;
    for (int d = 32; d > 0; d >>= 1) lmax = max(lmax, __shfl_xor(lmax, d, kWave));
    cands += (act && sub == 0) ? (unsigned long long)len : 0ull;
    double ax = 0.0, ay = 0.0, az = 0.0, du = 0.0, vmax = 0.0;
    if constexpr (MIXED) {
      const float al = (float)kp.alpha, be = (float)kp.beta, hau = (float)(0.5 * kp.alpha_u);
      const float vxi = ri.vx, vyi = ri.vy, vzi = ri.vz, hif = (float)hi;
      const float hinvi = ri.hinv, h4i = ri.hinv4pi, gi = ri.g, ki = ri.k;
      const float Pi = ri.P, rhoi = ri.rho, ui = ri.u;
      const float aci = al * ri.c, nhki = -0.5f * ki, S = (float)kp.support;
      // per-lane sums in FP32 (a lane takes one in LPI of the row's pairs),
      // combined across the slot's lanes in FP64 below
      float fax = 0.f, fay = 0.f, faz = 0.f, fdu = 0.f, fvmax = 0.f;
      uint32_t npr = 0;
      // The pair terms of eq:acc and eq:energy with the switch w_ = min(w, 0)
      // of the approaching pairs (w = v_ij . e_ij):
      //   t_i = g_i - k_i vsig_i w_ / 2,  A_i = t_i m_j F_i,  pa = A_i + t_j m_j F_j,
      //   a_i -= pa e_ij,  du_i += w A_i + (alpha_u / 2) v^u (u_i - u_j)
      //                                   (k_i m_j F_i + k_j m_j F_j);
      // the viscous heating of an approaching pair is the w_ part of w A_i.
      // The FP32 support test is settled in FP64 near its boundary, so the
      // accepted pairs are those of the FP64 predicate.
      const float qsx = ds->qf.step[0], qsy = ds->qf.step[1], qsz = ds->qf.step[2];
      auto pair = [&](const Rec& rj, int j) {
        const float dx = qsep(ri.qx, rj.qx, qsx);
        const float dy = qsep(ri.qy, rj.qy, qsy);
        const float dz = qsep(ri.qz, rj.qz, qsz);
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float sr = S * fmaxf(hif, rj.h);
        const float sr2 = sr * sr;
        bool in = r2 < sr2;
        const bool border = fabsf(r2 - sr2) <= kBorder * sr2;
        if (ballot64(border) != 0ull)
          if (border) in = exact_pair(kp, p.x, p.y, p.z, p.h, i, j, true);
        if (!in) return;
        ++npr;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;
        const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const float w = fmaf(vzi - rj.vz, ez, fmaf(vyi - rj.vy, ey, (vxi - rj.vx) * ex));
        const float mFi = rj.m * (kdf<KIND, float>(r * hinvi) * h4i);
        const float mFj = kdf<KIND, float>(r * rj.hinv) * (rj.m * rj.hinv4pi);
        const float aw = fabsf(w), wn = fminf(w, 0.f);
        const float vsi = fmaf(be, aw, aci);
        const float vsj = fmaf(be, aw, al * rj.c);
        const float ti = fmaf(nhki * vsi, wn, gi);
        const float tj = fmaf(-0.5f * rj.k * vsj, wn, rj.g);
        const float Ai = ti * mFi;
        const float pa = fmaf(tj, mFj, Ai);
        fax = fmaf(-pa, ex, fax);
        fay = fmaf(-pa, ey, fay);
        faz = fmaf(-pa, ez, faz);
        const float vu = fast_sqrt(fabsf(Pi - rj.P) * fast_rcp(0.5f * (rhoi + rj.rho)));
        const float X = fmaf(mFi, ki, mFj * rj.k);
        fdu = fmaf(w, Ai, fmaf(hau * vu * (ui - rj.u), X, fdu));
        fvmax = fmaxf(fvmax, vsi);
      };
      // row indices one iteration ahead, so that each iteration waits for
      // one gather of the two records only
      int j1 = (sub < len) ? row[sub] : i;
      int j2 = (sub + LPI < len) ? row[sub + LPI] : i;
      for (int k = sub; k < lmax; k += 2 * LPI) {
        const bool v1 = k < len, v2 = k + LPI < len;
        Rec r1, r2;
        if (v1) r1 = rec[j1];
        if (v2) r2 = rec[j2];
        const int kn = k + 2 * LPI;
        const int jn1 = (kn < len) ? row[kn] : i;
        const int jn2 = (kn + LPI < len) ? row[kn + LPI] : i;
        if (v1 && j1 != i) pair(r1, j1);
        if (v2 && j2 != i) pair(r2, j2);
        j1 = jn1;
        j2 = jn2;
      }
      ax = fax;
      ay = fay;
      az = faz;
      du = fdu;
      vmax = fvmax;
      pairs += npr;
    } else {
      const double al = kp.alpha, be = kp.beta, au = kp.alpha_u;
      const double vxi = ri.vx, vyi = ri.vy, vzi = ri.vz;
      const double hinvi = ri.hinv, h4i = ri.hinv4pi, gi = ri.g, ki = ri.k, ci = ri.c;
      const double Pi = ri.P, rhoi = ri.rho, ui = ri.u;
      auto pair = [&](const Rec& rj) {
        const double dx = fold(xi - rj.x, kp.len[0], kp.half[0], kp.periodic[0]);
        const double dy = fold(yi - rj.y, kp.len[1], kp.half[1], kp.periodic[1]);
        const double dz = fold(zi - rj.z, kp.len[2], kp.half[2], kp.periodic[2]);
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double sr = kp.support * (hi > rj.h ? hi : rj.h);
        if (!(r2 < sr * sr)) return;
        ++pairs;
        const double r = sqrt(r2);
        const double rinv = 1.0 / r;
        const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const double w = fma(vzi - rj.vz, ez, fma(vyi - rj.vy, ey, (vxi - rj.vx) * ex));
        const double Fi = kdf<KIND, double>(r * hinvi) * h4i;
        const double Fj = kdf<KIND, double>(r * rj.hinv) * rj.hinv4pi;
        const double aw = fabs(w);
        const bool app = w < 0.0;
        const double vsi = fma(be, aw, al * ci);
        const double vsj = fma(be, aw, al * rj.c);
        const double ti = app ? fma(-0.5 * vsi * w, ki, gi) : gi;
        const double tj = app ? fma(-0.5 * vsj * w, rj.k, rj.g) : rj.g;
        const double pa = rj.m * fma(ti, Fi, tj * Fj);
        ax -= pa * ex;
        ay -= pa * ey;
        az -= pa * ez;
        const double mwF = rj.m * w * Fi;
        double e = gi * mwF;
        if (app) e = fma(-0.5 * ki * vsi * w, mwF, e);
        const double vu = sqrt(fabs(Pi - rj.P) / (0.5 * (rhoi + rj.rho)));
        e = fma(rj.m * au * vu * (ui - rj.u), 0.5 * fma(Fi, ki, Fj * rj.k), e);
        du += e;
        vmax = fmax(vmax, vsi);
      };
      // one 128-byte record in flight per lane (registers); row index one
      // iteration ahead
      int j = (sub < len) ? row[sub] : i;
      for (int k = sub; k < lmax; k += LPI) {
        const bool v = k < len;
        const Rec rj = rec[j];
        const int jn = (k + LPI < len) ? row[k + LPI] : i;
        if (v && j != i) pair(rj);
        j = jn;
      }
    }
    ax = seg_sum<LPI>(ax);
    ay = seg_sum<LPI>(ay);
    az = seg_sum<LPI>(az);
    du = seg_sum<LPI>(du);
    vmax = seg_max<LPI>(vmax);
    if (act) {
      const double v0 = (kp.alpha == 0.0) ? (double)ri.c : kp.alpha * (double)ri.c;
      const double vs = fmax(vmax, v0);
      if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(du))) err |= kErrNonFinite;
      if (sub == 0) {
        out_ax[i] = ax;
        out_ay[i] = ay;
        out_az[i] = az;
        out_du[i] = du;
        p.vsig[i] = vs;
      }
      dtmin = fmin(dtmin, kp.c_cour * hi / vs);
    }
  }
  const uint64_t b = ballot64(err != 0);
  uint32_t eall = err;
  for (int d = 32; d > 0; d >>= 1) eall |= __shfl_xor(eall, d, kWave);
  unsigned long long pf = pairs, cd = cands;
  for (int d = 32; d > 0; d >>= 1) {
    pf += __shfl_xor(pf, d, kWave);
    cd += __shfl_xor(cd, d, kWave);
  }
  const double dm = wave_min_f64(dtmin);
  if (lane == 0) {
    if (b) atomicOr(&ds->err, eall);
    if (pf) atomicAdd(&ds->n_pairs_force, pf);
    if (pf) atomicAdd(&ds->tot_pairs_force, pf);
    if (cd) atomicAdd(&ds->n_cand_force, cd);
    if (dm < SPH_INF) dt_min_update(ds, dm);
  }
}

// ============================================================================
// The pairs the list kernels accept (Sect. 3.2), for inspection and for the
// adjoint's frozen neighbour sets: each particle's row filtered with the
// exact FP64 predicate at the h in p.h (the mixed force kernel settles its
// FP32 test in FP64 near the boundary, so it accepts the same pairs); mode
// 0: density set (r < S h_i, self included), 1: force set (j != i,
// r < S max(h_i, h_j)).  Particles of flagged groups (incomplete rows) get
// the count -1.  Indices are written at offsets[i] in row order.
// ============================================================================
template <int LPI>
__global__ __launch_bounds__(64) void k_row_sets(KParams kp, Parts p, int mode,
                                                 const int32_t* __restrict__ nl_idx,
                                                 const int32_t* __restrict__ nl_len,
                                                 const int32_t* __restrict__ gflag,
                                                 const int32_t* __restrict__ grp_of,
                                                 int32_t* __restrict__ counts,
                                                 int32_t* __restrict__ idx,
                                                 const int64_t* __restrict__ offsets) {
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  constexpr int CS = kWave / LPI;
  const int nch = (kp.n + CS - 1) / CS;
  const GroupRange gr = xcd_groups(nch);
  for (int g = gr.beg; g < gr.end; g += gr.step) {
    const int first = g * CS, count = min(CS, kp.n - first);
    const bool inr = slot < count;
    const int i = first + (inr ? slot : 0);
    const bool act = inr && gflag[grp_of[i]] == 0;
    const int len = act ? min(nl_len[i], kp.nl_cap) : 0;
    int lmax = len;
    for (int d = 32; d > 0; d >>= 1) lmax = max(lmax, __shfl_xor(lmax, d, kWave));
    const int32_t* __restrict__ row = nl_idx + (int64_t)i * kp.nl_cap;
    const int64_t base = (act && idx) ? offsets[i] : 0;
    int n = 0;  // accepted entries of this slot so far (uniform over the slot's lanes)
    for (int k0 = 0; k0 < lmax; k0 += LPI) {
      const int k = k0 + sub;
      bool hit = false;
      int j = i;
      if (k < len) {
        j = row[k];
        hit = exact_pair(kp, p.x, p.y, p.z, p.h, i, j, mode == 1) && (mode == 0 || j != i);
      }
      const uint64_t b = ballot64(hit);
      const uint32_t seg = (uint32_t)(b >> (slot * LPI)) & ((1u << LPI) - 1u);
      if (hit && idx) idx[base + n + __popc(seg & ((1u << sub) - 1u))] = j;
      n += __popc(seg);
    }
    if (inr && sub == 0) counts[i] = act ? n : -1;
  }
}

// ============================================================================
// Neighbour sets for inspection: the same walk, the exact FP64 predicates,
// counts (idx == nullptr) or indices written at offsets[i].
// ============================================================================
template <int LPI>
__global__ __launch_bounds__(64) void k_neighbours(KParams kp, Parts p, int mode,
                                                   const WalkNode* __restrict__ nodes,
                                                   const GroupInfo* __restrict__ groups,
                                                   int32_t* __restrict__ counts,
                                                   const int64_t* __restrict__ offsets,
                                                   int32_t* __restrict__ idx,
                                                   int32_t* __restrict__ walk_spill,
    DevState* __restrict__ ds) {
  int* __restrict__ spill = walk_spill + (int64_t)blockIdx.x * 2 * kSpill;
  __shared__ WalkLds L;
  __shared__ int s_front[2][kFCap];
  __shared__ TileOf<double> T;
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  const int ng = ds->n_groups;
  uint32_t err = 0;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    const GroupInfo G = groups[g];
    const bool act = slot < G.count;
    const int i = G.first + (act ? slot : 0);
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i], hi = p.h[i];
    int cnt = 0;
    const double hg = G.hmax;
    auto radius = [&](const WalkNode& nd) {
      return kp.support * (mode == 1 ? fmax(hg, (double)nd.hmax) : hg) * (1.0 + 4e-9);
    };
    auto flush = [&](int nleaf) {
      const int total = leaf_offsets(L, nleaf);
      for_tiles<LPI, double>(L, nleaf, total, sub, p.x, p.y, p.z, p.h, T, G, kp,
                             [&](bool valid, int c) {
        bool pred = false;
        const int j = valid ? T.j[c] : -1;
        if (valid && act) {
          const double dx = fold(xi - T.x[c], kp.len[0], kp.half[0], kp.periodic[0]);
          const double dy = fold(yi - T.y[c], kp.len[1], kp.half[1], kp.periodic[1]);
          const double dz = fold(zi - T.z[c], kp.len[2], kp.half[2], kp.periodic[2]);
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          if (mode == 0) {
            const double s = kp.support * hi;
            pred = r2 < s * s;
          } else {
            const double hj = T.a[c];
            const double s = kp.support * (hi > hj ? hi : hj);
            pred = (j != i) && r2 < s * s;
          }
        }
        const uint64_t b = ballot64(pred);
        const uint32_t seg = (uint32_t)((b >> (slot * LPI)) & ((LPI == 64) ? ~0ull : ((1ull << LPI) - 1ull)));
        const int pos = cnt + __popc(seg & ((1u << sub) - 1u));
        if (pred && idx) idx[offsets[i] + pos] = j;
        cnt += __popc(seg);
      });
      __syncthreads();
    };
    if (!group_walk(nodes, G, kp, L, s_front, spill, radius, flush)) err |= kErrFrontier;
    if (act && sub == 0 && !idx) counts[i] = cnt;
  }
  if (err) atomicOr(&ds->err, err);
}

// ============================================================================
// Integration and reductions (one thread per particle)
// ============================================================================
__global__ void k_set_leaf_state(DevState* ds, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ds->leaf_state = v;
    ds->lists_missing = 0;
    ds->n_flag_rows = 0;
    ds->n_flag_grew = 0;
    ds->n_flagged = 0;
  }
}

__global__ void k_reset_force_state(DevState* ds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ds->dt_min_enc = enc_f64(SPH_INF);
}

__device__ __forceinline__ void clear_counters(DevState* ds) {
  ds->max_iter = 0;
  ds->n_pairs_density = 0;
  ds->n_pairs_force = 0;
  ds->n_sums_density = 0;
  ds->n_cand_density = 0;
  ds->n_cand_force = 0;
  ds->n_rewalk = 0;
  ds->leaf_state = 0;
  ds->lists_missing = 0;
  ds->n_flag_rows = 0;
  ds->n_flag_grew = 0;
  ds->n_flagged = 0;
}

__global__ void k_reset_counters(DevState* ds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clear_counters(ds);
}

// Start of a step: counters cleared; the step's dt (the host's, or the
// previous force pass's Courant minimum) taken before that minimum is reset
// for this step's force pass; neighbour lists wanted (leaf_state 1: the tree
// kernels before the density do not read it).
__global__ void k_step_begin(DevState* ds, double dt_host) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ds->dt_cur = (dt_host > 0.0) ? dt_host : dec_f64(ds->dt_min_enc);
    ds->dt_min_enc = enc_f64(SPH_INF);
    clear_counters(ds);
    ds->leaf_state = 1;
  }
}

// v1 = v_p + (a1 - a0) dt/2, u1 = u_p + (du1 - du0) dt/2; a0 <- a1.
__global__ __launch_bounds__(256) void k_correct(Parts p, int n, const double* __restrict__ a1,
                                                  int64_t stride, const DevState* __restrict__ ds) {
  const double hdt = 0.5 * ds->dt_cur;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double nax = a1[i], nay = a1[stride + i], naz = a1[2 * stride + i],
                 ndu = a1[3 * stride + i];
    p.vx[i] = p.vx[i] + (nax - p.ax[i]) * hdt;
    p.vy[i] = p.vy[i] + (nay - p.ay[i]) * hdt;
    p.vz[i] = p.vz[i] + (naz - p.az[i]) * hdt;
    p.u[i] = p.u[i] + (ndu - p.dudt[i]) * hdt;
    p.ax[i] = nax;
    p.ay[i] = nay;
    p.az[i] = naz;
    p.dudt[i] = ndu;
  }
}

constexpr int kRedBlocks = 512;

// Fixed-order FP64 sums: thread t of block b owns particles b*256+t + k*stride.
__global__ __launch_bounds__(256) void k_reduce_part(Parts p, int n, double* __restrict__ part) {
  __shared__ double s[12][256];
  double acc[12];
  for (int q = 0; q < 12; ++q) acc[q] = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kRedBlocks * 256) {
    const double m = p.m[i], vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
    const double ax = p.ax[i], ay = p.ay[i], az = p.az[i], du = p.dudt[i], u = p.u[i];
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double va = vx * ax + vy * ay + vz * az;
    acc[1] += 0.5 * m * v2;
    acc[2] += m * u;
    acc[3] += m * vx;
    acc[4] += m * vy;
    acc[5] += m * vz;
    acc[6] += m * ax;
    acc[7] += m * ay;
    acc[8] += m * az;
    acc[9] += m * (va + du);
    acc[10] += m * sqrt(ax * ax + ay * ay + az * az);
    acc[11] += m * (fabs(va) + fabs(du));
  }
  for (int q = 0; q < 12; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 12; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 12) part[blockIdx.x * 12 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_reduce_final(const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x < 12) {
    double a = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) a += part[b * 12 + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) out[0] = out[1] + out[2];
}

// ============================================================================
// Allocation-free reduction: the partial sums of k_reduce_part and the 12
// results of k_reduce_final in a file-scope device array instead of context
// scratch.  Each GPU the library runs on holds its own copy, until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: it takes the array's device address on each device once
// (hipGetSymbolAddress, with that device current) and uses that address.
// ============================================================================
constexpr int kRedScratch = kRedBlocks * 12 + 16;  // doubles: partials, then the 12 sums
static __device__ __align__(256) double scratch[kRedScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on the first
// call there).
static hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// ============================================================================
// Host-side launchers
// ============================================================================
static Parts parts_of(const sph_particles* s) {
  Parts p;
  p.id = s->id;
  p.x = s->x;
  p.y = s->y;
  p.z = s->z;
  p.vx = s->vx;
  p.vy = s->vy;
  p.vz = s->vz;
  p.m = s->m;
  p.u = s->u;
  p.h = s->h;
  p.ax = s->ax;
  p.ay = s->ay;
  p.az = s->az;
  p.dudt = s->dudt;
  p.rho = s->rho;
  p.omega = s->omega;
  p.P = s->P;
  p.cs = s->cs;
  p.vsig = s->vsig_dt;
  return p;
}

static int stream_blocks(int n) {
  int b = (n + 255) / 256;
  return b < 1 ? 1 : (b > 8192 ? 8192 : b);
}

// The radix sort's workspace: look-back status words of every pass and tile,
// then the eight digit histograms, then the eight tile tickets.
struct SortWs {
  uint32_t *status, *ghist, *tickets;
};
static SortWs sort_ws(sph_ctx* c) {
  const int64_t nst = (int64_t)c->n_max_sort_blocks * 8 * 256;
  SortWs w;
  w.status = c->radix_cnt;
  w.ghist = c->radix_cnt + nst;
  w.tickets = w.ghist + 8 * 256;
  return w;
}

hipError_t launch_predict_keys(sph_ctx* c, const sph_particles* s, bool predict, double) {
  c->kp.n = c->n;
  const SortWs w = sort_ws(c);
  hipLaunchKernelGGL(k_predict_keys, dim3(stream_blocks(c->n)), dim3(256), 0, c->stream, c->kp,
                     parts_of(s), predict ? 1 : 0, c->ds, c->keys[0], c->vals[0], w.ghist,
                     w.tickets, &c->ds->err);
  return hipGetLastError();
}

// Follows launch_predict_keys, which cleared the histograms and tickets.
hipError_t launch_sort(sph_ctx* c) {
  const int n = c->n;
  const int nblk = (n + kSortTile - 1) / kSortTile;
  const SortWs w = sort_ws(c);
  uint32_t* status = w.status;
  uint32_t* ghist = w.ghist;
  uint32_t* tickets = w.tickets;
  const int pblocks = std::min(nblk, 4 * c->n_cu);
  hipLaunchKernelGGL(k_radix_prep, dim3(pblocks), dim3(256), 0, c->stream, c->keys[0], n, nblk,
                     status, ghist);
  for (int pass = 0; pass < 8; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    hipLaunchKernelGGL(k_radix_pass, dim3(nblk), dim3(256), 0, c->stream, c->keys[src],
                       c->vals[src], c->keys[dst], c->vals[dst], n, pass, nblk, status, ghist,
                       tickets, &c->ds->err);
  }
  return hipGetLastError();  // 8 passes: the result is back in buffer 0
}

hipError_t launch_permute(sph_ctx* c, const sph_particles* s, bool outputs_too) {
  FieldSet fs;
  fs.nf = 0;
  double* all[] = {s->x,  s->y,  s->z,    s->vx,  s->vy,   s->vz, s->m,  s->u,     s->h,
                   s->ax, s->ay, s->az,   s->dudt, s->rho, s->omega, s->P, s->cs, s->vsig_dt};
  const int n_in = 13;  // x..dudt are state; the rest are outputs
  fs.im = -1;
  for (int k = 0; k < (int)(sizeof(all) / sizeof(all[0])); ++k) {
    if (!all[k]) continue;
    if (k >= n_in && !outputs_too) continue;
    if (all[k] == s->m) fs.im = fs.nf;
    fs.f[fs.nf++] = all[k];
  }
  fs.xyzm = c->kp.precision == SPH_PREC_MIXED ? nullptr : c->xyzm;
  fs.id = s->id;
  const int nb = stream_blocks(c->n);
  hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, c->stream, fs, c->vals[0], c->gtmp,
                     c->gtmp_id, c->n, (int64_t)c->n_max);
  hipLaunchKernelGGL(k_copy_back, dim3(nb), dim3(256), 0, c->stream, fs, c->gtmp, c->gtmp_id,
                     c->n, (int64_t)c->n_max);
  return hipGetLastError();
}

// FP64 contexts: x, y, z, m packed for the density gather (the mixed code
// records are packed with each refresh of the nodes' h_max, node_props)
hipError_t launch_pack_xyzm(sph_ctx* c, const sph_particles* s) {
  if (c->kp.precision != SPH_PREC_MIXED)
    hipLaunchKernelGGL(k_pack_xyzm, dim3(stream_blocks(c->n)), dim3(256), 0, c->stream,
                       parts_of(s), c->n, c->xyzm);
  return hipGetLastError();
}

static void pack_q(sph_ctx* c, const sph_particles* s, int mode) {
  hipLaunchKernelGGL(k_pack_q, dim3(stream_blocks(c->n)), dim3(256), 0, c->stream, c->kp,
                     parts_of(s), c->n, c->ds, mode, c->qxyzm, c->qrec);
}

hipError_t launch_tree(sph_ctx* c) {
  const int n = c->n;
  const int nblk = (n + kTreeTile - 1) / kTreeTile;
  hipLaunchKernelGGL(k_tree_levels, dim3(nblk), dim3(256), 0, c->stream, c->keys[0], n,
                     c->kp.n_leaf, c->kp.n_group, c->dlev, c->lleaf, c->gsize, c->gstart,
                     c->tree_cnt, c->grp_cnt, nblk, c->node_nchild, c->node_cap);
  hipError_t e = scan_u32(c, c->tree_cnt, (int64_t)kLevels * nblk, nullptr, &c->ds->n_nodes);
  if (e != hipSuccess) return e;
  e = scan_u32(c, c->grp_cnt, nblk, nullptr, &c->ds->n_groups);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tree_emit, dim3(nblk), dim3(256), 0, c->stream, c->keys[0], n,
                     c->kp.n_group, c->dlev, c->lleaf, c->gsize, c->gstart, c->tree_cnt,
                     c->grp_cnt, nblk, c->node_cap, c->node_level, c->node_first,
                     c->node_count, c->node_parent, c->node_child, c->node_nchild,
                     c->grp_first, c->grp_count, c->ds);
  return hipGetLastError();  // node_props checks the node count (tree_guard)
}

// Node boxes (positions) and largest h; group boxes.  The positions are the
// current (sorted) ones; h may be the start value or the converged one.
static hipError_t node_props(sph_ctx* c, const sph_particles* s, int mode) {
  const int n = c->n;
  const bool small = n <= kSmallTree;
  // leaves and groups four per wavefront; small trees: their inner nodes one
  // per wavefront in the same launch (from chunk boxes), large trees: one
  // launch per level afterwards (the deepest first; the last level holds
  // leaves only; the level offsets are the scanned per-level node counts).
  // A new tree's node count is checked before the box kernels read it.
  if (small) {
    const int nch = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_chunk_boxes, dim3((nch + 3) / 4), dim3(256), 0, c->stream, s->x, s->y,
                       s->z, s->h, n, c->chunk_box, c->ds, mode, c->node_cap);
  } else if (mode == 1) {
    hipLaunchKernelGGL(k_tree_guard, dim3(1), dim3(64), 0, c->stream, c->ds, c->node_cap);
  }
  const int64_t items = c->node_cap + (int64_t)n;
  const int nb = (int)std::min<int64_t>(std::max<int64_t>((items / 4 + 15) / 16, 16), 4096);
  const int nbi =
      small ? (int)std::min<int64_t>(std::max<int64_t>((c->node_cap / 8 + 63) / 64, 16), 4096) : 0;
  hipLaunchKernelGGL(k_range_boxes, dim3(nb + nbi), dim3(256), 0, c->stream, s->x, s->y, s->z,
                     s->h, c->node_first, c->node_count, c->node_child, c->node_nchild, c->wnode,
                     c->grp_first, c->grp_count, c->ginfo, c->ds, mode, nb, n, c->chunk_box,
                     c->node_parent);
  if (!small) {
    const int nblk = (n + kTreeTile - 1) / kTreeTile;
    const int lb =
        (int)std::min<int64_t>(std::max<int64_t>((c->node_cap / 4 + 255) / 256, 1), 1024);
    for (int l = kLevels - 2; l >= 0; --l)
      hipLaunchKernelGGL(k_level_boxes, dim3(lb), dim3(256), 0, c->stream, l, c->tree_cnt, nblk,
                         c->node_first, c->node_child, c->node_nchild, c->wnode, c->ds, mode);
  }
  // mixed: the code records with the current h and m (a new tree's after its
  // frame, below)
  if (mode != 1 && c->kp.precision == SPH_PREC_MIXED) pack_q(c, s, mode);
  return hipGetLastError();
}

hipError_t launch_node_h(sph_ctx* c, const sph_particles* s, bool always) {
  return node_props(c, s, always ? 2 : 0);
}
hipError_t launch_node_boxes(sph_ctx* c, const sph_particles* s) {
  const hipError_t e = node_props(c, s, 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_qframe, dim3(1), dim3(64), 0, c->stream, c->kp, c->wnode, c->ds);
  // the mixed code records need the frame (the FP64 packed positions come
  // from the permute)
  if (c->kp.precision == SPH_PREC_MIXED) pack_q(c, s, 1);
  return hipGetLastError();
}

// Density and force of groups of 4 or 8 particles go through the neighbour
// lists; larger groups (and flagged groups) through the walking kernels.
bool lists_mode(const sph_ctx* c) { return c->kp.n_group == 4 || c->kp.n_group == 8; }

#define SPH_LPI_SWITCH(NG, BODY)      \
  switch (NG) {                       \
    case 4: {                         \
      constexpr int LPI = 16;         \
      BODY;                           \
    } break;                          \
    case 8: {                         \
      constexpr int LPI = 8;          \
      BODY;                           \
    } break;                          \
    case 16: {                        \
      constexpr int LPI = 4;          \
      BODY;                           \
    } break;                          \
    default: {                        \
      constexpr int LPI = 2;          \
      BODY;                           \
    } break;                          \
  }

#define SPH_LPI_SWITCH_LISTS(NG, BODY) \
  switch (NG) {                        \
    case 4: {                          \
      constexpr int LPI = 16;          \
      BODY;                            \
    } break;                           \
    default: {                         \
      constexpr int LPI = 8;           \
      BODY;                            \
    } break;                           \
  }

template <bool MIXED>
static hipError_t density_dispatch(sph_ctx* c, const sph_particles* s, const int32_t* gflag) {
  const Parts p = parts_of(s);
  // the flagged groups (usually none, at most a few per cent) are striped
  // over a quarter of the walk grid: an empty launch then costs less
  const dim3 grid(gflag ? std::max(c->walk_blocks / 4, 8) : c->walk_blocks), block(64);
  SPH_LPI_SWITCH(c->kp.n_group,
                 hipLaunchKernelGGL((k_density<MIXED, LPI>), grid, block, 0, c->stream, c->kp, p,
                                    c->wnode, c->ginfo, c->frec, c->leaf_pool, c->pool_cap,
                                    c->gl_off, c->gl_cnt, gflag, c->walk_spill, c->ds));
  return hipGetLastError();
}

hipError_t launch_density(sph_ctx* c, const sph_particles* s, bool flagged_only) {
  c->kp.n = c->n;
  const int32_t* gf = flagged_only ? c->flag_list : nullptr;
  return c->kp.precision == SPH_PREC_MIXED ? density_dispatch<true>(c, s, gf)
                                           : density_dispatch<false>(c, s, gf);
}

hipError_t launch_lists(sph_ctx* c, const sph_particles* s) {
  c->kp.n = c->n;
  const Parts p = parts_of(s);
  const dim3 grid(c->walk_blocks), block(64);
  if (c->kp.precision == SPH_PREC_MIXED) {
    SPH_LPI_SWITCH_LISTS(c->kp.n_group,
                         hipLaunchKernelGGL((k_lists<true, LPI>), grid, block, 0, c->stream,
                                            c->kp, p, c->wnode, c->ginfo, c->nl_idx, c->nl_len,
                                            c->gflag, c->flag_list, c->grp_of, c->qrec,
                                            c->walk_spill, c->ds));
  } else {
    SPH_LPI_SWITCH_LISTS(c->kp.n_group,
                         hipLaunchKernelGGL((k_lists<false, LPI>), grid, block, 0, c->stream,
                                            c->kp, p, c->wnode, c->ginfo, c->nl_idx, c->nl_len,
                                            c->gflag, c->flag_list, c->grp_of, c->qrec,
                                            c->walk_spill, c->ds));
  }
  return hipGetLastError();
}

// The list kernels are instantiated per smoothing kernel (Sect. 2.3).
#define SPH_KIND_SWITCH(KD, BODY) \
  switch (KD) {                   \
    case 1: {                     \
      constexpr int KIND = 1;     \
      BODY;                       \
    } break;                      \
    case 2: {                     \
      constexpr int KIND = 2;     \
      BODY;                       \
    } break;                      \
    default: {                    \
      constexpr int KIND = 0;     \
      BODY;                       \
    } break;                      \
  }

template <bool MIXED, int CAP, int KIND>
static void density_lists_kind(sph_ctx* c, const Parts& p) {
  const dim3 grid(c->walk_blocks), block(64);
  SPH_LPI_SWITCH_LISTS(c->kp.n_group,
                       hipLaunchKernelGGL((k_density_lists<MIXED, LPI, CAP, KIND>), grid, block,
                                          0, c->stream, c->kp, p, c->ginfo, c->nl_idx, c->nl_len,
                                          c->gflag, c->flag_list, c->grp_of,
                                          MIXED ? (const void*)c->qxyzm : (const void*)c->xyzm,
                                          c->frec, c->ds));
}

template <bool MIXED, int CAP>
static void density_lists_dispatch(sph_ctx* c, const Parts& p) {
  SPH_KIND_SWITCH(c->kp.kernel, (density_lists_kind<MIXED, CAP, KIND>(c, p)));
}

hipError_t launch_density_lists(sph_ctx* c, const sph_particles* s) {
  c->kp.n = c->n;
  const Parts p = parts_of(s);
  const bool wide = c->kp.nl_cap > 128;
  if (c->kp.precision == SPH_PREC_MIXED) {
    if (wide)
      density_lists_dispatch<true, 256>(c, p);
    else
      density_lists_dispatch<true, 128>(c, p);
  } else {
    if (wide)
      density_lists_dispatch<false, 256>(c, p);
    else
      density_lists_dispatch<false, 128>(c, p);
  }
  return hipGetLastError();
}

template <bool MIXED>
static hipError_t force_dispatch(sph_ctx* c, const sph_particles* s, double* oax, double* oay,
                                 double* oaz, double* odu, const int32_t* gflag) {
  const Parts p = parts_of(s);
  const dim3 grid(c->walk_blocks), block(64);
  SPH_LPI_SWITCH(c->kp.n_group,
                 hipLaunchKernelGGL((k_force<MIXED, LPI>), grid, block, 0, c->stream, c->kp, p,
                                    c->wnode, c->ginfo, c->frec, c->leaf_pool, c->gl_off,
                                    c->gl_cnt, oax, oay, oaz, odu, gflag, c->walk_spill, c->ds));
  return hipGetLastError();
}

static void force_outputs(sph_ctx* c, const sph_particles* s, bool step_mode, double** o) {
  o[0] = step_mode ? c->a1 : s->ax;
  o[1] = step_mode ? c->a1 + c->n_max : s->ay;
  o[2] = step_mode ? c->a1 + 2 * c->n_max : s->az;
  o[3] = step_mode ? c->a1 + 3 * c->n_max : s->dudt;
}

hipError_t launch_force(sph_ctx* c, const sph_particles* s, bool step_mode, bool flagged_only) {
  c->kp.n = c->n;
  double* o[4];
  force_outputs(c, s, step_mode, o);
  const int32_t* gf = flagged_only ? c->flag_list : nullptr;
  return c->kp.precision == SPH_PREC_MIXED ? force_dispatch<true>(c, s, o[0], o[1], o[2], o[3], gf)
                                           : force_dispatch<false>(c, s, o[0], o[1], o[2], o[3], gf);
}

template <bool MIXED, int KIND>
static void force_lists_kind(sph_ctx* c, const Parts& p, double* const* o) {
  const dim3 grid(c->walk_blocks), block(64);
  SPH_LPI_SWITCH_LISTS(c->kp.n_group,
                       hipLaunchKernelGGL((k_force_lists<MIXED, LPI, KIND>), grid, block, 0,
                                          c->stream, c->kp, p, c->ginfo, c->frec, c->nl_idx,
                                          c->nl_len, c->gflag, c->grp_of, o[0], o[1], o[2], o[3],
                                          c->ds));
}

hipError_t launch_force_lists(sph_ctx* c, const sph_particles* s, bool step_mode) {
  c->kp.n = c->n;
  double* o[4];
  force_outputs(c, s, step_mode, o);
  const Parts p = parts_of(s);
  if (c->kp.precision == SPH_PREC_MIXED) {
    SPH_KIND_SWITCH(c->kp.kernel, (force_lists_kind<true, KIND>(c, p, o)));
  } else {
    SPH_KIND_SWITCH(c->kp.kernel, (force_lists_kind<false, KIND>(c, p, o)));
  }
  return hipGetLastError();
}

// Each particle's pairs among its list row that pass the exact FP64
// predicate at the h in p->h (mode 0: density set, self included; 1: force
// set): counts, and the indices at offsets[i] when idx is given.
hipError_t launch_row_sets(sph_ctx* c, const sph_particles* s, int mode, int32_t* counts,
                           int32_t* idx, const int64_t* offsets) {
  c->kp.n = c->n;
  const Parts p = parts_of(s);
  const dim3 grid(c->walk_blocks), block(64);
  SPH_LPI_SWITCH_LISTS(c->kp.n_group,
                       hipLaunchKernelGGL((k_row_sets<LPI>), grid, block, 0, c->stream, c->kp, p,
                                          mode, c->nl_idx, c->nl_len, c->gflag, c->grp_of,
                                          counts, idx, offsets));
  return hipGetLastError();
}

hipError_t launch_leaf_state(sph_ctx* c, int v) {
  hipLaunchKernelGGL(k_set_leaf_state, dim3(1), dim3(64), 0, c->stream, c->ds, v);
  return hipGetLastError();
}

hipError_t launch_force_reset(sph_ctx* c) {
  hipLaunchKernelGGL(k_reset_force_state, dim3(1), dim3(64), 0, c->stream, c->ds);
  return hipGetLastError();
}

hipError_t launch_correct(sph_ctx* c, const sph_particles* s) {
  hipLaunchKernelGGL(k_correct, dim3(stream_blocks(c->n)), dim3(256), 0, c->stream, parts_of(s),
                     c->n, c->a1, (int64_t)c->n_max, c->ds);
  return hipGetLastError();
}

// The sums of launch_reduce with the partials in `scratch` (its device
// address on the current device), copied into the host array out; the
// stream is synchronised.  Allocates nothing.
hipError_t reduce_noalloc(const sph_particles* s, hipStream_t stream, double* out) {
  double* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  double* part = base;
  double* res = base + kRedBlocks * 12;
  hipLaunchKernelGGL(k_reduce_part, dim3(kRedBlocks), dim3(256), 0, stream, parts_of(s),
                     (int)s->n, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, stream, part, res);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, 12 * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

hipError_t launch_reduce(sph_ctx* c, const sph_particles* s, double* dev_out) {
  hipLaunchKernelGGL(k_reduce_part, dim3(kRedBlocks), dim3(256), 0, c->stream, parts_of(s),
                     (int)s->n, c->red_part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, c->stream, c->red_part, dev_out);
  return hipGetLastError();
}

hipError_t launch_step_begin(sph_ctx* c, double dt_host) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, c->stream, c->ds, dt_host);
  return hipGetLastError();
}

hipError_t launch_reset_counters(sph_ctx* c) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, c->stream, c->ds);
  return hipGetLastError();
}

hipError_t launch_neighbours(sph_ctx* c, const sph_particles* s, int mode, int32_t* counts,
                             const int64_t* offsets, int32_t* idx) {
  c->kp.n = c->n;
  const Parts p = parts_of(s);
  const dim3 grid(c->walk_blocks), block(64);
  switch (c->kp.n_group) {
    case 4:
      hipLaunchKernelGGL((k_neighbours<16>), grid, block, 0, c->stream, c->kp, p, mode, c->wnode,
                         c->ginfo, counts, offsets, idx, c->walk_spill, c->ds);
      break;
    case 8:
      hipLaunchKernelGGL((k_neighbours<8>), grid, block, 0, c->stream, c->kp, p, mode, c->wnode,
                         c->ginfo, counts, offsets, idx, c->walk_spill, c->ds);
      break;
    case 16:
      hipLaunchKernelGGL((k_neighbours<4>), grid, block, 0, c->stream, c->kp, p, mode, c->wnode,
                         c->ginfo, counts, offsets, idx, c->walk_spill, c->ds);
      break;
    default:
      hipLaunchKernelGGL((k_neighbours<2>), grid, block, 0, c->stream, c->kp, p, mode, c->wnode,
                         c->ginfo, counts, offsets, idx, c->walk_spill, c->ds);
      break;
  }
  return hipGetLastError();
}

}  // namespace sph
