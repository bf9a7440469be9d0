// sph_adjoint.hip -- gfx950 kernels of the adjoint (reverse-mode derivative)
// of one hydro evaluation and of one leapfrog step.
//
// The forward quantities differentiated are those of Sect. 2.2-2.6: the
// density sums S0 = sum m_j W(r_ij, h_i) (= rho_i) and S1 = sum m_j dW/dh,
// the smoothing length as the root of f(h) = S0(h) - m (hfact/h)^3, the
// grad-h term Omega = 1 + h S1 / (3 rho), the ideal-gas P and c_s, and the
// momentum and energy equations with viscosity (approaching pairs) and
// conductivity.  Held fixed: the neighbour sets of the forward evaluation, the
// viscosity switches (w < 0) and the step dt.  The root h enters through its
// implicit derivative dh = -(dS0/dx) dx / f'(h).
//
// Pass structure (gather form: every output belongs to one particle and is
// written by the lanes of that particle, so there are no atomics):
//   k_adj_seed   cotangents of a and du/dt in key order (AoS records)
//   k_adj_force  for particle k, both pair terms a_k(j) and a_j(k): the
//                cotangent of x_k, v_k and of k's own h, g = P/(rho^2 Omega),
//                kk = 1/(rho Omega), c, P, rho, u; in the same pair loop
//                S1, S2 = sum m_j d2W/dh2 over k's density set; then the
//                chain through P, c, g, kk, Omega and the root h gives the
//                coefficients alpha_k, beta_k of dS0_k/dx and dS1_k/dx
//   k_adj_dens2  x-cotangent through the density sums, from both directions
//                of each pair, and the final combination with the leapfrog
//                (Sect. 2.4) into the caller's cotangent arrays.
//
// Built with -ffp-contract=off: every fused multiply-add is an explicit fma().
#include <math.h>

#include <type_traits>

#include "sph_ctx.h"

namespace sph {

namespace {

// Nearest periodic image of a separation d (|d| < 1.5 len), without branches.
__device__ __forceinline__ double afold(double d, double len, double half, int periodic) {
  const double lp = periodic ? len : 0.0;
  double t = d > half ? d - lp : d;
  t = d < -half ? d + lp : t;
  return t;
}

template <typename R>
__device__ __forceinline__ R pos5(R t) {
  return t > R(0) ? t : R(0);
}

// Kernel shape f(q) and its first two derivatives (Sect. 2.3), W = C f(r/h)/h^3.
template <typename R>
__device__ __forceinline__ void kern3(int kind, R q, R& f, R& d1, R& d2) {
  if (kind == 1) {  // M6 quintic: (3-q)^5 - 6(2-q)^5 + 15(1-q)^5, each term where positive
    const R a = pos5<R>(R(3) - q), b = pos5<R>(R(2) - q), c = pos5<R>(R(1) - q);
    const R a2 = a * a, b2 = b * b, c2 = c * c;
    const R a3 = a2 * a, b3 = b2 * b, c3 = c2 * c;
    f = a3 * a2 - R(6) * b3 * b2 + R(15) * c3 * c2;
    d1 = R(-5) * a2 * a2 + R(30) * b2 * b2 - R(75) * c2 * c2;
    d2 = R(20) * a3 - R(120) * b3 + R(300) * c3;
  } else if (kind == 2) {  // Wendland C6: s^8 g, s = 1 - q/2, g = 4q^3 + 6.25q^2 + 4q + 1
    const R s = pos5<R>(R(1) - R(0.5) * q);
    const R s2 = s * s, s3 = s2 * s, s6 = s3 * s3, s7 = s6 * s;
    const R g = ((R(4) * q + R(6.25)) * q + R(4)) * q + R(1);
    const R p = ((R(8) * q + R(7)) * q + R(2)) * q;  // f' = -2.75 p s^7
    f = s7 * s * g;
    d1 = R(-2.75) * p * s7;
    // f'' = -2.75 s^6 [ p' s - 3.5 p ],  p' = 24 q^2 + 14 q + 2
    d2 = R(-2.75) * s6 * (((R(24) * q + R(14)) * q + R(2)) * s - R(3.5) * p);
  } else {  // M4 cubic spline
    if (q < R(1)) {
      f = R(1) - R(1.5) * q * q + R(0.75) * q * q * q;
      d1 = R(-3) * q + R(2.25) * q * q;
      d2 = R(-3) + R(4.5) * q;
    } else if (q < R(2)) {
      const R t = R(2) - q;
      f = R(0.25) * t * t * t;
      d1 = R(-0.75) * t * t;
      d2 = R(1.5) * t;
    } else {
      f = d1 = d2 = R(0);
    }
  }
}

// F = dW/dr, F_r = d2W/dr2, F_h = d2W/dr dh at (r, h); C = normalisation.
template <typename R>
__device__ __forceinline__ void kern_F3(int kind, R C, R r, R hinv, R& F, R& Fr, R& Fh) {
  const R q = r * hinv;
  R f, d1, d2;
  kern3<R>(kind, q, f, d1, d2);
  const R h4 = C * hinv * hinv * hinv * hinv, h5 = h4 * hinv;
  F = d1 * h4;
  Fr = d2 * h5;
  Fh = -(R(4) * d1 + q * d2) * h5;
}

template <int LPI>
__device__ __forceinline__ double seg_sum_d(double v) {
#pragma unroll
  for (int d = LPI / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Chunks of particles of this wavefront under the XCD-aware static schedule:
// block b works on the contiguous eighth of the chunks of XCD b mod 8.
struct ChunkRange {
  int beg, end, step;
};
__device__ __forceinline__ ChunkRange xcd_chunks(int nch) {
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int per = (nch + 7) >> 3;
  const int beg = xcd * per;
  return ChunkRange{beg + local, min(beg + per, nch), nloc};
}

template <bool MIXED>
struct ARecOf {
  using T = FRec64;
  using C = double4;
};
template <>
struct ARecOf<true> {
  using T = FRec32;
  using C = float4;
};

}  // namespace

// Cotangent arrays of the caller (sph_cotangents), indexed by original id.
struct Cot {
  double *x, *y, *z, *vx, *vy, *vz, *u, *ax, *ay, *az, *du;
};

// ---------------------------------------------------------------------------
// Seed: cotangents of the evaluation's outputs a, du/dt in key order.  In a
// step the corrector v1 = v_p + (a1 - a0) dt/2 (u likewise) adds dt/2 times
// the cotangents of v1, u1 to those of a1, du1.
// ---------------------------------------------------------------------------
template <bool MIXED>
__global__ __launch_bounds__(256) void k_adj_seed(int n, const int64_t* __restrict__ id, Cot g,
                                                  double hdt, int step_mode,
                                                  void* __restrict__ abar_out,
                                                  uint32_t* __restrict__ err) {
  using CT = typename ARecOf<MIXED>::C;
  CT* __restrict__ abar = reinterpret_cast<CT*>(abar_out);
  bool bad = false;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int64_t o = id[i];
    if ((uint64_t)o >= (uint64_t)n) {
      bad = true;
      abar[i] = CT{0, 0, 0, 0};
      continue;
    }
    double ax = g.ax[o], ay = g.ay[o], az = g.az[o], du = g.du[o];
    if (step_mode) {
      ax = fma(hdt, g.vx[o], ax);
      ay = fma(hdt, g.vy[o], ay);
      az = fma(hdt, g.vz[o], az);
      du = fma(hdt, g.u[o], du);
    }
    CT c;
    c.x = ax;
    c.y = ay;
    c.z = az;
    c.w = du;
    abar[i] = c;
  }
  if (bad) atomicOr(err, kErrIds);
}

// ---------------------------------------------------------------------------
// Force adjoint.  For the pair (k, j), with r_kj = x_k - x_j, e = r_kj / r,
// w = (v_k - v_j).e, F_k = F(r, h_k), vs_k = alpha c_k - beta w (w < 0),
// T_k = g_k - vs_k w kk_k / 2, v^u = sqrt(|P_k - P_j| / rhobar), the term of a_k
// is -m_j (T_k F_k + T_j F_j) e and that of du_k/dt is
//   m_j [ g_k w F_k - kk_k vs_k w^2 F_k / 2 + alpha_u v^u (u_k - u_j)(F_k kk_k + F_j kk_j)/2 ].
// Particle k differentiates its own term (cotangents abar_k) and the mirror
// term of a_j, du_j (cotangents abar_j), with respect to x_k, v_k and k's own
// per-particle quantities.
// ---------------------------------------------------------------------------
template <bool MIXED, int LPI>
__global__ __launch_bounds__(64) void k_adj_force(KParams kp, Parts p,
                                                  const void* __restrict__ frec_in,
                                                  const void* __restrict__ abar_in,
                                                  const int32_t* __restrict__ nl_idx,
                                                  const int32_t* __restrict__ nl_len,
                                                  double* __restrict__ raw, int64_t ns,
                                                  double2* __restrict__ ab,
                                                  const QFrame* __restrict__ qf) {
  using Rec = typename ARecOf<MIXED>::T;
  using CT = typename ARecOf<MIXED>::C;
  using R = typename std::conditional<MIXED, float, double>::type;
  const Rec* __restrict__ rec = reinterpret_cast<const Rec*>(frec_in);
  float qs[3] = {0.f, 0.f, 0.f};  // code steps of the mixed records' positions
  if constexpr (MIXED)
    for (int a = 0; a < 3; ++a) qs[a] = qf->step[a];
  const CT* __restrict__ abar = reinterpret_cast<const CT*>(abar_in);
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  constexpr int CS = kWave / LPI;
  const int nch = (kp.n + CS - 1) / CS;
  const ChunkRange cr = xcd_chunks(nch);
  const R al = (R)kp.alpha, be = (R)kp.beta, au = (R)kp.alpha_u, C = (R)kp.knorm;
  const R S = (R)kp.support;
  const int kind = kp.kernel;

  for (int ch = cr.beg; ch < cr.end; ch += cr.step) {
    const int first = ch * CS, count = min(CS, kp.n - first);
    const bool act = slot < count;
    const int k = first + (act ? slot : 0);
    const Rec rk = rec[k];
    const CT ak = abar[k];
    // position: FP64 (folded per pair) or the mixed record's codes
    double xk = 0.0, yk = 0.0, zk = 0.0;
    int32_t qxk = 0, qyk = 0, qzk = 0;
    if constexpr (MIXED) {
      qxk = rk.qx;
      qyk = rk.qy;
      qzk = rk.qz;
    } else {
      xk = rk.x;
      yk = rk.y;
      zk = rk.z;
    }
    const R hk = (R)rk.h, hinvk = R(1) / hk, mk = (R)rk.m;
    const R h4k = C * hinvk * hinvk * hinvk * hinvk, h5k = h4k * hinvk;
    const R srk = S * hk, srk2 = srk * srk;
    const R vxk = (R)rk.vx, vyk = (R)rk.vy, vzk = (R)rk.vz, uk = (R)rk.u;
    const R gk = (R)rk.g, kk = (R)rk.k, ck = (R)rk.c, Pk = (R)rk.P, rhok = (R)rk.rho;
    const R Axk = (R)ak.x, Ayk = (R)ak.y, Azk = (R)ak.z, Dk = (R)ak.w;
    const int len = act ? min(nl_len[k], kp.nl_cap) : 0;
    const int32_t* __restrict__ row = nl_idx + (int64_t)k * kp.nl_cap;
    R bx = 0, by = 0, bz = 0, bvx = 0, bvy = 0, bvz = 0;
    R bh = 0, bg = 0, bk = 0, bc = 0, bp = 0, br = 0, bu = 0;
    R s1 = 0, s2 = 0;  // density sums of dW/dh and d2W/dh2 (without C / h^4, C / h^5)
    // row index one iteration ahead
    int jn = (sub < len) ? row[sub] : k;
    for (int t = sub; t < len; t += LPI) {
      const int j = jn;
      jn = (t + LPI < len) ? row[t + LPI] : k;
      if (j == k) continue;
      const Rec rj = rec[j];
      R dx, dy, dz;
      if constexpr (MIXED) {
        dx = qsep(qxk, rj.qx, qs[0]);
        dy = qsep(qyk, rj.qy, qs[1]);
        dz = qsep(qzk, rj.qz, qs[2]);
      } else {
        dx = afold(xk - rj.x, kp.len[0], kp.half[0], kp.periodic[0]);
        dy = afold(yk - rj.y, kp.len[1], kp.half[1], kp.periodic[1]);
        dz = afold(zk - rj.z, kp.len[2], kp.half[2], kp.periodic[2]);
      }
      const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      const R hj = (R)rj.h;
      const R sr = S * (hk > hj ? hk : hj);
      if (!(r2 < sr * sr)) continue;
      const CT aj = abar[j];
      const R r = sqrt(r2), rinv = R(1) / r;
      const R ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
      const R vx = vxk - (R)rj.vx, vy = vyk - (R)rj.vy, vz = vzk - (R)rj.vz;
      const R w = fma(vz, ez, fma(vy, ey, vx * ex));
      R Fk, Frk, Fhk, Fj, Frj, Fhj;
      {
        const R q = r * hinvk;
        R f, d1, d2;
        kern3<R>(kind, q, f, d1, d2);
        Fk = d1 * h4k;
        Frk = d2 * h5k;
        Fhk = -(R(4) * d1 + q * d2) * h5k;
        if (r2 < srk2) {  // k's density set
          const R mjd = (R)rj.m;
          s1 += mjd * (R(3) * f + q * d1);
          s2 += mjd * ((R(12) * f + R(8) * q * d1) + q * q * d2);
        }
      }
      kern_F3<R>(kind, C, r, R(1) / hj, Fj, Frj, Fhj);
      const R mj = (R)rj.m, gj = (R)rj.g, kj = (R)rj.k, cj = (R)rj.c;
      const bool chi = w < R(0);
      const R vsk = chi ? al * ck - be * w : R(0);
      const R vsj = chi ? al * (R)cj - be * w : R(0);
      const R Tk = gk - R(0.5) * vsk * w * kk;
      const R Tj = gj - R(0.5) * vsj * w * kj;
      const R dTk = chi ? R(-0.5) * kk * (al * ck - R(2) * be * w) : R(0);
      const R dTj = chi ? R(-0.5) * kj * (al * cj - R(2) * be * w) : R(0);
      const R rbar = R(0.5) * (rhok + (R)rj.rho);
      const R dP = Pk - (R)rj.P;
      const R adP = dP < R(0) ? -dP : dP;
      const R vu = adP > R(0) ? sqrt(adP / rbar) : R(0);
      const R dvu_dP = adP > R(0) ? (dP > R(0) ? R(1) : R(-1)) / (R(2) * vu * rbar) : R(0);
      const R dvu_dr = -vu / (R(4) * rbar);
      const R du = uk - (R)rj.u;
      const R Kb = R(0.5) * (Fk * kk + Fj * kj);
      const R Kbr = R(0.5) * (Frk * kk + Frj * kj);
      const R Ajx = (R)aj.x, Ajy = (R)aj.y, Ajz = (R)aj.z, Dj = (R)aj.w;
      const R wvx = (vx - w * ex) * rinv, wvy = (vy - w * ey) * rinv, wvz = (vz - w * ez) * rinv;
      const R w2 = w * w;
      const R avw = chi ? R(2) * al * w : R(0), bw2 = chi ? R(3) * be * w2 : R(0);
      // term of particle k: loss -m_j (T_k F_k + T_j F_j) s + D_k E_k
      {
        const R s = fma(Azk, ez, fma(Ayk, ey, Axk * ex));
        const R pa = mj * fma(Tk, Fk, Tj * Fj);
        const R Lr = -mj * fma(Tk, Frk, Tj * Frj) * s +
                     Dk * mj * (gk * w * Frk - R(0.5) * kk * vsk * w2 * Frk + au * vu * du * Kbr);
        const R Lw = -mj * fma(dTk, Fk, dTj * Fj) * s +
                     Dk * mj * (gk * Fk - R(0.5) * kk * (avw * ck - bw2) * Fk);
        const R Ls = -pa * rinv;
        bx += Lr * ex + Lw * wvx + Ls * (Axk - s * ex);
        by += Lr * ey + Lw * wvy + Ls * (Ayk - s * ey);
        bz += Lr * ez + Lw * wvz + Ls * (Azk - s * ez);
        bvx += Lw * ex;
        bvy += Lw * ey;
        bvz += Lw * ez;
        bh += -mj * Tk * Fhk * s +
              Dk * mj * (gk * w * Fhk - R(0.5) * kk * vsk * w2 * Fhk + au * vu * du * R(0.5) * Fhk * kk);
        bg += -mj * Fk * s + Dk * mj * w * Fk;
        bk += mj * R(0.5) * vsk * w * Fk * s + Dk * mj * (R(-0.5) * vsk * w2 * Fk + au * vu * du * R(0.5) * Fk);
        if (chi) bc += mj * R(0.5) * al * w * kk * Fk * s - Dk * R(0.5) * kk * mj * al * w2 * Fk;
        const R Cc = Dk * mj * au * du * Kb;
        bp += Cc * dvu_dP;
        br += Cc * dvu_dr;
        bu += Dk * mj * au * vu * Kb;
      }
      // mirror term of particle j (owner j, separation -r_kj, same w)
      {
        const R sj = fma(Ajz, ez, fma(Ajy, ey, Ajx * ex));  // s' = -sj
        const R Lr = mk * fma(Tj, Frj, Tk * Frk) * sj +
                     Dj * mk * (gj * w * Frj - R(0.5) * kj * vsj * w2 * Frj - au * vu * du * Kbr);
        const R Lw = mk * fma(dTj, Fj, dTk * Fk) * sj +
                     Dj * mk * (gj * Fj - R(0.5) * kj * (avw * cj - bw2) * Fj);
        const R Ls = -mk * fma(Tj, Fj, Tk * Fk) * rinv;
        bx += Lr * ex + Lw * wvx - Ls * (Ajx - sj * ex);
        by += Lr * ey + Lw * wvy - Ls * (Ajy - sj * ey);
        bz += Lr * ez + Lw * wvz - Ls * (Ajz - sj * ez);
        bvx += Lw * ex;
        bvy += Lw * ey;
        bvz += Lw * ez;
        bh += mk * Tk * Fhk * sj - Dj * mk * au * vu * du * R(0.5) * Fhk * kk;
        bg += mk * Fk * sj;
        bk += -mk * R(0.5) * vsk * w * Fk * sj - Dj * mk * au * vu * du * R(0.5) * Fk;
        if (chi) bc += -mk * R(0.5) * al * w * kk * Fk * sj;
        const R Cc = -Dj * mk * au * du * Kb;
        bp += Cc * dvu_dP;
        br += Cc * dvu_dr;
        bu += -Dj * mk * au * vu * Kb;
      }
    }
    double o[15] = {(double)bx, (double)by, (double)bz, (double)bvx, (double)bvy, (double)bvz,
                    (double)bh, (double)bg, (double)bk, (double)bc, (double)bp, (double)br,
                    (double)bu, (double)s1, (double)s2};
#pragma unroll
    for (int q = 0; q < 15; ++q) o[q] = seg_sum_d<LPI>(o[q]);
    if (act && sub == 0) {
      // the chain through g, kk, P, c, Omega and the root h (see below)
      const double hd = p.h[k], hinv = 1.0 / hd;
      double f0, d10, d20;
      kern3<double>(kind, 0.0, f0, d10, d20);  // the self term (r = 0, f'(0) = 0)
      const double md = p.m[k];
      const double h4 = kp.knorm * hinv * hinv * hinv * hinv;
      const double S1 = -(o[13] + 3.0 * md * f0) * h4;
      const double S2 = (o[14] + 12.0 * md * f0) * h4 * hinv;
      const double rho = p.rho[k], om = p.omega[k], P = p.P[k], u = p.u[k], c = p.cs[k];
      const double gb = o[7], kb = o[8], cb = o[9], pb = o[10], rb = o[11], ub = o[12];
      const double r2o = rho * rho * om;
      const double Ptot = pb + gb / r2o;
      double rtot = rb - 2.0 * gb * P / (r2o * rho) - kb / (om * rho * rho);
      const double Ob = -gb * P / (r2o * om) - kb / (om * om * rho);
      rtot += Ptot * kp.gm1 * u;
      const double utot =
          ub + Ptot * kp.gm1 * rho + (c > 0.0 ? cb * kp.gamma * kp.gm1 / (2.0 * c) : 0.0);
      const double S1b = Ob * hd / (3.0 * rho);
      rtot -= Ob * hd * S1 / (3.0 * rho * rho);
      const double hb = o[6] + Ob * S1 / (3.0 * rho);
      const double S0b = rtot;
      const double H = hb + S0b * S1 + S1b * S2;
      const double hr = kp.hfact * hinv;
      const double rho_h = md * hr * hr * hr;
      const double fp = S1 + 3.0 * rho_h * hinv;
      const double lam = -H / fp;
      ab[k] = make_double2(S0b + lam, S1b);
#pragma unroll
      for (int q = 0; q < 6; ++q) raw[q * ns + k] = o[q];
      raw[6 * ns + k] = utot;
    }
  }
}

// The density adjoint's first half -- S1, S2 = sum m_j d2W/dh2 over k's
// density set (self included) and the chain of per-particle relations
//   g = P/(rho^2 Omega), kk = 1/(rho Omega), P = (gamma-1) rho u,
//   c = sqrt(gamma (gamma-1) u), Omega = 1 + h S1/(3 rho), rho = S0,
// and the root h (f(h) = S0 - m (hfact/h)^3 = 0):
//   H = hbar + S0bar S1 + S1bar S2,  lambda = -H / (S1 + 3 m (hfact/h)^3 / h),
//   alpha = S0bar + lambda,  beta = S1bar,
// so that the x-cotangent through the density is alpha_k dS0_k/dx +
// beta_k dS1_k/dx summed over k -- runs at the end of k_adj_force, whose
// pair loop visits every density pair of k (the force set holds it).
// raw rows: xb yb zb vxb vyb vzb and the evaluation's final u-cotangent.

// ---------------------------------------------------------------------------
// Density adjoint, second half: for particle k over its row (j != k),
//   xbar_k += m_j [alpha_k F(r, h_k) + beta_k F_h(r, h_k)] e    (r < S h_k)
//           + m_k [alpha_j F(r, h_j) + beta_j F_h(r, h_j)] e    (r < S h_j)
// with e = (x_k - x_j)/r, F = dW/dr, F_h = d2W/dr dh; then the evaluation's
// cotangents are complete and are combined into the caller's arrays:
//   evaluation:  xbar += xbar_eval, vbar += vbar_eval, ubar += ubar_eval
//   step (reverse of predictor, evaluation, corrector with cotangents
//   X1, V1, U1, A1, D1 of the step's outputs):
//     Vp = V1 + vbar_eval, Xt = X1 + xbar_eval, Up = U1 + ubar_eval,
//     X0 = Xt, V0 = dt Xt + Vp, U0 = Up,
//     A0 = -dt/2 V1 + dt^2/2 Xt + dt Vp,  D0 = -dt/2 U1 + dt Up.
// ---------------------------------------------------------------------------
template <bool MIXED, int LPI>
__global__ __launch_bounds__(64) void k_adj_dens2(KParams kp, Parts p,
                                                  const void* __restrict__ frec_in,
                                                  const int32_t* __restrict__ nl_idx,
                                                  const int32_t* __restrict__ nl_len,
                                                  const double* __restrict__ raw, int64_t ns,
                                                  const double2* __restrict__ ab, Cot g,
                                                  double dt, int step_mode,
                                                  const QFrame* __restrict__ qf) {
  using Rec = typename ARecOf<MIXED>::T;
  using R = typename std::conditional<MIXED, float, double>::type;
  const Rec* __restrict__ rec = reinterpret_cast<const Rec*>(frec_in);
  float qs[3] = {0.f, 0.f, 0.f};  // code steps of the mixed records' positions
  if constexpr (MIXED)
    for (int a = 0; a < 3; ++a) qs[a] = qf->step[a];
  const int lane = threadIdx.x;
  const int slot = lane / LPI, sub = lane % LPI;
  constexpr int CS = kWave / LPI;
  const int nch = (kp.n + CS - 1) / CS;
  const ChunkRange cr = xcd_chunks(nch);
  const double C = kp.knorm, S = kp.support;
  for (int ch = cr.beg; ch < cr.end; ch += cr.step) {
    const int first = ch * CS, count = min(CS, kp.n - first);
    const bool act = slot < count;
    const int k = first + (act ? slot : 0);
    const double xk = p.x[k], yk = p.y[k], zk = p.z[k];
    // the mixed records hold position codes; k's are those its record holds
    int32_t qxk = 0, qyk = 0, qzk = 0;
    if constexpr (MIXED) {
      qxk = qcode(xk, *qf, 0, kp.periodic[0]);
      qyk = qcode(yk, *qf, 1, kp.periodic[1]);
      qzk = qcode(zk, *qf, 2, kp.periodic[2]);
    }
    const R hk = (R)p.h[k], mk = (R)p.m[k], Cr = (R)C;
    const R hinvk = R(1) / hk, srk = (R)S * hk, srk2 = srk * srk;
    const double2 abk = ab[k];
    const R ak = (R)abk.x, bk = (R)abk.y;
    const int len = act ? min(nl_len[k], kp.nl_cap) : 0;
    const int32_t* __restrict__ row = nl_idx + (int64_t)k * kp.nl_cap;
    R sx = 0, sy = 0, sz = 0;
    // row index one iteration ahead
    int jn = (sub < len) ? row[sub] : k;
    for (int t = sub; t < len; t += LPI) {
      const int j = jn;
      jn = (t + LPI < len) ? row[t + LPI] : k;
      if (j == k) continue;
      const Rec rj = rec[j];
      R dx, dy, dz;
      if constexpr (MIXED) {
        dx = qsep(qxk, rj.qx, qs[0]);
        dy = qsep(qyk, rj.qy, qs[1]);
        dz = qsep(qzk, rj.qz, qs[2]);
      } else {
        dx = afold(xk - rj.x, kp.len[0], kp.half[0], kp.periodic[0]);
        dy = afold(yk - rj.y, kp.len[1], kp.half[1], kp.periodic[1]);
        dz = afold(zk - rj.z, kp.len[2], kp.half[2], kp.periodic[2]);
      }
      const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      const R hj = (R)rj.h;
      const R srj = (R)S * hj;
      const bool ink = r2 < srk2, inj = r2 < srj * srj;
      if (!(ink || inj)) continue;
      const R r = sqrt(r2);
      R coef = 0;
      if (ink) {
        R F, Fr, Fh;
        kern_F3<R>(kp.kernel, Cr, r, hinvk, F, Fr, Fh);
        coef += (R)rj.m * (ak * F + bk * Fh);
      }
      if (inj) {
        const double2 abj = ab[j];
        R F, Fr, Fh;
        kern_F3<R>(kp.kernel, Cr, r, R(1) / hj, F, Fr, Fh);
        coef += mk * ((R)abj.x * F + (R)abj.y * Fh);
      }
      coef /= r;
      sx += coef * dx;
      sy += coef * dy;
      sz += coef * dz;
    }
    const double bx = seg_sum_d<LPI>((double)sx);
    const double by = seg_sum_d<LPI>((double)sy);
    const double bz = seg_sum_d<LPI>((double)sz);
    if (act && sub == 0) {
      const double ex = bx + raw[k], ey = by + raw[ns + k], ez = bz + raw[2 * ns + k];
      const double evx = raw[3 * ns + k], evy = raw[4 * ns + k], evz = raw[5 * ns + k];
      const double eu = raw[6 * ns + k];
      const int64_t o = p.id[k];
      if ((uint64_t)o >= (uint64_t)kp.n) {
        // reported by the seed kernel
      } else if (step_mode) {
        const double hdt = 0.5 * dt, hdt2 = 0.5 * dt * dt;
        const double X[3] = {g.x[o] + ex, g.y[o] + ey, g.z[o] + ez};
        const double V1[3] = {g.vx[o], g.vy[o], g.vz[o]};
        const double Vp[3] = {V1[0] + evx, V1[1] + evy, V1[2] + evz};
        const double U1 = g.u[o], Up = U1 + eu;
        double* const gx[3] = {g.x, g.y, g.z};
        double* const gv[3] = {g.vx, g.vy, g.vz};
        double* const ga[3] = {g.ax, g.ay, g.az};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gx[a][o] = X[a];
          gv[a][o] = fma(dt, X[a], Vp[a]);
          ga[a][o] = fma(dt, Vp[a], fma(hdt2, X[a], -hdt * V1[a]));
        }
        g.u[o] = Up;
        g.du[o] = fma(dt, Up, -hdt * U1);
      } else {
        g.x[o] += ex;
        g.y[o] += ey;
        g.z[o] += ez;
        g.vx[o] += evx;
        g.vy[o] += evy;
        g.vz[o] += evz;
        g.u[o] += eu;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static Parts adj_parts(const sph_particles* s) {
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

static Cot cot_of(const sph_cotangents* g) {
  return Cot{g->x, g->y, g->z, g->vx, g->vy, g->vz, g->u, g->ax, g->ay, g->az, g->dudt};
}

// Three launches: the seed, the force adjoint (the dominant kernel, timed on
// its own by the host) and the two density passes with the final combination.
hipError_t launch_adjoint(sph_ctx* c, const sph_particles* s, const sph_cotangents* gc, double dt,
                          bool step_mode, int part) {
  c->kp.n = c->n;
  const Parts p = adj_parts(s);
  const Cot g = cot_of(gc);
  const int n = c->n;
  const int64_t ns = c->n_max;
  const bool mixed = c->kp.precision == SPH_PREC_MIXED;
  const dim3 grid(c->walk_blocks), block(64);
  // the density pass has little arithmetic per gathered neighbour: more
  // wavefronts in flight hide the gathers' latency
  const dim3 dgrid(4 * c->walk_blocks);
  constexpr int LPI = 8;
  if (part == 0) {
    const int sblocks = (int)std::min<int64_t>((n + 255) / 256, 8 * (int64_t)c->n_cu);
    if (mixed)
      hipLaunchKernelGGL(k_adj_seed<true>, dim3(sblocks), dim3(256), 0, c->stream, n, p.id, g,
                         0.5 * dt, step_mode ? 1 : 0, c->adj_abar, &c->ds->err);
    else
      hipLaunchKernelGGL(k_adj_seed<false>, dim3(sblocks), dim3(256), 0, c->stream, n, p.id, g,
                         0.5 * dt, step_mode ? 1 : 0, c->adj_abar, &c->ds->err);
  } else if (part == 1) {
    if (mixed)
      hipLaunchKernelGGL((k_adj_force<true, LPI>), grid, block, 0, c->stream, c->kp, p, c->frec,
                         c->adj_abar, c->nl_idx, c->nl_len, c->adj_raw, ns, c->adj_ab,
                         &c->ds->qf);
    else
      hipLaunchKernelGGL((k_adj_force<false, LPI>), grid, block, 0, c->stream, c->kp, p, c->frec,
                         c->adj_abar, c->nl_idx, c->nl_len, c->adj_raw, ns, c->adj_ab,
                         &c->ds->qf);
  } else if (mixed) {
    hipLaunchKernelGGL((k_adj_dens2<true, LPI>), dgrid, block, 0, c->stream, c->kp, p, c->frec,
                       c->nl_idx, c->nl_len, c->adj_raw, ns, c->adj_ab, g, dt,
                       step_mode ? 1 : 0, &c->ds->qf);
  } else {
    hipLaunchKernelGGL((k_adj_dens2<false, LPI>), dgrid, block, 0, c->stream, c->kp, p, c->frec,
                       c->nl_idx, c->nl_len, c->adj_raw, ns, c->adj_ab, g, dt,
                       step_mode ? 1 : 0, &c->ds->qf);
  }
  return hipGetLastError();
}

}  // namespace sph
