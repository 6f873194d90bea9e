// wcc_cell.hpp -- per-cell arithmetic of the WCC half-step on gfx950.
//
// Everything here is register resident and fully unrolled for a compile-time
// degree P: the Taylor triangles of the Cauchy-Kovalewski expansion live in
// VGPRs, there is no dynamic indexing and no LDS.  The two scalar types are
//   A = double : point values, half-cell averages and the cell-average update
//                (the conservative part; binary64 in both precision modes);
//   R          : the bulk type of the expansion, derivatives and limiter
//                (double in FP64 mode, float in FP32-mixed mode).
//
// Operation order (binary64 mode): every quantity is evaluated with the same
// sequence of correctly rounded operations as the written arithmetic of the
// scheme -- sums of products as s = c0*x0; s = fma(ci, xi, s) in index order,
// no other contraction (the library is compiled with -ffp-contract=off), so
// the binary64 results are reproducible bit for bit on any IEEE machine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_rn.hpp"

namespace wcc {

constexpr int kAdvection = 0, kBurgers = 1, kEuler = 2;
constexpr int kPeriodic = 0, kTransmissive = 1, kDirichlet = 2;

template <int EQ>
constexpr int ncomp() { return EQ == kEuler ? 3 : 1; }

// ---------------------------------------------------------------------------
// Exact rationals of the scheme, rounded once (constant-folded by the compiler).
// ---------------------------------------------------------------------------
// Non-recursive so that they inline into the unrolled loops and fold to
// immediates (a recursive constexpr function called with a loop index is
// compiled as a real call).
__host__ __device__ constexpr double fac(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return f;
}
__host__ __device__ constexpr double two_pow(int k) {
  double p = 1.0;
  for (int i = 0; i < k; ++i) p *= 2.0;
  return p;
}
// 1/k!  (normalised Taylor coefficient)
__host__ __device__ constexpr double inv_fac(int k) { return 1.0 / fac(k); }
// weight of u_kx in the right half-cell average, Eq. SubEq:1DCellAVGR
__host__ __device__ constexpr double half_avg(int k) { return 1.0 / (fac(k + 1) * two_pow(k)); }
// weight of u_kx in the left half-cell average, Eq. SubEq:1DCellAVGL
__host__ __device__ constexpr double half_avg_left(int k) { return (k % 2 == 0) ? half_avg(k) : -half_avg(k); }
// minus the weight of u_kx in the cell average (Eq. SubEq:1DCellAVG -> Eq. 1DCalU)
__host__ __device__ constexpr double neg_avg(int k) { return -half_avg(k); }
// minus the odd-moment weight of Eq. SubEq:Cal_1D_Derivatives_3
__host__ __device__ constexpr double neg_odd(int m) { return (m % 2 == 1) ? -(2.0 / (fac(m) * two_pow(m))) : 0.0; }
// m!/(m+1)! of Eq. Cal1DFlux
__host__ __device__ constexpr double flux_w(int m) { return 1.0 / (double)(m + 1); }
// (k+1)/m of the normalised CK identity
__host__ __device__ constexpr double ck_ratio(int k, int m) { return (double)(k + 1) / (double)m; }
// (+-1/2)^k/k!: the cell polynomial at the right / left edge
__host__ __device__ constexpr double edge_plus(int k) { return 1.0 / (fac(k) * two_pow(k)); }
__host__ __device__ constexpr double edge_minus(int k) { return (k % 2 == 0) ? edge_plus(k) : -edge_plus(k); }
// int_{-1/2}^{1/2} xi^s dxi for even s
__host__ __device__ constexpr double even_moment(int s) { return 1.0 / ((double)(s + 1) * two_pow(s)); }

// fused multiply-add in the bulk type (v_fma_f64 / v_fma_f32)
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double absT(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float absT(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double sqrtT(double a) { return sqrt_rn(a); }
__device__ __forceinline__ float sqrtT(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ bool finiteT(double a) { return __builtin_isfinite(a); }

// Division in the bulk type.  binary64: the correctly rounded quotient
// (div_rn; the binary64 mode is bit-reproducible).  binary32 (FP32-mixed mode, checked against the FP64
// oracle with a tolerance): the hardware reciprocal (1 ulp) times the
// numerator, both scaled by 2^100 when the divisor is below 2^-100 so that
// subnormal divisors (the limiter's epsilon is a binary32 subnormal) do not
// overflow the reciprocal; the scaling by a power of two is exact.
__device__ __forceinline__ double divT(double a, double b) { return div_rn(a, b); }
__device__ __forceinline__ float divT(float a, float b) {
  const bool tiny = __builtin_fabsf(b) < 0x1p-100f;
  const float s = tiny ? 0x1p100f : 1.0f;
  return (a * s) * __builtin_amdgcn_rcpf(b * s);
}
__device__ __forceinline__ bool finiteT(float a) { return __builtin_isfinite(a); }

// Physical parameters in the bulk type.
template <class R>
struct Phys {
  R a;      // advection speed
  R gamma;
  R gm1;    // gamma - 1
  R eps;    // limiter epsilon
};

// ---------------------------------------------------------------------------
// Register triangle of normalised Taylor coefficients X[k][m] = u_{kx,mt}/(k!m!),
// k + m <= P.  Stored square for simple constant indexing; unused entries are
// never touched.
// ---------------------------------------------------------------------------
template <class R, int P>
struct Tri {
  R v[P + 1][P + 1];
};

// (X o Y)[k][m] = sum_{a<=k} sum_{b<=m} X[a][b] Y[k-a][m-b], a outer, b inner.
template <int P, class R>
__device__ __forceinline__ R tri_mul(const Tri<R, P>& X, const Tri<R, P>& Y, int k, int m) {
  R s = X.v[0][0] * Y.v[k][m];
#pragma unroll
  for (int a = 0; a <= k; ++a) {
#pragma unroll
    for (int b = 0; b <= m; ++b) {
      if (a == 0 && b == 0) continue;
      s = fmaT(X.v[a][b], Y.v[k - a][m - b], s);
    }
  }
  return s;
}

// Quotient entry V[k][m] of V = M / Rho, given V at all lower entries.
template <int P, class R>
__device__ __forceinline__ R tri_div(const Tri<R, P>& M, const Tri<R, P>& Rho, const Tri<R, P>& V, R rinv,
                                     int k, int m) {
  R s = M.v[k][m];
#pragma unroll
  for (int a = 0; a <= k; ++a) {
#pragma unroll
    for (int b = 0; b <= m; ++b) {
      if (a == 0 && b == 0) continue;
      s = fmaT(-Rho.v[a][b], V.v[k - a][m - b], s);
    }
  }
  return s * rinv;
}

// What one old cell hands to the two new cells it overlaps.
template <int EQ, int P, class R>
struct OldOut {
  static constexpr int NC = ncomp<EQ>();
  double uR[NC];             // right half-cell average (Eq. SubEq:1DCellAVGR)
  double uL[NC];             // left half-cell average (Eq. SubEq:1DCellAVGL)
  R fbar[NC];                // time-averaged flux through the cell centre (Eq. Cal1DFlux)
  R V[NC][P > 0 ? P : 1];    // (u_kx) at the centre at t^{n+1/2}, k < P (Eq. SubEq:Cal_1D_Derivatives_4)
};

// ---------------------------------------------------------------------------
// Old cell: Cauchy-Kovalewski expansion and the derived interface quantities.
//   p[c]    : point value (binary64)
//   d[c][k] : scaled derivatives, k = 1..P (bulk type)
//   nlam    : -dt/dx in the bulk type
// ---------------------------------------------------------------------------
template <int EQ, int P, class R>
__device__ __forceinline__ void old_cell(const double (&p)[ncomp<EQ>()], const R (&d)[ncomp<EQ>()][P + 1],
                                         R nlam, const Phys<R>& ph, OldOut<EQ, P, R>& out) {
  constexpr int NC = ncomp<EQ>();
  Tri<R, P> T[NC];   // u
  Tri<R, P> G[NC];   // f(u)
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T[c].v[0][0] = (R)p[c];
#pragma unroll
    for (int k = 1; k <= P; ++k) T[c].v[k][0] = (k <= 1) ? d[c][k] : d[c][k] * (R)inv_fac(k);
  }

  // Euler work triangles: velocity, rho*u^2 is folded into the momentum flux,
  // W = rho e + p.
  Tri<R, P> vel, W;
  R rinv = (R)0;
  R fsum[NC];

#pragma unroll
  for (int m = 1; m <= P + 1; ++m) {
    const int j = m - 1;  // flux column formed at this level
#pragma unroll
    for (int k = 0; k + j <= P; ++k) {
      if constexpr (EQ == kAdvection) {
        G[0].v[k][j] = ph.a * T[0].v[k][j];
      } else if constexpr (EQ == kBurgers) {
        G[0].v[k][j] = (R)0.5 * tri_mul<P>(T[0], T[0], k, j);
      } else {
        if (k == 0 && j == 0) rinv = divT((R)1.0, T[0].v[0][0]);
        vel.v[k][j] = tri_div<P>(T[1], T[0], vel, rinv, k, j);
        const R kin = tri_mul<P>(T[1], vel, k, j);                     // rho u^2
        const R pre = ph.gm1 * (T[2].v[k][j] - (R)0.5 * kin);           // p
        W.v[k][j] = T[2].v[k][j] + pre;                                 // rho e + p
        G[0].v[k][j] = T[1].v[k][j];
        G[1].v[k][j] = kin + pre;
        G[2].v[k][j] = tri_mul<P>(W, vel, k, j);
      }
    }
    // time-averaged flux, accumulated as soon as G[.][0][j] exists
#pragma unroll
    for (int c = 0; c < NC; ++c) fsum[c] = (j == 0) ? G[c].v[0][0] : fmaT((R)flux_w(j), G[c].v[0][j], fsum[c]);
    if (m <= P) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int k = 0; k + m <= P; ++k) T[c].v[k][m] = (nlam * (R)ck_ratio(k, m)) * G[c].v[k + 1][m - 1];
      }
    }
  }

#pragma unroll
  for (int c = 0; c < NC; ++c) {
    out.fbar[c] = fsum[c];
    double r = p[c], l = p[c];
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      r = __builtin_fma(half_avg(k), (double)d[c][k], r);
      l = __builtin_fma(half_avg_left(k), (double)d[c][k], l);
    }
    out.uR[c] = r;
    out.uL[c] = l;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      R s = T[c].v[k][0];
#pragma unroll
      for (int m = 1; k + m <= P; ++m) s = s + T[c].v[k][m];
      out.V[c][k] = (k <= 1) ? s : (R)fac(k) * s;
    }
  }
}

// ---------------------------------------------------------------------------
// Jiang-Shu indicator of a degree-P polynomial in scaled derivatives d[1..P]
// (Eq. 1DSmoothIndicator): squared derivative polynomials integrated term by
// term over the unit cell.
// ---------------------------------------------------------------------------
template <int P, class R>
__device__ __forceinline__ R smoothness(const R (&d)[P + 1]) {
  R beta = (R)0;
#pragma unroll
  for (int k = 1; k <= P; ++k) {
    const int deg = P - k;
    R cp[P + 1];
#pragma unroll
    for (int n = 0; n <= deg; ++n) cp[n] = (n <= 1) ? d[k + n] : d[k + n] * (R)inv_fac(n);
    R integral = (R)0;
#pragma unroll
    for (int s = 0; s <= 2 * deg; s += 2) {
      const int n0 = (s > deg) ? s - deg : 0;
      const int n1 = (s < deg) ? s : deg;
      R sq = cp[n0] * cp[s - n0];
#pragma unroll
      for (int n = n0 + 1; n <= n1; ++n) sq = fmaT(cp[n], cp[s - n], sq);
      integral = (s == 0) ? sq : fmaT((R)even_moment(s), sq, integral);
    }
    beta = (k == 1) ? integral : beta + integral;
  }
  return beta;
}

// Normalised weights (w0, w1, w2) of Eq. 1DLimitedPolynomial.
//   binary64: the formulas of Eq. 1D2ndOrderWeights (P = 1) and
//             Eq. 1DHighOrderWeights (P >= 2) with alpha = 2, literally.
//   binary32: the same weights after dividing every unnormalised weight by
//             the largest one, so that the tiny epsilon (a binary32 subnormal)
//             and ratios up to 1e80 neither overflow nor give inf/inf.
template <int P>
__device__ __forceinline__ void limiter_weights(double b0, double b1, double b2, double st, double eps,
                                                double& w0, double& w1, double& w2) {
  double wh0, wh1, wh2;
  if (P == 1) {
    const double q0 = div_rn(1.0, b0 + eps), q1 = div_rn(1.0, b1 + eps), q2 = div_rn(1.0, b2 + eps);
    wh0 = q0 * q0;
    wh1 = q1 * q1;
    wh2 = q2 * q2;
  } else {
    const double r0 = div_rn(st, __builtin_fma(b0, b0, eps));
    const double r1 = div_rn(st, __builtin_fma(b1, b1, eps));
    const double r2 = div_rn(st, __builtin_fma(b2, b2, eps));
    wh0 = __builtin_fma(r0, r0, 1.0);
    wh1 = r1 * r1;
    wh2 = r2 * r2;
  }
  const double inv = div_rn(1.0, (wh0 + wh1) + wh2);
  w0 = wh0 * inv;
  w1 = wh1 * inv;
  w2 = wh2 * inv;
}

template <int P>
__device__ __forceinline__ void limiter_weights(float b0, float b1, float b2, float st, float eps,
                                                float& w0, float& w1, float& w2) {
  float wh0, wh1, wh2;
  if (P == 1) {
    // w_m = (1/q_m)^2 / sum_l (1/q_l)^2 = (qmin/q_m)^2 / sum_l (qmin/q_l)^2
    const float q0 = b0 + eps, q1 = b1 + eps, q2 = b2 + eps;
    const float qm = __builtin_fminf(q0, __builtin_fminf(q1, q2));
    const float x0 = divT(qm, q0), x1 = divT(qm, q1), x2 = divT(qm, q2);
    wh0 = x0 * x0;
    wh1 = x1 * x1;
    wh2 = x2 * x2;
  } else {
    // w_hat = (1 + r0^2, r1^2, r2^2) with r_m = st/q_m; if st >= qmin divide
    // all by (st/qmin)^2 first.
    const float q0 = __builtin_fmaf(b0, b0, eps), q1 = __builtin_fmaf(b1, b1, eps),
                q2 = __builtin_fmaf(b2, b2, eps);
    const float qm = __builtin_fminf(q0, __builtin_fminf(q1, q2));
    if (st >= qm) {
      const float g = divT(qm, st), x0 = divT(qm, q0), x1 = divT(qm, q1), x2 = divT(qm, q2);
      wh0 = __builtin_fmaf(x0, x0, g * g);
      wh1 = x1 * x1;
      wh2 = x2 * x2;
    } else {
      const float r0 = divT(st, q0), r1 = divT(st, q1), r2 = divT(st, q2);
      wh0 = __builtin_fmaf(r0, r0, 1.0f);
      wh1 = r1 * r1;
      wh2 = r2 * r2;
    }
  }
  const float inv = divT(1.0f, (wh0 + wh1) + wh2);
  w0 = wh0 * inv;
  w1 = wh1 * inv;
  w2 = wh2 * inv;
}

// The WENO-type limiter on one scalar (or characteristic) field of a new cell
// (Section 2.2): candidates of Eq. 1D_U012 built from the average abar and the
// vertex values vl, vr; the limited polynomial keeps abar and replaces
// d1 <- w0 d1 + w1 s1 + w2 s2, dk <- w0 dk.
template <int P, class R>
__device__ __forceinline__ void limit_field(R (&d)[P + 1], R abar, R vl, R vr, R eps) {
  const R s1 = (abar - vl) * (R)2.0;
  const R s2 = (vr - abar) * (R)2.0;
  R b0, st = (R)0;
  if constexpr (P == 1) {
    b0 = d[1] * d[1];
  } else {
    R pc = abar;
#pragma unroll
    for (int k = 2; k <= P; k += 2) pc = fmaT((R)neg_avg(k), d[k], pc);
    R ep = pc, em = pc;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      ep = fmaT((R)edge_plus(k), d[k], ep);
      em = fmaT((R)edge_minus(k), d[k], em);
    }
    const R rp = ep - vr, rm = em - vl;
    const R sigma = fmaT(rm, rm, rp * rp);
    const R tau = d[P] * d[P];
    b0 = smoothness<P>(d);
    st = sigma * tau;
  }
  const R b1 = s1 * s1, b2 = s2 * s2;
  R w0, w1, w2;
  limiter_weights<P>(b0, b1, b2, st, eps, w0, w1, w2);
  R d1 = w0 * d[1];
  d1 = fmaT(w1, s1, d1);
  d1 = fmaT(w2, s2, d1);
  d[1] = d1;
#pragma unroll
  for (int k = 2; k <= P; ++k) d[k] = w0 * d[k];
}

// Velocity, pressure and sound speed of a conserved Euler state.
template <class R>
__device__ __forceinline__ void euler_uc(const Phys<R>& ph, R rho, R mom, R ene, R& u, R& p, R& c) {
  u = divT(mom, rho);
  p = ph.gm1 * (ene - (R)0.5 * mom * u);
  c = sqrtT(divT(ph.gamma * p, rho));
}

template <class R>
__device__ __forceinline__ void mat3_apply(const R (&M)[3][3], R x0, R x1, R x2, R& y0, R& y1, R& y2) {
  R s;
  s = M[0][0] * x0; s = fmaT(M[0][1], x1, s); y0 = fmaT(M[0][2], x2, s);
  s = M[1][0] * x0; s = fmaT(M[1][1], x1, s); y1 = fmaT(M[1][2], x2, s);
  s = M[2][0] * x0; s = fmaT(M[2][1], x1, s); y2 = fmaT(M[2][2], x2, s);
}

// ---------------------------------------------------------------------------
// New cell from its left parent L (own lane) and right parent Rt (neighbour).
// Writes the new point values pn[c], derivatives dn[c][1..P], the wave speed
// and the status bits (1: non-finite, 2: rho <= 0 or p <= 0).
// ---------------------------------------------------------------------------
template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ int new_cell(const OldOut<EQ, P, R>& L, const double (&uL_R)[ncomp<EQ>()],
                                        const R (&fbar_R)[ncomp<EQ>()], const R (&V_R)[ncomp<EQ>()][P > 0 ? P : 1],
                                        double lam, const Phys<R>& ph, double (&pn)[ncomp<EQ>()],
                                        R (&dn)[ncomp<EQ>()][P + 1], double& speed) {
  constexpr int NC = ncomp<EQ>();
  double abar[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double h = 0.5 * (L.uR[c] + uL_R[c]);
    abar[c] = __builtin_fma(lam, (double)L.fbar[c] - (double)fbar_R[c], h);
    dn[c][0] = (R)0;
#pragma unroll
    for (int k = P - 1; k >= 0; --k) {
      R s = V_R[c][k] - L.V[c][k];
#pragma unroll
      for (int m = 3; m <= P - k; m += 2) s = fmaT((R)neg_odd(m), dn[c][k + m], s);
      dn[c][k + 1] = s;
    }
  }
  int flag = 0;
  R eu = (R)0, ep = (R)0, ec = (R)0;
  if constexpr (EQ == kEuler) {
    euler_uc(ph, (R)abar[0], (R)abar[1], (R)abar[2], eu, ep, ec);
    speed = (double)(absT(eu) + ec);
    if (!(abar[0] > 0.0) || !(ep > (R)0)) flag |= 2;
  } else if constexpr (EQ == kBurgers) {
    speed = __builtin_fabs(abar[0]);
  } else {
    speed = (double)absT(ph.a);
  }

  if constexpr (LIM && P >= 1) {
    if constexpr (EQ != kEuler) {
      R df[P + 1];
#pragma unroll
      for (int k = 0; k <= P; ++k) df[k] = dn[0][k];
      limit_field<P>(df, (R)abar[0], L.V[0][0], V_R[0][0], ph.eps);
#pragma unroll
      for (int k = 1; k <= P; ++k) dn[0][k] = df[k];
    } else {
      // Characteristic decomposition at the new cell average (Section 4),
      // one characteristic field at a time: row f of L projects the average,
      // the two vertex values and the derivatives; the limited field is added
      // into R*cd column by column (the same order as a full 3x3 product).
      const R rho = (R)abar[0];
      const R H = divT((R)abar[2] + ep, rho);
      const R ic = divT((R)1.0, ec);
      const R b1 = ph.gm1 * (ic * ic);
      const R b2 = (R)0.5 * b1 * (eu * eu);
      const R uic = eu * ic, b1u = b1 * eu;
      const R uc = eu * ec;
      R dout[3][P + 1];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        R l0, l1, l2, r0, r1, r2;
        if (f == 0) {
          l0 = (R)0.5 * (b2 + uic); l1 = (R)(-0.5) * (b1u + ic); l2 = (R)0.5 * b1;
          r0 = (R)1.0; r1 = eu - ec; r2 = H - uc;
        } else if (f == 1) {
          l0 = (R)1.0 - b2; l1 = b1u; l2 = -b1;
          r0 = (R)1.0; r1 = eu; r2 = (R)0.5 * (eu * eu);
        } else {
          l0 = (R)0.5 * (b2 - uic); l1 = (R)(-0.5) * (b1u - ic); l2 = (R)0.5 * b1;
          r0 = (R)1.0; r1 = eu + ec; r2 = H + uc;
        }
        R s;
        s = l0 * (R)abar[0]; s = fmaT(l1, (R)abar[1], s); const R ca = fmaT(l2, (R)abar[2], s);
        s = l0 * L.V[0][0]; s = fmaT(l1, L.V[1][0], s); const R cl = fmaT(l2, L.V[2][0], s);
        s = l0 * V_R[0][0]; s = fmaT(l1, V_R[1][0], s); const R cr = fmaT(l2, V_R[2][0], s);
        R cd[P + 1];
        cd[0] = (R)0;
#pragma unroll
        for (int k = 1; k <= P; ++k) {
          s = l0 * dn[0][k]; s = fmaT(l1, dn[1][k], s); cd[k] = fmaT(l2, dn[2][k], s);
        }
        limit_field<P>(cd, ca, cl, cr, ph.eps);
#pragma unroll
        for (int k = 1; k <= P; ++k) {
          if (f == 0) {
            dout[0][k] = r0 * cd[k];
            dout[1][k] = r1 * cd[k];
            dout[2][k] = r2 * cd[k];
          } else {
            dout[0][k] = fmaT(r0, cd[k], dout[0][k]);
            dout[1][k] = fmaT(r1, cd[k], dout[1][k]);
            dout[2][k] = fmaT(r2, cd[k], dout[2][k]);
          }
        }
        // Keep the three fields in sequence: interleaving them only raises
        // register pressure (and costs occupancy) in this latency-bound phase.
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int k = 1; k <= P; ++k) dn[c][k] = dout[c][k];
      }
    }
  }

#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double pv = abar[c];
#pragma unroll
    for (int k = 2; k <= P; k += 2) pv = __builtin_fma(neg_avg(k), (double)dn[c][k], pv);
    pn[c] = pv;
    bool ok = __builtin_isfinite(pv);
#pragma unroll
    for (int k = 1; k <= P; ++k) ok = ok && finiteT(dn[c][k]);
    if (!ok) flag |= 1;
  }
  if (!__builtin_isfinite(speed)) flag |= 1;
  return flag;
}

// Wave speed of a stored cell (used once per write for the first time step):
// the average from Eq. SubEq:1DCellAVG, then |a|, |u| or |u| + c.
template <int EQ, int P, class R>
__device__ __forceinline__ double stored_speed(const double (&p)[ncomp<EQ>()], const R (&d)[ncomp<EQ>()][P + 1],
                                               const Phys<R>& ph) {
  constexpr int NC = ncomp<EQ>();
  double abar[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double s = p[c];
#pragma unroll
    for (int k = 2; k <= P; k += 2) s = __builtin_fma(half_avg(k), (double)d[c][k], s);
    abar[c] = s;
  }
  if constexpr (EQ == kEuler) {
    R u, pr, c;
    euler_uc(ph, (R)abar[0], (R)abar[1], (R)abar[2], u, pr, c);
    return (double)(absT(u) + c);
  } else if constexpr (EQ == kBurgers) {
    return __builtin_fabs(abar[0]);
  }
  return (double)absT(ph.a);
}

}  // namespace wcc
