// wcc2d_cell.hpp -- per-cell arithmetic of the 2D WCC half-step (Section 3,
// Appendix B; the 2D Euler step of Section 4), binary64.
//
// State of a cell: the point value and the scaled derivatives
// u_{kx,ly} = dx^k dy^l d^{k+l}u/dx^k dy^l at the centre, k + l <= P, stored
// in "DOF order" (total degree n = k + l ascending, then l ascending).
//
// Arithmetic rules (shared with the rest of this library): binary64, no
// contraction; a sum of products is s = c0*x0; s = fma(ci, xi, s) in the
// index order written here; constants are exact rationals rounded once
// (compile-time division of exact integers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_rn.hpp"

namespace wcc2d {

enum { kAdvection = 0, kBurgers = 1, kEuler = 2 };

template <int EQ>
__host__ __device__ constexpr int ncomp() { return EQ == kEuler ? 4 : 1; }
__host__ __device__ constexpr int ndof(int P) { return (P + 1) * (P + 2) / 2; }
__host__ __device__ constexpr int dof(int k, int l) { return (k + l) * (k + l + 1) / 2 + l; }
__host__ __device__ constexpr int nvert(int P) { return P * (P + 1) / 2; }   // (k, l) with k + l < P

// ---- exact rational constants -------------------------------------------
__host__ __device__ constexpr double fac(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}
__host__ __device__ constexpr double p2(int n) {
  double f = 1.0;
  for (int i = 0; i < n; ++i) f *= 2.0;
  return f;
}
// 1/(k! l!)
__host__ __device__ constexpr double iff(int k, int l) { return 1.0 / (fac(k) * fac(l)); }
// k! l!
__host__ __device__ constexpr double ff(int k, int l) { return fac(k) * fac(l); }
// quarter-cell average weight 1/((k+1)! 2^k (l+1)! 2^l)   (Eq. SubEq:2DCellAVGRU)
__host__ __device__ constexpr double qa(int k, int l) { return 1.0 / (fac(k + 1) * p2(k) * fac(l + 1) * p2(l)); }
// point value from the average: -qa for even k, l
__host__ __device__ constexpr double nqa(int k, int l) { return (k % 2 == 0 && l % 2 == 0) ? -qa(k, l) : 0.0; }
// half-edge space-time moment weight 1/((s+1) 2^s (m+1))   (Eq. SubEq:2DFluxFU)
__host__ __device__ constexpr double fi(int s, int m) { return 1.0 / ((double)(s + 1) * p2(s) * (double)(m + 1)); }
// Cauchy-Kovalewski ratio (k+1)/m
__host__ __device__ constexpr double ckr(int k, int m) { return m > 0 ? (double)(k + 1) / (double)m : 0.0; }
// derivative corrections of Eq. SubEq:2DUx / 2DUy
__host__ __device__ constexpr double cx1(int s) { return (s % 2 == 1 && s >= 3) ? -(2.0 / (fac(s) * p2(s))) : 0.0; }
__host__ __device__ constexpr double cx2(int s, int t) {
  return (s % 2 == 1 && t % 2 == 0 && t >= 2) ? -(2.0 / (fac(s) * fac(t) * p2(s + t))) : 0.0;
}
// polynomial at a vertex: 1/(2^{k+l} k! l!)
__host__ __device__ constexpr double ev(int k, int l) { return 1.0 / (p2(k + l) * fac(k) * fac(l)); }
// moments over the unit square of xi^a eta^b (a, b even)
__host__ __device__ constexpr double w2(int a, int b) {
  return (a % 2 == 0 && b % 2 == 0) ? 1.0 / ((double)(a + 1) * p2(a) * (double)(b + 1) * p2(b)) : 0.0;
}

struct Phys2 {
  double a, b;        // advection velocity
  double gamma, gm1;  // gm1 = gamma - 1
  double eps;         // limiter epsilon
};

template <int P>
struct Tri3 {
  double v[P + 1][P + 1][P + 1];   // [k][l][m], k + l + m <= P
};

template <int P>
__device__ __forceinline__ double tprod3(const Tri3<P>& X, const Tri3<P>& Y, int k, int l, int m) {
  double s = X.v[0][0][0] * Y.v[k][l][m];
#pragma unroll
  for (int a = 0; a <= k; ++a)
#pragma unroll
    for (int b = 0; b <= l; ++b)
#pragma unroll
      for (int c = 0; c <= m; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        s = __builtin_fma(X.v[a][b][c], Y.v[k - a][l - b][m - c], s);
      }
  return s;
}

template <int P>
__device__ __forceinline__ double tquot3(const Tri3<P>& M, const Tri3<P>& Rho, const Tri3<P>& V, double rinv, int k,
                                         int l, int m) {
  double s = M.v[k][l][m];
#pragma unroll
  for (int a = 0; a <= k; ++a)
#pragma unroll
    for (int b = 0; b <= l; ++b)
#pragma unroll
      for (int c = 0; c <= m; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        s = __builtin_fma(-Rho.v[a][b][c], V.v[k - a][l - b][m - c], s);
      }
  return s * rinv;
}

// What one old cell hands to the four new cells it overlaps.
template <int EQ, int P>
struct Old2 {
  static constexpr int NC = ncomp<EQ>();
  double RU[NC], RD[NC], LU[NC], LD[NC];   // quarter-cell averages (Eq. SubEq:2DCellAVGRU/RD/LU/LD)
  double fU[NC], fD[NC], gR[NC], gL[NC];   // half-edge flux averages (Eq. SubEq:2DFluxFU/FD/GR/GL)
  double V[NC][nvert(P) > 0 ? nvert(P) : 1];   // (u_{kx,ly})^{n+1/2}, k + l < P, DOF order (Eq. SubEq:2DUij)
};

// Cauchy-Kovalewski expansion of one old cell and the quantities derived from
// it.  q[c][dof]: the cell's state; cx(k,m) = -(dt/dx)(k+1)/m etc. are formed
// from nlx = -dt/dx, nly = -dt/dy.
template <int EQ, int P>
__device__ __forceinline__ void old_cell2(const double (&q)[ncomp<EQ>()][ndof(P)], double nlx, double nly,
                                          const Phys2& ph, Old2<EQ, P>& o) {
  constexpr int NC = ncomp<EQ>();
  Tri3<P> T[NC];
  double Fl[NC][ndof(P)], Gl[NC][ndof(P)];   // flux coefficients of one time level
  Tri3<P> u, v, W;                            // Euler work triangles
  double rinv = 0.0;
  double fu[NC], fd[NC], gr[NC], gl[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int n = 0; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        const double x = q[c][dof(k, l)];
        T[c].v[k][l][0] = (k <= 1 && l <= 1) ? x : x * iff(k, l);
      }

#pragma unroll
  for (int m = 0; m <= P; ++m) {
    // fluxes at time level m, entries k + l <= P - m
#pragma unroll
    for (int n = 0; n <= P - m; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const int k = n - l, d = dof(k, l);
        if constexpr (EQ == kAdvection) {
          Fl[0][d] = ph.a * T[0].v[k][l][m];
          Gl[0][d] = ph.b * T[0].v[k][l][m];
        } else if constexpr (EQ == kBurgers) {
          const double h = 0.5 * tprod3<P>(T[0], T[0], k, l, m);
          Fl[0][d] = h;
          Gl[0][d] = h;
        } else {
          if (k == 0 && l == 0 && m == 0) rinv = wcc::div_rn(1.0, T[0].v[0][0][0]);
          u.v[k][l][m] = tquot3<P>(T[1], T[0], u, rinv, k, l, m);
          v.v[k][l][m] = tquot3<P>(T[2], T[0], v, rinv, k, l, m);
          const double kx = tprod3<P>(T[1], u, k, l, m);
          const double ky = tprod3<P>(T[2], v, k, l, m);
          const double kxy = tprod3<P>(T[1], v, k, l, m);
          const double p = ph.gm1 * (T[3].v[k][l][m] - 0.5 * (kx + ky));
          W.v[k][l][m] = T[3].v[k][l][m] + p;
          Fl[0][d] = T[1].v[k][l][m];
          Fl[1][d] = kx + p;
          Fl[2][d] = kxy;
          Fl[3][d] = tprod3<P>(W, u, k, l, m);
          Gl[0][d] = T[2].v[k][l][m];
          Gl[1][d] = kxy;
          Gl[2][d] = ky + p;
          Gl[3][d] = tprod3<P>(W, v, k, l, m);
        }
      }
    // half-edge averages, this level's moments (time index outer, offset inner)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int s = 0; s <= P - m; ++s) {
        const double w = fi(s, m), ws = (s % 2) ? -w : w;
        const double F0 = Fl[c][dof(0, s)], G0 = Gl[c][dof(s, 0)];
        if (m == 0 && s == 0) {
          fu[c] = F0; fd[c] = F0; gr[c] = G0; gl[c] = G0;
        } else {
          fu[c] = __builtin_fma(w, F0, fu[c]);
          fd[c] = __builtin_fma(ws, F0, fd[c]);
          gr[c] = __builtin_fma(w, G0, gr[c]);
          gl[c] = __builtin_fma(ws, G0, gl[c]);
        }
      }
    // next level of the expansion:
    //   T[k][l][m+1] = -((dt/dx)(k+1) F[k+1][l][m] + (dt/dy)(l+1) G[k][l+1][m]) / (m+1)
    if (m < P) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int n = 0; n <= P - m - 1; ++n)
#pragma unroll
          for (int l = 0; l <= n; ++l) {
            const int k = n - l;
            T[c].v[k][l][m + 1] = __builtin_fma(nly * ckr(l, m + 1), Gl[c][dof(k, l + 1)],
                                                (nlx * ckr(k, m + 1)) * Fl[c][dof(k + 1, l)]);
          }
    }
  }

#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double ru = q[c][0], rd = q[c][0], lu = q[c][0], ld = q[c][0];
#pragma unroll
    for (int n = 1; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        const double x = q[c][dof(k, l)];
        ru = __builtin_fma(qa(k, l), x, ru);
        rd = __builtin_fma((l % 2) ? -qa(k, l) : qa(k, l), x, rd);
        lu = __builtin_fma((k % 2) ? -qa(k, l) : qa(k, l), x, lu);
        ld = __builtin_fma(((k + l) % 2) ? -qa(k, l) : qa(k, l), x, ld);
      }
    o.RU[c] = ru; o.RD[c] = rd; o.LU[c] = lu; o.LD[c] = ld;
    o.fU[c] = fu[c]; o.fD[c] = fd[c]; o.gR[c] = gr[c]; o.gL[c] = gl[c];
#pragma unroll
    for (int n = 0; n < P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        double s = T[c].v[k][l][0];
#pragma unroll
        for (int m = 1; m <= P - n; ++m) s = s + T[c].v[k][l][m];
        o.V[c][dof(k, l)] = (k <= 1 && l <= 1) ? s : ff(k, l) * s;
      }
  }
}

// Eq. 2DSmoothIndicator: sum over 1 <= k + l <= P of the integral over the
// unit square of (d^k_xi d^l_eta p)^2, each derivative polynomial squared
// pair by pair.
template <int P>
__device__ __forceinline__ double js2d(const double (&D)[P + 1][P + 1]) {
  double beta = 0.0;
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int l = 0; l <= n; ++l) {
      const int k = n - l, d = P - n;
      constexpr int NCF = ndof(P);
      double cf[NCF];
#pragma unroll
      for (int e = 0; e <= d; ++e)
#pragma unroll
        for (int t = 0; t <= e; ++t) {
          const int s = e - t;
          const double x = D[k + s][l + t];
          cf[dof(s, t)] = (s <= 1 && t <= 1) ? x : x * iff(s, t);
        }
      double acc = cf[0] * cf[0];
#pragma unroll
      for (int e1 = 0; e1 <= d; ++e1)
#pragma unroll
        for (int t1 = 0; t1 <= e1; ++t1)
#pragma unroll
          for (int e2 = 0; e2 <= d; ++e2)
#pragma unroll
            for (int t2 = 0; t2 <= e2; ++t2) {
              const int s1 = e1 - t1, s2 = e2 - t2;
              if (e1 == 0 && e2 == 0) continue;
              if ((s1 + s2) % 2 || (t1 + t2) % 2) continue;
              acc = __builtin_fma(w2(s1 + s2, t1 + t2), cf[dof(s1, t1)] * cf[dof(s2, t2)], acc);
            }
      beta = (n == 1 && l == 0) ? acc : beta + acc;
    }
  return beta;
}

// The 2D limiter of Section 3.2 on one new cell (Eq. 2DLimitedPolynomial,
// 2DLowOrderPolynomial, 2D2ndOrderWeights, high-order weights with sigma and
// tau); D holds the unlimited scaled derivatives and is modified in place.
template <int P>
__device__ __forceinline__ void limit2d(double eps, double abar, double (&D)[P + 1][P + 1], double vld, double vrd,
                                        double vru, double vlu) {
  const double a2 = abar * 2.0;
  const double ux1 = a2 - (vld + vlu), uy1 = vlu - vld;
  const double ux2 = vrd - vld, uy2 = a2 - (vld + vrd);
  const double ux3 = (vrd + vru) - a2, uy3 = vru - vrd;
  const double ux4 = vru - vlu, uy4 = (vlu + vru) - a2;
  const double b0 = js2d<P>(D);
  const double b1 = __builtin_fma(uy1, uy1, ux1 * ux1), b2 = __builtin_fma(uy2, uy2, ux2 * ux2);
  const double b3 = __builtin_fma(uy3, uy3, ux3 * ux3), b4 = __builtin_fma(uy4, uy4, ux4 * ux4);
  double wh0, wh1, wh2, wh3, wh4;
  if constexpr (P == 1) {
    const double q0 = wcc::div_rn(1.0, b0 + eps), q1 = wcc::div_rn(1.0, b1 + eps), q2 = wcc::div_rn(1.0, b2 + eps),
                 q3 = wcc::div_rn(1.0, b3 + eps), q4 = wcc::div_rn(1.0, b4 + eps);
    wh0 = q0 * q0; wh1 = q1 * q1; wh2 = q2 * q2; wh3 = q3 * q3; wh4 = q4 * q4;
  } else {
    double p0 = abar;
#pragma unroll
    for (int n = 2; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        if (k % 2 == 0 && l % 2 == 0) p0 = __builtin_fma(nqa(k, l), D[k][l], p0);
      }
    double sigma = 0.0;
    const double vv[4] = {vld, vrd, vru, vlu};
#pragma unroll
    for (int vtx = 0; vtx < 4; ++vtx) {
      const int sx = (vtx == 0 || vtx == 3) ? -1 : 1, sy = (vtx < 2) ? -1 : 1;   // LD, RD, RU, LU
      double s = p0;
#pragma unroll
      for (int n = 1; n <= P; ++n)
#pragma unroll
        for (int l = 0; l <= n; ++l) {
          const int k = n - l;
          const int sg = ((k % 2) ? sx : 1) * ((l % 2) ? sy : 1);
          s = __builtin_fma(sg > 0 ? ev(k, l) : -ev(k, l), D[k][l], s);
        }
      const double r = s - vv[vtx];
      sigma = (vtx == 0) ? r * r : __builtin_fma(r, r, sigma);
    }
    double tau = D[0][P] * D[0][P];
#pragma unroll
    for (int k = 1; k <= P; ++k) tau = __builtin_fma(D[k][P - k], D[k][P - k], tau);
    const double st = sigma * tau;
    const double r0 = wcc::div_rn(st, __builtin_fma(b0, b0, eps)), r1 = wcc::div_rn(st, __builtin_fma(b1, b1, eps)),
                 r2 = wcc::div_rn(st, __builtin_fma(b2, b2, eps)), r3 = wcc::div_rn(st, __builtin_fma(b3, b3, eps)),
                 r4 = wcc::div_rn(st, __builtin_fma(b4, b4, eps));
    wh0 = __builtin_fma(r0, r0, 1.0); wh1 = r1 * r1; wh2 = r2 * r2; wh3 = r3 * r3; wh4 = r4 * r4;
  }
  const double inv = wcc::div_rn(1.0, (((wh0 + wh1) + wh2) + wh3) + wh4);
  const double w0 = wh0 * inv, w1 = wh1 * inv, w2_ = wh2 * inv, w3 = wh3 * inv, w4 = wh4 * inv;
  double dx1 = w0 * D[1][0], dy1 = w0 * D[0][1];
  dx1 = __builtin_fma(w1, ux1, dx1); dy1 = __builtin_fma(w1, uy1, dy1);
  dx1 = __builtin_fma(w2_, ux2, dx1); dy1 = __builtin_fma(w2_, uy2, dy1);
  dx1 = __builtin_fma(w3, ux3, dx1); dy1 = __builtin_fma(w3, uy3, dy1);
  dx1 = __builtin_fma(w4, ux4, dx1); dy1 = __builtin_fma(w4, uy4, dy1);
  D[1][0] = dx1;
  D[0][1] = dy1;
#pragma unroll
  for (int n = 2; n <= P; ++n)
#pragma unroll
    for (int l = 0; l <= n; ++l) D[n - l][l] = w0 * D[n - l][l];
}

// Rotated characteristic limiting of a 2D Euler new cell (Section 4): the
// direction n = grad(phi)/|grad(phi)| with phi = rho e from the new cell's
// central-difference derivatives (Eq. RotatedNormal; n = (1, 0) where the
// gradient vanishes); the eigenvectors of A cos(theta) + B sin(theta) at the
// new average; every characteristic field through limit2d; back with R.
// v[c][vtx]: vertex values, vtx = LD, RD, RU, LU.
template <int P>
__device__ __forceinline__ void char_limit2d(const Phys2& ph, double dx, double dy, const double (&ab)[4],
                                             double (&D)[4][P + 1][P + 1], const double (&v)[4][4]) {
  const double gx = wcc::div_rn(D[3][1][0], dx), gy = wcc::div_rn(D[3][0][1], dy);
  const double g2 = __builtin_fma(gy, gy, gx * gx);
  double nx = 1.0, ny = 0.0;
  if (g2 > 0.0) {
    const double gn = wcc::sqrt_rn(g2);
    nx = wcc::div_rn(gx, gn);
    ny = wcc::div_rn(gy, gn);
  }
  const double rho = ab[0], u = wcc::div_rn(ab[1], rho), vv = wcc::div_rn(ab[2], rho);
  const double p = ph.gm1 * (ab[3] - 0.5 * __builtin_fma(ab[2], vv, ab[1] * u));
  const double c = wcc::sqrt_rn(wcc::div_rn(ph.gamma * p, rho));
  const double H = wcc::div_rn(ab[3] + p, rho);
  const double un = __builtin_fma(vv, ny, u * nx), ut = __builtin_fma(vv, nx, -(u * ny));
  const double q2 = __builtin_fma(vv, vv, u * u);
  const double ic = wcc::div_rn(1.0, c);
  const double b1 = ph.gm1 * (ic * ic), b2 = 0.5 * (q2 * b1);
  const double uic = un * ic, nxic = nx * ic, nyic = ny * ic, b1u = b1 * u, b1v = b1 * vv;
  const double L[4][4] = {{0.5 * (b2 + uic), -0.5 * (b1u + nxic), -0.5 * (b1v + nyic), 0.5 * b1},
                          {1.0 - b2, b1u, b1v, -b1},
                          {-ut, -ny, nx, 0.0},
                          {0.5 * (b2 - uic), -0.5 * (b1u - nxic), -0.5 * (b1v - nyic), 0.5 * b1}};
  const double cun = c * un;
  const double R[4][4] = {{1.0, u - c * nx, vv - c * ny, H - cun},
                          {1.0, u, vv, 0.5 * q2},
                          {0.0, -ny, nx, ut},
                          {1.0, u + c * nx, vv + c * ny, H + cun}};
  double out[4][P + 1][P + 1];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    auto proj = [&](double x0, double x1, double x2, double x3) {
      double s = L[f][0] * x0;
      s = __builtin_fma(L[f][1], x1, s);
      s = __builtin_fma(L[f][2], x2, s);
      if (f != 2) s = __builtin_fma(L[f][3], x3, s);
      return s;
    };
    const double ca = proj(ab[0], ab[1], ab[2], ab[3]);
    double cv[4];
#pragma unroll
    for (int vtx = 0; vtx < 4; ++vtx) cv[vtx] = proj(v[0][vtx], v[1][vtx], v[2][vtx], v[3][vtx]);
    double cD[P + 1][P + 1];
#pragma unroll
    for (int n = 1; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) cD[n - l][l] = proj(D[0][n - l][l], D[1][n - l][l], D[2][n - l][l], D[3][n - l][l]);
    limit2d<P>(ph.eps, ca, cD, cv[0], cv[1], cv[2], cv[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (f == 2 && r == 0) continue;
#pragma unroll
      for (int n = 1; n <= P; ++n)
#pragma unroll
        for (int l = 0; l <= n; ++l) {
          const int k = n - l;
          out[r][k][l] = (f == 0) ? R[f][r] * cD[k][l] : __builtin_fma(R[f][r], cD[k][l], out[r][k][l]);
        }
    }
    // keep the four fields in sequence (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int n = 1; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) D[r][n - l][l] = out[r][n - l][l];
}

// New derivatives of one component, highest total order first (Eq.
// SubEq:2DUx, SubEq:2DUy; cross derivatives as the mean of the two).  Parents:
// A lower-left, B upper-left, C lower-right, E upper-right vertex of the new
// cell; their vertex values in DOF order.
template <int P>
__device__ __forceinline__ void new_derivatives(const double* VA, const double* VB, const double* VC,
                                                const double* VE, double (&D)[P + 1][P + 1]) {
#pragma unroll
  for (int n = P; n >= 1; --n)
#pragma unroll
    for (int l = 0; l <= n; ++l) {
      const int k = n - l;
      double X = 0.0, Y = 0.0;
      if (k >= 1) {
        const int kb = k - 1, r = P - kb - l, i = dof(kb, l);
        X = 0.5 * ((VC[i] - VA[i]) + (VE[i] - VB[i]));
#pragma unroll
        for (int s = 3; s <= r; s += 2) X = __builtin_fma(cx1(s), D[kb + s][l], X);
#pragma unroll
        for (int t = 2; t <= r; t += 2)
#pragma unroll
          for (int s = 1; s <= r - t; s += 2) X = __builtin_fma(cx2(s, t), D[kb + s][l + t], X);
      }
      if (l >= 1) {
        const int lb = l - 1, r = P - k - lb, i = dof(k, lb);
        Y = 0.5 * ((VB[i] - VA[i]) + (VE[i] - VC[i]));
#pragma unroll
        for (int t = 3; t <= r; t += 2) Y = __builtin_fma(cx1(t), D[k][lb + t], Y);
#pragma unroll
        for (int t = 1; t <= r; t += 2)
#pragma unroll
          for (int s = 2; s <= r - t; s += 2) Y = __builtin_fma(cx2(t, s), D[k + s][lb + t], Y);
      }
      D[k][l] = (k >= 1 && l >= 1) ? 0.5 * (X + Y) : (k >= 1 ? X : Y);
    }
}

// Point value from the average (inverse of Eq. SubEq:2DCellAVG).
template <int P>
__device__ __forceinline__ double point_value(double abar, const double (&D)[P + 1][P + 1]) {
  double pv = abar;
#pragma unroll
  for (int n = 2; n <= P; ++n)
#pragma unroll
    for (int l = 0; l <= n; ++l) {
      const int k = n - l;
      if (k % 2 == 0 && l % 2 == 0) pv = __builtin_fma(nqa(k, l), D[k][l], pv);
    }
  return pv;
}

// Wave-speed rate s_x/dx + s_y/dy of a conserved average; status bit 2 for a
// non-positive density or pressure.
template <int EQ>
__device__ __forceinline__ double speed_rate(const double (&ab)[ncomp<EQ>()], const Phys2& ph, double idx,
                                             double idy, unsigned& flag) {
  if constexpr (EQ == kAdvection) {
    return __builtin_fma(__builtin_fabs(ph.b), idy, __builtin_fabs(ph.a) * idx);
  } else if constexpr (EQ == kBurgers) {
    const double s = __builtin_fabs(ab[0]);
    return __builtin_fma(s, idy, s * idx);
  } else {
    const double rho = ab[0];
    const double u = wcc::div_rn(ab[1], rho), v = wcc::div_rn(ab[2], rho);
    const double p = ph.gm1 * (ab[3] - 0.5 * __builtin_fma(ab[2], v, ab[1] * u));
    const double c = wcc::sqrt_rn(wcc::div_rn(ph.gamma * p, rho));
    if (!(rho > 0.0) || !(p > 0.0)) flag |= 2u;
    return __builtin_fma(__builtin_fabs(v) + c, idy, (__builtin_fabs(u) + c) * idx);
  }
}

}  // namespace wcc2d
