// wcc2d_oracle.cpp -- plain FP64 CPU reference of the 2D weighted compact
// central (WCC) half-step on Cartesian meshes (Section 3 and Appendix B of
// Shen & Parsani, arXiv:2104.04347), including the 2D Euler half-step of
// Section 4, unlimited (LCCS) or limited in the rotated characteristic
// decomposition (WCCS).
//
// TEST INFRASTRUCTURE ONLY, like the 1D oracle in this directory: tests, the
// smoke check and the CPU-baseline leg of the benchmark use it; the product
// never links or calls it, and it shares no code with the GPU path.
//
// What one half-step computes (periodic mesh, Section 3.1):
//   * state of a cell: the point value and the scaled derivatives
//     u_{kx,ly} = dx^k dy^l d^{k+l}u/dx^k dy^l at the centre, k + l <= P
//     (Eq. 2DPolynomial_Space);
//   * Cauchy-Kovalewski expansion of every old cell in normalised trivariate
//     Taylor arithmetic, T[k][l][m] = u_{kx,ly,mt}/(k! l! m!), from
//     u_t = -f_x - g_y (Eq. SubEq:2DHCL_Eq);
//   * quarter-cell averages (Eq. SubEq:2DCellAVGRU/RD/LU/LD) and
//     half-edge space-time flux averages (Eq. SubEq:2DFluxFD/FU/GL/GR)
//     -> new cell average by the balance on the staggered control volume
//     (Eq. 2DIntegral);
//   * vertex values at the half time level (Eq. SubEq:2DUij) -> new
//     derivatives, highest total order first, x-formula (Eq. SubEq:2DUx),
//     y-formula (Eq. SubEq:2DUy), cross derivatives as the mean of the two
//     (the remark after Eq. 2DDerivatives);
//   * the 2D limiter of Section 3.2 (five candidates, Eq.
//     2DLimitedPolynomial, 2DLowOrderPolynomial, 2D2ndOrderWeights for P = 1,
//     the high-order weights with sigma and tau for P >= 2, smoothness
//     indicator Eq. 2DSmoothIndicator); for the Euler equations applied to
//     the characteristic fields of the rotated decomposition of Section 4;
//   * new point value from the new average (inverse of Eq. SubEq:2DCellAVG).
//
// Canonical arithmetic: the rules of the 1D oracle (binary64, no
// contraction; sums of products left to right as s = c0*x0; s = fma(ci, xi, s);
// constants exact rationals rounded once).  Index order of every sum: over
// (k, l) pairs by total degree n = k + l ascending, then l ascending (the
// "DOF order"); over (a, b, c) in Taylor products a outer, b, c inner; the
// half-edge flux averages time index outer, offset inner (Appendix B).
//
// Readings (design notes of the repository): state = point value; time step
// dt = cfl / max_cells(s_x/dx + s_y/dy) from the cell averages, recomputed
// every half-step and clipped to t_end; periodic or transmissive edges, per
// direction.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace w2d {

constexpr int PMAX = 4;
constexpr int NCMAX = 4;
enum { EQ_ADVECTION = 0, EQ_BURGERS = 1, EQ_EULER = 2 };

inline int ndof(int P) { return (P + 1) * (P + 2) / 2; }
inline int dof(int k, int l) { const int n = k + l; return n * (n + 1) / 2 + l; }

// Exact rational constants, each rounded once to binary64.
struct Consts {
  double fact[2 * PMAX + 3];
  double IFF[PMAX + 1][PMAX + 1];   // 1/(k! l!)
  double FF[PMAX + 1][PMAX + 1];    // k! l!
  double QA[PMAX + 1][PMAX + 1];    // 1/((k+1)! 2^k (l+1)! 2^l)    Eq. SubEq:2DCellAVGRU
  double NQA[PMAX + 1][PMAX + 1];   // -QA for even k, l (point value from the average), else 0
  double FI[PMAX + 1][PMAX + 1];    // 1/((s+1) 2^s (m+1))           Eq. SubEq:2DFluxFU (normalised)
  double CKR[PMAX + 1][PMAX + 1];   // (k+1)/m
  double CX1[PMAX + 1];             // -2/(s! 2^s) for odd s >= 3     Eq. SubEq:2DUx, first sum
  double CX2[PMAX + 1][PMAX + 1];   // -2/(s! t! 2^{s+t}), s odd, t even >= 2 (and transposed use)
  double EV[PMAX + 1][PMAX + 1];    // 1/(2^{k+l} k! l!)             polynomial at a vertex
  double W2[2 * PMAX + 1][2 * PMAX + 1];  // int xi^n1 eta^n2 over the unit square, n1, n2 even
  Consts() {
    fact[0] = 1.0;
    for (int k = 1; k < 2 * PMAX + 3; ++k) fact[k] = fact[k - 1] * (double)k;
    for (int k = 0; k <= PMAX; ++k)
      for (int l = 0; l <= PMAX; ++l) {
        IFF[k][l] = 1.0 / (fact[k] * fact[l]);
        FF[k][l] = fact[k] * fact[l];
        QA[k][l] = 1.0 / (fact[k + 1] * std::ldexp(1.0, k) * fact[l + 1] * std::ldexp(1.0, l));
        NQA[k][l] = (k % 2 == 0 && l % 2 == 0) ? -QA[k][l] : 0.0;
        FI[k][l] = 1.0 / ((double)(k + 1) * std::ldexp(1.0, k) * (double)(l + 1));
        CKR[k][l] = (l > 0) ? (double)(k + 1) / (double)l : 0.0;
        EV[k][l] = 1.0 / (std::ldexp(1.0, k + l) * fact[k] * fact[l]);
        CX2[k][l] = (k % 2 == 1 && l % 2 == 0 && l >= 2)
                        ? -(2.0 / (fact[k] * fact[l] * std::ldexp(1.0, k + l))) : 0.0;
      }
    for (int s = 0; s <= PMAX; ++s) CX1[s] = (s % 2 == 1 && s >= 3) ? -(2.0 / (fact[s] * std::ldexp(1.0, s))) : 0.0;
    for (int a = 0; a <= 2 * PMAX; ++a)
      for (int b = 0; b <= 2 * PMAX; ++b)
        W2[a][b] = (a % 2 == 0 && b % 2 == 0)
                       ? 1.0 / ((double)(a + 1) * std::ldexp(1.0, a) * (double)(b + 1) * std::ldexp(1.0, b)) : 0.0;
  }
};
const Consts K;

}  // namespace w2d

extern "C" {
typedef struct {
  int32_t equation;  // 0 advection (f = a u, g = b u), 1 Burgers (f = g = u^2/2), 2 Euler
  int32_t P;         // degree 0..4
  int64_t Nx, Ny;    // mesh intervals per direction
  int32_t limiter;
  int32_t bc;        // x edges: 0 periodic, 1 transmissive (see Mesh below)
  int32_t bc_y;      // y edges: likewise; -1: as bc
  int32_t pad2;
  double x_left, x_right, y_left, y_right;
  double a, b;       // advection velocity
  double gamma;
  double eps;        // limiter epsilon (1e-40)
} wcc2d_oracle_problem;
}

namespace w2d {

using Tri3 = double[PMAX + 1][PMAX + 1][PMAX + 1];   // [k][l][m], k + l + m <= P

inline int ncomp(const wcc2d_oracle_problem& pb) { return pb.equation == EQ_EULER ? 4 : 1; }

// (X o Y)[k][l][m] = sum_{a<=k} sum_{b<=l} sum_{c<=m} X[a][b][c] Y[k-a][l-b][m-c]
double tprod3(const Tri3& X, const Tri3& Y, int k, int l, int m) {
  double s = X[0][0][0] * Y[k][l][m];
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= l; ++b)
      for (int c = 0; c <= m; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        s = std::fma(X[a][b][c], Y[k - a][l - b][m - c], s);
      }
  return s;
}

// Quotient V = M / Rho at [k][l][m], lower entries of V known.
double tquot3(const Tri3& M, const Tri3& Rho, const Tri3& V, double rinv, int k, int l, int m) {
  double s = M[k][l][m];
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= l; ++b)
      for (int c = 0; c <= m; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        s = std::fma(-Rho[a][b][c], V[k - a][l - b][m - c], s);
      }
  return s * rinv;
}

struct Work {
  Tri3 u, v, W;   // Euler: velocities, energy + pressure
  double rinv;
};

// Flux coefficients F = f(U), G = g(U) at time level m, entries k + l <= P - m.
void flux_level(const wcc2d_oracle_problem& pb, int P, Tri3* T, Tri3* F, Tri3* G, Work& w, int m) {
  for (int n = 0; n <= P - m; ++n)
    for (int l = 0; l <= n; ++l) {
      const int k = n - l;
      if (pb.equation == EQ_ADVECTION) {
        F[0][k][l][m] = pb.a * T[0][k][l][m];
        G[0][k][l][m] = pb.b * T[0][k][l][m];
      } else if (pb.equation == EQ_BURGERS) {
        const double h = 0.5 * tprod3(T[0], T[0], k, l, m);
        F[0][k][l][m] = h;
        G[0][k][l][m] = h;
      } else {
        const Tri3 &rho = T[0], &mx = T[1], &my = T[2], &E = T[3];
        if (k == 0 && l == 0 && m == 0) w.rinv = 1.0 / rho[0][0][0];
        w.u[k][l][m] = tquot3(mx, rho, w.u, w.rinv, k, l, m);     // u = (rho u)/rho
        w.v[k][l][m] = tquot3(my, rho, w.v, w.rinv, k, l, m);     // v = (rho v)/rho
        const double kx = tprod3(mx, w.u, k, l, m);                // rho u^2
        const double ky = tprod3(my, w.v, k, l, m);                // rho v^2
        const double kxy = tprod3(mx, w.v, k, l, m);               // rho u v
        const double p = (pb.gamma - 1.0) * (E[k][l][m] - 0.5 * (kx + ky));
        w.W[k][l][m] = E[k][l][m] + p;                              // rho e + p
        F[0][k][l][m] = mx[k][l][m];
        F[1][k][l][m] = kx + p;
        F[2][k][l][m] = kxy;
        F[3][k][l][m] = tprod3(w.W, w.u, k, l, m);
        G[0][k][l][m] = my[k][l][m];
        G[1][k][l][m] = kxy;
        G[2][k][l][m] = ky + p;
        G[3][k][l][m] = tprod3(w.W, w.v, k, l, m);
      }
    }
}

// What one old cell hands to the four new cells it overlaps.
struct Old {
  double RU[NCMAX], RD[NCMAX], LU[NCMAX], LD[NCMAX];   // quarter-cell averages
  double fU[NCMAX], fD[NCMAX], gR[NCMAX], gL[NCMAX];   // half-edge space-time flux averages
  double V[NCMAX][PMAX + 1][PMAX + 1];                  // (u_{kx,ly})^{n+1/2} at the centre, k + l < P
};

// q[c][dof]: the cell's state.  cx[k][m] = -(dt/dx)(k+1)/m, cy[l][m] = -(dt/dy)(l+1)/m.
void old_cell(const wcc2d_oracle_problem& pb, const double q[NCMAX][32], const double cx[PMAX + 1][PMAX + 1],
              const double cy[PMAX + 1][PMAX + 1], Old& o) {
  const int P = pb.P, nc = ncomp(pb);
  static thread_local Tri3 T[NCMAX], F[NCMAX], G[NCMAX];
  static thread_local Work w;
  for (int c = 0; c < nc; ++c)
    for (int n = 0; n <= P; ++n)
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        const double x = q[c][dof(k, l)];
        T[c][k][l][0] = (k <= 1 && l <= 1) ? x : x * K.IFF[k][l];
      }
  // Level m of the expansion: fluxes at level m-1, then
  //   T[k][l][m] = -( (dt/dx)(k+1) F[k+1][l][m-1] + (dt/dy)(l+1) G[k][l+1][m-1] ) / m.
  for (int m = 1; m <= P; ++m) {
    flux_level(pb, P, T, F, G, w, m - 1);
    for (int c = 0; c < nc; ++c)
      for (int n = 0; n <= P - m; ++n)
        for (int l = 0; l <= n; ++l) {
          const int k = n - l;
          T[c][k][l][m] = std::fma(cy[l][m], G[c][k][l + 1][m - 1], cx[k][m] * F[c][k + 1][l][m - 1]);
        }
  }
  flux_level(pb, P, T, F, G, w, P);

  for (int c = 0; c < nc; ++c) {
    // quarter-cell averages from the stored state, DOF order
    double ru = q[c][0], rd = q[c][0], lu = q[c][0], ld = q[c][0];
    for (int n = 1; n <= P; ++n)
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        const double x = q[c][dof(k, l)], qa = K.QA[k][l];
        ru = std::fma(qa, x, ru);
        rd = std::fma((l % 2) ? -qa : qa, x, rd);
        lu = std::fma((k % 2) ? -qa : qa, x, lu);
        ld = std::fma(((k + l) % 2) ? -qa : qa, x, ld);
      }
    o.RU[c] = ru; o.RD[c] = rd; o.LU[c] = lu; o.LD[c] = ld;
    // half-edge flux averages: f along the line x = x_i (y offset s, time m),
    // g along y = y_j (x offset s, time m); time index outer, offset inner,
    // the order of the double sums of Appendix B
    double fu = F[c][0][0][0], fd = F[c][0][0][0], gr = G[c][0][0][0], gl = G[c][0][0][0];
    for (int m = 0; m <= P; ++m)
      for (int s = (m == 0) ? 1 : 0; s <= P - m; ++s) {
        const double fi = K.FI[s][m];
        fu = std::fma(fi, F[c][0][s][m], fu);
        fd = std::fma((s % 2) ? -fi : fi, F[c][0][s][m], fd);
        gr = std::fma(fi, G[c][s][0][m], gr);
        gl = std::fma((s % 2) ? -fi : fi, G[c][s][0][m], gl);
      }
    o.fU[c] = fu; o.fD[c] = fd; o.gR[c] = gr; o.gL[c] = gl;
    // Eq. SubEq:2DUij: (u_{kx,ly})^{n+1/2} = k! l! sum_m T[k][l][m]
    for (int n = 0; n < P; ++n)
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        double s = T[c][k][l][0];
        for (int m = 1; m <= P - n; ++m) s = s + T[c][k][l][m];
        o.V[c][k][l] = (k <= 1 && l <= 1) ? s : K.FF[k][l] * s;
      }
  }
}

// 2D smoothness indicator (Eq. 2DSmoothIndicator) of the polynomial with
// scaled derivatives D[k][l], 1 <= k + l <= P:
//   beta = sum_{1<=k+l<=P} int int (d^k_xi d^l_eta p)^2 over [-1/2,1/2]^2,
// each derivative polynomial c(xi, eta) = sum_{s+t<=P-k-l} D[k+s][l+t]/(s! t!) xi^s eta^t
// squared pair by pair (DOF order, both indices) and integrated term by term.
double js2d(int P, const double D[PMAX + 1][PMAX + 1]) {
  double beta = 0.0;
  bool first = true;
  for (int n = 1; n <= P; ++n)
    for (int l = 0; l <= n; ++l) {
      const int k = n - l, d = P - n;
      double cf[32] = {};
      int cs[32], ct[32], nc = 0;
      for (int e = 0; e <= d; ++e)
        for (int t = 0; t <= e; ++t) {
          const int s = e - t;
          const double x = D[k + s][l + t];
          cf[nc] = (s <= 1 && t <= 1) ? x : x * K.IFF[s][t];
          cs[nc] = s;
          ct[nc] = t;
          ++nc;
        }
      double acc = cf[0] * cf[0];
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
          if (i == 0 && j == 0) continue;
          if ((cs[i] + cs[j]) % 2 || (ct[i] + ct[j]) % 2) continue;
          acc = std::fma(K.W2[cs[i] + cs[j]][ct[i] + ct[j]], cf[i] * cf[j], acc);
        }
      beta = first ? acc : beta + acc;
      first = false;
    }
  return beta;
}

// The 2D limiter (Section 3.2) on one new cell: abar the average, D the
// unlimited scaled derivatives (modified in place), vertex values
// vld = u(x_{i-1/2}, y_{j-1/2}), vrd, vru, vlu from Eq. SubEq:2DUij.
void limit2d(int P, double eps, double abar, double D[PMAX + 1][PMAX + 1], double vld, double vrd, double vru,
             double vlu) {
  const double a2 = abar * 2.0;
  // Eq. 2DLowOrderPolynomial: slopes (u_x^m, u_y^m) of the four edge candidates
  const double ux[5] = {0.0, a2 - (vld + vlu), vrd - vld, (vrd + vru) - a2, vru - vlu};
  const double uy[5] = {0.0, vlu - vld, a2 - (vld + vrd), vru - vrd, (vlu + vru) - a2};
  double beta[5];
  beta[0] = js2d(P, D);
  for (int m = 1; m <= 4; ++m) beta[m] = std::fma(uy[m], uy[m], ux[m] * ux[m]);
  double wh[5];
  if (P == 1) {
    // Eq. 2D2ndOrderWeights, alpha = 2
    for (int m = 0; m <= 4; ++m) {
      const double qm = 1.0 / (beta[m] + eps);
      wh[m] = qm * qm;
    }
  } else {
    // high-order weights: w0 = 1 + (sigma tau/(beta0^2 + eps))^2,
    // wm = (sigma tau/(betam^2 + eps))^2
    double p0 = abar;
    for (int n = 2; n <= P; ++n)
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        if (k % 2 == 0 && l % 2 == 0) p0 = std::fma(K.NQA[k][l], D[k][l], p0);
      }
    const int sx[4] = {-1, 1, 1, -1}, sy[4] = {-1, -1, 1, 1};   // LD, RD, RU, LU
    const double vv[4] = {vld, vrd, vru, vlu};
    double sigma = 0.0;
    for (int vtx = 0; vtx < 4; ++vtx) {
      double s = p0;
      for (int n = 1; n <= P; ++n)
        for (int l = 0; l <= n; ++l) {
          const int k = n - l;
          const int sg = ((k % 2) ? sx[vtx] : 1) * ((l % 2) ? sy[vtx] : 1);
          s = std::fma(sg > 0 ? K.EV[k][l] : -K.EV[k][l], D[k][l], s);
        }
      const double r = s - vv[vtx];
      sigma = (vtx == 0) ? r * r : std::fma(r, r, sigma);
    }
    double tau = D[0][P] * D[0][P];
    for (int k = 1; k <= P; ++k) tau = std::fma(D[k][P - k], D[k][P - k], tau);
    const double st = sigma * tau;
    const double r0 = st / std::fma(beta[0], beta[0], eps);
    wh[0] = std::fma(r0, r0, 1.0);
    for (int m = 1; m <= 4; ++m) {
      const double rm = st / std::fma(beta[m], beta[m], eps);
      wh[m] = rm * rm;
    }
  }
  const double inv = 1.0 / ((((wh[0] + wh[1]) + wh[2]) + wh[3]) + wh[4]);
  double w[5];
  for (int m = 0; m <= 4; ++m) w[m] = wh[m] * inv;
  // Eq. 2DLimitedPolynomial: average kept; first derivatives mix all five,
  // higher ones keep only u_0's share
  double dx1 = w[0] * D[1][0], dy1 = w[0] * D[0][1];
  for (int m = 1; m <= 4; ++m) {
    dx1 = std::fma(w[m], ux[m], dx1);
    dy1 = std::fma(w[m], uy[m], dy1);
  }
  D[1][0] = dx1;
  D[0][1] = dy1;
  for (int n = 2; n <= P; ++n)
    for (int l = 0; l <= n; ++l) D[n - l][l] = w[0] * D[n - l][l];
}

// Rotated characteristic limiting of a 2D Euler new cell (Section 4):
// direction n = grad(phi)/|grad(phi)| with phi = rho e (Section 5.3) from the
// new cell's central-difference derivatives (Eq. RotatedNormal; n = (1, 0)
// where the gradient vanishes); left/right eigenvectors of
// A cos(theta) + B sin(theta) at the new average; every candidate of
// Eq. 2DLowOrderPolynomial / 2DHighOrderPolynomial projected with L, each
// characteristic field limited by limit2d, the result projected back with R.
// ab: conserved average; D[c]: unlimited derivatives (modified in place);
// v[c][vtx]: vertex values, vtx = LD, RD, RU, LU.
void char_limit2d(int P, double gamma, double eps, double dx, double dy, const double ab[4],
                  double D[4][PMAX + 1][PMAX + 1], const double v[4][4]) {
  const double gx = D[3][1][0] / dx, gy = D[3][0][1] / dy;
  const double g2 = std::fma(gy, gy, gx * gx);
  double nx = 1.0, ny = 0.0;
  if (g2 > 0.0) {
    const double gn = std::sqrt(g2);
    nx = gx / gn;
    ny = gy / gn;
  }
  const double rho = ab[0], u = ab[1] / rho, vv = ab[2] / rho;
  const double p = (gamma - 1.0) * (ab[3] - 0.5 * std::fma(ab[2], vv, ab[1] * u));
  const double c = std::sqrt((gamma * p) / rho);
  const double H = (ab[3] + p) / rho;
  const double un = std::fma(vv, ny, u * nx), ut = std::fma(vv, nx, -(u * ny));
  const double q2 = std::fma(vv, vv, u * u);
  const double ic = 1.0 / c;
  const double b1 = (gamma - 1.0) * (ic * ic), b2 = 0.5 * (q2 * b1);
  const double uic = un * ic, nxic = nx * ic, nyic = ny * ic, b1u = b1 * u, b1v = b1 * vv;
  // rows of L; the third row has no energy entry
  const double L[4][4] = {{0.5 * (b2 + uic), -0.5 * (b1u + nxic), -0.5 * (b1v + nyic), 0.5 * b1},
                          {1.0 - b2, b1u, b1v, -b1},
                          {-ut, -ny, nx, 0.0},
                          {0.5 * (b2 - uic), -0.5 * (b1u - nxic), -0.5 * (b1v - nyic), 0.5 * b1}};
  // columns of R; the third column has no density entry
  const double cun = c * un;
  const double R[4][4] = {{1.0, u - c * nx, vv - c * ny, H - cun},
                          {1.0, u, vv, 0.5 * q2},
                          {0.0, -ny, nx, ut},
                          {1.0, u + c * nx, vv + c * ny, H + cun}};
  auto proj = [&](int f, const double x[4]) {
    double s = L[f][0] * x[0];
    s = std::fma(L[f][1], x[1], s);
    s = std::fma(L[f][2], x[2], s);
    if (f != 2) s = std::fma(L[f][3], x[3], s);
    return s;
  };
  double out[4][PMAX + 1][PMAX + 1] = {};
  for (int f = 0; f < 4; ++f) {
    double x[4];
    for (int r = 0; r < 4; ++r) x[r] = ab[r];
    const double ca = proj(f, x);
    double cv[4];
    for (int vtx = 0; vtx < 4; ++vtx) {
      for (int r = 0; r < 4; ++r) x[r] = v[r][vtx];
      cv[vtx] = proj(f, x);
    }
    double cD[PMAX + 1][PMAX + 1] = {};
    for (int n = 1; n <= P; ++n)
      for (int l = 0; l <= n; ++l) {
        for (int r = 0; r < 4; ++r) x[r] = D[r][n - l][l];
        cD[n - l][l] = proj(f, x);
      }
    limit2d(P, eps, ca, cD, cv[0], cv[1], cv[2], cv[3]);
    for (int r = 0; r < 4; ++r) {
      if (f == 2 && r == 0) continue;
      for (int n = 1; n <= P; ++n)
        for (int l = 0; l <= n; ++l) {
          const int k = n - l;
          out[r][k][l] = (f == 0) ? R[f][r] * cD[k][l] : std::fma(R[f][r], cD[k][l], out[r][k][l]);
        }
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int n = 1; n <= P; ++n)
      for (int l = 0; l <= n; ++l) D[r][n - l][l] = out[r][n - l][l];
}

// The two meshes of Section 3.1, direction by direction.  Periodic: Nx cells
// on both meshes, centred at x_left + i dx (parity 0) and shifted by dx/2
// (parity 1), indices wrapped.  Transmissive: parity 0 has the Nx+1 cells
// centred at the mesh points x_i (the domain's edges included), parity 1 the
// Nx cells between them; a new parity-0 cell on an edge has parents outside
// the staggered mesh, which are copies (all DOFs) of the adjacent staggered
// cell -- the 1D transmissive ghost rule, corners included.  Likewise in y.
struct Mesh {
  int64_t nx, ny;     // cells of this mesh
  bool periodic_x, periodic_y;
  int64_t mapx(int64_t i) const {
    if (periodic_x) return (i % nx + nx) % nx;
    return i < 0 ? 0 : (i >= nx ? nx - 1 : i);
  }
  int64_t mapy(int64_t j) const {
    if (periodic_y) return (j % ny + ny) % ny;
    return j < 0 ? 0 : (j >= ny ? ny - 1 : j);
  }
};

inline int bc_y_of(const wcc2d_oracle_problem& pb) { return pb.bc_y < 0 ? pb.bc : pb.bc_y; }

inline Mesh mesh_of(const wcc2d_oracle_problem& pb, int parity) {
  const bool px = pb.bc == 0, py = bc_y_of(pb) == 0;
  const int64_t ex = (px || parity == 1) ? 0 : 1, ey = (py || parity == 1) ? 0 : 1;
  return Mesh{pb.Nx + ex, pb.Ny + ey, px, py};
}

// Wave-speed rate s_x/dx + s_y/dy of a conserved average (1/time units).
double speed_rate(const wcc2d_oracle_problem& pb, const double* ab, double idx, double idy, int& flag) {
  if (pb.equation == EQ_ADVECTION) return std::fma(std::fabs(pb.b), idy, std::fabs(pb.a) * idx);
  if (pb.equation == EQ_BURGERS) {
    const double s = std::fabs(ab[0]);
    return std::fma(s, idy, s * idx);
  }
  const double rho = ab[0];
  const double u = ab[1] / rho, v = ab[2] / rho;
  const double p = (pb.gamma - 1.0) * (ab[3] - 0.5 * std::fma(ab[2], v, ab[1] * u));
  const double c = std::sqrt((pb.gamma * p) / rho);
  if (!(rho > 0.0) || !(p > 0.0)) flag |= 2;
  return std::fma(std::fabs(v) + c, idy, (std::fabs(u) + c) * idx);
}

// Cell average of a stored state (inverse of the point-value relation).
void stored_average(int P, int nc, const double q[NCMAX][32], double* ab) {
  for (int c = 0; c < nc; ++c) {
    double s = q[c][0];
    for (int n = 2; n <= P; ++n)
      for (int l = 0; l <= n; ++l) {
        const int k = n - l;
        if (k % 2 == 0 && l % 2 == 0) s = std::fma(-K.NQA[k][l], q[c][dof(k, l)], s);
      }
    ab[c] = s;
  }
}

// State of cell (i, j) of mesh M: planes [c][dof] of M.nx * M.ny values,
// row-major (x fastest).
void load(const wcc2d_oracle_problem& pb, const Mesh& M, const double* qs, int64_t i, int64_t j,
          double q[NCMAX][32]) {
  const int nd = ndof(pb.P), nc = ncomp(pb);
  const int64_t plane = M.nx * M.ny;
  for (int c = 0; c < nc; ++c)
    for (int d = 0; d < nd; ++d) q[c][d] = qs[((int64_t)(c * nd + d)) * plane + j * M.nx + i];
}

// One half-step from mesh `parity` with time step dt.  Returns the largest
// wave-speed rate of the new averages in *smax and status bits in *flags
// (1: non-finite, 2: rho <= 0 or p <= 0).
void half_step(const wcc2d_oracle_problem& pb, int parity, const double* qin, double dt, double* qout, double* smax,
               int* flags) {
  const int P = pb.P, nd = ndof(P), nc = ncomp(pb);
  const double dx = (pb.x_right - pb.x_left) / (double)pb.Nx, dy = (pb.y_right - pb.y_left) / (double)pb.Ny;
  const double lamx = dt / dx, lamy = dt / dy, hx = 0.5 * lamx, hy = 0.5 * lamy;
  const double idx = 1.0 / dx, idy = 1.0 / dy;
  double cx[PMAX + 1][PMAX + 1], cy[PMAX + 1][PMAX + 1];
  for (int k = 0; k <= PMAX; ++k)
    for (int m = 0; m <= PMAX; ++m) {
      cx[k][m] = -lamx * K.CKR[k][m];
      cy[k][m] = -lamy * K.CKR[k][m];
    }
  const Mesh M = mesh_of(pb, parity), MN = mesh_of(pb, 1 - parity);
  std::vector<Old> old((size_t)(M.nx * M.ny));
  double q[NCMAX][32];
  for (int64_t j = 0; j < M.ny; ++j)
    for (int64_t i = 0; i < M.nx; ++i) {
      load(pb, M, qin, i, j, q);
      old_cell(pb, q, cx, cy, old[(size_t)(j * M.nx + i)]);
    }
  // parents of new cell (i, j): old cells (i+off .. i+off+1, j+off .. j+off+1)
  const int64_t off = parity == 0 ? 0 : -1;
  const int64_t plane = MN.nx * MN.ny;
  double sm = 0.0;
  int fl = 0;
  for (int64_t j = 0; j < MN.ny; ++j)
    for (int64_t i = 0; i < MN.nx; ++i) {
      const int64_t i0 = M.mapx(i + off), i1 = M.mapx(i + off + 1), j0 = M.mapy(j + off), j1 = M.mapy(j + off + 1);
      const Old& A = old[(size_t)(j0 * M.nx + i0)];   // lower-left vertex of the new cell
      const Old& B = old[(size_t)(j1 * M.nx + i0)];   // upper-left
      const Old& C = old[(size_t)(j0 * M.nx + i1)];   // lower-right
      const Old& Dd = old[(size_t)(j1 * M.nx + i1)];  // upper-right
      double ab[NCMAX];
      double D[NCMAX][PMAX + 1][PMAX + 1] = {};
      for (int c = 0; c < nc; ++c) {
        // Eq. 2DIntegral; the flux terms are grouped as differences of the
        // same half-edge flux on opposite faces, so that data uniform in the
        // transverse direction cancels exactly
        const double h = 0.25 * (((A.RU[c] + B.RD[c]) + C.LU[c]) + Dd.LD[c]);
        const double fx = (A.fU[c] - C.fU[c]) + (B.fD[c] - Dd.fD[c]);
        const double gy = (A.gR[c] - B.gR[c]) + (C.gL[c] - Dd.gL[c]);
        ab[c] = std::fma(hy, gy, std::fma(hx, fx, h));
        // Eq. 2DDerivatives, total order n = P down to 1
        for (int n = P; n >= 1; --n)
          for (int l = 0; l <= n; ++l) {
            const int k = n - l;
            double X = 0.0, Y = 0.0;
            if (k >= 1) {
              const int kb = k - 1, r = P - kb - l;
              X = 0.5 * ((C.V[c][kb][l] - A.V[c][kb][l]) + (Dd.V[c][kb][l] - B.V[c][kb][l]));
              for (int s = 3; s <= r; s += 2) X = std::fma(K.CX1[s], D[c][kb + s][l], X);
              for (int t = 2; t <= r; t += 2)
                for (int s = 1; s <= r - t; s += 2) X = std::fma(K.CX2[s][t], D[c][kb + s][l + t], X);
            }
            if (l >= 1) {
              const int lb = l - 1, r = P - k - lb;
              Y = 0.5 * ((B.V[c][k][lb] - A.V[c][k][lb]) + (Dd.V[c][k][lb] - C.V[c][k][lb]));
              for (int t = 3; t <= r; t += 2) Y = std::fma(K.CX1[t], D[c][k][lb + t], Y);
              for (int t = 1; t <= r; t += 2)
                for (int s = 2; s <= r - t; s += 2) Y = std::fma(K.CX2[t][s], D[c][k + s][lb + t], Y);
            }
            D[c][k][l] = (k >= 1 && l >= 1) ? 0.5 * (X + Y) : (k >= 1 ? X : Y);
          }
      }
      if (pb.limiter && P >= 1) {
        if (pb.equation == EQ_EULER) {
          double vtx[4][4];
          for (int c = 0; c < 4; ++c) {
            vtx[c][0] = A.V[c][0][0];
            vtx[c][1] = C.V[c][0][0];
            vtx[c][2] = Dd.V[c][0][0];
            vtx[c][3] = B.V[c][0][0];
          }
          char_limit2d(P, pb.gamma, pb.eps, dx, dy, ab, D, vtx);
        } else {
          limit2d(P, pb.eps, ab[0], D[0], A.V[0][0][0], C.V[0][0][0], Dd.V[0][0][0], B.V[0][0][0]);
        }
      }
      for (int c = 0; c < nc; ++c) {
        double pv = ab[c];
        for (int n = 2; n <= P; ++n)
          for (int l = 0; l <= n; ++l) {
            const int k = n - l;
            if (k % 2 == 0 && l % 2 == 0) pv = std::fma(K.NQA[k][l], D[c][k][l], pv);
          }
        const int64_t cell = j * MN.nx + i;
        qout[((int64_t)(c * nd)) * plane + cell] = pv;
        bool ok = std::isfinite(pv);
        for (int n = 1; n <= P; ++n)
          for (int l = 0; l <= n; ++l) {
            const double x = D[c][n - l][l];
            qout[((int64_t)(c * nd + dof(n - l, l))) * plane + cell] = x;
            ok = ok && std::isfinite(x);
          }
        if (!ok) fl |= 1;
      }
      const double sr = speed_rate(pb, ab, idx, idy, fl);
      if (!std::isfinite(sr)) fl |= 1;
      sm = std::fmax(sm, sr);
    }
  *smax = sm;
  *flags = fl;
}

}  // namespace w2d

extern "C" {

int64_t wcc2d_oracle_ndof(int32_t P) { return w2d::ndof(P); }

// Eq. 2DSmoothIndicator of the polynomial with scaled derivatives d (DOF
// order, entry 0 ignored).
double wcc2d_oracle_js_indicator(int32_t P, const double* d) {
  double D[w2d::PMAX + 1][w2d::PMAX + 1] = {};
  for (int n = 0; n <= P; ++n)
    for (int l = 0; l <= n; ++l) D[n - l][l] = d[w2d::dof(n - l, l)];
  return w2d::js2d(P, D);
}

// Largest wave-speed rate s_x/dx + s_y/dy over the averages of a stored
// state on mesh `parity`.
double wcc2d_oracle_max_speed(const wcc2d_oracle_problem* pb, int32_t parity, const double* q, int32_t* flags) {
  const int nc = w2d::ncomp(*pb);
  const double dx = (pb->x_right - pb->x_left) / (double)pb->Nx, dy = (pb->y_right - pb->y_left) / (double)pb->Ny;
  const double idx = 1.0 / dx, idy = 1.0 / dy;
  const w2d::Mesh M = w2d::mesh_of(*pb, parity);
  double sm = 0.0;
  int fl = 0;
  double qc[w2d::NCMAX][32], ab[w2d::NCMAX];
  for (int64_t j = 0; j < M.ny; ++j)
    for (int64_t i = 0; i < M.nx; ++i) {
      w2d::load(*pb, M, q, i, j, qc);
      w2d::stored_average(pb->P, nc, qc, ab);
      sm = std::fmax(sm, w2d::speed_rate(*pb, ab, idx, idy, fl));
    }
  if (flags) *flags = fl;
  return sm;
}

// The per-old-cell quantities of one cell with state q (DOF order, nc x ndof)
// and time step dt: out = [RU, RD, LU, LD, fU, fD, gR, gL] per component
// (8 nc values), then the vertex values V[c][k][l], k + l < P, DOF order.
int32_t wcc2d_oracle_old_cell(const wcc2d_oracle_problem* pb, const double* q, double dt, double* out) {
  if (!pb || pb->P < 0 || pb->P > w2d::PMAX) return -1;
  const int P = pb->P, nd = w2d::ndof(P), nc = w2d::ncomp(*pb);
  const double dx = (pb->x_right - pb->x_left) / (double)pb->Nx, dy = (pb->y_right - pb->y_left) / (double)pb->Ny;
  const double lamx = dt / dx, lamy = dt / dy;
  double cx[w2d::PMAX + 1][w2d::PMAX + 1], cy[w2d::PMAX + 1][w2d::PMAX + 1];
  for (int k = 0; k <= w2d::PMAX; ++k)
    for (int m = 0; m <= w2d::PMAX; ++m) {
      cx[k][m] = -lamx * w2d::K.CKR[k][m];
      cy[k][m] = -lamy * w2d::K.CKR[k][m];
    }
  double qc[w2d::NCMAX][32];
  for (int c = 0; c < nc; ++c)
    for (int d = 0; d < nd; ++d) qc[c][d] = q[c * nd + d];
  w2d::Old o;
  w2d::old_cell(*pb, qc, cx, cy, o);
  int idx = 0;
  for (int c = 0; c < nc; ++c) {
    const double v[8] = {o.RU[c], o.RD[c], o.LU[c], o.LD[c], o.fU[c], o.fD[c], o.gR[c], o.gL[c]};
    for (int i = 0; i < 8; ++i) out[idx++] = v[i];
  }
  for (int c = 0; c < nc; ++c)
    for (int n = 0; n < P; ++n)
      for (int l = 0; l <= n; ++l) out[idx++] = o.V[c][n - l][l];
  return 0;
}

int32_t wcc2d_oracle_half_step(const wcc2d_oracle_problem* pb, int32_t parity, const double* qin, double dt,
                               double* qout, double* smax, int32_t* flags) {
  if (!pb || pb->P < 0 || pb->P > w2d::PMAX || pb->Nx < 2 || pb->Ny < 2 || pb->bc < 0 || pb->bc > 1 || pb->bc_y < -1 || pb->bc_y > 1) return -1;
  int fl = 0;
  w2d::half_step(*pb, parity, qin, dt, qout, smax, &fl);
  if (flags) *flags = fl;
  return 0;
}

// March half-steps: dt = cfl / smax (smax: wave-speed rate of the current
// state), clipped to t_end; or dt_fixed when > 0.  q (in/out) holds the state
// of mesh *parity and has room for the larger mesh.  Stops at t_end, after
// max_half_steps, or when a status bit is raised.  Returns the number of
// half-steps taken, -1 on bad input.
int64_t wcc2d_oracle_run(const wcc2d_oracle_problem* pb, int32_t* parity, double* t, double* smax, double* q,
                         double t_end, double cfl, double dt_fixed, int64_t max_half_steps, int32_t* flags) {
  if (!pb || pb->P < 0 || pb->P > w2d::PMAX || pb->Nx < 2 || pb->Ny < 2 || pb->bc < 0 || pb->bc > 1 || pb->bc_y < -1 || pb->bc_y > 1) return -1;
  const size_t per_cell = (size_t)(w2d::ncomp(*pb) * w2d::ndof(pb->P));
  std::vector<double> tmp(per_cell * (size_t)((pb->Nx + 1) * (pb->Ny + 1)));
  int64_t taken = 0;
  *flags = 0;
  while (taken < max_half_steps && *t < t_end) {
    double dt, tn;
    if (dt_fixed > 0.0) {
      dt = dt_fixed;
      tn = *t + dt;
    } else {
      dt = cfl / *smax;
      const double rem = t_end - *t;
      if (dt >= rem) {
        dt = rem;
        tn = t_end;
      } else {
        tn = *t + dt;
      }
    }
    int fl = 0;
    double sm = 0.0;
    w2d::half_step(*pb, *parity, q, dt, tmp.data(), &sm, &fl);
    const w2d::Mesh MN = w2d::mesh_of(*pb, 1 - *parity);
    std::memcpy(q, tmp.data(), per_cell * (size_t)(MN.nx * MN.ny) * sizeof(double));
    *parity ^= 1;
    *t = tn;
    *smax = sm;
    ++taken;
    if (fl) {
      *flags = fl;
      break;
    }
  }
  return taken;
}

}  // extern "C"
