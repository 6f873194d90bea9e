// wcc_oracle.cpp -- plain FP64 CPU reference of the 1D weighted compact central
// (WCC) half-step of Shen & Parsani, "A class of high-order weighted compact
// central schemes for solving hyperbolic conservation laws" (arXiv:2104.04347).
//
// TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
// leg of the benchmark are its only users; the product library never links,
// loads or calls it, and it shares no code, header or constant table with the
// GPU path.  It is written to be read against the paper, not to be fast:
// every cell of a half-step is processed by the same scalar code in the order
// the paper derives the quantities.
//
// What one half-step computes (Section 2.1 and 2.2 of the paper):
//   * state on a cell: q = [u, u_x, ..., u_Px], the point value and the scaled
//     spatial derivatives at the cell centre (Eq. 1D_Derivative_DEF,
//     Eq. 1DPolynomial_Space; the same vector q appears in
//     Eq. 1DSchemeMatrixForm);
//   * Cauchy-Kovalewski expansion of every old cell (Eq. 1DCauchy_Kovalewski;
//     for systems the generalised Leibniz rule named in Section 4), carried
//     out in truncated bivariate Taylor arithmetic;
//   * time-averaged interface flux (Eq. Cal1DFlux) and half-cell averages
//     (Eq. SubEq:1DCellAVGR, SubEq:1DCellAVGL) -> new cell average by the
//     finite-volume balance on the staggered control volume
//     (Eq. SubEq:1DIntegral);
//   * vertex values at the half time level (Eq. SubEq:Cal_1D_Derivatives_4)
//     -> new derivatives by central differences, highest order first
//     (Eq. SubEq:Cal_1D_Derivatives_3);
//   * the compact WENO-type limiter (Eq. 1D_U012, 1DLimitedPolynomial,
//     1D2ndOrderWeights for P=1, 1DHighOrderWeights for P>=2), applied to
//     characteristic variables for the Euler equations (Section 4);
//   * new point value from the new average (Eq. 1DCalU).
//
// Canonical arithmetic (the GPU path follows the same written rules):
//   * IEEE binary64, round to nearest even, no contraction (-ffp-contract=off)
//     and no fast-math.
//   * Every sum of products sum_i c_i*x_i is evaluated left to right in the
//     index order written here as  s = c_0*x_0;  s = fma(c_i, x_i, s).
//     A chain that starts from a plain value y evaluates  s = y;
//     s = fma(c_i, x_i, s).  Everything else is plain +, -, *, / and sqrt,
//     each correctly rounded.
//   * Constants are exact rationals rounded once (integer numerator divided by
//     integer denominator in binary64).
//   * alpha = 2 is evaluated as x*x.
//
// Readings of the paper that this file implements are listed in the design
// notes of the repository (CFL per half-step, point-value state, wave-speed
// estimator, boundary ghosts, time-step clipping).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int PMAX = 4;
constexpr int NCMAX = 3;

enum { EQ_ADVECTION = 0, EQ_BURGERS = 1, EQ_EULER = 2 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_DIRICHLET = 2 };

// ---------------------------------------------------------------------------
// Flop-counting real type: the same templated code computes in double for the
// reference results and in Counted to count the algorithm's floating-point
// operations per cell (used for the arithmetic-intensity figures).
// ---------------------------------------------------------------------------
struct OpCount {
  double add = 0, mul = 0, fma = 0, div = 0, sqrt = 0;
};
OpCount g_ops;

struct Counted {
  double v;
  Counted() : v(0) {}
  Counted(double x) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { g_ops.add += 1; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { g_ops.add += 1; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { g_ops.mul += 1; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { g_ops.div += 1; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
inline Counted fmaR(Counted a, Counted b, Counted c) { g_ops.fma += 1; return Counted(std::fma(a.v, b.v, c.v)); }
inline Counted sqrtR(Counted a) { g_ops.sqrt += 1; return Counted(std::sqrt(a.v)); }
inline Counted absR(Counted a) { return Counted(std::fabs(a.v)); }
inline double val(Counted a) { return a.v; }

inline double fmaR(double a, double b, double c) { return std::fma(a, b, c); }
inline double sqrtR(double a) { return std::sqrt(a); }
inline double absR(double a) { return std::fabs(a); }
inline double val(double a) { return a; }

// ---------------------------------------------------------------------------
// Exact rational constants, each rounded once to binary64.
// ---------------------------------------------------------------------------
struct Consts {
  double fact[2 * PMAX + 3];       // k!
  double IF[PMAX + 1];             // 1/k!
  double CA[PMAX + 1];             // 1/((k+1)! 2^k)      Eq. SubEq:1DCellAVGR
  double SCA[PMAX + 1];            // (-1)^k/((k+1)! 2^k) Eq. SubEq:1DCellAVGL
  double NCA[PMAX + 1];            // -1/((k+1)! 2^k), used for Eq. 1DCalU
  double NCO[PMAX + 1];            // -(1-(-1)^m)/(m! 2^m) Eq. SubEq:Cal_1D_Derivatives_3
  double RM[PMAX + 1];             // m!/(m+1)! = 1/(m+1)  Eq. Cal1DFlux
  double CKR[PMAX + 1][PMAX + 1];  // (k+1)/m              Eq. 1DCauchy_Kovalewski
  double EP[PMAX + 1];             // (+1/2)^k/k!          Eq. 1DPolynomial_Space at x_i + dx/2
  double EM[PMAX + 1];             // (-1/2)^k/k!          Eq. 1DPolynomial_Space at x_i - dx/2
  double JI[2 * PMAX + 1];         // int_{-1/2}^{1/2} xi^s dxi = 1/((s+1) 2^s), s even
  Consts() {
    fact[0] = 1.0;
    for (int k = 1; k < 2 * PMAX + 3; ++k) fact[k] = fact[k - 1] * (double)k;
    for (int k = 0; k <= PMAX; ++k) {
      double p2 = std::ldexp(1.0, k);
      IF[k] = 1.0 / fact[k];
      CA[k] = 1.0 / (fact[k + 1] * p2);
      SCA[k] = (k % 2 == 0) ? CA[k] : -CA[k];
      NCA[k] = -CA[k];
      NCO[k] = (k % 2 == 1) ? -(2.0 / (fact[k] * p2)) : 0.0;
      RM[k] = 1.0 / (double)(k + 1);
      EP[k] = 1.0 / (fact[k] * p2);
      EM[k] = (k % 2 == 0) ? EP[k] : -EP[k];
      for (int m = 0; m <= PMAX; ++m) CKR[k][m] = (m > 0) ? (double)(k + 1) / (double)m : 0.0;
    }
    for (int s = 0; s <= 2 * PMAX; ++s)
      JI[s] = (s % 2 == 0) ? 1.0 / ((double)(s + 1) * std::ldexp(1.0, s)) : 0.0;
  }
};
const Consts K;

// ---------------------------------------------------------------------------
// Problem description (mirrors the ctypes structure of the Python wrapper).
// ---------------------------------------------------------------------------
}  // namespace

extern "C" {
typedef struct {
  int32_t equation;  // 0 advection f=a*u, 1 Burgers f=u^2/2, 2 Euler
  int32_t P;         // polynomial degree 0..4
  int64_t N;         // number of mesh intervals, dx = (x_right-x_left)/N
  int32_t bc;        // 0 periodic, 1 transmissive, 2 Dirichlet
  int32_t limiter;   // 0/1
  double x_left, x_right;
  double a;          // advection speed
  double gamma;      // ratio of specific heats
  double eps;        // limiter epsilon (1e-40 in the paper)
  double left_state[3], right_state[3];  // Dirichlet ghost states (conserved)
} wcc_oracle_problem;
}

namespace {

inline int ncomp(const wcc_oracle_problem& pb) { return pb.equation == EQ_EULER ? 3 : 1; }

// Number of cells on the original mesh (parity 0) or the staggered mesh
// (parity 1).  Periodic: N on both.  Otherwise the original mesh has the N+1
// cells centred at x_1 = x_L ... x_{N+1} = x_R and the staggered mesh the N
// cells centred at x_{3/2} ... x_{N+1/2} (Section 2.1, mesh definition).
inline int64_t ncells(const wcc_oracle_problem& pb, int parity) {
  if (pb.bc == BC_PERIODIC) return pb.N;
  return parity == 0 ? pb.N + 1 : pb.N;
}

template <class R>
using Tri = R[PMAX + 1][PMAX + 1];  // Taylor triangle, entry [k][m] with k+m <= P

// Truncated bivariate Taylor product (X o Y)[k][m] = sum_{a<=k} sum_{b<=m}
// X[a][b] Y[k-a][m-b]: the generalised Leibniz rule for the normalised
// coefficients  X[k][m] = u_{kx,mt}/(k! m!).  a outer, b inner.
template <class R>
R tprod(const Tri<R>& X, const Tri<R>& Y, int k, int m) {
  R s = X[0][0] * Y[k][m];
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= m; ++b) {
      if (a == 0 && b == 0) continue;
      s = fmaR(X[a][b], Y[k - a][m - b], s);
    }
  return s;
}

// Taylor quotient V = M / Rho at entry [k][m], from M = Rho o V solved for the
// highest coefficient:  V[k][m] = (M[k][m] - sum_{(a,b)!=(0,0)} Rho[a][b]
// V[k-a][m-b]) * (1/Rho[0][0]).  Needs V at all lower entries.
template <class R>
R tquot(const Tri<R>& M, const Tri<R>& Rho, const Tri<R>& V, R rinv, int k, int m) {
  R s = M[k][m];
  for (int a = 0; a <= k; ++a)
    for (int b = 0; b <= m; ++b) {
      if (a == 0 && b == 0) continue;
      s = fmaR(-Rho[a][b], V[k - a][m - b], s);
    }
  return s * rinv;
}

// Flux Taylor coefficients G = f(U) in Taylor arithmetic, one time column j,
// rows k = 0..P-j.  The Euler quantities follow F = [rho u, rho u^2 + p,
// (rho e + p) u] with p = (gamma-1)(rho e - rho u^2/2) (Section 5.2).
template <class R>
struct FluxWork {
  Tri<R> v, Kin, Pi, W;  // Euler: velocity, rho u^2 (momentum*velocity), pressure, energy+pressure
  R rinv;
};

template <class R>
void flux_column(const wcc_oracle_problem& pb, int P, Tri<R>* T, Tri<R>* G, FluxWork<R>& w, int j) {
  if (pb.equation == EQ_ADVECTION) {
    R a = pb.a;
    for (int k = 0; k + j <= P; ++k) G[0][k][j] = a * T[0][k][j];
  } else if (pb.equation == EQ_BURGERS) {
    R half = 0.5;
    for (int k = 0; k + j <= P; ++k) G[0][k][j] = half * tprod(T[0], T[0], k, j);
  } else {
    R gm1 = R(pb.gamma) - R(1.0);
    R half = 0.5;
    Tri<R>& rho = T[0];
    Tri<R>& mom = T[1];
    Tri<R>& ene = T[2];
    if (j == 0) w.rinv = R(1.0) / rho[0][0];
    for (int k = 0; k + j <= P; ++k) {
      w.v[k][j] = tquot(mom, rho, w.v, w.rinv, k, j);          // u = (rho u)/rho
      w.Kin[k][j] = tprod(mom, w.v, k, j);                     // rho u^2
      w.Pi[k][j] = gm1 * (ene[k][j] - half * w.Kin[k][j]);     // p
      w.W[k][j] = ene[k][j] + w.Pi[k][j];                      // rho e + p
      G[0][k][j] = mom[k][j];                                  // rho u
      G[1][k][j] = w.Kin[k][j] + w.Pi[k][j];                   // rho u^2 + p
      G[2][k][j] = tprod(w.W, w.v, k, j);                      // (rho e + p) u
    }
  }
}

// Per old cell: everything the two new cells that overlap it need.
template <class R>
struct OldCell {
  R uR[NCMAX];              // (u_R)_i, Eq. SubEq:1DCellAVGR
  R uL[NCMAX];              // (u_L)_i, Eq. SubEq:1DCellAVGL
  R fbar[NCMAX];            // time-averaged flux at the cell centre, Eq. Cal1DFlux
  R V[NCMAX][PMAX + 1];     // (u_kx)_i^{n+1/2}, Eq. SubEq:Cal_1D_Derivatives_4
};

// Cauchy-Kovalewski expansion of one old cell and the quantities derived from
// it.  q[c][k] is the cell's state (k=0: point value).  ck[k][m] holds
// (-dt/dx) * (k+1)/m, the factor of the scaled CK identity
// u_{kx,mt} = -(dt/dx) f_{(k+1)x,(m-1)t} written for normalised coefficients.
template <class R>
void old_cell(const wcc_oracle_problem& pb, const R q[NCMAX][PMAX + 1], const R ck[PMAX + 1][PMAX + 1],
              OldCell<R>& out) {
  const int P = pb.P, nc = ncomp(pb);
  Tri<R> T[NCMAX], G[NCMAX];
  FluxWork<R> w;
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k) T[c][k][0] = (k <= 1) ? q[c][k] : q[c][k] * R(K.IF[k]);  // 1/0! = 1/1! = 1
  // Level m: flux column m-1, then u_{kx,mt} from Eq. 1DCauchy_Kovalewski.
  for (int m = 1; m <= P; ++m) {
    flux_column(pb, P, T, G, w, m - 1);
    for (int c = 0; c < nc; ++c)
      for (int k = 0; k + m <= P; ++k) T[c][k][m] = ck[k][m] * G[c][k + 1][m - 1];
  }
  flux_column(pb, P, T, G, w, P);  // only G[.][0][P] is formed here

  for (int c = 0; c < nc; ++c) {
    // Eq. Cal1DFlux: fbar = sum_m f_mt/(m+1)! = sum_m G[0][m]/(m+1).
    R f = G[c][0][0];  // 1/(0+1) = 1
    for (int m = 1; m <= P; ++m) f = fmaR(R(K.RM[m]), G[c][0][m], f);
    out.fbar[c] = f;
    // Eq. SubEq:1DCellAVGR / SubEq:1DCellAVGL with (u_0x) the point value.
    R r = q[c][0], l = q[c][0];
    for (int k = 1; k <= P; ++k) {
      r = fmaR(R(K.CA[k]), q[c][k], r);
      l = fmaR(R(K.SCA[k]), q[c][k], l);
    }
    out.uR[c] = r;
    out.uL[c] = l;
    // Eq. SubEq:Cal_1D_Derivatives_4: (u_kx)^{n+1/2} = sum_m u_{kx,mt}/m!
    //   = k! * sum_m T[k][m].
    for (int k = 0; k < P; ++k) {
      R s = T[c][k][0];
      for (int m = 1; k + m <= P; ++m) s = s + T[c][k][m];
      out.V[c][k] = (k <= 1) ? s : R(K.fact[k]) * s;  // 0! = 1! = 1
    }
  }
}

// Jiang-Shu smoothness indicator (Eq. 1DSmoothIndicator) of the degree-P
// polynomial with scaled derivatives d[1..P] on a cell of unit scaled width:
//   beta = sum_{k=1}^{P} int_{-1/2}^{1/2} ( sum_{n=0}^{P-k} d_{k+n} xi^n/n! )^2 dxi.
// The square of the inner polynomial is formed coefficient by coefficient
// (only even powers integrate to a non-zero value) and integrated term by term.
template <class R>
R js_indicator(int P, const R d[PMAX + 1]) {
  R beta = 0.0;
  for (int k = 1; k <= P; ++k) {
    R cpoly[PMAX + 1];
    const int deg = P - k;
    for (int n = 0; n <= deg; ++n) cpoly[n] = (n <= 1) ? d[k + n] : d[k + n] * R(K.IF[n]);
    R integral = 0.0;
    for (int s = 0; s <= 2 * deg; s += 2) {
      // coefficient of xi^s in cpoly^2
      int n0 = (s > deg) ? s - deg : 0;
      int n1 = (s < deg) ? s : deg;
      R sq = cpoly[n0] * cpoly[s - n0];
      for (int n = n0 + 1; n <= n1; ++n) sq = fmaR(cpoly[n], cpoly[s - n], sq);
      integral = (s == 0) ? sq : fmaR(R(K.JI[s]), sq, integral);  // JI[0] = 1
    }
    beta = (k == 1) ? integral : beta + integral;
  }
  return beta;
}

// The WENO-type limiter for one scalar field on one new cell (Section 2.2).
//   abar: cell average of u_0 (Eq. SubEq:1DIntegral),
//   d[1..P]: scaled derivatives of u_0, modified in place,
//   vl, vr: vertex values u_{i-1/2}, u_{i+1/2} from Eq. SubEq:Cal_1D_Derivatives_4.
// Candidates (Eq. 1D_U012): u_0 itself; u_1, u_2 linear with average abar and
// slopes 2(abar - vl), 2(vr - abar).  Limited polynomial (Eq. 1DLimitedPolynomial):
// sum_m w_m u_m, so the average is kept and d_1 <- w0 d1 + w1 s1 + w2 s2,
// d_k <- w0 d_k (k >= 2).
template <class R>
void limit_field(int P, R eps, R abar, R d[PMAX + 1], R vl, R vr) {
  R s1 = (abar - vl) * R(2.0);
  R s2 = (vr - abar) * R(2.0);
  R wh0, wh1, wh2;
  if (P == 1) {
    // Eq. 1D2ndOrderWeights with alpha = 2; beta_m of a linear polynomial is its
    // squared scaled slope (Eq. 1DSmoothIndicator with P = 1).
    R b0 = d[1] * d[1], b1 = s1 * s1, b2 = s2 * s2;
    R q0 = R(1.0) / (b0 + eps), q1 = R(1.0) / (b1 + eps), q2 = R(1.0) / (b2 + eps);
    wh0 = q0 * q0;
    wh1 = q1 * q1;
    wh2 = q2 * q2;
  } else {
    // Eq. 1DHighOrderWeights with alpha = 2.
    // Point value of u_0 (Eq. 1DCalU applied to u_0), then u_0 at x_{i+-1/2}.
    R pc = abar;
    for (int k = 2; k <= P; k += 2) pc = fmaR(R(K.NCA[k]), d[k], pc);
    R ep = pc, em = pc;
    for (int k = 1; k <= P; ++k) {
      ep = fmaR(R(K.EP[k]), d[k], ep);
      em = fmaR(R(K.EM[k]), d[k], em);
    }
    R rp = ep - vr, rm = em - vl;
    R sigma = fmaR(rm, rm, rp * rp);
    R tau = d[P] * d[P];
    R b0 = js_indicator(P, d);
    R b1 = s1 * s1, b2 = s2 * s2;
    R st = sigma * tau;
    R r0 = st / fmaR(b0, b0, eps);
    R r1 = st / fmaR(b1, b1, eps);
    R r2 = st / fmaR(b2, b2, eps);
    wh0 = fmaR(r0, r0, R(1.0));
    wh1 = r1 * r1;
    wh2 = r2 * r2;
  }
  R inv = R(1.0) / ((wh0 + wh1) + wh2);
  R w0 = wh0 * inv, w1 = wh1 * inv, w2 = wh2 * inv;
  R d1 = w0 * d[1];
  d1 = fmaR(w1, s1, d1);
  d1 = fmaR(w2, s2, d1);
  d[1] = d1;
  for (int k = 2; k <= P; ++k) d[k] = w0 * d[k];
}

// Eigen-structure of the 1D Euler flux Jacobian at the conserved state
// U = (rho, rho u, rho e) with velocity u, pressure p and sound speed c:
// A = R diag(u-c, u, u+c) L (Section 4, limiting of systems).
template <class R>
struct EulerEig {
  R L[3][3], Rm[3][3];
};

template <class R>
void euler_primitive(R gamma, const R U[3], R& u, R& p, R& c) {
  R gm1 = gamma - R(1.0);
  u = U[1] / U[0];
  p = gm1 * (U[2] - R(0.5) * U[1] * u);
  c = sqrtR((gamma * p) / U[0]);
}

template <class R>
void euler_eigen(R gamma, const R U[3], R u, R p, R c, EulerEig<R>& e) {
  R gm1 = gamma - R(1.0);
  R H = (U[2] + p) / U[0];
  R ic = R(1.0) / c;
  R b1 = gm1 * (ic * ic);
  R b2 = R(0.5) * b1 * (u * u);
  R uic = u * ic, b1u = b1 * u;
  e.L[0][0] = R(0.5) * (b2 + uic);
  e.L[0][1] = R(-0.5) * (b1u + ic);
  e.L[0][2] = R(0.5) * b1;
  e.L[1][0] = R(1.0) - b2;
  e.L[1][1] = b1u;
  e.L[1][2] = -b1;
  e.L[2][0] = R(0.5) * (b2 - uic);
  e.L[2][1] = R(-0.5) * (b1u - ic);
  e.L[2][2] = R(0.5) * b1;
  R uc = u * c;
  e.Rm[0][0] = 1.0;     e.Rm[0][1] = 1.0;               e.Rm[0][2] = 1.0;
  e.Rm[1][0] = u - c;   e.Rm[1][1] = u;                 e.Rm[1][2] = u + c;
  e.Rm[2][0] = H - uc;  e.Rm[2][1] = R(0.5) * (u * u);  e.Rm[2][2] = H + uc;
}

// y = M x for a 3x3 matrix, rows evaluated as sums of products.
template <class R>
void mat3(const R M[3][3], const R x[3], R y[3]) {
  for (int i = 0; i < 3; ++i) {
    R s = M[i][0] * x[0];
    s = fmaR(M[i][1], x[1], s);
    s = fmaR(M[i][2], x[2], s);
    y[i] = s;
  }
}

// Wave speed used for the CFL time step, from a cell average.
template <class R>
R cell_speed(const wcc_oracle_problem& pb, const R abar[NCMAX]) {
  if (pb.equation == EQ_ADVECTION) return absR(R(pb.a));
  if (pb.equation == EQ_BURGERS) return absR(abar[0]);
  R u, p, c;
  euler_primitive(R(pb.gamma), abar, u, p, c);
  return absR(u) + c;
}

// New cell from its left parent L and right parent R (the two old cells whose
// centres are the new cell's vertices).  Writes the new state q[c][k]
// (k=0: point value), its wave speed and a status flag
// (bit 0: non-finite value, bit 1: rho <= 0 or p <= 0).
template <class R>
int new_cell(const wcc_oracle_problem& pb, R lam, const OldCell<R>& Lc, const OldCell<R>& Rc,
             R q[NCMAX][PMAX + 1], R& speed) {
  const int P = pb.P, nc = ncomp(pb);
  R abar[NCMAX];
  R d[NCMAX][PMAX + 1];
  for (int c = 0; c < nc; ++c) {
    // Eq. SubEq:1DIntegral.
    R h = R(0.5) * (Lc.uR[c] + Rc.uL[c]);
    abar[c] = fmaR(lam, Lc.fbar[c] - Rc.fbar[c], h);
    // Eq. SubEq:Cal_1D_Derivatives_3, from the highest derivative down.
    d[c][0] = 0.0;
    for (int k = P - 1; k >= 0; --k) {
      R s = Rc.V[c][k] - Lc.V[c][k];
      for (int m = 3; m <= P - k; m += 2) s = fmaR(R(K.NCO[m]), d[c][k + m], s);
      d[c][k + 1] = s;
    }
  }
  int flag = 0;
  // Wave speed of the new cell average: |a|, |u| or |u| + c.
  R eu = 0.0, ep = 0.0, ec = 0.0;
  if (pb.equation == EQ_EULER) {
    euler_primitive(R(pb.gamma), abar, eu, ep, ec);
    speed = absR(eu) + ec;
    if (!(val(abar[0]) > 0.0) || !(val(ep) > 0.0)) flag |= 2;
  } else {
    speed = cell_speed(pb, abar);
  }
  if (pb.limiter && P >= 1) {
    R eps = pb.eps;
    if (pb.equation != EQ_EULER) {
      limit_field(P, eps, abar[0], d[0], Lc.V[0][0], Rc.V[0][0]);
    } else {
      EulerEig<R> e;
      euler_eigen(R(pb.gamma), abar, eu, ep, ec, e);
      R ca[3], cl[3], cr[3], cd[PMAX + 1][3];
      R vl[3] = {Lc.V[0][0], Lc.V[1][0], Lc.V[2][0]};
      R vr[3] = {Rc.V[0][0], Rc.V[1][0], Rc.V[2][0]};
      mat3(e.L, abar, ca);
      mat3(e.L, vl, cl);
      mat3(e.L, vr, cr);
      for (int k = 1; k <= P; ++k) {
        R x[3] = {d[0][k], d[1][k], d[2][k]};
        mat3(e.L, x, cd[k]);
      }
      for (int f = 0; f < 3; ++f) {
        R df[PMAX + 1];
        df[0] = 0.0;
        for (int k = 1; k <= P; ++k) df[k] = cd[k][f];
        limit_field(P, eps, ca[f], df, cl[f], cr[f]);
        for (int k = 1; k <= P; ++k) cd[k][f] = df[k];
      }
      for (int k = 1; k <= P; ++k) {
        R y[3];
        mat3(e.Rm, cd[k], y);
        d[0][k] = y[0];
        d[1][k] = y[1];
        d[2][k] = y[2];
      }
    }
  }
  for (int c = 0; c < nc; ++c) {
    // Eq. 1DCalU: point value from the average.
    R p = abar[c];
    for (int k = 2; k <= P; k += 2) p = fmaR(R(K.NCA[k]), d[c][k], p);
    q[c][0] = p;
    for (int k = 1; k <= P; ++k) q[c][k] = d[c][k];
    for (int k = 0; k <= P; ++k)
      if (!std::isfinite(val(q[c][k]))) flag |= 1;
  }
  if (!std::isfinite(val(speed))) flag |= 1;
  return flag;
}

template <class R>
void ck_factors(R lam, R ck[PMAX + 1][PMAX + 1]) {
  R nlam = -lam;
  for (int k = 0; k <= PMAX; ++k)
    for (int m = 0; m <= PMAX; ++m) ck[k][m] = (m > 0) ? nlam * R(K.CKR[k][m]) : R(0.0);
}

inline void load_cell(const wcc_oracle_problem& pb, const double* dofs, int64_t n, int64_t j,
                      double q[NCMAX][PMAX + 1]) {
  const int P = pb.P, nc = ncomp(pb);
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k) q[c][k] = dofs[((int64_t)c * (P + 1) + k) * n + j];
}

// One half-step (Section 2.1): old state on the mesh of the given parity ->
// new state on the other mesh.  dofs layout: [c][k][j], k=0 the point value.
int half_step(const wcc_oracle_problem& pb, int parity, const double* old_dofs, double dt,
              double* new_dofs, double* smax_out) {
  const int P = pb.P, nc = ncomp(pb);
  const int64_t n_old = ncells(pb, parity), n_new = ncells(pb, 1 - parity);
  const double dx = (pb.x_right - pb.x_left) / (double)pb.N;
  const double lam = dt / dx;
  double ck[PMAX + 1][PMAX + 1];
  ck_factors(lam, ck);

  // Old cells, with one ghost on each side for the non-periodic odd->even step.
  // (Cells are independent: the optional OpenMP build splits the loops over
  // threads without changing any operation; the serial build ignores it.)
  std::vector<OldCell<double>> oc((size_t)n_old + 2);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t j = 0; j < n_old; ++j) {
    double q[NCMAX][PMAX + 1];
    load_cell(pb, old_dofs, n_old, j, q);
    old_cell(pb, q, ck, oc[(size_t)j + 1]);
  }
  if (pb.bc != BC_PERIODIC && parity == 1) {
    if (pb.bc == BC_TRANSMISSIVE) {
      // Ghost staggered cells at x_{1/2} and x_{N+3/2}: copies of the adjacent cells.
      oc[0] = oc[1];
      oc[(size_t)n_old + 1] = oc[(size_t)n_old];
    } else {
      // Dirichlet: constant boundary state, zero derivatives.
      double q[NCMAX][PMAX + 1];
      for (int side = 0; side < 2; ++side) {
        const double* st = side == 0 ? pb.left_state : pb.right_state;
        for (int c = 0; c < nc; ++c)
          for (int k = 0; k <= P; ++k) q[c][k] = (k == 0) ? st[c] : 0.0;
        old_cell(pb, q, ck, oc[side == 0 ? 0 : (size_t)n_old + 1]);
      }
    }
  }

  // Largest new wave speed, NaN if any speed is NaN: the result does not
  // depend on the order in which the cells are visited.
  double smax = 0.0;
  int flags = 0;
#ifdef _OPENMP
#pragma omp parallel
#endif
  {
  double smax_t = 0.0;
  int flags_t = 0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
  for (int64_t j = 0; j < n_new; ++j) {
    int64_t jl, jr;  // indices of the parents in the old cell array (no ghost offset)
    if (pb.bc == BC_PERIODIC) {
      if (parity == 0) { jl = j; jr = (j + 1) % pb.N; }
      else { jl = (j - 1 + pb.N) % pb.N; jr = j; }
    } else {
      if (parity == 0) { jl = j; jr = j + 1; }
      else { jl = j - 1; jr = j; }
    }
    double q[NCMAX][PMAX + 1], sp;
    flags_t |= new_cell(pb, lam, oc[(size_t)(jl + 1)], oc[(size_t)(jr + 1)], q, sp);
    if (sp > smax_t || std::isnan(sp)) smax_t = std::isnan(smax_t) ? smax_t : sp;
    for (int c = 0; c < nc; ++c)
      for (int k = 0; k <= P; ++k) new_dofs[((int64_t)c * (P + 1) + k) * n_new + j] = q[c][k];
  }
#ifdef _OPENMP
#pragma omp critical
#endif
  {
    flags |= flags_t;
    if (smax_t > smax || std::isnan(smax_t)) smax = std::isnan(smax) ? smax : smax_t;
  }
  }
  *smax_out = smax;
  return flags;
}

// Largest wave speed over the cell averages of a state (Eq. SubEq:1DCellAVG
// gives the average from q).
double max_speed(const wcc_oracle_problem& pb, int parity, const double* dofs) {
  const int P = pb.P, nc = ncomp(pb);
  const int64_t n = ncells(pb, parity);
  double smax = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double q[NCMAX][PMAX + 1], abar[NCMAX];
    load_cell(pb, dofs, n, j, q);
    for (int c = 0; c < nc; ++c) {
      double s = q[c][0];
      for (int k = 2; k <= P; k += 2) s = std::fma(K.CA[k], q[c][k], s);
      abar[c] = s;
    }
    double sp = cell_speed(pb, abar);
    if (sp > smax || std::isnan(sp)) smax = std::isnan(smax) ? smax : sp;
  }
  return smax;
}

bool valid(const wcc_oracle_problem* pb) {
  if (!pb) return false;
  if (pb->equation < 0 || pb->equation > 2) return false;
  if (pb->P < 0 || pb->P > PMAX) return false;
  if (pb->N < 2) return false;
  if (pb->bc < 0 || pb->bc > 2) return false;
  if (!(pb->x_right > pb->x_left)) return false;
  return true;
}

}  // namespace

extern "C" {

// Threads a half-step uses: 1 in the serial build, the OpenMP team size in
// the OpenMP build.
int wcc_oracle_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t wcc_oracle_ncells(const wcc_oracle_problem* pb, int parity) {
  if (!valid(pb)) return -1;
  return ncells(*pb, parity & 1);
}

// One half-step with the given dt.  Returns the status flags (>= 0) or -1.
int wcc_oracle_half_step(const wcc_oracle_problem* pb, int parity, const double* old_dofs, double dt,
                         double* new_dofs, double* smax_out) {
  if (!valid(pb) || !old_dofs || !new_dofs || !smax_out) return -1;
  return half_step(*pb, parity & 1, old_dofs, dt, new_dofs, smax_out);
}

double wcc_oracle_max_speed(const wcc_oracle_problem* pb, int parity, const double* dofs) {
  if (!valid(pb) || !dofs) return -1.0;
  return max_speed(*pb, parity & 1, dofs);
}

// Time marching (CFL number per half-step, Section 5).  State in/out:
// *parity, *t, *smax (wave speed of the current state) and dofs, which must
// hold max(ncells(0), ncells(1)) cells per row ([c][k][j] with the row length
// of the current parity).  dt_fixed > 0 uses that dt and ignores t_end;
// otherwise dt = (cfl*dx)/smax, clipped so the last step ends on t_end.
// Runs at most max_half_steps.  Returns the number of half-steps taken and
// stores the status flags of the last step in *flags (the run stops at the
// first step that raises a flag).
int64_t wcc_oracle_run(const wcc_oracle_problem* pb, int* parity, double* t, double* smax, double* dofs,
                       double t_end, double cfl, double dt_fixed, int64_t max_half_steps, int* flags) {
  if (!valid(pb) || !parity || !t || !smax || !dofs || !flags) return -1;
  const int P = pb->P, nc = ncomp(*pb);
  const double dx = (pb->x_right - pb->x_left) / (double)pb->N;
  const int64_t nmax = ncells(*pb, 0) > ncells(*pb, 1) ? ncells(*pb, 0) : ncells(*pb, 1);
  std::vector<double> tmp((size_t)(nc * (P + 1)) * (size_t)nmax);
  *flags = 0;
  int64_t taken = 0;
  for (; taken < max_half_steps; ++taken) {
    double dt, tn;
    if (dt_fixed > 0.0) {
      dt = dt_fixed;
      tn = *t + dt;
    } else {
      if (!(*t < t_end)) break;
      dt = (cfl * dx) / *smax;
      double rem = t_end - *t;
      if (dt >= rem) { dt = rem; tn = t_end; }
      else tn = *t + dt;
    }
    double sm;
    int f = half_step(*pb, *parity, dofs, dt, tmp.data(), &sm);
    const int64_t nn = ncells(*pb, 1 - *parity);
    std::memcpy(dofs, tmp.data(), sizeof(double) * (size_t)(nc * (P + 1)) * (size_t)nn);
    *parity ^= 1;
    *t = tn;
    *smax = sm;
    if (f) { *flags = f; ++taken; break; }
  }
  return taken;
}

// Intermediate quantities of one half-step, per new cell j (limiter not
// applied): the new average abar[c][j] (Eq. SubEq:1DIntegral), the new
// derivatives d[c][k][j] (k=1..P, Eq. SubEq:Cal_1D_Derivatives_3; k=0 unused)
// and the vertex values vl[c][j], vr[c][j] (Eq. SubEq:Cal_1D_Derivatives_4 at
// the left and right parent).  Used to read off the linear candidates of
// Eq. 1D_U012.
int wcc_oracle_half_step_parts(const wcc_oracle_problem* pb, int parity, const double* old_dofs, double dt,
                               double* abar, double* d, double* vl, double* vr) {
  if (!valid(pb) || !old_dofs || !abar || !d || !vl || !vr) return -1;
  wcc_oracle_problem q = *pb;
  q.limiter = 0;
  const int P = q.P, nc = ncomp(q);
  const int64_t n_old = ncells(q, parity & 1), n_new = ncells(q, 1 - (parity & 1));
  if (q.bc != BC_PERIODIC) return -1;
  const double dx = (q.x_right - q.x_left) / (double)q.N;
  const double lam = dt / dx;
  double ck[PMAX + 1][PMAX + 1];
  ck_factors(lam, ck);
  std::vector<OldCell<double>> oc((size_t)n_old);
  for (int64_t j = 0; j < n_old; ++j) {
    double qq[NCMAX][PMAX + 1];
    load_cell(q, old_dofs, n_old, j, qq);
    old_cell(q, qq, ck, oc[(size_t)j]);
  }
  for (int64_t j = 0; j < n_new; ++j) {
    int64_t jl = (parity & 1) == 0 ? j : (j - 1 + q.N) % q.N;
    int64_t jr = (parity & 1) == 0 ? (j + 1) % q.N : j;
    const OldCell<double>& L = oc[(size_t)jl];
    const OldCell<double>& R = oc[(size_t)jr];
    for (int c = 0; c < nc; ++c) {
      double h = 0.5 * (L.uR[c] + R.uL[c]);
      abar[(int64_t)c * n_new + j] = std::fma(lam, L.fbar[c] - R.fbar[c], h);
      double dd[PMAX + 1];
      dd[0] = 0.0;
      for (int k = P - 1; k >= 0; --k) {
        double s = R.V[c][k] - L.V[c][k];
        for (int m = 3; m <= P - k; m += 2) s = std::fma(K.NCO[m], dd[k + m], s);
        dd[k + 1] = s;
      }
      for (int k = 0; k <= P; ++k) d[((int64_t)c * (P + 1) + k) * n_new + j] = dd[k];
      vl[(int64_t)c * n_new + j] = P >= 1 ? L.V[c][0] : L.uR[c];
      vr[(int64_t)c * n_new + j] = P >= 1 ? R.V[c][0] : R.uL[c];
    }
  }
  return 0;
}

// Normalised Cauchy-Kovalewski triangle of one cell state q[c][k]:
// T[c][k][m] = u_{kx,mt}/(k! m!) for k+m <= P (other entries zero), lam = dt/dx.
int wcc_oracle_ck_triangle(const wcc_oracle_problem* pb, const double* qin, double lam, double* Tout) {
  if (!valid(pb) || !qin || !Tout) return -1;
  const int P = pb->P, nc = ncomp(*pb);
  double q[NCMAX][PMAX + 1];
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k) q[c][k] = qin[c * (P + 1) + k];
  double ck[PMAX + 1][PMAX + 1];
  ck_factors(lam, ck);
  Tri<double> T[NCMAX], G[NCMAX];
  FluxWork<double> w;
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= PMAX; ++k)
      for (int m = 0; m <= PMAX; ++m) T[c][k][m] = 0.0;
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k) T[c][k][0] = (k <= 1) ? q[c][k] : q[c][k] * K.IF[k];
  for (int m = 1; m <= P; ++m) {
    flux_column(*pb, P, T, G, w, m - 1);
    for (int c = 0; c < nc; ++c)
      for (int k = 0; k + m <= P; ++k) T[c][k][m] = ck[k][m] * G[c][k + 1][m - 1];
  }
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k)
      for (int m = 0; m <= P; ++m) Tout[(c * (P + 1) + k) * (P + 1) + m] = (k + m <= P) ? T[c][k][m] : 0.0;
  return 0;
}

double wcc_oracle_js_indicator(int P, const double* d) {
  if (P < 1 || P > PMAX || !d) return -1.0;
  double dd[PMAX + 1];
  for (int k = 0; k <= P; ++k) dd[k] = d[k];
  return js_indicator(P, dd);
}

// The limiter on one scalar field: d[0..P] (d[0] ignored) modified in place.
int wcc_oracle_limit_field(int P, double eps, double abar, double* d, double vl, double vr) {
  if (P < 1 || P > PMAX || !d) return -1;
  double dd[PMAX + 1];
  for (int k = 0; k <= P; ++k) dd[k] = d[k];
  limit_field(P, eps, abar, dd, vl, vr);
  for (int k = 1; k <= P; ++k) d[k] = dd[k];
  return 0;
}

// Left and right eigenvector matrices of the Euler flux Jacobian at U.
int wcc_oracle_euler_eigen(double gamma, const double* U, double* Lout, double* Rout) {
  if (!U || !Lout || !Rout) return -1;
  double UU[3] = {U[0], U[1], U[2]}, u, p, c;
  euler_primitive(gamma, UU, u, p, c);
  EulerEig<double> e;
  euler_eigen(gamma, UU, u, p, c, e);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Lout[i * 3 + j] = e.L[i][j];
      Rout[i * 3 + j] = e.Rm[i][j];
    }
  return 0;
}

// Floating-point operations of the half-step per new cell for this problem,
// counted by running one interior new cell in the counting type:
// out = {add/sub, mul, fma, div, sqrt, flops} with flops = add+mul+2*fma+div+sqrt
// (the per-old-cell work, done once per old cell, is included once).
int wcc_oracle_count_flops(const wcc_oracle_problem* pb, const double* q_left, const double* q_right,
                           double lam, double* out) {
  if (!valid(pb) || !q_left || !q_right || !out) return -1;
  const int P = pb->P, nc = ncomp(*pb);
  Counted ck[PMAX + 1][PMAX + 1];
  Counted ql[NCMAX][PMAX + 1], qr[NCMAX][PMAX + 1];
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k <= P; ++k) {
      ql[c][k] = q_left[c * (P + 1) + k];
      qr[c][k] = q_right[c * (P + 1) + k];
    }
  ck_factors(Counted(lam), ck);  // per-step constant: not counted per cell
  OldCell<Counted> a, b;
  old_cell(*pb, qr, ck, b);
  g_ops = OpCount();
  old_cell(*pb, ql, ck, a);
  Counted q[NCMAX][PMAX + 1], sp;
  new_cell(*pb, Counted(lam), a, b, q, sp);
  out[0] = g_ops.add;
  out[1] = g_ops.mul;
  out[2] = g_ops.fma;
  out[3] = g_ops.div;
  out[4] = g_ops.sqrt;
  out[5] = g_ops.add + g_ops.mul + 2 * g_ops.fma + g_ops.div + g_ops.sqrt;
  return 0;
}

}  // extern "C"
