// CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, double-precision reference of the p-adaptive implicit flux
// reconstruction (FR/CPR) hot path of Wang, Gobbert & Yu (arXiv 1910.03693).
// Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
// load it.  It shares no source with the HIP library: every operator, geometric
// quantity, flux, solver and indicator below is written out again from the
// paper's definitions, in the paper's order, with no blocking or fusion.
//
// The residual is templated on the scalar so that the very same code also runs
// in std::complex<double> and gives the exact tangent by the complex step
// (Squire & Trapp 1998): J v = Im R(U + i h v) / h with h = 1e-30.
//
// Readings of points the paper leaves open (each one listed in the design notes):
//  * solution points: tensor Gauss-Legendre; correction function: the DG one
//    (right/left Radau polynomials), which is what the Galerkin definition of the
//    correction field in section 2.2 yields;
//  * common solution: average of the conservative states (eq. com_q);
//  * BR2 (eq. com_grad_q): grad q^{+/-} are face extrapolations of the
//    uncorrected physical gradient, r^{+/-} the lifting of this face's jump
//    alone, penalty factor 1;
//  * Roe flux (eq. invis_com) without low-Mach preconditioning or entropy fix;
//  * faces whose sides differ in degree: the face points are the higher side's
//    Gauss points; the lower side is interpolated there, and what it receives
//    back (jump, common flux) is the L2 projection onto its own degree;
//  * boundary states: no-slip adiabatic wall (interior density and temperature,
//    zero velocity, zero heat flux) and far field (common solution halfway to
//    the free stream); the common gradient there is grad q_i + r_i.
#include <algorithm>
#include <cmath>
#include <complex>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace orc {

using cplx = std::complex<double>;

// ------------------------------------------------------------ scalar helpers
inline double re(double x) { return x; }
inline double re(long double x) { return (double)x; }
inline double re(const cplx& x) { return x.real(); }
// |x| and max() choose by the real part, which makes them complex-step safe
template <class S> S sabs(const S& x) { return re(x) < 0 ? S(-x) : x; }
template <class S> S smax(const S& a, const S& b) { return re(a) >= re(b) ? a : b; }
inline double ssqrt(double x) { return std::sqrt(x); }
inline long double ssqrt(long double x) { return std::sqrt(x); }
inline cplx ssqrt(const cplx& x) { return std::sqrt(x); }

// ------------------------------------------------------- operation counting
// Scalars that count the floating-point operations of the code that runs on
// them (one per +, -, *, / and square root; a sign change or a comparison is
// none), for the work model of the measured kernels.  Cnt is a counted real;
// DCnt is a counted forward-mode dual number (value and derivative), with
// each operation charged what it costs in that arithmetic: a product 3 (+1
// for the value), a quotient 4, a square root 3, an operation with a plain
// double half of that or less.  The counter is global: the counting entry
// points run their residual with one thread.
static long long g_flops = 0;
struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_flops; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_flops; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_flops; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_flops; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline double re(const Cnt& x) { return x.v; }
inline Cnt ssqrt(const Cnt& x) { ++g_flops; return Cnt(std::sqrt(x.v)); }

struct DCnt {
  double v, d;
  DCnt() : v(0.0), d(0.0) {}
  DCnt(double x) : v(x), d(0.0) {}
  DCnt(double x, double y) : v(x), d(y) {}
};
inline DCnt operator+(DCnt a, DCnt b) { g_flops += 2; return DCnt(a.v + b.v, a.d + b.d); }
inline DCnt operator-(DCnt a, DCnt b) { g_flops += 2; return DCnt(a.v - b.v, a.d - b.d); }
inline DCnt operator*(DCnt a, DCnt b) { g_flops += 4; return DCnt(a.v * b.v, a.d * b.v + a.v * b.d); }
inline DCnt operator/(DCnt a, DCnt b) {
  g_flops += 4;
  const double q = a.v / b.v;
  return DCnt(q, (a.d - q * b.d) / b.v);
}
inline DCnt operator+(DCnt a, double b) { g_flops += 1; return DCnt(a.v + b, a.d); }
inline DCnt operator+(double a, DCnt b) { g_flops += 1; return DCnt(a + b.v, b.d); }
inline DCnt operator-(DCnt a, double b) { g_flops += 1; return DCnt(a.v - b, a.d); }
inline DCnt operator-(double a, DCnt b) { g_flops += 1; return DCnt(a - b.v, -b.d); }
inline DCnt operator*(DCnt a, double b) { g_flops += 2; return DCnt(a.v * b, a.d * b); }
inline DCnt operator*(double a, DCnt b) { g_flops += 2; return DCnt(a * b.v, a * b.d); }
inline DCnt operator/(DCnt a, double b) { g_flops += 2; return DCnt(a.v / b, a.d / b); }
inline DCnt operator/(double a, DCnt b) {
  g_flops += 4;
  const double q = a / b.v;
  return DCnt(q, -q * b.d / b.v);
}
inline DCnt operator-(DCnt a) { return DCnt(-a.v, -a.d); }
inline DCnt& operator+=(DCnt& a, DCnt b) { a = a + b; return a; }
inline DCnt& operator-=(DCnt& a, DCnt b) { a = a - b; return a; }
inline DCnt& operator*=(DCnt& a, DCnt b) { a = a * b; return a; }
inline double re(const DCnt& x) { return x.v; }
inline DCnt ssqrt(const DCnt& x) {
  g_flops += 3;
  const double r = std::sqrt(x.v);
  return DCnt(r, x.d / (2.0 * r));
}

// ------------------------------------------------------- 1-D polynomial tools
// Legendre P_k(x) and P_k'(x) for k = 0..K by the three-term recurrence.
template <class R> static void legendre(int K, R x, R* P, R* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (K >= 1) { P[1] = x; dP[1] = 1.0; }
  for (int k = 1; k < K; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}

// Operators in the real type R: double for the double and complex-step
// residuals, long double for the extended-precision reference used to size
// rounding errors.
template <class R> struct Ops1DT {
  int n = 0;
  std::vector<R> x, w;  // Gauss-Legendre nodes (ascending) and weights
  std::vector<R> D;     // D[k*n + j] = l_j'(x_k)
  std::vector<R> lm, lp;  // l_j(-1), l_j(+1)
  std::vector<R> gLp, gRp;  // g_L'(x_k), g_R'(x_k)
  std::vector<R> V;       // V[k*n + m] = P_m(x_k)  (Legendre Vandermonde)
};
using Ops1D = Ops1DT<double>;

template <class R> static R lagrange(const std::vector<R>& x, int j, R t) {
  R v = 1.0;
  for (size_t m = 0; m < x.size(); ++m)
    if ((int)m != j) v *= (t - x[m]) / (x[j] - x[m]);
  return v;
}

template <class R> static R lagrange_d(const std::vector<R>& x, int j, R t) {
  R s = 0.0;
  for (size_t l = 0; l < x.size(); ++l) {
    if ((int)l == j) continue;
    R prod = R(1.0) / (x[j] - x[l]);
    for (size_t m = 0; m < x.size(); ++m)
      if ((int)m != j && m != l) prod *= (t - x[m]) / (x[j] - x[m]);
    s += prod;
  }
  return s;
}

// DG correction function g_L = right Radau polynomial of degree p+1:
// g_L(x) = (-1)^(p+1)/2 (P_{p+1}(x) - P_p(x)); g_L(-1) = 1, g_L(+1) = 0.
template <class R> static R radau_gL_d(int p, R x) {
  R P[16], dP[16];
  legendre<R>(p + 1, x, P, dP);
  R sgn = ((p + 1) % 2 == 0) ? 1.0 : -1.0;
  return 0.5 * sgn * (dP[p + 1] - dP[p]);
}

template <class R> static Ops1DT<R> make_ops(int n) {
  Ops1DT<R> o;
  o.n = n;
  o.x.resize(n);
  o.w.resize(n);
  R P[16], dP[16];
  for (int i = 0; i < n; ++i) {  // Newton on P_n from the usual cosine guess
    R t = -std::cos(R(M_PI) * (i + R(0.75)) / (n + R(0.5)));
    for (int it = 0; it < 100; ++it) {
      legendre<R>(n, t, P, dP);
      R dt = P[n] / dP[n];
      t -= dt;
      if (std::fabs(dt) < R(1e-19)) break;
    }
    legendre<R>(n, t, P, dP);
    o.x[i] = t;
    o.w[i] = R(2.0) / ((R(1.0) - t * t) * dP[n] * dP[n]);
  }
  o.D.resize(n * n);
  o.lm.resize(n);
  o.lp.resize(n);
  o.gLp.resize(n);
  o.gRp.resize(n);
  o.V.resize(n * n);
  int p = n - 1;
  for (int k = 0; k < n; ++k) {
    for (int j = 0; j < n; ++j) o.D[k * n + j] = lagrange_d<R>(o.x, j, o.x[k]);
    o.lm[k] = lagrange<R>(o.x, k, R(-1.0));
    o.lp[k] = lagrange<R>(o.x, k, R(1.0));
    o.gLp[k] = radau_gL_d<R>(p, o.x[k]);
    o.gRp[k] = -radau_gL_d<R>(p, -o.x[k]);  // g_R(x) = g_L(-x)
    legendre<R>(n - 1, o.x[k], P, dP);
    for (int m = 0; m < n; ++m) o.V[k * n + m] = P[m];
  }
  return o;
}

template <class R = double> static const Ops1DT<R>& ops(int n) {
  static Ops1DT<R> table[8];
  static bool init = false;
  if (!init) {
    for (int m = 1; m < 8; ++m) table[m] = make_ops<R>(m);
    init = true;
  }
  return table[n];
}

// Interpolation from the n_from Gauss points to the n_to Gauss points:
// I[a*n_from + b] = l^{from}_b(x^{to}_a).
template <class R = double> static std::vector<R> interp_matrix(int n_from, int n_to) {
  const Ops1DT<R>& f = ops<R>(n_from);
  const Ops1DT<R>& t = ops<R>(n_to);
  std::vector<R> I(n_to * n_from);
  for (int a = 0; a < n_to; ++a)
    for (int b = 0; b < n_from; ++b) I[a * n_from + b] = lagrange<R>(f.x, b, t.x[a]);
  return I;
}

// L2 projection onto degree n_lo-1 of values at the n_hi Gauss points, returned
// at the n_lo Gauss points; the n_lo-point rule makes the mass matrix diagonal:
// Pr[k*n_hi + m] = w^hi_m l^lo_k(x^hi_m) / w^lo_k.
template <class R = double> static std::vector<R> project_matrix(int n_hi, int n_lo) {
  const Ops1DT<R>& h = ops<R>(n_hi);
  const Ops1DT<R>& l = ops<R>(n_lo);
  std::vector<R> Pr(n_lo * n_hi);
  for (int k = 0; k < n_lo; ++k)
    for (int m = 0; m < n_hi; ++m) Pr[k * n_hi + m] = h.w[m] * lagrange<R>(l.x, k, h.x[m]) / l.w[k];
  return Pr;
}

// ------------------------------------------------------------------ geometry
// Trilinear map of a hexahedron; vertex v = a + 2b + 4c sits at reference
// (2a-1, 2b-1, 2c-1).  dx[i][c] = d x_c / d xi^i.
template <class R> static void trilinear(const double* X, const R r[3], R x[3], R dx[3][3]) {
  for (int c = 0; c < 3; ++c) {
    x[c] = 0;
    for (int i = 0; i < 3; ++i) dx[i][c] = 0;
  }
  for (int v = 0; v < 8; ++v) {
    R s[3] = {(v & 1) ? R(1.0) : R(-1.0), (v & 2) ? R(1.0) : R(-1.0), (v & 4) ? R(1.0) : R(-1.0)};
    R f[3] = {1 + s[0] * r[0], 1 + s[1] * r[1], 1 + s[2] * r[2]};
    R N = R(0.125) * f[0] * f[1] * f[2];
    R dN[3] = {R(0.125) * s[0] * f[1] * f[2], R(0.125) * f[0] * s[1] * f[2], R(0.125) * f[0] * f[1] * s[2]};
    for (int c = 0; c < 3; ++c) {
      x[c] += N * X[3 * v + c];
      for (int i = 0; i < 3; ++i) dx[i][c] += dN[i] * X[3 * v + c];
    }
  }
}

template <class R> static void cross(const R a[3], const R b[3], R o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Metric cofactors Ja^i = x_{xi^(i+1)} x x_{xi^(i+2)} and J = det(dx/dxi) at r.
template <class R> static void metrics(const double* X, const R r[3], R Ja[3][3], R* J) {
  R x[3], dx[3][3];
  trilinear<R>(X, r, x, dx);
  for (int i = 0; i < 3; ++i) cross(dx[(i + 1) % 3], dx[(i + 2) % 3], Ja[i]);
  *J = dx[0][0] * Ja[0][0] + dx[0][1] * Ja[0][1] + dx[0][2] * Ja[0][2];
}

// -------------------------------------------------------------------- mesh
struct Elem {
  int n;             // p + 1
  long off;          // first solution point
  const double* X;   // 8 vertices
  std::vector<double> J, Ja;  // per solution point: J, Ja[i][c]
  std::vector<long double> Jl, Jal;  // the same in extended precision
  template <class R> const R* Jp() const;
  template <class R> const R* Jap() const;
};
template <> const double* Elem::Jp<double>() const { return J.data(); }
template <> const long double* Elem::Jp<long double>() const { return Jl.data(); }
template <> const double* Elem::Jap<double>() const { return Ja.data(); }
template <> const long double* Elem::Jap<long double>() const { return Jal.data(); }

template <class S> struct real_of { using type = double; };
template <> struct real_of<long double> { using type = long double; };

struct IFace { int L, R, d; };        // L's +d face is R's -d face
struct BFace { int e, f, bc; };       // element face f = 2d + s, bc -1 wall, -2 far field

struct Mesh {
  int n_elem = 0;
  long n_sp = 0;
  int physics = 0, flux = 0;
  double gamma = 1.4, mu = 0, prandtl = 0.72;
  double farfield[5] = {0, 0, 0, 0, 0};
  std::vector<double> xyz;
  std::vector<int> nbr;
  std::vector<Elem> el;
  std::vector<IFace> ifaces;
  std::vector<BFace> bfaces;
};

// Index of the solution point at position m along reference direction d on the
// line through face point (a, b); tangential directions are the other two in
// increasing order.
static inline int line_idx(int n, int d, int a, int b, int m) {
  int id[3];
  id[d] = m;
  id[d == 0 ? 1 : 0] = a;
  id[d == 2 ? 1 : 2] = b;
  return id[0] + n * (id[1] + n * id[2]);
}

// Reference coordinates of face point (a, b) of the n-point rule on face (d, side).
template <class R> static void face_point(int n, int d, int side, int a, int b, R r[3]) {
  const Ops1DT<R>& o = ops<R>(n);
  r[d] = side ? 1.0 : -1.0;
  r[d == 0 ? 1 : 0] = o.x[a];
  r[d == 2 ? 1 : 2] = o.x[b];
}

// ------------------------------------------------------------------ physics
template <class S> struct Phys {
  double g, mu, pr;
  S pressure(const S* q) const {
    return (g - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
  }
  // inviscid flux in physical direction c (section 2.1, the Euler part)
  void inviscid(const S* q, int c, S* f) const {
    S p = pressure(q);
    S uc = q[1 + c] / q[0];
    f[0] = q[1 + c];
    for (int a = 0; a < 3; ++a) f[1 + a] = q[1 + a] * uc + (a == c ? p : S(0.0));
    f[4] = (q[4] + p) * uc;
  }
  // viscous flux fv[c][v] from the conservative state and its physical gradient
  // G[v][c]: Stokes stress with constant mu, Fourier heat flux with constant Pr,
  // gas constant 1 (T = p / rho), cp = gamma / (gamma - 1).
  void viscous(const S* q, const S G[5][3], S fv[3][5], bool adiabatic = false) const {
    S rho = q[0];
    S u[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
    S gu[3][3];  // gu[a][c] = d u_a / d x_c
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) gu[a][c] = (G[1 + a][c] - u[a] * G[0][c]) / rho;
    S e = q[4] / rho;
    S gT[3];
    for (int c = 0; c < 3; ++c) {
      S ge = (G[4][c] - e * G[0][c]) / rho;
      S uu = u[0] * gu[0][c] + u[1] * gu[1][c] + u[2] * gu[2][c];
      gT[c] = (g - 1.0) * (ge - uu);
    }
    S div = gu[0][0] + gu[1][1] + gu[2][2];
    double kappa = mu * g / ((g - 1.0) * pr);
    for (int c = 0; c < 3; ++c) {
      S tau[3];
      for (int a = 0; a < 3; ++a) tau[a] = mu * (gu[a][c] + gu[c][a] - (a == c ? (2.0 / 3.0) * div : S(0.0)));
      fv[c][0] = 0.0;
      for (int a = 0; a < 3; ++a) fv[c][1 + a] = tau[a];
      fv[c][4] = adiabatic ? S(0.0) : S(u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + kappa * gT[c]);
    }
  }
  // common inviscid flux dotted with the (unnormalised) area vector Sv.
  template <class R> void roe(const S* qL, const S* qR, const R* Sv, S* out) const {
    R area = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
    R nv[3] = {Sv[0] / area, Sv[1] / area, Sv[2] / area};
    S fL[5], fR[5];
    for (int v = 0; v < 5; ++v) fL[v] = fR[v] = 0.0;
    for (int c = 0; c < 3; ++c) {
      S a[5], b[5];
      inviscid(qL, c, a);
      inviscid(qR, c, b);
      for (int v = 0; v < 5; ++v) {
        fL[v] += nv[c] * a[v];
        fR[v] += nv[c] * b[v];
      }
    }
    S pL = pressure(qL), pR = pressure(qR);
    S sL = ssqrt(qL[0]), sR = ssqrt(qR[0]);
    S uL[3], uR[3], ut[3];
    for (int a = 0; a < 3; ++a) {
      uL[a] = qL[1 + a] / qL[0];
      uR[a] = qR[1 + a] / qR[0];
      ut[a] = (sL * uL[a] + sR * uR[a]) / (sL + sR);
    }
    S HL = (qL[4] + pL) / qL[0], HR = (qR[4] + pR) / qR[0];
    S Ht = (sL * HL + sR * HR) / (sL + sR);
    S rhot = sL * sR;
    S q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    S ct = ssqrt((g - 1.0) * (Ht - 0.5 * q2));
    S un = ut[0] * nv[0] + ut[1] * nv[1] + ut[2] * nv[2];
    S dp = pR - pL, drho = qR[0] - qL[0];
    S du[3];
    for (int a = 0; a < 3; ++a) du[a] = uR[a] - uL[a];
    S dun = du[0] * nv[0] + du[1] * nv[1] + du[2] * nv[2];
    S l1 = sabs(S(un - ct)), l2 = sabs(un), l5 = sabs(S(un + ct));
    S a1 = (dp - rhot * ct * dun) / (2.0 * ct * ct);
    S a5 = (dp + rhot * ct * dun) / (2.0 * ct * ct);
    S a2 = drho - dp / (ct * ct);
    S diss[5];
    diss[0] = l1 * a1 + l2 * a2 + l5 * a5;
    for (int a = 0; a < 3; ++a)
      diss[1 + a] = l1 * a1 * (ut[a] - ct * nv[a]) + l2 * (a2 * ut[a] + rhot * (du[a] - dun * nv[a])) +
                    l5 * a5 * (ut[a] + ct * nv[a]);
    S udu = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
    diss[4] = l1 * a1 * (Ht - un * ct) + l2 * (a2 * 0.5 * q2 + rhot * (udu - un * dun)) + l5 * a5 * (Ht + un * ct);
    for (int v = 0; v < 5; ++v) out[v] = area * (0.5 * (fL[v] + fR[v]) - 0.5 * diss[v]);
  }
  template <class R> void rusanov(const S* qL, const S* qR, const R* Sv, S* out) const {
    R area = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
    R nv[3] = {Sv[0] / area, Sv[1] / area, Sv[2] / area};
    S fL[5], fR[5];
    for (int v = 0; v < 5; ++v) fL[v] = fR[v] = 0.0;
    for (int c = 0; c < 3; ++c) {
      S a[5], b[5];
      inviscid(qL, c, a);
      inviscid(qR, c, b);
      for (int v = 0; v < 5; ++v) {
        fL[v] += nv[c] * a[v];
        fR[v] += nv[c] * b[v];
      }
    }
    S cL = ssqrt(g * pressure(qL) / qL[0]), cR = ssqrt(g * pressure(qR) / qR[0]);
    S unL = (qL[1] * nv[0] + qL[2] * nv[1] + qL[3] * nv[2]) / qL[0];
    S unR = (qR[1] * nv[0] + qR[2] * nv[1] + qR[3] * nv[2]) / qR[0];
    S lam = smax(S(sabs(unL) + cL), S(sabs(unR) + cR));
    for (int v = 0; v < 5; ++v) out[v] = area * (0.5 * (fL[v] + fR[v]) - 0.5 * lam * (qR[v] - qL[v]));
  }
};

// ----------------------------------------------------------------- residual
// R = -(P(div f) + delta) of eq. FR_diff, written in the reference element:
// R = -(1/J) [ sum_i D_i Ft^i + sum_faces (f_com.S - f_loc) g' ], with the
// contravariant flux Ft^i = Ja^i . f and the DG correction functions.
template <class S> struct Work {
  // per element, per face (6), per variable, per own face point
  std::vector<std::vector<S>> qf, gf, dq, fS;
};

// tabs (optional): at every solution point, the sum of the absolute values of
// the terms that the last step adds up, divided by |J| (the scale against
// which the rounding of R is judged where the terms cancel).
// The element loops and the interior-face loop run with OpenMP when the
// library is built with it; every iteration writes only its own element's or
// face's entries, so the result does not depend on the thread count.
template <class S>
static void residual(const Mesh& M, const S* U, S* Rout, double* bflux = nullptr, double* tabs = nullptr) {
  using R = typename real_of<S>::type;
  (void)ops<R>(1);  // the operator tables are built once, before any thread starts
  Phys<S> ph{M.gamma, M.mu, M.prandtl};
  const bool ns = M.physics == 1;
  if (bflux)
    for (int v = 0; v < 5; ++v) bflux[v] = 0.0;
  const long N = M.n_sp;
  const int E = M.n_elem;
  auto Uv = [&](int v, long k) -> const S& { return U[v * N + k]; };
  Work<S> W;
  W.qf.resize(E);
  W.gf.resize(E);
  W.dq.resize(E);
  W.fS.resize(E);
  std::vector<std::vector<S>> gphys(E);  // uncorrected physical gradient [k][v][c]

  // 1. Traces of q at the faces, and (Navier-Stokes) the uncorrected physical
  //    gradient at the solution points and its face traces.
#pragma omp parallel for schedule(dynamic, 16)
  for (int e = 0; e < E; ++e) {
    const Elem& el = M.el[e];
    int n = el.n, n2 = n * n, n3 = n2 * n;
    const Ops1DT<R>& o = ops<R>(n);
    const R* eJ = el.Jp<R>();
    const R* eJa = el.Jap<R>();
    W.qf[e].assign(6 * 5 * n2, S(0.0));
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      const std::vector<R>& l = (f % 2) ? o.lp : o.lm;
      for (int v = 0; v < 5; ++v)
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            S s = 0.0;
            for (int m = 0; m < n; ++m) s += l[m] * Uv(v, el.off + line_idx(n, d, a, b, m));
            W.qf[e][(f * 5 + v) * n2 + a + n * b] = s;
          }
    }
    if (!ns) continue;
    gphys[e].assign(n3 * 15, S(0.0));
    for (int k = 0; k < n3; ++k) {
      int id[3] = {k % n, (k / n) % n, k / n2};
      for (int v = 0; v < 5; ++v) {
        S dxi[3];
        for (int i = 0; i < 3; ++i) {
          dxi[i] = 0.0;
          for (int m = 0; m < n; ++m) {
            int jd[3] = {id[0], id[1], id[2]};
            jd[i] = m;
            dxi[i] += o.D[id[i] * n + m] * Uv(v, el.off + jd[0] + n * (jd[1] + n * jd[2]));
          }
        }
        for (int c = 0; c < 3; ++c) {
          S s = 0.0;
          for (int i = 0; i < 3; ++i) s += eJa[k * 9 + i * 3 + c] * dxi[i];
          gphys[e][k * 15 + v * 3 + c] = s / eJ[k];
        }
      }
    }
    W.gf[e].assign(6 * 15 * n2, S(0.0));
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      const std::vector<R>& l = (f % 2) ? o.lp : o.lm;
      for (int vc = 0; vc < 15; ++vc)
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            S s = 0.0;
            for (int m = 0; m < n; ++m) s += l[m] * gphys[e][line_idx(n, d, a, b, m) * 15 + vc];
            W.gf[e][(f * 15 + vc) * n2 + a + n * b] = s;
          }
    }
  }

  // 2. Faces: common solution, BR2 common gradient, common normal flux.
  for (int e = 0; e < E; ++e) {
    int n2 = M.el[e].n * M.el[e].n;
    W.dq[e].assign(6 * 5 * n2, S(0.0));
    W.fS[e].assign(6 * 5 * n2, S(0.0));
  }
  // values of side (e, f) at the face's nh x nh points (tensor interpolation)
  auto to_face = [&](const std::vector<S>& src, int e, int f, int nvals, int nh, std::vector<S>& dst) {
    int n = M.el[e].n, n2 = n * n;
    std::vector<R> I = interp_matrix<R>(n, nh);
    dst.assign(nvals * nh * nh, S(0.0));
    for (int v = 0; v < nvals; ++v)
      for (int B = 0; B < nh; ++B)
        for (int A = 0; A < nh; ++A) {
          S s = 0.0;
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) s += I[A * n + a] * I[B * n + b] * src[(f * nvals + v) * n2 + a + n * b];
          dst[v * nh * nh + A + nh * B] = s;
        }
  };
  // store values given at the nh x nh face points into side (e, f), projecting
  // onto the side's own degree
  auto from_face = [&](const std::vector<S>& src, int e, int f, int nh, std::vector<S>& dst) {
    int n = M.el[e].n, n2 = n * n;
    std::vector<R> P = project_matrix<R>(nh, n);
    for (int v = 0; v < 5; ++v)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          S s = 0.0;
          for (int B = 0; B < nh; ++B)
            for (int A = 0; A < nh; ++A) s += P[a * nh + A] * P[b * nh + B] * src[v * nh * nh + A + nh * B];
          dst[(f * 5 + v) * n2 + a + n * b] = s;
        }
  };
  auto common_inviscid = [&](const S* qm, const S* qp, const R* Sv, S* out) {
    if (M.flux == 0) ph.roe(qm, qp, Sv, out);
    else ph.rusanov(qm, qp, Sv, out);
  };

#pragma omp parallel for schedule(dynamic, 16)
  for (size_t fi = 0; fi < M.ifaces.size(); ++fi) {
    const IFace& F = M.ifaces[fi];
    int fL = 2 * F.d + 1, fR = 2 * F.d;
    int nL = M.el[F.L].n, nR = M.el[F.R].n, nh = std::max(nL, nR), nh2 = nh * nh;
    std::vector<S> qL, qR, gL, gR;
    to_face(W.qf[F.L], F.L, fL, 5, nh, qL);
    to_face(W.qf[F.R], F.R, fR, 5, nh, qR);
    if (ns) {
      to_face(W.gf[F.L], F.L, fL, 15, nh, gL);
      to_face(W.gf[F.R], F.R, fR, 15, nh, gR);
    }
    std::vector<S> fs(5 * nh2), jL(5 * nh2), jR(5 * nh2);
    for (int B = 0; B < nh; ++B)
      for (int A = 0; A < nh; ++A) {
        int pt = A + nh * B;
        R rL[3], rR[3], Sv[3], JaL[3][3], JaR[3][3], JL, JR;
        face_point<R>(nh, F.d, 1, A, B, rL);
        face_point<R>(nh, F.d, 0, A, B, rR);
        metrics<R>(M.el[F.L].X, rL, JaL, &JL);  // area vector from the minus side
        metrics<R>(M.el[F.R].X, rR, JaR, &JR);
        for (int c = 0; c < 3; ++c) Sv[c] = JaL[F.d][c];
        S qm[5], qp[5], qc[5], out[5];
        for (int v = 0; v < 5; ++v) {
          qm[v] = qL[v * nh2 + pt];
          qp[v] = qR[v * nh2 + pt];
          qc[v] = 0.5 * (qm[v] + qp[v]);  // eq. com_q
        }
        common_inviscid(qm, qp, Sv, out);
        if (ns) {
          // BR2 liftings of this face's jump: r = (S / J_f) (q_com - q) g'(face)
          R cL = R(0.5) * nL * nL / JL;   // g_R'(+1) = (p+1)^2/2 on L's + face
          R cR = R(-0.5) * nR * nR / JR;  // g_L'(-1) = -(p+1)^2/2 on R's - face
          S Gc[5][3];
          for (int v = 0; v < 5; ++v)
            for (int c = 0; c < 3; ++c) {
              S rl = Sv[c] * cL * (qc[v] - qm[v]);
              S rr = Sv[c] * cR * (qc[v] - qp[v]);
              Gc[v][c] = 0.5 * (gL[(v * 3 + c) * nh2 + pt] + rl + gR[(v * 3 + c) * nh2 + pt] + rr);  // eq. com_grad_q
            }
          S fv[3][5];
          ph.viscous(qc, Gc, fv);
          for (int v = 0; v < 5; ++v) out[v] -= fv[0][v] * Sv[0] + fv[1][v] * Sv[1] + fv[2][v] * Sv[2];
        }
        for (int v = 0; v < 5; ++v) {
          fs[v * nh2 + pt] = out[v];
          jL[v * nh2 + pt] = qc[v] - qm[v];
          jR[v * nh2 + pt] = qc[v] - qp[v];
        }
      }
    from_face(fs, F.L, fL, nh, W.fS[F.L]);
    from_face(fs, F.R, fR, nh, W.fS[F.R]);
    from_face(jL, F.L, fL, nh, W.dq[F.L]);
    from_face(jR, F.R, fR, nh, W.dq[F.R]);
  }

  for (const BFace& F : M.bfaces) {
    const Elem& el = M.el[F.e];
    int n = el.n, n2 = n * n, d = F.f / 2, side = F.f % 2;
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) {
        int pt = a + n * b;
        R r[3], Ja[3][3], J;
        face_point<R>(n, d, side, a, b, r);
        metrics<R>(el.X, r, Ja, &J);
        const R* Sv = Ja[d];
        S qi[5], qb[5], out[5];
        for (int v = 0; v < 5; ++v) qi[v] = W.qf[F.e][(F.f * 5 + v) * n2 + pt];
        bool wall = F.bc == -1;
        if (wall) {
          S ke = 0.5 * (qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]) / qi[0];
          qb[0] = qi[0];
          qb[1] = qb[2] = qb[3] = 0.0;
          qb[4] = qi[4] - ke;
          S p = ph.pressure(qi);
          out[0] = out[4] = 0.0;
          for (int c = 0; c < 3; ++c) out[1 + c] = p * Sv[c];
        } else {
          S qinf[5];
          for (int v = 0; v < 5; ++v) {
            qinf[v] = M.farfield[v];
            qb[v] = 0.5 * (qi[v] + qinf[v]);
          }
          if (side) common_inviscid(qi, qinf, Sv, out);
          else common_inviscid(qinf, qi, Sv, out);
        }
        if (ns) {
          R cf = R(side ? 0.5 : -0.5) * n * n / J;
          S Gc[5][3];
          for (int v = 0; v < 5; ++v)
            for (int c = 0; c < 3; ++c)
              Gc[v][c] = W.gf[F.e][(F.f * 15 + v * 3 + c) * n2 + pt] + Sv[c] * cf * (qb[v] - qi[v]);
          S fv[3][5];
          ph.viscous(qb, Gc, fv, wall);
          for (int v = 0; v < 5; ++v) out[v] -= fv[0][v] * Sv[0] + fv[1][v] * Sv[1] + fv[2][v] * Sv[2];
        }
        for (int v = 0; v < 5; ++v) {
          W.fS[F.e][(F.f * 5 + v) * n2 + pt] = out[v];
          W.dq[F.e][(F.f * 5 + v) * n2 + pt] = qb[v] - qi[v];
          if (bflux) bflux[v] += (side ? 1.0 : -1.0) * ops(n).w[a] * ops(n).w[b] * re(out[v]);
        }
      }
  }

  // 3. Per element: corrected gradient, volume flux, divergence and correction.
#pragma omp parallel for schedule(dynamic, 16)
  for (int e = 0; e < E; ++e) {
    const Elem& el = M.el[e];
    int n = el.n, n2 = n * n, n3 = n2 * n;
    const Ops1DT<R>& o = ops<R>(n);
    const R* eJ = el.Jp<R>();
    const R* eJa = el.Jap<R>();
    std::vector<S> Ft(n3 * 15);  // Ft[k][i][v]
    for (int k = 0; k < n3; ++k) {
      int id[3] = {k % n, (k / n) % n, k / n2};
      S q[5];
      for (int v = 0; v < 5; ++v) q[v] = Uv(v, el.off + k);
      S f[3][5];
      for (int c = 0; c < 3; ++c) ph.inviscid(q, c, f[c]);
      if (ns) {
        S G[5][3];
        for (int v = 0; v < 5; ++v) {
          S dxi[3];
          for (int i = 0; i < 3; ++i) {
            S s = 0.0;
            for (int m = 0; m < n; ++m) {
              int jd[3] = {id[0], id[1], id[2]};
              jd[i] = m;
              s += o.D[id[i] * n + m] * Uv(v, el.off + jd[0] + n * (jd[1] + n * jd[2]));
            }
            // face point of this line on the faces of direction i
            int a = id[i == 0 ? 1 : 0], b = id[i == 2 ? 1 : 2];
            s += W.dq[e][((2 * i) * 5 + v) * n2 + a + n * b] * o.gLp[id[i]];
            s += W.dq[e][((2 * i + 1) * 5 + v) * n2 + a + n * b] * o.gRp[id[i]];
            dxi[i] = s;
          }
          for (int c = 0; c < 3; ++c) {
            S s = 0.0;
            for (int i = 0; i < 3; ++i) s += eJa[k * 9 + i * 3 + c] * dxi[i];
            G[v][c] = s / eJ[k];
          }
        }
        S fv[3][5];
        ph.viscous(q, G, fv);
        for (int c = 0; c < 3; ++c)
          for (int v = 0; v < 5; ++v) f[c][v] -= fv[c][v];
      }
      for (int i = 0; i < 3; ++i)
        for (int v = 0; v < 5; ++v) {
          S s = 0.0;
          for (int c = 0; c < 3; ++c) s += eJa[k * 9 + i * 3 + c] * f[c][v];
          Ft[k * 15 + i * 5 + v] = s;
        }
    }
    // flux jumps at the element's own face points
    std::vector<S> df(6 * 5 * n2);
    for (int f = 0; f < 6; ++f) {
      int d = f / 2;
      const std::vector<R>& l = (f % 2) ? o.lp : o.lm;
      for (int v = 0; v < 5; ++v)
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            S floc = 0.0;
            for (int m = 0; m < n; ++m) floc += l[m] * Ft[line_idx(n, d, a, b, m) * 15 + d * 5 + v];
            df[(f * 5 + v) * n2 + a + n * b] = W.fS[e][(f * 5 + v) * n2 + a + n * b] - floc;
          }
    }
    for (int k = 0; k < n3; ++k) {
      int id[3] = {k % n, (k / n) % n, k / n2};
      for (int v = 0; v < 5; ++v) {
        S s = 0.0;
        double ta = 0.0;
        for (int i = 0; i < 3; ++i) {
          for (int m = 0; m < n; ++m) {
            int jd[3] = {id[0], id[1], id[2]};
            jd[i] = m;
            const S t = o.D[id[i] * n + m] * Ft[(jd[0] + n * (jd[1] + n * jd[2])) * 15 + i * 5 + v];
            s += t;
            ta += std::fabs(re(t));
          }
          int a = id[i == 0 ? 1 : 0], b = id[i == 2 ? 1 : 2];
          const S tl = df[((2 * i) * 5 + v) * n2 + a + n * b] * o.gLp[id[i]];
          const S tr = df[((2 * i + 1) * 5 + v) * n2 + a + n * b] * o.gRp[id[i]];
          s += tl;
          s += tr;
          ta += std::fabs(re(tl)) + std::fabs(re(tr));
        }
        Rout[v * N + el.off + k] = -s / eJ[k];
        if (tabs) tabs[v * N + el.off + k] = ta / std::fabs(re(S(eJ[k])));
      }
    }
  }
}

}  // namespace orc

using namespace orc;

// ======================================================================= C ABI
extern "C" {

// Build the oracle's mesh: geometry at every solution point and the face lists.
// Returns NULL on an invalid description.
void* oracle_create(int n_elem, const double* elem_xyz, const int32_t* elem_nbr, const int8_t* elem_p,
                    int physics, int flux, double gamma, double mu, double prandtl, const double* farfield) {
  Mesh* M = new Mesh;
  M->n_elem = n_elem;
  M->physics = physics;
  M->flux = flux;
  M->gamma = gamma;
  M->mu = mu;
  M->prandtl = prandtl;
  for (int v = 0; v < 5; ++v) M->farfield[v] = farfield ? farfield[v] : 0.0;
  M->xyz.assign(elem_xyz, elem_xyz + 24L * n_elem);
  M->nbr.assign(elem_nbr, elem_nbr + 6L * n_elem);
  M->el.resize(n_elem);
  long off = 0;
  for (int e = 0; e < n_elem; ++e) {
    Elem& el = M->el[e];
    if (elem_p[e] < 1 || elem_p[e] > 5) { delete M; return nullptr; }
    el.n = elem_p[e] + 1;
    el.off = off;
    el.X = &M->xyz[24L * e];
    int n = el.n, n3 = n * n * n;
    off += n3;
    el.J.resize(n3);
    el.Ja.resize(9 * n3);
    el.Jl.resize(n3);
    el.Jal.resize(9 * n3);
    const Ops1D& o = ops(n);
    const Ops1DT<long double>& ol = ops<long double>(n);
    for (int k = 0; k < n3; ++k) {
      double r[3] = {o.x[k % n], o.x[(k / n) % n], o.x[k / (n * n)]};
      double Ja[3][3], J;
      metrics<double>(el.X, r, Ja, &J);
      el.J[k] = J;
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) el.Ja[k * 9 + i * 3 + c] = Ja[i][c];
      long double rl[3] = {ol.x[k % n], ol.x[(k / n) % n], ol.x[k / (n * n)]};
      long double Jal[3][3], Jl;
      metrics<long double>(el.X, rl, Jal, &Jl);
      el.Jl[k] = Jl;
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) el.Jal[k * 9 + i * 3 + c] = Jal[i][c];
    }
  }
  M->n_sp = off;
  for (int e = 0; e < n_elem; ++e)
    for (int f = 0; f < 6; ++f) {
      int nb = M->nbr[6 * e + f];
      if (nb >= 0) {
        if (f % 2 == 1) M->ifaces.push_back({e, nb, f / 2});
      } else {
        M->bfaces.push_back({e, f, nb});
      }
    }
  return M;
}

void oracle_destroy(void* h) { delete (Mesh*)h; }
long oracle_nsp(void* h) { return ((Mesh*)h)->n_sp; }

void oracle_residual(void* h, const double* U, double* R) { residual<double>(*(Mesh*)h, U, R); }

// The residual and, at every solution point, the sum of the absolute values of
// the terms it adds up, over |J| (see residual()).
void oracle_residual_terms(void* h, const double* U, double* R, double* T) {
  residual<double>(*(Mesh*)h, U, R, nullptr, T);
}

// Floating-point operations of one residual evaluation (mode 0, counted
// reals) or of one residual-and-tangent evaluation in forward-mode dual
// arithmetic along v (mode 1), at the state U: the work model of the
// measured kernels.  R receives the residual (mode 0) or the tangent (mode
// 1).  Runs with one thread (the counter is global).
long long oracle_count_flops(void* h, const double* U, const double* v, int mode, double* R) {
  Mesh& M = *(Mesh*)h;
  const long N = 5 * M.n_sp;
#ifdef _OPENMP
  const int nt = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  g_flops = 0;
  if (mode == 0) {
    std::vector<Cnt> Uc(U, U + N), Rc(N);
    residual<Cnt>(M, Uc.data(), Rc.data());
    for (long i = 0; i < N; ++i) R[i] = Rc[i].v;
  } else {
    std::vector<DCnt> Uc(N), Rc(N);
    for (long i = 0; i < N; ++i) Uc[i] = DCnt(U[i], v[i]);
    residual<DCnt>(M, Uc.data(), Rc.data());
    for (long i = 0; i < N; ++i) R[i] = Rc[i].d;
  }
  const long long f = g_flops;
#ifdef _OPENMP
  omp_set_num_threads(nt);
#endif
  return f;
}

// Threads an OpenMP region of the oracle uses (1 without OpenMP).
int oracle_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Sets the threads of the following OpenMP regions (no effect without OpenMP).
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// The same residual evaluated in extended precision (x87 long double, 64-bit
// significand) from the same double inputs: a reference for sizing the
// rounding error of double-precision evaluations.
void oracle_residual_ld(void* h, const double* U, double* R) {
  Mesh& M = *(Mesh*)h;
  long N = 5 * M.n_sp;
  std::vector<long double> Ul(U, U + N), Rl(N);
  residual<long double>(M, Ul.data(), Rl.data());
  for (long i = 0; i < N; ++i) R[i] = (double)Rl[i];
}

// Complex-step tangent: J v = Im R(U + i h v) / h.
void oracle_jvp_cs(void* h, const double* U, const double* v, double* Jv) {
  Mesh& M = *(Mesh*)h;
  long N = 5 * M.n_sp;
  const double hs = 1e-30;
  std::vector<cplx> Uc(N), Rc(N);
  for (long i = 0; i < N; ++i) Uc[i] = cplx(U[i], hs * v[i]);
  residual<cplx>(M, Uc.data(), Rc.data());
  for (long i = 0; i < N; ++i) Jv[i] = Rc[i].imag() / hs;
}

// Finite-difference product of section 2.3: (R(U + eps v) - R(U)) / eps.
void oracle_jvp_fd(void* h, const double* U, const double* v, double eps, double* Jv) {
  Mesh& M = *(Mesh*)h;
  long N = 5 * M.n_sp;
  std::vector<double> Up(N), R0(N), R1(N);
  for (long i = 0; i < N; ++i) Up[i] = U[i] + eps * v[i];
  residual<double>(M, U, R0.data());
  residual<double>(M, Up.data(), R1.data());
  for (long i = 0; i < N; ++i) Jv[i] = (R1[i] - R0[i]) / eps;
}

// Dense Jacobian dR/dU (row-major, N x N), one complex-step column at a time.
void oracle_jacobian(void* h, const double* U, double* Jd) {
  Mesh& M = *(Mesh*)h;
  long N = 5 * M.n_sp;
  std::vector<double> e(N, 0.0), col(N);
  for (long j = 0; j < N; ++j) {
    e[j] = 1.0;
    oracle_jvp_cs(h, U, e.data(), col.data());
    e[j] = 0.0;
    for (long i = 0; i < N; ++i) Jd[i * N + j] = col[i];
  }
}

// 1-D operators for the pins: nodes, weights, D (n x n), l(-1), l(+1), g_L', g_R'.
void oracle_ops1d(int n, double* x, double* w, double* D, double* lm, double* lp, double* gLp, double* gRp) {
  const Ops1D& o = ops(n);
  for (int k = 0; k < n; ++k) {
    x[k] = o.x[k];
    w[k] = o.w[k];
    lm[k] = o.lm[k];
    lp[k] = o.lp[k];
    gLp[k] = o.gLp[k];
    gRp[k] = o.gRp[k];
    for (int j = 0; j < n; ++j) D[k * n + j] = o.D[k * n + j];
  }
}

// g_L'(x) of degree p at an arbitrary point (pins: value at -1).
double oracle_radau_gL_d(int p, double x) { return radau_gL_d(p, x); }

void oracle_interp_project(int n_lo, int n_hi, double* I /* n_hi x n_lo */, double* P /* n_lo x n_hi */) {
  std::vector<double> a = interp_matrix(n_lo, n_hi), b = project_matrix(n_hi, n_lo);
  std::copy(a.begin(), a.end(), I);
  std::copy(b.begin(), b.end(), P);
}

// Quadrature weight times J at every solution point: w_i w_j w_k J_k.
void oracle_mass(void* h, double* wJ) {
  Mesh& M = *(Mesh*)h;
  for (const Elem& el : M.el) {
    int n = el.n;
    const Ops1D& o = ops(n);
    for (int k = 0; k < n * n * n; ++k)
      wJ[el.off + k] = o.w[k % n] * o.w[(k / n) % n] * o.w[k / (n * n)] * el.J[k];
  }
}

// Net flux leaving through the boundary faces, per variable, with the common
// flux of the residual: sum over boundary face points of w_a w_b (f_com . n_out) dA.
// (Conservation pin: sum_k w J R = -this.)
void oracle_boundary_flux(void* h, const double* U, double* out5) {
  Mesh& M = *(Mesh*)h;
  std::vector<double> R(5 * M.n_sp);
  residual<double>(M, U, R.data(), out5);
}

// Spectral-decay smoothness indicator of section 3.1 for variable `var`:
// eta_e = ||s_p - s_{p-1}|| / ||s_p|| with the |J|-weighted Gauss "L2" of the
// paper (a ratio of weighted sums of squares; the normalising sums cancel),
// s_{p-1} = projection onto tensor degree p-1 = Legendre modes with every index < p.
void oracle_indicator(void* h, const double* U, int var, double* eta, double* eta_max) {
  Mesh& M = *(Mesh*)h;
  (void)ops(1);  // the operator tables are built before any thread starts
  // every element writes only its own eta (OpenMP when built with it)
#pragma omp parallel for schedule(dynamic, 16)
  for (int e = 0; e < M.n_elem; ++e) {
    const Elem& el = M.el[e];
    int n = el.n, n3 = n * n * n;
    const Ops1D& o = ops(n);
    // inverse of the 1-D Legendre Vandermonde by Gauss-Jordan elimination
    std::vector<double> A(o.V), Vi(n * n, 0.0);
    for (int i = 0; i < n; ++i) Vi[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
      for (int j = 0; j < n; ++j) {
        std::swap(A[c * n + j], A[piv * n + j]);
        std::swap(Vi[c * n + j], Vi[piv * n + j]);
      }
      double dgn = A[c * n + c];
      for (int j = 0; j < n; ++j) {
        A[c * n + j] /= dgn;
        Vi[c * n + j] /= dgn;
      }
      for (int r = 0; r < n; ++r) {
        if (r == c) continue;
        double fct = A[r * n + c];
        for (int j = 0; j < n; ++j) {
          A[r * n + j] -= fct * A[c * n + j];
          Vi[r * n + j] -= fct * Vi[c * n + j];
        }
      }
    }
    // modal coefficients c_abc = sum_ijk Vi[a,i] Vi[b,j] Vi[c,k] s_ijk
    std::vector<double> s(n3), cm(n3, 0.0);
    for (int k = 0; k < n3; ++k) s[k] = U[(long)var * M.n_sp + el.off + k];
    for (int m = 0; m < n3; ++m) {
      int ma = m % n, mb = (m / n) % n, mc = m / (n * n);
      double acc = 0.0;
      for (int k = 0; k < n3; ++k) acc += Vi[ma * n + k % n] * Vi[mb * n + (k / n) % n] * Vi[mc * n + k / (n * n)] * s[k];
      cm[m] = acc;
    }
    // s - s_{p-1}: the modes with some index equal to p, back at the points
    double num = 0.0, den = 0.0;
    for (int k = 0; k < n3; ++k) {
      int i = k % n, j = (k / n) % n, l = k / (n * n);
      double top = 0.0;
      for (int m = 0; m < n3; ++m) {
        int ma = m % n, mb = (m / n) % n, mc = m / (n * n);
        if (ma < n - 1 && mb < n - 1 && mc < n - 1) continue;
        top += cm[m] * o.V[i * n + ma] * o.V[j * n + mb] * o.V[l * n + mc];
      }
      double wJ = o.w[i] * o.w[j] * o.w[l] * std::fabs(el.J[k]);
      num += top * top * wJ;
      den += s[k] * s[k] * wJ;
    }
    eta[e] = den > 0.0 ? num / den : 0.0;
  }
  double mx = 0.0;
  for (int e = 0; e < M.n_elem; ++e) mx = std::max(mx, eta[e]);
  *eta_max = mx;
}

}  // extern "C"

// ------------------------------------------------------ implicit time stepping
namespace orc {

static double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}
static double norm2(const std::vector<double>& a) { return std::sqrt(dot(a, a)); }

// Jacobian-vector products used by the Krylov solver: exact (complex step) or
// the finite difference of section 2.3 with the residual at U cached.
struct JvCtx {
  Mesh* M;
  const double* U;
  int mode;  // 0 exact, 1 finite difference
  double eps;
  std::vector<double> R0;
};

static void jv(JvCtx& c, const double* v, double* out) {
  long N = 5 * c.M->n_sp;
  if (c.mode == 0) {
    std::vector<cplx> Uc(N), Rc(N);
    for (long i = 0; i < N; ++i) Uc[i] = cplx(c.U[i], 1e-30 * v[i]);
    residual<cplx>(*c.M, Uc.data(), Rc.data());
    for (long i = 0; i < N; ++i) out[i] = Rc[i].imag() / 1e-30;
  } else {
    if (c.R0.empty()) {
      c.R0.resize(N);
      residual<double>(*c.M, c.U, c.R0.data());
    }
    // the step eps is taken along the unit vector v/||v|| and the difference
    // quotient scaled back by ||v||, so every product sees the same relative step
    double nv = 0.0;
    for (long i = 0; i < N; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    if (nv == 0.0) {
      for (long i = 0; i < N; ++i) out[i] = 0.0;
      return;
    }
    std::vector<double> Up(N), R1(N);
    for (long i = 0; i < N; ++i) Up[i] = c.U[i] + c.eps * v[i] / nv;
    residual<double>(*c.M, Up.data(), R1.data());
    for (long i = 0; i < N; ++i) out[i] = nv * (R1[i] - c.R0[i]) / c.eps;
  }
}

// Restarted GMRES(m) (Saad & Schultz) for (shift I - dR/dU) x = F with x0 = 0:
// modified Gram-Schmidt Arnoldi, Givens rotations, stop when the residual
// estimate falls to tol ||F|| or after max_it products (section 2.3).
// Returns 0 on convergence, 1 otherwise.
static int gmres(JvCtx& c, double shift, const double* F, double* x, int m, int max_it, double tol,
                 int* iters, double* rel_res) {
  long N = 5 * c.M->n_sp;
  std::vector<double> f(F, F + N), r(f), w(N);
  for (long i = 0; i < N; ++i) x[i] = 0.0;
  double nF = norm2(f);
  *iters = 0;
  *rel_res = 0.0;
  if (nF == 0.0) return 0;
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(N));
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1);
  int total = 0;
  double res = nF;
  while (true) {
    double beta = norm2(r);
    res = beta;
    if (beta <= tol * nF) break;
    if (total >= max_it) break;
    for (long i = 0; i < N; ++i) V[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      jv(c, V[j].data(), w.data());
      for (long i = 0; i < N; ++i) w[i] = shift * V[j][i] - w[i];
      ++total;
      for (int i = 0; i <= j; ++i) {
        double h = dot(w, V[i]);
        H[i * m + j] = h;
        for (long l = 0; l < N; ++l) w[l] -= h * V[i][l];
      }
      double hn = norm2(w);
      H[(j + 1) * m + j] = hn;
      for (long l = 0; l < N; ++l) V[j + 1][l] = hn > 0 ? w[l] / hn : 0.0;
      for (int i = 0; i < j; ++i) {  // previous rotations
        double a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * b;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      double a = H[j * m + j], b = H[(j + 1) * m + j];
      double den = std::sqrt(a * a + b * b);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? b / den : 0.0;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      res = std::fabs(g[j + 1]);
      k = j + 1;
      if (res <= tol * nF || total >= max_it) break;
    }
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[i * m + l] * y[l];
      y[i] = s / H[i * m + i];
    }
    for (int i = 0; i < k; ++i)
      for (long l = 0; l < N; ++l) x[l] += y[i] * V[i][l];
    // stop on the Arnoldi residual estimate (as a matrix-free Krylov solver
    // does); otherwise restart from the true residual
    if (res <= tol * nF || total >= max_it) break;
    jv(c, x, w.data());
    for (long l = 0; l < N; ++l) r[l] = f[l] - (shift * x[l] - w[l]);
  }
  *iters = total;
  *rel_res = res / nF;
  return res <= tol * nF ? 0 : 1;
}

}  // namespace orc

extern "C" {

int oracle_gmres(void* h, const double* U, double shift, const double* F, double* x, int m, int max_it,
                 double tol, int jv_mode, double fd_eps, int* iters, double* rel_res) {
  JvCtx c{(Mesh*)h, U, jv_mode, fd_eps, {}};
  return gmres(c, shift, F, x, m, max_it, tol, iters, rel_res);
}

// Butcher tableau of the ESDIRK schemes of section 2.3 (explicit first
// stage, one diagonal coefficient, stiffly accurate: b = last row).  Scheme 0:
// the three-stage, second-order ESDIRK2 (gamma = 1 - sqrt(2)/2); scheme 1: the
// six-stage, fourth-order ESDIRK4 the paper takes from Bijl et al., the
// implicit tableau of Kennedy and Carpenter's ARK4(3)6L[2]SA (gamma = 1/4).
// Returns the number of stages, 0 for an unknown scheme.
static int esdirk_tableau(int scheme, double A[6][6], double b[6]) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = 0.0;
  int s = 0;
  if (scheme == 0) {
    const double g = 1.0 - std::sqrt(2.0) / 2.0;
    A[1][0] = g; A[1][1] = g;
    A[2][0] = (1 - g) / 2; A[2][1] = (1 - g) / 2; A[2][2] = g;
    s = 3;
  } else if (scheme == 1) {
    const double g = 0.25;
    A[1][0] = g; A[1][1] = g;
    A[2][0] = 8611.0 / 62500.0; A[2][1] = -1743.0 / 31250.0; A[2][2] = g;
    A[3][0] = 5012029.0 / 34652500.0; A[3][1] = -654441.0 / 2922500.0; A[3][2] = 174375.0 / 388108.0; A[3][3] = g;
    A[4][0] = 15267082809.0 / 155376265600.0; A[4][1] = -71443401.0 / 120774400.0;
    A[4][2] = 730878875.0 / 902184768.0; A[4][3] = 2285395.0 / 8070912.0; A[4][4] = g;
    A[5][0] = 82889.0 / 524892.0; A[5][1] = 0.0; A[5][2] = 15625.0 / 83664.0; A[5][3] = 69875.0 / 102672.0;
    A[5][4] = -2260.0 / 8211.0; A[5][5] = g;
    s = 6;
  }
  for (int j = 0; j < 6; ++j) b[j] = s ? A[s - 1][j] : 0.0;
  return s;
}

// One step of an ESDIRK scheme (eq. ESDIRK_ns): stages 2..s each solved by
// pseudo-transient continuation on eq. ESDIRK_conservative (Newton steps of
// eq. pseudo_transient linearised as in eq. linearized_pseudo_transient_final)
// with the SER update of eq. ser and restarted GMRES; a GMRES failure within
// max_gmres_it halves dtau and redoes the iterate.  If 2 <= last_stage < s the
// stage solution q^{last_stage} is returned instead of q^{n+1}.
// opts: [dtau_init, dtau_max, dtau_min, tol_pseudo, tol_gmres, restart, max_gmres_it,
//        max_ptc_it, jv_mode, fd_eps, last_stage]
// stats: [ptc_iterations, gmres_iterations, halvings, final ||F||/||F0|| of the last stage]
int oracle_esdirk_step(void* h, double* U, double dt, const double* opts, double* stats, int scheme) {
  Mesh& M = *(Mesh*)h;
  long N = 5 * M.n_sp;
  double A[6][6], b[6];
  const int ns = esdirk_tableau(scheme, A, b);
  if (!ns) return 3;
  double dtau_init = opts[0], dtau_max = opts[1], dtau_min = opts[2], tol_p = opts[3], tol_g = opts[4];
  int restart = (int)opts[5], max_git = (int)opts[6], max_ptc = (int)opts[7], mode = (int)opts[8];
  double fd_eps = opts[9];
  int last_stage = (int)opts[10];
  if (last_stage < 2 || last_stage > ns) last_stage = ns;
  for (int i = 0; i < 4; ++i) stats[i] = 0;
  std::vector<double> qn(U, U + N), q(qn), rhs(N), F(N), dq(N), Rq(N);
  std::vector<std::vector<double>> Rs(ns, std::vector<double>(N));
  residual<double>(M, qn.data(), Rs[0].data());
  const double w = A[1][1];
  int status = 0;
  for (int i = 1; i < last_stage; ++i) {
    for (long l = 0; l < N; ++l) {
      double s = qn[l];
      for (int j = 0; j < i; ++j) s += dt * A[i][j] * Rs[j][l];
      rhs[l] = s;
    }
    double dtau = dtau_init, nF0 = 0, nFprev = 0;
    for (int m = 0;; ++m) {
      residual<double>(M, q.data(), Rq.data());
      for (long l = 0; l < N; ++l) F[l] = -q[l] / (w * dt) + Rq[l] + rhs[l] / (w * dt);  // eq. ESDIRK_conservative
      double nF = std::sqrt(dot(F, F));
      if (m == 0) nF0 = nF;
      else dtau = std::min(dtau * nFprev / nF, dtau_max);  // eq. ser
      stats[3] = nF0 > 0 ? nF / nF0 : 0.0;
      if (nF <= tol_p * nF0 || nF == 0.0) break;
      if (m >= max_ptc) { status = 1; break; }
      while (true) {
        JvCtx c{&M, q.data(), mode, fd_eps, {}};
        if (mode == 1) c.R0 = Rq;
        int its;
        double rr;
        int st = gmres(c, 1.0 / (w * dt) + 1.0 / dtau, F.data(), dq.data(), restart, max_git, tol_g, &its, &rr);
        stats[1] += its;
        if (st == 0) break;
        dtau *= 0.5;  // Delta tau halving
        stats[2] += 1;
        if (dtau < dtau_min) { status = 2; break; }
      }
      if (status) break;
      for (long l = 0; l < N; ++l) q[l] += dq[l];
      nFprev = nF;
      stats[0] += 1;
    }
    if (status) break;
    residual<double>(M, q.data(), Rs[i].data());
  }
  if (last_stage < ns) {
    for (long l = 0; l < N; ++l) U[l] = q[l];
  } else {
    for (long l = 0; l < N; ++l) {
      double s = qn[l];
      for (int j = 0; j < ns; ++j) s += dt * b[j] * Rs[j][l];
      U[l] = s;
    }
  }
  return status;
}

int oracle_esdirk2_step(void* h, double* U, double dt, const double* opts, double* stats) {
  return oracle_esdirk_step(h, U, dt, opts, stats, 0);
}

}  // extern "C"

extern "C" {

// Common inviscid flux dotted with the area vector S (flux 0 Roe, 1 Rusanov),
// exported for the algebraic pins of the Riemann solvers.
void oracle_common_flux(int flux, double gamma, const double* qL, const double* qR, const double* S, double* out) {
  Phys<double> ph{gamma, 0.0, 1.0};
  if (flux == 0) ph.roe(qL, qR, S, out);
  else ph.rusanov(qL, qR, S, out);
}

// Physical flux f_c(q) (inviscid) and viscous flux from (q, grad q): for pins.
void oracle_physical_flux(double gamma, double mu, double prandtl, const double* q, const double* G /*[5][3]*/,
                          double* f /*[3][5]*/) {
  Phys<double> ph{gamma, mu, prandtl};
  double Gm[5][3], fv[3][5];
  for (int v = 0; v < 5; ++v)
    for (int c = 0; c < 3; ++c) Gm[v][c] = G[v * 3 + c];
  ph.viscous(q, Gm, fv);
  for (int c = 0; c < 3; ++c) {
    double fi[5];
    ph.inviscid(q, c, fi);
    for (int v = 0; v < 5; ++v) f[c * 5 + v] = fi[v] - fv[c][v];
  }
}

// Vectorised form of oracle_physical_flux over npts points: q [npts][5],
// G [npts][5][3], f [npts][3][5].
void oracle_physical_flux_n(long npts, double gamma, double mu, double prandtl, const double* q, const double* G,
                            double* f) {
  for (long i = 0; i < npts; ++i) oracle_physical_flux(gamma, mu, prandtl, q + 5 * i, G + 15 * i, f + 15 * i);
}

// The tableau used by oracle_esdirk_step (A row-major s x s, b, c); returns s.
int oracle_esdirk_tableau(int scheme, double* A, double* b, double* c) {
  double T[6][6], bb[6];
  const int s = esdirk_tableau(scheme, T, bb);
  for (int i = 0; i < s; ++i) {
    b[i] = bb[i];
    c[i] = 0.0;
    for (int j = 0; j < s; ++j) {
      A[i * s + j] = T[i][j];
      c[i] += T[i][j];
    }
  }
  return s;
}

// The ESDIRK2 tableau (A row-major 3x3, b, c).
void oracle_esdirk2_tableau(double* A, double* b, double* c) { oracle_esdirk_tableau(0, A, b, c); }

}  // extern "C"
