// Device-side building blocks of the FR hot path for CDNA4 (gfx950):
// scalar types (plain and dual numbers for the exact tangent), the per-degree
// 1-D operator tables, trilinear metrics and the pointwise fluxes.
//
// Paper: Wang, Gobbert & Yu, arXiv 1910.03693, section 2 (governing equations,
// FR/CPR method, Roe common flux, BR2 common gradient).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace frx {

constexpr int NMAX = 6;  // n = p + 1 <= 6 (p <= 5)
#define FRX_MAX_THREADS 256  // launch bound of every residual-stage kernel

// Waves per SIMD that each fused residual stage is built for, per scalar
// kind (double, Dual<double>, Dual<float>) and stage (trace, face,
// divergence).  A 256-thread block is one wave on each of the CU's four
// SIMDs, so the target is also the number of blocks per CU: the kernel gets
// the register budget of that many waves (amdgpu_waves_per_eu) and the fused
// plan keeps every tile's LDS within 160 KB / waves (64 KB at most).
constexpr int FRX_STAGE_WAVES[3][3] = {{4, 4, 3}, {4, 2, 3}, {4, 4, 4}};

// LDS scalars per element of the trace stage for Navier-Stokes (ns) at n
// points per direction and sb bytes per scalar: q and the uncorrected
// gradient (20 n^3) up to FRX_TRACE_LDS_ALL bytes, else q alone with the
// gradient passed through it one variable at a time (5 n^3); Euler: q (5 n^3).
// (The one-variable rounds double the elements per CU at p = 3 and 4, and
// were slower there: the 128x128x8 float64-dual trace took 0.92 ms with a
// 32 KB limit and 1.05 ms with 16 KB, against 0.84 ms.)
constexpr int FRX_TRACE_LDS_ALL = 65536;
__host__ __device__ constexpr int trace_lds_vals(bool ns, int n, int sb) {
  return (ns && 20 * n * n * n * sb > FRX_TRACE_LDS_ALL) ? 5 : (ns ? 20 : 5);
}

// ------------------------------------------------------------------ scalars
// Forward-mode dual number: value and directional derivative.  The residual
// kernels instantiated with Dual<B> compute R(U) and J(U) v in one sweep.
template <class B> struct Dual {
  B v, d;
  __host__ __device__ Dual() {}
  __host__ __device__ Dual(B a) : v(a), d(B(0)) {}
  __host__ __device__ Dual(B a, B b) : v(a), d(b) {}
};

template <class T> struct base_of { using type = T; };
template <class B> struct base_of<Dual<B>> { using type = B; };
template <class T> using base_t = typename base_of<T>::type;
template <class T> struct scalar_kind;
template <> struct scalar_kind<double> { static constexpr int value = 0; };
template <> struct scalar_kind<Dual<double>> { static constexpr int value = 1; };
template <> struct scalar_kind<Dual<float>> { static constexpr int value = 2; };
template <class T, int ST> struct StageWaves { static constexpr int value = FRX_STAGE_WAVES[scalar_kind<T>::value][ST]; };
template <class T> struct is_dual { static constexpr bool value = false; };
template <class B> struct is_dual<Dual<B>> { static constexpr bool value = true; };

template <class B> __device__ __forceinline__ Dual<B> operator+(Dual<B> a, Dual<B> b) { return {a.v + b.v, a.d + b.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator-(Dual<B> a, Dual<B> b) { return {a.v - b.v, a.d - b.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator-(Dual<B> a) { return {-a.v, -a.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator*(Dual<B> a, Dual<B> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator/(Dual<B> a, Dual<B> b) {
  B q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class B> __device__ __forceinline__ Dual<B> operator+(Dual<B> a, B b) { return {a.v + b, a.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator+(B b, Dual<B> a) { return {a.v + b, a.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator-(Dual<B> a, B b) { return {a.v - b, a.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator-(B b, Dual<B> a) { return {b - a.v, -a.d}; }
template <class B> __device__ __forceinline__ Dual<B> operator*(Dual<B> a, B b) { return {a.v * b, a.d * b}; }
template <class B> __device__ __forceinline__ Dual<B> operator*(B b, Dual<B> a) { return {a.v * b, a.d * b}; }
template <class B> __device__ __forceinline__ Dual<B> operator/(Dual<B> a, B b) { return {a.v / b, a.d / b}; }
template <class B> __device__ __forceinline__ Dual<B> operator/(B b, Dual<B> a) {
  B q = b / a.v;
  return {q, -q * a.d / a.v};
}
template <class B> __device__ __forceinline__ Dual<B>& operator+=(Dual<B>& a, Dual<B> b) { a.v += b.v; a.d += b.d; return a; }
template <class B> __device__ __forceinline__ Dual<B>& operator-=(Dual<B>& a, Dual<B> b) { a.v -= b.v; a.d -= b.d; return a; }
template <class B> __device__ __forceinline__ Dual<B>& operator+=(Dual<B>& a, B b) { a.v += b; return a; }

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <class B> __device__ __forceinline__ B val(Dual<B> x) { return x.v; }

__device__ __forceinline__ double ssqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float ssqrt(float x) { return sqrtf(x); }
template <class B> __device__ __forceinline__ Dual<B> ssqrt(Dual<B> x) {
  B s = ssqrt(x.v);
  return {s, x.d / (B(2) * s)};
}
// |x| and max() take the branch of the value: the derivative of the branch
// that is active (the convention of the complex step as well).
template <class T> __device__ __forceinline__ T sabs(T x) { return val(x) < 0 ? T(-x) : x; }
template <class T> __device__ __forceinline__ T smax(T a, T b) { return val(a) >= val(b) ? a : b; }
// c ? a : b on values (a select between two arrays' addresses would put both
// arrays in scratch)
__device__ __forceinline__ double sel(bool c, double a, double b) { return c ? a : b; }
__device__ __forceinline__ float sel(bool c, float a, float b) { return c ? a : b; }
template <class B> __device__ __forceinline__ Dual<B> sel(bool c, Dual<B> a, Dual<B> b) {
  return {c ? a.v : b.v, c ? a.d : b.d};
}

// Fused multiply-add on the base type, plain multiply-add on duals.
template <class T, class B> __device__ __forceinline__ T fmab(B a, T x, T acc) { return acc + a * x; }
__device__ __forceinline__ double fmab(double a, double x, double acc) { return fma(a, x, acc); }
__device__ __forceinline__ float fmab(float a, float x, float acc) { return fmaf(a, x, acc); }

// ---------------------------------------------------------- operator tables
// Per n (index n = p + 1, 1..6): Gauss-Legendre nodes and weights, the
// differentiation matrix D[k][j] = l_j'(x_k), extrapolation rows l_j(-1),
// l_j(+1), the derivatives of the DG correction functions at the nodes,
// the Legendre Vandermonde and its inverse, and for every pair of sizes
// nlo < nhi the face interpolation (lo -> hi) and L2 projection (hi -> lo).
template <class B> struct OpsTab {
  B x[NMAX + 1][NMAX], w[NMAX + 1][NMAX];
  B D[NMAX + 1][NMAX][NMAX];
  B lm[NMAX + 1][NMAX], lp[NMAX + 1][NMAX];
  B gL[NMAX + 1][NMAX], gR[NMAX + 1][NMAX];
  B V[NMAX + 1][NMAX][NMAX];     // V[k][m] = P_m(x_k)
  B Vinv[NMAX + 1][NMAX][NMAX];  // Vinv[m][k] = (2m+1)/2 w_k P_m(x_k)
  B I[NMAX - 1][NMAX - 1][NMAX][NMAX];  // [nlo-2][nhi-2][A][a]: l^lo_a(x^hi_A)
  B P[NMAX - 1][NMAX - 1][NMAX][NMAX];  // [nlo-2][nhi-2][a][A]: w^hi_A l^lo_a(x^hi_A) / w^lo_a
};

// one copy per translation unit (each kernel unit uploads its own)
static __constant__ OpsTab<double> c_ops_d;
static __constant__ OpsTab<float> c_ops_f;
template <class B> __device__ __forceinline__ const OpsTab<B>& ops();
template <> __device__ __forceinline__ const OpsTab<double>& ops<double>() { return c_ops_d; }
template <> __device__ __forceinline__ const OpsTab<float>& ops<float>() { return c_ops_f; }

// ------------------------------------------------------------------ physics
template <class B> struct Gas {
  B gamma, gm1, mu, kappa;  // kappa = mu cp / Pr with cp = gamma / (gamma - 1), gas constant 1
  B ff[5];                  // far-field conservative state
};

// Trilinear map stored as monomial coefficients per element:
// x(r) = a0 + a1 r0 + a2 r1 + a3 r2 + a4 r0 r1 + a5 r1 r2 + a6 r0 r2 + a7 r0 r1 r2,
// geo[e][m][c] = a_m component c.  Returns Ja^i = x_{r(i+1)} x x_{r(i+2)} and J.
template <class B>
__device__ __forceinline__ void tri_metrics(const B* __restrict__ g, B r0, B r1, B r2, B Ja[3][3], B& J) {
  B d[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    d[0][c] = g[3 + c] + g[12 + c] * r1 + g[18 + c] * r2 + g[21 + c] * (r1 * r2);
    d[1][c] = g[6 + c] + g[12 + c] * r0 + g[15 + c] * r2 + g[21 + c] * (r0 * r2);
    d[2][c] = g[9 + c] + g[15 + c] * r1 + g[18 + c] * r0 + g[21 + c] * (r0 * r1);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const B* a = d[(i + 1) % 3];
    const B* b = d[(i + 2) % 3];
    Ja[i][0] = a[1] * b[2] - a[2] * b[1];
    Ja[i][1] = a[2] * b[0] - a[0] * b[2];
    Ja[i][2] = a[0] * b[1] - a[1] * b[0];
  }
  J = d[0][0] * Ja[0][0] + d[0][1] * Ja[0][1] + d[0][2] * Ja[0][2];
}

// Area vector S = Ja^d and Jacobian J at the face point (r_d = rd, tangential
// coordinates ta, tb in increasing direction order) of the face of direction d;
// selects instead of indexing so that nothing is spilled to scratch.
template <class B>
__device__ __forceinline__ void face_geom(const B* __restrict__ g, int d, B rd, B ta, B tb, B S[3], B& J) {
  const B r0 = d == 0 ? rd : ta;
  const B r1 = d == 1 ? rd : (d == 0 ? ta : tb);
  const B r2 = d == 2 ? rd : tb;
  B Ja[3][3];
  tri_metrics<B>(g, r0, r1, r2, Ja, J);
#pragma unroll
  for (int c = 0; c < 3; ++c) S[c] = d == 0 ? Ja[0][c] : (d == 1 ? Ja[1][c] : Ja[2][c]);
}

template <class T, class B> __device__ __forceinline__ T pressure(const T q[5], const Gas<B>& G) {
  return G.gm1 * (q[4] - B(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// Viscous stress tensor (symmetric, tau[a][c]) and energy flux vector
// e[c] = u_a tau_ac + kappa dT/dx_c from q and its physical gradient Gq[v][c]
// (section 2.1: Stokes hypothesis, Fourier law, constant mu and Pr).
template <class T, class B>
__device__ __forceinline__ void viscous_terms(const T q[5], const T Gq[5][3], const Gas<B>& G, T tau[3][3], T e[3],
                                              bool adiabatic = false) {
  T ir = B(1) / q[0];
  T u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  T du[3][3];  // du[a][c] = d u_a / d x_c
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) du[a][c] = (Gq[1 + a][c] - u[a] * Gq[0][c]) * ir;
  T dil = du[0][0] + du[1][1] + du[2][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = a; c < 3; ++c) {
      T s = G.mu * (du[a][c] + du[c][a]);
      if (a == c) s = s - (B(2) / B(3)) * G.mu * dil;
      tau[a][c] = s;
      tau[c][a] = s;
    }
  if (adiabatic) {
    e[0] = e[1] = e[2] = T(B(0));
    return;
  }
  T E = q[4] * ir;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // T = (gamma-1)(E - |u|^2/2)  =>  dT = (gamma-1)(dE - u . du)
    T dE = (Gq[4][c] - E * Gq[0][c]) * ir;
    T dT = G.gm1 * (dE - (u[0] * du[0][c] + u[1] * du[1][c] + u[2] * du[2][c]));
    e[c] = u[0] * tau[0][c] + u[1] * tau[1][c] + u[2] * tau[2][c] + G.kappa * dT;
  }
}

// Contravariant total flux Ft^i = Ja^i . (f_inv - f_vis) at a solution point.
template <class T, class B, bool NS>
__device__ __forceinline__ void volume_flux(const T q[5], const T Gq[5][3], const B Ja[3][3], const Gas<B>& G,
                                            T Ft[3][5]) {
  T ir = B(1) / q[0];
  T u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  T p = G.gm1 * (q[4] - B(0.5) * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
  T h = q[4] + p;
  T tau[3][3], e[3];
  if (NS) viscous_terms<T, B>(q, Gq, G, tau, e);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T Uc = Ja[i][0] * u[0] + Ja[i][1] * u[1] + Ja[i][2] * u[2];  // contravariant velocity
    Ft[i][0] = q[0] * Uc;
#pragma unroll
    for (int a = 0; a < 3; ++a) Ft[i][1 + a] = q[1 + a] * Uc + Ja[i][a] * p;
    Ft[i][4] = h * Uc;
    if (NS) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        Ft[i][1 + a] = Ft[i][1 + a] - (Ja[i][0] * tau[a][0] + Ja[i][1] * tau[a][1] + Ja[i][2] * tau[a][2]);
      Ft[i][4] = Ft[i][4] - (Ja[i][0] * e[0] + Ja[i][1] * e[1] + Ja[i][2] * e[2]);
    }
  }
}

// Normal inviscid flux (f . S) of one state.
template <class T, class B>
__device__ __forceinline__ void normal_flux(const T q[5], const B S[3], const Gas<B>& G, T f[5], T& p, T& un) {
  T ir = B(1) / q[0];
  un = (q[1] * S[0] + q[2] * S[1] + q[3] * S[2]) * ir;
  p = G.gm1 * (q[4] - B(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * ir);
  f[0] = q[0] * un;
#pragma unroll
  for (int a = 0; a < 3; ++a) f[1 + a] = q[1 + a] * un + p * S[a];
  f[4] = (q[4] + p) * un;
}

// Common inviscid flux dotted with the area vector S (eq. invis_com).
// flux 0: Roe, with the wave decomposition written as a symmetric and an
// antisymmetric acoustic part; no entropy fix.  flux 1: Rusanov.  FLUX >= 0
// fixes the choice at compile time (the argument is then ignored): a kernel
// that holds both solvers behind a branch on the argument keeps values of
// both alive and needs far more registers.
template <class T, class B, int FLUX = -1>
__device__ __forceinline__ void riemann(const T qL[5], const T qR[5], const B S[3], const Gas<B>& G, int flux,
                                       T out[5]) {
  B area = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  B n[3] = {S[0] / area, S[1] / area, S[2] / area};
  T fL[5], fR[5], pL, pR, unL, unR;
  normal_flux<T, B>(qL, S, G, fL, pL, unL);  // un here carries the factor |S|
  normal_flux<T, B>(qR, S, G, fR, pR, unR);
  if ((FLUX < 0 ? flux : FLUX) == 1) {
    T cL = ssqrt(G.gamma * pL / qL[0]), cR = ssqrt(G.gamma * pR / qR[0]);
    T lam = smax(T(sabs(unL) + area * cL), T(sabs(unR) + area * cR));
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = B(0.5) * (fL[v] + fR[v] - lam * (qR[v] - qL[v]));
    return;
  }
  T sL = ssqrt(qL[0]), sR = ssqrt(qR[0]);
  T wL = sL / (sL + sR), wR = sR / (sL + sR);
  T iL = B(1) / qL[0], iR = B(1) / qR[0];
  T uL[3] = {qL[1] * iL, qL[2] * iL, qL[3] * iL};
  T uR[3] = {qR[1] * iR, qR[2] * iR, qR[3] * iR};
  T ut[3], du[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ut[a] = wL * uL[a] + wR * uR[a];
    du[a] = uR[a] - uL[a];
  }
  T Ht = wL * ((qL[4] + pL) * iL) + wR * ((qR[4] + pR) * iR);
  T rt = sL * sR;
  T k2 = B(0.5) * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  T c2 = G.gm1 * (Ht - k2);
  T c = ssqrt(c2);
  T un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  T dp = pR - pL;
  T a1 = (dp - rt * c * dun) / (B(2) * c2);   // wave u - c
  T a3 = (dp + rt * c * dun) / (B(2) * c2);   // wave u + c
  T a2 = (qR[0] - qL[0]) - dp / c2;           // entropy wave
  T l1 = sabs(T(un - c)), l2 = sabs(un), l3 = sabs(T(un + c));
  T As = l1 * a1 + l3 * a3;          // symmetric acoustic part
  T Aa = (l3 * a3 - l1 * a1) * c;    // antisymmetric acoustic part
  T ud = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
  T diss[5];
  diss[0] = As + l2 * a2;
#pragma unroll
  for (int a = 0; a < 3; ++a) diss[1 + a] = As * ut[a] + Aa * n[a] + l2 * (a2 * ut[a] + rt * (du[a] - dun * n[a]));
  diss[4] = As * Ht + Aa * un + l2 * (a2 * k2 + rt * (ud - un * dun));
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = B(0.5) * (fL[v] + fR[v]) - (B(0.5) * area) * diss[v];
}

// Solution jumps q_com - q of both sides of an interior face point, with the
// common solution q_com = (q^- + q^+)/2 (eq. com_q).
template <class T, class B>
__device__ __forceinline__ void face_jumps(const T qL[5], const T qR[5], T jL[5], T jR[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T qc = B(0.5) * (qL[v] + qR[v]);
    jL[v] = qc - qL[v];
    jR[v] = qc - qR[v];
  }
}

// Face function at one face point of an interior face (L on the minus side of
// S, R on the plus side): common solution (eq. com_q), BR2 common gradient
// (eq. com_grad_q) from gLR = grad q^- + grad q^+ and the liftings
// r = S (q_com - q) g'(face) / J_f, and the common normal flux
// f_com . S = Riemann(qL, qR) - f_vis(q_com, grad q_com) . S.  The jumps that
// the face slots also receive come from face_jumps.  cL = g_R'(+1)/J_L > 0,
// cR = g_L'(-1)/J_R < 0.  The viscous flux is evaluated before the Riemann
// flux and the scheduler is kept from interleaving the two: each needs about
// 200 registers per lane with float64 duals, the two interleaved over 320.
template <bool NS, class T, class B, int FLUX = -1>
__device__ __forceinline__ void face_fn(const T qL[5], const T qR[5], const T gLR[5][3], const B S[3], B cL, B cR,
                                        const Gas<B>& G, int flux, T fS[5]) {
  T qc[5], jL[5], jR[5];
  face_jumps<T, B>(qL, qR, jL, jR);
#pragma unroll
  for (int v = 0; v < 5; ++v) qc[v] = B(0.5) * (qL[v] + qR[v]);
  T fv[4];  // f_vis(q_com, grad q_com) . S, momentum and energy
  if (NS) {
    T Gc[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T lift = cL * jL[v] + cR * jR[v];
#pragma unroll
      for (int c = 0; c < 3; ++c) Gc[v][c] = B(0.5) * (gLR[v][c] + S[c] * lift);
    }
    T tau[3][3], e[3];
    viscous_terms<T, B>(qc, Gc, G, tau, e);
#pragma unroll
    for (int a = 0; a < 3; ++a) fv[a] = tau[a][0] * S[0] + tau[a][1] * S[1] + tau[a][2] * S[2];
    fv[3] = e[0] * S[0] + e[1] * S[1] + e[2] * S[2];
    __builtin_amdgcn_sched_barrier(0);
  }
  riemann<T, B, FLUX>(qL, qR, S, G, flux, fS);
  if (NS) {
#pragma unroll
    for (int a = 0; a < 3; ++a) fS[1 + a] = fS[1 + a] - fv[a];
    fS[4] = fS[4] - fv[3];
  }
}

// Boundary face point: BC -1 no-slip adiabatic wall (interior density and
// temperature, zero velocity, inviscid flux p S, no heat flux), BC -2 far
// field (Riemann problem with the free stream, common solution halfway).
// side = 1 if the element lies on the minus side of S (its +xi^d face).
// cf = g'(face)/J_f of the element.
template <bool NS, class T, class B, int FLUX = -1>
__device__ __forceinline__ void bface_fn(const T qi[5], const T gi[5][3], const B S[3], B cf, int bc, int side,
                                         const Gas<B>& G, int flux, T fS[5], T jump[5]) {
  T qb[5];
  if (bc == -1) {
    T p = pressure<T, B>(qi, G);
    qb[0] = qi[0];
    qb[1] = qb[2] = qb[3] = T(B(0));
    qb[4] = p / G.gm1;
    fS[0] = fS[4] = T(B(0));
#pragma unroll
    for (int a = 0; a < 3; ++a) fS[1 + a] = p * S[a];
  } else {
    // minus / plus states chosen value by value (a pointer select would put
    // the arrays in scratch)
    T qm[5], qp[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T qf = T(G.ff[v]);
      qb[v] = B(0.5) * (qi[v] + qf);
      qm[v] = side ? qi[v] : qf;
      qp[v] = side ? qf : qi[v];
    }
    riemann<T, B, FLUX>(qm, qp, S, G, flux, fS);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) jump[v] = qb[v] - qi[v];
  if (NS) {
    T Gc[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) Gc[v][c] = gi[v][c] + S[c] * (cf * jump[v]);
    T tau[3][3], e[3];
    viscous_terms<T, B>(qb, Gc, G, tau, e, bc == -1);
#pragma unroll
    for (int a = 0; a < 3; ++a) fS[1 + a] = fS[1 + a] - (tau[a][0] * S[0] + tau[a][1] * S[1] + tau[a][2] * S[2]);
    fS[4] = fS[4] - (e[0] * S[0] + e[1] * S[1] + e[2] * S[2]);
  }
}

}  // namespace frx

