// Reverse mode of the FR residual: J(U)^T w in float64.
//
// The forward stages (traces, faces) are recomputed inside the call to give
// the face intermediates; then the stages run backwards:
//   div_rev:   w -> adjoints of the volume flux (transposed D along each line,
//              the flux jumps and the extrapolated local flux), pointwise
//              adjoint of the flux, transposed corrected gradient -> partial
//              U-bar, adjoints of f_com . S and of the solution jumps;
//   face_rev:  pointwise adjoint of the face function (common solution, BR2
//              common gradient, Roe/Rusanov and viscous flux), with the
//              transposed projection / interpolation of mixed-degree faces;
//   trace_rev: transposed extrapolation and transposed gradient -> U-bar.
// Adjoints overwrite the forward face buffers slot by slot (every face slot
// belongs to one face and one element), so no extra face storage is needed
// and no atomics are used.  Pointwise adjoints are formed by forward sweeps
// of dual numbers over the inputs of the pointwise function.
#pragma once
#include "frx_residual.hpp"

namespace frx {

struct VjpArgs {
  const double* U;
  const double* W;   // adjoint seed [5][nsp]
  double* out;       // J^T W [5][nsp]
  int nsp, nfp, flux;
  const int* sp_off;
  const int* fp_off;
  const double* geo;
  // face-slot buffers, nv values per slot laid out by fslot()
  const double* fgeo;  // nv 5: face-point geometry (k_face_geo)
  double* QF;  // forward q traces, then their adjoints
  double* GF;  // forward gradient traces, then their adjoints
  double* DQ;  // forward solution jumps, then their adjoints
  double* FS;  // forward f_com . S, then its adjoint
  Gas<double> gas;
};

using D64 = Dual<double>;

// Adjoint of viscous_terms with respect to the gradient Gq at fixed q: the
// stress and energy flux are linear in Gq, so G-bar follows from the
// adjoints of tau[a][c] (taub, as the consumers read tau; viscous_terms
// stores one value in tau[a][c] and tau[c][a]) and of e[c] (eb) through the
// transposed chain: e -> (tau, dT), tau -> du, dT -> (dE, du), du and dE -> Gq.
__device__ __forceinline__ void visc_grad_adjoint(const double q[5], const double taub[3][3], const double eb[3],
                                                  const Gas<double>& gas, double Gb[5][3]) {
  const double ir = 1.0 / q[0];
  const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  const double E = q[4] * ir;
  double T[3][3];  // adjoint of tau[a][c] including e[c] = u_a tau[a][c] + ...
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) T[a][c] = taub[a][c] + u[a] * eb[c];
  const double tr = T[0][0] + T[1][1] + T[2][2];
  double dub[3][3];  // adjoint of du[a][c] = d u_a / d x_c
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) dub[a][c] = gas.mu * (T[a][c] + T[c][a]) - (a == c ? (2.0 / 3.0) * gas.mu * tr : 0.0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double dTb = gas.kappa * eb[c];
    const double dEb = gas.gm1 * dTb;
    double g0 = -E * dEb * ir;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double d = dub[a][c] - gas.gm1 * u[a] * dTb;
      Gb[1 + a][c] = d * ir;
      g0 -= u[a] * d * ir;
    }
    Gb[4][c] = dEb * ir;
    Gb[0][c] = g0;
  }
}

// Adjoint of viscous_terms with respect to the state q at fixed Gq: given the
// adjoints taub (of tau[a][c], as in visc_grad_adjoint) and eb (of e[c]),
// adds q-bar through u = m / rho, E / rho and 1 / rho in the velocity and
// energy gradients and in e = u . tau + kappa grad T.
__device__ __forceinline__ void visc_q_adjoint(const double q[5], const double G[5][3], const double taub[3][3],
                                               const double eb[3], const Gas<double>& gas, double qb[5]) {
  const double gm1 = gas.gm1, ir = 1.0 / q[0];
  const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  const double E = q[4] * ir;
  double du[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) du[a][c] = (G[1 + a][c] - u[a] * G[0][c]) * ir;
  const double dil = du[0][0] + du[1][1] + du[2][2];
  double T[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) T[a][c] = taub[a][c] + u[a] * eb[c];
  const double tr = T[0][0] + T[1][1] + T[2][2];
  double ub[3] = {0.0, 0.0, 0.0}, irb = 0.0, Eb = 0.0;
  // e = u_a tau[a][c] + kappa dT: u-bar from the stress
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double tau = gas.mu * (du[a][c] + du[c][a]) - (a == c ? (2.0 / 3.0) * gas.mu * dil : 0.0);
      ub[a] += tau * eb[c];
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double dTb = gas.kappa * eb[c];
    const double dEb = gm1 * dTb;
    Eb -= dEb * G[0][c] * ir;
    irb += dEb * (G[4][c] - E * G[0][c]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double dub = gas.mu * (T[a][c] + T[c][a]) - (a == c ? (2.0 / 3.0) * gas.mu * tr : 0.0) - gm1 * u[a] * dTb;
      ub[a] -= gm1 * dTb * du[a][c] + dub * G[0][c] * ir;
      irb += dub * (G[1 + a][c] - u[a] * G[0][c]);
    }
  }
  qb[4] += Eb * ir;
  irb += Eb * q[4];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qb[1 + a] += ub[a] * ir;
    irb += ub[a] * q[1 + a];
  }
  qb[0] -= irb * ir * ir;
}

// q-bar of Ft = volume_flux(q, G, Ja) at fixed G for the output adjoint Fb,
// in closed form: the inviscid contravariant flux through Uc = Ja^i . u, p and
// h = E + p, and for Navier-Stokes the state dependence of tau and e (through
// u = m / rho, E / rho and 1 / rho in the velocity and energy gradients).
template <bool NS>
__device__ __forceinline__ void volume_flux_q_adjoint(const double q[5], const double G[5][3], const double Ja[3][3],
                                                      const Gas<double>& gas, const double Fb[3][5], double qb[5]) {
  const double gm1 = gas.gm1, ir = 1.0 / q[0];
  const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  const double p = gm1 * (q[4] - 0.5 * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
  const double h = q[4] + p;
  double ub[3] = {0.0, 0.0, 0.0}, irb = 0.0, pb = 0.0, hb = 0.0;  // inviscid part
#pragma unroll
  for (int v = 0; v < 5; ++v) qb[v] = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double Uc = Ja[i][0] * u[0] + Ja[i][1] * u[1] + Ja[i][2] * u[2];
    const double Ucb = Fb[i][0] * q[0] + Fb[i][1] * q[1] + Fb[i][2] * q[2] + Fb[i][3] * q[3] + Fb[i][4] * h;
    qb[0] += Fb[i][0] * Uc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qb[1 + a] += Fb[i][1 + a] * Uc;
      pb += Fb[i][1 + a] * Ja[i][a];
      ub[a] += Ucb * Ja[i][a];
    }
    hb += Fb[i][4] * Uc;
  }
  qb[4] += hb;
  pb += hb;
  qb[4] += gm1 * pb;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qb[1 + a] -= gm1 * pb * 0.5 * u[a];
    ub[a] -= gm1 * pb * 0.5 * q[1 + a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qb[1 + a] += ub[a] * ir;
    irb += ub[a] * q[1 + a];
  }
  qb[0] -= irb * ir * ir;
  if (NS) {
    double taub[3][3], eb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      eb[c] = -(Fb[0][4] * Ja[0][c] + Fb[1][4] * Ja[1][c] + Fb[2][4] * Ja[2][c]);
#pragma unroll
      for (int a = 0; a < 3; ++a) taub[a][c] = -(Fb[0][1 + a] * Ja[0][c] + Fb[1][1 + a] * Ja[1][c] + Fb[2][1 + a] * Ja[2][c]);
    }
    visc_q_adjoint(q, G, taub, eb, gas, qb);
  }
}

// q-bar, G-bar of Ft = volume_flux(q, G, Ja) for the output adjoint Fb
template <bool NS>
__device__ void volume_flux_vjp(const double q[5], const double G[5][3], const double Ja[3][3], const Gas<double>& gas,
                                const double Fb[3][5], double qb[5], double Gb[5][3]) {
  volume_flux_q_adjoint<NS>(q, G, Ja, gas, Fb, qb);
  if (NS) {
    // G-bar: Ft^i -= Ja^i . tau and Ja^i . e, linear in G
    double taub[3][3], eb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      eb[c] = -(Fb[0][4] * Ja[0][c] + Fb[1][4] * Ja[1][c] + Fb[2][4] * Ja[2][c]);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        taub[a][c] = -(Fb[0][1 + a] * Ja[0][c] + Fb[1][1 + a] * Ja[1][c] + Fb[2][1 + a] * Ja[2][c]);
    }
    visc_grad_adjoint(q, taub, eb, gas, Gb);
  } else {
    for (int v = 0; v < 5; ++v)
      for (int c = 0; c < 3; ++c) Gb[v][c] = 0.0;
  }
}

// Adjoint of the normal inviscid flux (f . S, normal_flux) of one state: the
// output adjoint fb to the state adjoint qb (accumulated).
__device__ __forceinline__ void normal_flux_vjp(const double q[5], const double S[3], const Gas<double>& gas,
                                                const double fb[5], double qb[5]) {
  const double i0 = 1.0 / q[0];
  const double m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const double mS = q[1] * S[0] + q[2] * S[1] + q[3] * S[2];
  const double un = mS * i0;
  const double p = gas.gm1 * (q[4] - 0.5 * m2 * i0);
  const double unb = fb[0] * q[0] + fb[1] * q[1] + fb[2] * q[2] + fb[3] * q[3] + fb[4] * (q[4] + p);
  const double pb = fb[1] * S[0] + fb[2] * S[1] + fb[3] * S[2] + fb[4] * un;
  double i0b = unb * mS - gas.gm1 * pb * 0.5 * m2;
  qb[0] += fb[0] * un;
#pragma unroll
  for (int a = 0; a < 3; ++a) qb[1 + a] += fb[1 + a] * un + unb * i0 * S[a] - gas.gm1 * pb * q[1 + a] * i0;
  qb[4] += fb[4] * un + gas.gm1 * pb;
  qb[0] -= i0b * i0 * i0;
}

// Adjoint of the Roe flux of riemann (flux 0) in closed form: given the
// adjoint ob of f_com . S, the adjoints of both states.  The forward
// quantities are recomputed, then the chain is walked back: dissipation ->
// (wave strengths, |lambda|, Roe averages) -> (pressures, velocities, rho^1/2)
// -> states; the normal fluxes' adjoints are added by normal_flux_vjp.  |x|
// takes the derivative sign as sabs does (+1 at 0).
__device__ __forceinline__ void roe_vjp(const double qL[5], const double qR[5], const double S[3],
                                        const Gas<double>& gas, const double ob[5], double qLb[5], double qRb[5]) {
  const double gm1 = gas.gm1;
  const double area = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  const double n[3] = {S[0] / area, S[1] / area, S[2] / area};
  const double iL = 1.0 / qL[0], iR = 1.0 / qR[0];
  const double pL = gm1 * (qL[4] - 0.5 * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]) * iL);
  const double pR = gm1 * (qR[4] - 0.5 * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]) * iR);
  const double sL = sqrt(qL[0]), sR = sqrt(qR[0]), D = sL + sR;
  const double wL = sL / D, wR = sR / D;
  double uL[3], uR[3], ut[3], du[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uL[a] = qL[1 + a] * iL;
    uR[a] = qR[1 + a] * iR;
    ut[a] = wL * uL[a] + wR * uR[a];
    du[a] = uR[a] - uL[a];
  }
  const double hL = (qL[4] + pL) * iL, hR = (qR[4] + pR) * iR;
  const double Ht = wL * hL + wR * hR, rt = sL * sR;
  const double k2 = 0.5 * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  const double c2 = gm1 * (Ht - k2), c = sqrt(c2);
  const double un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  const double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const double dp = pR - pL;
  const double a1 = (dp - rt * c * dun) / (2.0 * c2), a3 = (dp + rt * c * dun) / (2.0 * c2);
  const double a2 = (qR[0] - qL[0]) - dp / c2;
  const double s1 = (un - c) < 0.0 ? -1.0 : 1.0, s2 = un < 0.0 ? -1.0 : 1.0, s3 = (un + c) < 0.0 ? -1.0 : 1.0;
  const double l1 = s1 * (un - c), l2 = s2 * un, l3 = s3 * (un + c);
  const double As = l1 * a1 + l3 * a3, Aa = (l3 * a3 - l1 * a1) * c;
  const double ud = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
  // out = (fL + fR)/2 - area/2 diss
  double db[5], fb[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    fb[v] = 0.5 * ob[v];
    db[v] = -0.5 * area * ob[v];
  }
  const double dbu = db[1] * ut[0] + db[2] * ut[1] + db[3] * ut[2];
  const double dbn = db[1] * n[0] + db[2] * n[1] + db[3] * n[2];
  const double Asb = db[0] + dbu + db[4] * Ht;
  const double Aab = dbn + db[4] * un;
  double l2b = db[0] * a2 + db[4] * (a2 * k2 + rt * (ud - un * dun));
  double rtb = db[4] * l2 * (ud - un * dun);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    l2b += db[1 + a] * (a2 * ut[a] + rt * (du[a] - dun * n[a]));
    rtb += db[1 + a] * l2 * (du[a] - dun * n[a]);
  }
  const double a2b = l2 * (db[0] + dbu + db[4] * k2);
  double dunb = -l2 * rt * (dbn + db[4] * un);
  double Htb = db[4] * As;
  double unb = db[4] * (Aa - l2 * rt * dun);
  double k2b = db[4] * l2 * a2;
  const double udb = db[4] * l2 * rt;
  double utb[3], dub[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    utb[a] = db[1 + a] * (As + l2 * a2) + udb * du[a];
    dub[a] = db[1 + a] * l2 * rt + udb * ut[a];
  }
  const double l1b = Asb * a1 - Aab * a1 * c, l3b = Asb * a3 + Aab * a3 * c;
  const double a1b = Asb * l1 - Aab * l1 * c, a3b = Asb * l3 + Aab * l3 * c;
  double cb = Aab * (l3 * a3 - l1 * a1);
  unb += l1b * s1 + l2b * s2 + l3b * s3;
  cb += -l1b * s1 + l3b * s3;
  // wave strengths
  double q0b_R = a2b, q0b_L = -a2b;
  double dpb = -a2b / c2;
  double c2b = a2b * dp / (c2 * c2);
  const double t1 = a1b / (2.0 * c2), t3 = a3b / (2.0 * c2);
  dpb += t1 + t3;
  rtb += (t3 - t1) * c * dun;
  cb += (t3 - t1) * rt * dun;
  dunb += (t3 - t1) * rt * c;
  c2b -= (a1b * a1 + a3b * a3) / c2;
  double pRb = dpb, pLb = -dpb;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dub[a] += dunb * n[a];
    utb[a] += unb * n[a];
  }
  c2b += cb / (2.0 * c);
  Htb += gm1 * c2b;
  k2b -= gm1 * c2b;
#pragma unroll
  for (int a = 0; a < 3; ++a) utb[a] += k2b * ut[a];
  double sLb = rtb * sR, sRb = rtb * sL;
  double wLb = Htb * hL, wRb = Htb * hR;
  const double hLb = Htb * wL, hRb = Htb * wR;
  double qLb4 = hLb * iL, qRb4 = hRb * iR;
  pLb += hLb * iL;
  pRb += hRb * iR;
  double iLb = hLb * (qL[4] + pL), iRb = hRb * (qR[4] + pR);
  double qLbm[3], qRbm[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double uLb = -dub[a] + utb[a] * wL, uRb = dub[a] + utb[a] * wR;
    wLb += utb[a] * uL[a];
    wRb += utb[a] * uR[a];
    qLbm[a] = uLb * iL;
    qRbm[a] = uRb * iR;
    iLb += uLb * qL[1 + a];
    iRb += uRb * qR[1 + a];
  }
  q0b_L -= iLb * iL * iL;
  q0b_R -= iRb * iR * iR;
  sLb += (wLb - wRb) * sR / (D * D);
  sRb += (wRb - wLb) * sL / (D * D);
  q0b_L += sLb / (2.0 * sL);
  q0b_R += sRb / (2.0 * sR);
  // pressures p = gm1 (q4 - |m|^2 / (2 q0))
  const double m2L = qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3];
  const double m2R = qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3];
  qLb4 += gm1 * pLb;
  qRb4 += gm1 * pRb;
  q0b_L += gm1 * pLb * 0.5 * m2L * iL * iL;
  q0b_R += gm1 * pRb * 0.5 * m2R * iR * iR;
  qLb[0] = q0b_L;
  qRb[0] = q0b_R;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qLb[1 + a] = qLbm[a] - gm1 * pLb * qL[1 + a] * iL;
    qRb[1 + a] = qRbm[a] - gm1 * pRb * qR[1 + a] * iR;
  }
  qLb[4] = qLb4;
  qRb[4] = qRb4;
  normal_flux_vjp(qL, S, gas, fb, qLb);
  normal_flux_vjp(qR, S, gas, fb, qRb);
}

// Adjoint of face_fn at one point: given fSb, jLb, jRb return qLb, qRb, gLb, gRb.
// FLUX >= 0 fixes the Riemann solver at compile time (as in riemann).
template <bool NS, int FLUX = -1>
__device__ void face_fn_vjp(const double qL[5], const double qR[5], const double gL[5][3], const double gR[5][3],
                            const double S[3], double cL, double cR, const Gas<double>& gas, int flux,
                            const double fSb[5], const double jLb[5], const double jRb[5], double qLb[5],
                            double qRb[5], double gLb[5][3], double gRb[5][3]) {
  // Riemann part: the Roe flux's adjoint in closed form; Rusanov by 10
  // forward sweeps
  if ((FLUX < 0 ? flux : FLUX) == 0) {
    roe_vjp(qL, qR, S, gas, fSb, qLb, qRb);
  } else {
#pragma unroll 1
    for (int j = 0; j < 10; ++j) {
      D64 a[5], b[5], o[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        a[v] = D64(qL[v], j == v ? 1.0 : 0.0);
        b[v] = D64(qR[v], j == 5 + v ? 1.0 : 0.0);
      }
      riemann<D64, double, (FLUX < 0 ? 1 : FLUX)>(a, b, S, gas, flux, o);
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < 5; ++v) s += o[v].d * fSb[v];
      if (j < 5) qLb[j] = s;
      else qRb[j - 5] = s;
    }
  }
  double jl[5], jr[5], qcb[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    jl[v] = jLb[v];
    jr[v] = jRb[v];
    qcb[v] = 0.0;
  }
  if (NS) {
    // forward intermediates
    double qc[5], Gc[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      qc[v] = 0.5 * (qL[v] + qR[v]);
      const double lift = cL * (qc[v] - qL[v]) + cR * (qc[v] - qR[v]);
#pragma unroll
      for (int c = 0; c < 3; ++c) Gc[v][c] = 0.5 * (gL[v][c] + gR[v][c] + S[c] * lift);
    }
    // the viscous flux (tau . S, e . S) of fS = Riemann - visc: adjoints of
    // tau and e, then q_com-bar at fixed G_com and G_com-bar (linear in it)
    double taub[3][3], eb[3], Gcb[5][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      eb[c] = -fSb[4] * S[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) taub[a][c] = -fSb[1 + a] * S[c];
    }
    visc_q_adjoint(qc, Gc, taub, eb, gas, qcb);
    visc_grad_adjoint(qc, taub, eb, gas, Gcb);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double sg = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gLb[v][c] = 0.5 * Gcb[v][c];
        gRb[v][c] = 0.5 * Gcb[v][c];
        sg += S[c] * Gcb[v][c];
      }
      jl[v] += 0.5 * cL * sg;
      jr[v] += 0.5 * cR * sg;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) gLb[v][c] = gRb[v][c] = 0.0;
  }
  // jL = qc - qL, jR = qc - qR, qc = (qL + qR) / 2
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    qcb[v] += jl[v] + jr[v];
    qLb[v] += -jl[v] + 0.5 * qcb[v];
    qRb[v] += -jr[v] + 0.5 * qcb[v];
  }
}

// ---------------------------------------------------------------- div_rev
template <int N, bool NS>
__device__ __forceinline__ void div_rev_body(const VjpArgs& a, const int* __restrict__ elems, int nel, int epb,
                                             int blk, unsigned char* smem) {
  constexpr int N2 = N * N, N3 = N2 * N;
  double* sX = reinterpret_cast<double*>(smem);  // [epb][5][N3]
  double* sY = sX + epb * 5 * N3;                // [epb][6][5][N2]
  const OpsTab<double>& O = ops<double>();
  const int tid = threadIdx.x;
  const int le = tid / N3, k = tid - le * N3;
  const int slot = blk * epb + le;
  const bool act = le < epb && slot < nel;
  const int e = act ? elems[slot] : 0;
  const long off = act ? (long)a.sp_off[e] + k : 0;
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = a.U[(long)v * a.nsp + off];
  }
  if (NS) {
    for (int it = tid; it < epb * 30 * N2; it += blockDim.x) {
      const int l2 = it / (30 * N2), rem = it - l2 * 30 * N2;
      const int s2 = blk * epb + l2;
      if (s2 >= nel) continue;
      sY[it] = a.DQ[5L * a.fp_off[elems[s2]] + rem];  // the element's [6][5][n^2] block
    }
  }
  __syncthreads();
  const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
  const int id[3] = {i0, i1, i2};
  double Ja[3][3], J = 1.0, q[5], G[5][3], Ab[5];
  if (act) {
    tri_metrics<double>(a.geo + 24L * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
    const double* qs = sX + le * 5 * N3;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      q[v] = qs[v * N3 + k];
      Ab[v] = -a.W[(long)v * a.nsp + off] / J;
    }
    if (NS) {
      const double* jm = sY + le * 30 * N2;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
          d0 = fma(O.D[N][i0][m], qs[v * N3 + m + N * (i1 + N * i2)], d0);
          d1 = fma(O.D[N][i1][m], qs[v * N3 + i0 + N * (m + N * i2)], d1);
          d2 = fma(O.D[N][i2][m], qs[v * N3 + i0 + N * (i1 + N * m)], d2);
        }
        d0 = fma(O.gL[N][i0], jm[(0 * 5 + v) * N2 + i1 + N * i2], d0);
        d0 = fma(O.gR[N][i0], jm[(1 * 5 + v) * N2 + i1 + N * i2], d0);
        d1 = fma(O.gL[N][i1], jm[(2 * 5 + v) * N2 + i0 + N * i2], d1);
        d1 = fma(O.gR[N][i1], jm[(3 * 5 + v) * N2 + i0 + N * i2], d1);
        d2 = fma(O.gL[N][i2], jm[(4 * 5 + v) * N2 + i0 + N * i1], d2);
        d2 = fma(O.gR[N][i2], jm[(5 * 5 + v) * N2 + i0 + N * i1], d2);
#pragma unroll
        for (int c = 0; c < 3; ++c) G[v][c] = (Ja[0][c] * d0 + Ja[1][c] * d1 + Ja[2][c] * d2) / J;
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = Ab[v];
  }
  __syncthreads();
  // adjoint of the flux jumps: sum of Ab g_face along each normal line; it is
  // also the adjoint of f_com . S
  for (int it = tid; it < epb * 30 * N2; it += blockDim.x) {
    const int l2 = it / (30 * N2), rem = it - l2 * 30 * N2;
    const int fv = rem / N2, p2 = rem - fv * N2;
    const int s2 = blk * epb + l2;
    if (s2 >= nel) continue;
    const int f = fv / 5, v = fv - f * 5, d = f >> 1;
    const double* gf = (f & 1) ? O.gR[N] : O.gL[N];
    const double* X = sX + (l2 * 5 + v) * N3;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) s = fma(gf[m], X[line_pt<N>(d, p2 % N, p2 / N, m)], s);
    sY[it] = s;
    a.FS[5L * a.fp_off[elems[s2]] + rem] = s;
  }
  __syncthreads();
  double Ub[5];
  double dqb[3][5];
  if (act) {
    const double* X = sX + le * 5 * N3;
    const double* Z = sY + le * 30 * N2;
    double Fb[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int fp = i == 0 ? i1 + N * i2 : (i == 1 ? i0 + N * i2 : i0 + N * i1);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
          const int kk = i == 0 ? m + N * (i1 + N * i2) : (i == 1 ? i0 + N * (m + N * i2) : i0 + N * (i1 + N * m));
          s = fma(O.D[N][m][id[i]], X[v * N3 + kk], s);  // transposed D
        }
        s -= O.lm[N][id[i]] * Z[((2 * i) * 5 + v) * N2 + fp];
        s -= O.lp[N][id[i]] * Z[((2 * i + 1) * 5 + v) * N2 + fp];
        Fb[i][v] = s;
      }
    }
    double qb[5], Gb[5][3];
    volume_flux_vjp<NS>(q, G, Ja, a.gas, Fb, qb, Gb);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Ub[v] = qb[v];
#pragma unroll
      for (int i = 0; i < 3; ++i) dqb[i][v] = NS ? (Ja[i][0] * Gb[v][0] + Ja[i][1] * Gb[v][1] + Ja[i][2] * Gb[v][2]) / J : 0.0;
    }
  }
  if (NS) {
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      __syncthreads();
      if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = i == 0 ? dqb[0][v] : (i == 1 ? dqb[1][v] : dqb[2][v]);
      }
      __syncthreads();
      if (act) {
        const double* X = sX + le * 5 * N3;
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const int kk = i == 0 ? m + N * (i1 + N * i2) : (i == 1 ? i0 + N * (m + N * i2) : i0 + N * (i1 + N * m));
            Ub[v] = fma(O.D[N][m][i == 0 ? i0 : (i == 1 ? i1 : i2)], X[v * N3 + kk], Ub[v]);
          }
      }
      // adjoint of the solution jumps of the two faces of direction i
      for (int it = tid; it < epb * 10 * N2; it += blockDim.x) {
        const int l2 = it / (10 * N2), rem = it - l2 * 10 * N2;
        const int sv = rem / N2, p2 = rem - sv * N2;
        const int s2 = blk * epb + l2;
        if (s2 >= nel) continue;
        const int side = sv / 5, v = sv - side * 5;
        const double* gf = side ? O.gR[N] : O.gL[N];
        const double* X = sX + (l2 * 5 + v) * N3;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) s = fma(gf[m], X[line_pt<N>(i, p2 % N, p2 / N, m)], s);
        a.DQ[5L * a.fp_off[elems[s2]] + 10 * i * N2 + rem] = s;
      }
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) a.out[(long)v * a.nsp + off] = Ub[v];
  }
}
template <int N, bool NS>
__global__ void __launch_bounds__(256) k_div_rev(VjpArgs a, const int* __restrict__ elems, int nel, int epb) {
  extern __shared__ __align__(16) unsigned char smem[];
  div_rev_body<N, NS>(a, elems, nel, epb, blockIdx.x, smem);
}

// --------------------------------------------------------------- face_rev
// Like the forward face stage, in three phases: face_rev_gather (forward
// inputs and output adjoints of the face point, interpolated from the low
// side of a mixed face), face_fn_vjp (once per point; the fused kernel holds
// a single copy after its switch over the tile kinds), face_rev_scatter (the
// adjoints to the face slots, transposed interpolation to the low side).
struct FaceRevPt {
  double q[2][5], g[2][5][3];  // forward q and gradient traces of both sides
  double fSb[5], jb[2][5];     // adjoints of f_com . S and of both jumps
  double S[3], cL, cR;
  int oL, oR, lf, pt;
  bool act, lowL, lowR;
};

template <int NL, int NH, bool NS>
__device__ __forceinline__ void face_rev_gather(const VjpArgs& a, const int4* __restrict__ faces, int nf, int fpb,
                                                int blk, unsigned char* smem, FaceRevPt& P) {
  constexpr int NH2 = NH * NH, NL2 = NL * NL;
  constexpr bool MIX = NL < NH;
  constexpr int NV = NS ? 20 : 5;
  double* slow = reinterpret_cast<double*>(smem);           // [fpb][NV][NL2] forward low-side traces
  double* sadj = slow + (MIX ? fpb * NV * NL2 : 0);          // [fpb][10][NL2] low-side fS-bar, jump-bar
  const OpsTab<double>& O = ops<double>();
  const int tid = threadIdx.x;
  P.lf = tid / NH2;
  P.pt = tid - P.lf * NH2;
  const int fi = blk * fpb + P.lf;
  P.act = P.lf < fpb && fi < nf;
  const FaceRec F = face_rec(P.act ? faces[fi] : make_int4(0, 0, 0, 0));
  P.oL = F.oL;
  P.oR = F.oR;
  P.lowR = MIX && F.low_is_R;
  P.lowL = MIX && !F.low_is_R;
  if (MIX) {
    for (int it = tid; it < fpb * (NV + 10) * NL2; it += blockDim.x) {
      const int l2 = it / ((NV + 10) * NL2), rem = it - l2 * (NV + 10) * NL2;
      const int vv = rem / NL2, p2 = rem - vv * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      double val;
      if (vv < 5) val = a.QF[fslot(5, fs, NL2, vv, p2)];
      else if (vv < NV) val = a.GF[fslot(15, fs, NL2, vv - 5, p2)];
      else if (vv < NV + 5) val = a.FS[fslot(5, fs, NL2, vv - NV, p2)];
      else val = a.DQ[fslot(5, fs, NL2, vv - NV - 5, p2)];
      if (vv < NV) slow[(l2 * NV + vv) * NL2 + p2] = val;
      else sadj[(l2 * 10 + vv - NV) * NL2 + p2] = val;
    }
    __syncthreads();
  }
  if (!P.act) return;
  const int pt = P.pt, A = pt % NH, Bq = pt / NH;
#pragma unroll
  for (int v = 0; v < 5; ++v) P.fSb[v] = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool low = s ? P.lowR : P.lowL;
    if (low) {
      const double* src = slow + P.lf * NV * NL2;
#pragma unroll
      for (int vv = 0; vv < NV; ++vv) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NL; ++b) {
          double row = 0.0;
#pragma unroll
          for (int aa = 0; aa < NL; ++aa) row = fma(O.I[NL - 2][NH - 2][A][aa], src[vv * NL2 + aa + NL * b], row);
          acc = fma(O.I[NL - 2][NH - 2][Bq][b], row, acc);
        }
        if (vv < 5) P.q[s][vv] = acc;
        else P.g[s][(vv - 5) / 3][(vv - 5) % 3] = acc;
      }
      // transposed projection of the low side's adjoints
      const double* adj = sadj + P.lf * 10 * NL2;
#pragma unroll
      for (int w = 0; w < 10; ++w) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NL; ++b)
#pragma unroll
          for (int aa = 0; aa < NL; ++aa)
            acc += O.P[NL - 2][NH - 2][aa][A] * O.P[NL - 2][NH - 2][b][Bq] * adj[w * NL2 + aa + NL * b];
        if (w < 5) P.fSb[w] += acc;
        else P.jb[s][w - 5] = NS ? acc : 0.0;
      }
    } else {
      const long fs = s ? F.oR : F.oL;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        P.q[s][v] = a.QF[fslot(5, fs, NH2, v, pt)];
        P.fSb[v] += a.FS[fslot(5, fs, NH2, v, pt)];
        P.jb[s][v] = NS ? a.DQ[fslot(5, fs, NH2, v, pt)] : 0.0;  // Euler: jumps do not enter R
      }
      if (NS) {
#pragma unroll
        for (int vc = 0; vc < 15; ++vc) P.g[s][vc / 3][vc % 3] = a.GF[fslot(15, fs, NH2, vc, pt)];
      } else {
#pragma unroll
        for (int vc = 0; vc < 15; ++vc) P.g[s][vc / 3][vc % 3] = 0.0;
      }
    }
  }
  // geometry of the face point, kept at the high side's slot
  const long og = P.lowL ? F.oR : F.oL;
  P.S[0] = a.fgeo[fslot(5, og, NH2, 0, pt)];
  P.S[1] = a.fgeo[fslot(5, og, NH2, 1, pt)];
  P.S[2] = a.fgeo[fslot(5, og, NH2, 2, pt)];
  P.cL = NS ? a.fgeo[fslot(5, og, NH2, 3, pt)] : 0.0;
  P.cR = NS ? a.fgeo[fslot(5, og, NH2, 4, pt)] : 0.0;
}

template <int NL, int NH, bool NS>
__device__ __forceinline__ void face_rev_scatter(const VjpArgs& a, const int4* __restrict__ faces, int nf, int fpb,
                                                 int blk, unsigned char* smem, const FaceRevPt& P,
                                                 const double qb[2][5], const double gb[2][5][3]) {
  constexpr int NH2 = NH * NH, NL2 = NL * NL;
  constexpr bool MIX = NL < NH;
  constexpr int NV = NS ? 20 : 5;
  double* sres = reinterpret_cast<double*>(smem) + (MIX ? fpb * (NV + 10) * NL2 : 0);  // [fpb][NV][NH2]
  const OpsTab<double>& O = ops<double>();
  const int tid = threadIdx.x, pt = P.pt;
  if (P.act) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const bool low = s ? P.lowR : P.lowL;
      if (!low) {
        const long fs = s ? P.oR : P.oL;
#pragma unroll
        for (int v = 0; v < 5; ++v) a.QF[fslot(5, fs, NH2, v, pt)] = qb[s][v];
        if (NS)
#pragma unroll
          for (int vc = 0; vc < 15; ++vc) a.GF[fslot(15, fs, NH2, vc, pt)] = gb[s][vc / 3][vc % 3];
      } else {
        double* dst = sres + P.lf * NV * NH2;
#pragma unroll
        for (int v = 0; v < 5; ++v) dst[v * NH2 + pt] = qb[s][v];
        if (NS)
#pragma unroll
          for (int vc = 0; vc < 15; ++vc) dst[(5 + vc) * NH2 + pt] = gb[s][vc / 3][vc % 3];
      }
    }
  }
  if (MIX) {
    __syncthreads();
    // transposed interpolation back to the low side's own points
    for (int it = tid; it < fpb * NL2; it += blockDim.x) {
      const int l2 = it / NL2, p2 = it - l2 * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      const int aa = p2 % NL, bb = p2 / NL;
      const double* src = sres + l2 * NV * NH2;
      for (int vv = 0; vv < NV; ++vv) {
        double acc = 0.0;
        for (int Bq = 0; Bq < NH; ++Bq)
          for (int A = 0; A < NH; ++A)
            acc += O.I[NL - 2][NH - 2][A][aa] * O.I[NL - 2][NH - 2][Bq][bb] * src[vv * NH2 + A + NH * Bq];
        if (vv < 5) a.QF[fslot(5, fs, NL2, vv, p2)] = acc;
        else a.GF[fslot(15, fs, NL2, vv - 5, p2)] = acc;
      }
    }
  }
}

template <int NL, int NH, bool NS>
__device__ __forceinline__ void face_rev_body(const VjpArgs& a, const int4* __restrict__ faces, int nf, int fpb,
                                              int blk, unsigned char* smem) {
  FaceRevPt P;
  face_rev_gather<NL, NH, NS>(a, faces, nf, fpb, blk, smem, P);
  double qb[2][5], gb[2][5][3];
  if (P.act)
    face_fn_vjp<NS>(P.q[0], P.q[1], P.g[0], P.g[1], P.S, P.cL, P.cR, a.gas, a.flux, P.fSb, P.jb[0], P.jb[1], qb[0],
                    qb[1], gb[0], gb[1]);
  face_rev_scatter<NL, NH, NS>(a, faces, nf, fpb, blk, smem, P, qb, gb);
}
template <int NL, int NH, bool NS>
__global__ void __launch_bounds__(256) k_face_rev(VjpArgs a, const int4* __restrict__ faces, int nf, int fpb) {
  extern __shared__ __align__(16) unsigned char smem[];
  face_rev_body<NL, NH, NS>(a, faces, nf, fpb, blockIdx.x, smem);
}

// -------------------------------------------------------------- bface_rev
template <int N, bool NS>
__device__ __forceinline__ void bface_rev_body(const VjpArgs& a, const int4* __restrict__ faces, int nf, int blk) {
  constexpr int N2 = N * N;
  const int gid = blk * blockDim.x + threadIdx.x;
  if (gid >= nf * N2) return;
  const int fi = gid / N2, pt = gid - fi * N2;
  const int4 F = faces[fi];
  const int e = F.x, f = F.y, bc = F.z, d = f >> 1, side = f & 1;
  const OpsTab<double>& O = ops<double>();
  const long fs = F.w;
  double q[5], g[5][3], fSb[5], jb[5];
  for (int v = 0; v < 5; ++v) {
    q[v] = a.QF[fslot(5, fs, N2, v, pt)];
    fSb[v] = a.FS[fslot(5, fs, N2, v, pt)];
    jb[v] = NS ? a.DQ[fslot(5, fs, N2, v, pt)] : 0.0;
  }
  for (int vc = 0; vc < 15; ++vc) g[vc / 3][vc % 3] = NS ? a.GF[fslot(15, fs, N2, vc, pt)] : 0.0;
  double S[3], J;
  face_geom<double>(a.geo + 24L * e, d, side ? 1.0 : -1.0, O.x[N][pt % N], O.x[N][pt / N], S, J);
  const double cf = (side ? 0.5 : -0.5) * (double)(N * N) / J;
  constexpr int NI = NS ? 20 : 5;
  double qb[5], gb[5][3];
  for (int v = 0; v < 5; ++v)
    for (int c = 0; c < 3; ++c) gb[v][c] = 0.0;
  for (int j = 0; j < NI; ++j) {
    D64 qd[5], gd[5][3], fS[5], jm[5];
    for (int v = 0; v < 5; ++v) qd[v] = D64(q[v], j == v ? 1.0 : 0.0);
    for (int v = 0; v < 5; ++v)
      for (int c = 0; c < 3; ++c) gd[v][c] = D64(g[v][c], j == 5 + v * 3 + c ? 1.0 : 0.0);
    bface_fn<NS, D64, double>(qd, gd, S, cf, bc, side, a.gas, a.flux, fS, jm);
    double s = 0.0;
    for (int v = 0; v < 5; ++v) s += fS[v].d * fSb[v] + jm[v].d * jb[v];
    if (j < 5) qb[j] = s;
    else gb[(j - 5) / 3][(j - 5) % 3] = s;
  }
  for (int v = 0; v < 5; ++v) a.QF[fslot(5, fs, N2, v, pt)] = qb[v];
  if (NS)
    for (int vc = 0; vc < 15; ++vc) a.GF[fslot(15, fs, N2, vc, pt)] = gb[vc / 3][vc % 3];
}
template <int N, bool NS>
__global__ void __launch_bounds__(256) k_bface_rev(VjpArgs a, const int4* __restrict__ faces, int nf) {
  bface_rev_body<N, NS>(a, faces, nf, blockIdx.x);
}

// -------------------------------------------------------------- trace_rev
// out += transposed extrapolation of the q-trace adjoints + transposed
// uncorrected gradient of the gradient-trace adjoints.
template <int N, bool NS>
__device__ __forceinline__ void trace_rev_body(const VjpArgs& a, const int* __restrict__ elems, int nel, int epb,
                                               int blk, unsigned char* smem) {
  constexpr int N2 = N * N, N3 = N2 * N;
  double* sX = reinterpret_cast<double*>(smem);  // [epb][5][N3]
  const OpsTab<double>& O = ops<double>();
  const int tid = threadIdx.x;
  const int le = tid / N3, k = tid - le * N3;
  const int slot = blk * epb + le;
  const bool act = le < epb && slot < nel;
  const int e = act ? elems[slot] : 0;
  const long off = act ? (long)a.sp_off[e] + k : 0;
  const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
  const int id[3] = {i0, i1, i2};
  double Ub[5], dqb[3][5];
  if (act) {
    const long fb = a.fp_off[e];
    double gbar[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Ub[v] = a.out[(long)v * a.nsp + off];
#pragma unroll
      for (int c = 0; c < 3; ++c) gbar[v][c] = 0.0;
    }
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
      const int fp = dd == 0 ? i1 + N * i2 : (dd == 1 ? i0 + N * i2 : i0 + N * i1);
      const long fm = fb + (2 * dd) * N2, fq = fb + (2 * dd + 1) * N2;
      const double wm = O.lm[N][id[dd]], wp = O.lp[N][id[dd]];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        Ub[v] += wm * a.QF[fslot(5, fm, N2, v, fp)] + wp * a.QF[fslot(5, fq, N2, v, fp)];
      if (NS) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            gbar[v][c] += wm * a.GF[fslot(15, fm, N2, v * 3 + c, fp)] + wp * a.GF[fslot(15, fq, N2, v * 3 + c, fp)];
      }
    }
    if (NS) {
      double Ja[3][3], J;
      tri_metrics<double>(a.geo + 24L * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dqb[i][v] = (Ja[i][0] * gbar[v][0] + Ja[i][1] * gbar[v][1] + Ja[i][2] * gbar[v][2]) / J;
    }
  }
  if (NS) {
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      __syncthreads();
      if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = i == 0 ? dqb[0][v] : (i == 1 ? dqb[1][v] : dqb[2][v]);
      }
      __syncthreads();
      if (act) {
        const double* X = sX + le * 5 * N3;
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const int kk = i == 0 ? m + N * (i1 + N * i2) : (i == 1 ? i0 + N * (m + N * i2) : i0 + N * (i1 + N * m));
            Ub[v] = fma(O.D[N][m][i == 0 ? i0 : (i == 1 ? i1 : i2)], X[v * N3 + kk], Ub[v]);
          }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) a.out[(long)v * a.nsp + off] = Ub[v];
  }
}
template <int N, bool NS>
__global__ void __launch_bounds__(256) k_trace_rev(VjpArgs a, const int* __restrict__ elems, int nel, int epb) {
  extern __shared__ __align__(16) unsigned char smem[];
  trace_rev_body<N, NS>(a, elems, nel, epb, blockIdx.x, smem);
}

// ------------------------------------------------------- fused launches
// One launch per reverse stage over every degree bucket, as in the forward
// pass: tiles[blockIdx.x] = (code, first, count, per) with code n for element
// tiles, 8 nl + nh for interior faces, 64 + n for boundary faces.
#define FRX_VCASE(N) \
  case N:            \
    if constexpr (TRACE) trace_rev_body<N, NS>(a, elems + t.y, t.z, t.w, 0, smem); \
    else div_rev_body<N, NS>(a, elems + t.y, t.z, t.w, 0, smem);                   \
    break;
template <bool NS, bool TRACE>
__global__ void __launch_bounds__(256) k_elem_rev_fused(VjpArgs a, const int* __restrict__ elems,
                                                        const int4* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_VCASE(2) FRX_VCASE(3) FRX_VCASE(4) FRX_VCASE(5) FRX_VCASE(6)
    default: break;
  }
}
#undef FRX_VCASE

#define FRX_VFLIST(X)                                           \
  X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(3, 3) X(3, 4) X(3, 5) \
  X(3, 6) X(4, 4) X(4, 5) X(4, 6) X(5, 5) X(5, 6) X(6, 6)
#define FRX_VGCASE(NL, NH) \
  case 8 * NL + NH: face_rev_gather<NL, NH, NS>(a, faces + t.y, t.z, t.w, 0, smem, P); break;
#define FRX_VSCASE(NL, NH) \
  case 8 * NL + NH: face_rev_scatter<NL, NH, NS>(a, faces + t.y, t.z, t.w, 0, smem, P, qb, gb); break;
// Interior-face tiles (the plan puts them first); boundary-face tiles go to
// k_bface_rev_fused.
template <bool NS, int FLUX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_face_rev_fused(VjpArgs a, const int4* __restrict__ faces, const int4* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  FaceRevPt P;
  switch (t.x) {
    FRX_VFLIST(FRX_VGCASE)
    default: return;
  }
  double qb[2][5], gb[2][5][3];
  if (P.act)
    face_fn_vjp<NS, FLUX>(P.q[0], P.q[1], P.g[0], P.g[1], P.S, P.cL, P.cR, a.gas, a.flux, P.fSb, P.jb[0], P.jb[1],
                          qb[0], qb[1], gb[0], gb[1]);
  switch (t.x) {
    FRX_VFLIST(FRX_VSCASE)
    default: break;
  }
}
#undef FRX_VGCASE
#undef FRX_VSCASE
#undef FRX_VFLIST

#define FRX_VBCASE(N) \
  case 64 + N: bface_rev_body<N, NS>(a, faces + t.y, t.z, 0); break;
template <bool NS>
__global__ void __launch_bounds__(256) k_bface_rev_fused(VjpArgs a, const int4* __restrict__ faces,
                                                         const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_VBCASE(2) FRX_VBCASE(3) FRX_VBCASE(4) FRX_VBCASE(5) FRX_VBCASE(6)
    default: break;
  }
}
#undef FRX_VBCASE

}  // namespace frx
