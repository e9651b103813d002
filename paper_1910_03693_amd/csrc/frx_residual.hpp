// FR/CPR residual kernels for hexahedra of degree p = N - 1 (section 2.2 of
// the paper), instantiated per N and per scalar T in {double, float,
// Dual<double>, Dual<float>}; with a dual scalar the same kernels return the
// exact tangent J(U) v next to R(U).
//
// The residual in the reference element (differential form eq. FR_diff with
// the DG correction field, contravariant flux Ft^i = Ja^i . f):
//   R = -(1/J) [ sum_i D_i Ft^i + sum_faces (f_com . S - f_loc) g'_face ]
// is evaluated in three stages over HBM-resident structure-of-arrays buffers:
//   trace: q (and, for Navier-Stokes, the uncorrected physical gradient) at
//          every element's own face points;
//   face:  common solution, BR2 common gradient and common normal flux per
//          face point, returned to each side at its own face points (the lower
//          degree side of a mixed face is interpolated to the higher side's
//          Gauss points and receives the L2 projection back);
//   div:   corrected gradient, volume flux, sum-factorised divergence and the
//          correction, written as R (or through an epilogue out = a*x + b*R).
#pragma once
#include "frx_device.hpp"

namespace frx {

// Load/store of the scalar T from base-type buffers: a dual reads (U, V) and
// stores its derivative part; a plain scalar reads U and stores its value.
template <class T> struct IO;
template <> struct IO<double> {
  static __device__ __forceinline__ double load(const double* U, const double*, long i) { return U[i]; }
  static __device__ __forceinline__ double out(double x) { return x; }
  static __device__ __forceinline__ double value(double x) { return x; }
};
template <> struct IO<float> {
  static __device__ __forceinline__ float load(const float* U, const float*, long i) { return U[i]; }
  static __device__ __forceinline__ float out(float x) { return x; }
  static __device__ __forceinline__ float value(float x) { return x; }
};
template <class B> struct IO<Dual<B>> {
  static __device__ __forceinline__ Dual<B> load(const B* U, const B* V, long i) { return Dual<B>(U[i], V[i]); }
  static __device__ __forceinline__ B out(Dual<B> x) { return x.d; }
  static __device__ __forceinline__ B value(Dual<B> x) { return x.v; }
};

template <class T> struct ResArgs {
  using B = base_t<T>;
  const B* U;      // state [5][nsp]
  const B* V;      // tangent direction [5][nsp] (dual scalars only)
  B* out;          // output [5][nsp]: out = alpha * in2 + beta * result
  B* out_val;      // optional (dual scalars): the value part of the result, i.e. R(U)
  const B* in2;    // optional second input of the epilogue
  const B* alpha_dev;  // if set, alpha is read from device memory
  B alpha, beta;
  int nsp, nfp;
  int flux;            // 0 Roe, 1 Rusanov
  const int* sp_off;   // [E] first solution point of each element
  const int* fp_off;   // [E] first face-slot point (6 n^2 per element)
  const B* geo;        // [E][24] trilinear monomial coefficients
  // face-slot buffers, nv values per slot laid out by fslot()
  const B* fgeo;       // nv 5: face-point geometry (k_face_geo)
  T* QF;               // nv 5: q traces
  T* GF;               // nv 15: gradient traces (Navier-Stokes)
  T* DQ;               // nv 5: q_com - q at own face points
  T* FS;               // nv 5: f_com . S at own face points
  Gas<B> gas;
  int* flag;           // set to 1 on a non-physical state (rho <= 0 or p <= 0)
  const int* skip;     // if set and nonzero the kernels return at once
};

// solution point on the line through face point (a, b) of direction d
template <int N> __device__ __forceinline__ int line_pt(int d, int a, int b, int m) {
  return d == 0 ? m + N * (a + N * b) : (d == 1 ? a + N * (m + N * b) : a + N * (b + N * m));
}

// Interior-face record (L, R, oL, pack): L's +d face is R's -d face; oL and
// oR are the first face slots of that face on L and on R, and
// pack = oR | d << 28 | low_is_R << 30, so that a face point's slots need no
// second dependent load.  Boundary-face record (e, f, bc, o), o the first slot
// of face f of e.
struct FaceRec {
  int L, R, oL, oR, d;
  bool low_is_R;
};
__device__ __forceinline__ FaceRec face_rec(const int4 F) {
  FaceRec r;
  r.L = F.x;
  r.R = F.y;
  r.oL = F.z;
  r.oR = F.w & 0x0fffffff;
  r.d = (F.w >> 28) & 3;
  r.low_is_R = (F.w >> 30) & 1;
  return r;
}

// Face-slot buffers hold nv values per slot.  A face side (first slot fs,
// n2 points) keeps its values as one [nv][n2] block at nv fs, so that the
// variables of a face point share cache lines, and an element's six sides,
// whose slots are consecutive, form one [6][nv][n2] block.
__device__ __forceinline__ long fslot(int nv, long fs, int n2, int v, int pt) {
  return (long)nv * fs + (v * n2 + pt);
}

// ---------------------------------------------------------------- trace stage
// Block: epb elements x N^3 threads (one solution point each).  LDS per
// element: q (5 N^3) and, for Navier-Stokes, the uncorrected physical
// gradient (15 N^3).  After one barrier every face item (element, face,
// point) extrapolates all of its values along the face-normal line.  Where
// 20 N^3 scalars of one element exceed FRX_TRACE_LDS_ALL bytes the gradient
// goes through a 5 N^3 region one variable at a time instead.
template <class T, int N, bool NS> __host__ __device__ constexpr bool trace_in_rounds() {
  return trace_lds_vals(NS, N, (int)sizeof(T)) == 5 && NS;
}
template <class T, int N, bool NS> __host__ __device__ constexpr int trace_vals() {
  return trace_in_rounds<T, N, NS>() ? 5 : (NS ? 20 : 5);
}

template <int N, class T, bool NS>
__device__ __forceinline__ void trace_body_rounds(const ResArgs<T>& a, const int4* __restrict__ elems, int nel, int epb,
                                           int blk, unsigned char* smem) {
  using B = base_t<T>;
  constexpr int N2 = N * N, N3 = N2 * N;
  T* sq = reinterpret_cast<T*>(smem);  // [epb][5][N3]
  const OpsTab<B>& O = ops<B>();
  const int tid = threadIdx.x;
  const int le = tid / N3, k = tid - le * N3;
  const int slot = blk * epb + le;
  const bool act = le < epb && slot < nel;
  const int4 ER = act ? elems[slot] : make_int4(0, 0, 0, 0);
  const int e = ER.x;
  if (act) {
    const long off = (long)ER.y + k;
#pragma unroll
    for (int v = 0; v < 5; ++v) sq[(le * 5 + v) * N3 + k] = IO<T>::load(a.U, a.V, (long)v * a.nsp + off);
  }
  __syncthreads();
  const int items = epb * 6 * N2;
  for (int it = tid; it < items; it += blockDim.x) {
    const int l2 = it / (6 * N2), rem = it - l2 * 6 * N2;
    const int f = rem / N2, pt = rem - f * N2;
    const int s2 = blk * epb + l2;
    if (s2 >= nel) continue;
    const long fs = elems[s2].z + f * N2;
    const int d = f >> 1, fa = pt % N, fb = pt / N;
    const B* lf = (f & 1) ? O.lp[N] : O.lm[N];
    const T* q = sq + l2 * 5 * N3;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T s = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) s = fmab(lf[m], q[v * N3 + line_pt<N>(d, fa, fb, m)], s);
      a.QF[fslot(5, fs, N2, v, pt)] = s;
    }
  }
  if (!NS) return;
  // uncorrected physical gradient at the point, kept in registers
  const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
  T gq[5][3];
  if (act) {
    B Ja[3][3], J;
    tri_metrics<B>(a.geo + 24L * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
    const B iJ = B(1) / J;
    const T* q = sq + le * 5 * N3;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T d0 = T(B(0)), d1 = T(B(0)), d2 = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) {
        d0 = fmab(O.D[N][i0][m], q[v * N3 + m + N * (i1 + N * i2)], d0);
        d1 = fmab(O.D[N][i1][m], q[v * N3 + i0 + N * (m + N * i2)], d1);
        d2 = fmab(O.D[N][i2][m], q[v * N3 + i0 + N * (i1 + N * m)], d2);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) gq[v][c] = (Ja[0][c] * d0 + Ja[1][c] * d1 + Ja[2][c] * d2) * iJ;
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    __syncthreads();  // previous readers of the region are done
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sq[(le * 5 + c) * N3 + k] = gq[v][c];
    }
    __syncthreads();
    for (int it = tid; it < epb * 18 * N2; it += blockDim.x) {
      const int l2 = it / (18 * N2), rem = it - l2 * 18 * N2;
      const int c = rem / (6 * N2), fp = rem - c * 6 * N2;
      const int f = fp / N2, pt = fp - f * N2;
      const int s2 = blk * epb + l2;
      if (s2 >= nel) continue;
      const long fs = elems[s2].z + f * N2;
      const int d = f >> 1;
      const B* lf = (f & 1) ? O.lp[N] : O.lm[N];
      const T* g = sq + (l2 * 5 + c) * N3;
      T s = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) s = fmab(lf[m], g[line_pt<N>(d, pt % N, pt / N, m)], s);
      a.GF[fslot(15, fs, N2, v * 3 + c, pt)] = s;
    }
  }
}


template <int N, class T, bool NS>
__device__ __forceinline__ void trace_body(const ResArgs<T>& a, const int4* __restrict__ elems, int nel, int epb,
                                           int blk, unsigned char* smem) {
  using B = base_t<T>;
  if constexpr (trace_in_rounds<T, N, NS>()) {
    trace_body_rounds<N, T, NS>(a, elems, nel, epb, blk, smem);
    return;
  }
  constexpr int N2 = N * N, N3 = N2 * N, NV = trace_vals<T, N, NS>();
  T* sq = reinterpret_cast<T*>(smem);  // [epb][NV][N3]
  const OpsTab<B>& O = ops<B>();
  const int tid = threadIdx.x;
  const int le = tid / N3, k = tid - le * N3;
  const int slot = blk * epb + le;
  const bool act = le < epb && slot < nel;
  const int4 ER = act ? elems[slot] : make_int4(0, 0, 0, 0);
  const int e = ER.x;
  T* q = sq + le * NV * N3;
  if (act) {
    const int off = ER.y + k;
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v * N3 + k] = IO<T>::load(a.U, a.V, (long)(v * a.nsp + off));
  }
  if (NS) {
    __syncthreads();
    if (act) {
      const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
      B Ja[3][3], J;
      tri_metrics<B>(a.geo + 24 * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
      const B iJ = B(1) / J;
      T g[15];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        T d0 = T(B(0)), d1 = T(B(0)), d2 = T(B(0));
#pragma unroll
        for (int m = 0; m < N; ++m) {
          d0 = fmab(O.D[N][i0][m], q[v * N3 + m + N * (i1 + N * i2)], d0);
          d1 = fmab(O.D[N][i1][m], q[v * N3 + i0 + N * (m + N * i2)], d1);
          d2 = fmab(O.D[N][i2][m], q[v * N3 + i0 + N * (i1 + N * m)], d2);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) g[v * 3 + c] = (Ja[0][c] * d0 + Ja[1][c] * d1 + Ja[2][c] * d2) * iJ;
      }
#pragma unroll
      for (int vc = 0; vc < 15; ++vc) q[(5 + vc) * N3 + k] = g[vc];
    }
  }
  __syncthreads();
  // items (element, face, point): a wave covers runs of contiguous slots
  for (int it = tid; it < epb * 6 * N2; it += blockDim.x) {
    const int l2 = it / (6 * N2), fp = it - l2 * 6 * N2;
    const int s2 = blk * epb + l2;
    if (s2 >= nel) continue;
    const int f = fp / N2, pt = fp - f * N2;
    const int d = f >> 1, fa = pt % N, fb = pt / N;
    const long fs = elems[s2].z + f * N2;
    const B* lf = (f & 1) ? O.lp[N] : O.lm[N];
    // start and stride of the normal line through (fa, fb)
    const int base = d == 0 ? N * (fa + N * fb) : (d == 1 ? fa + N2 * fb : fa + N * fb);
    const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
    const T* src = sq + l2 * NV * N3 + base;
    B w[N];
#pragma unroll
    for (int m = 0; m < N; ++m) w[m] = lf[m];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T s = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) s = fmab(w[m], src[v * N3 + m * stride], s);
      if (v < 5) a.QF[fslot(5, fs, N2, v, pt)] = s;
      else a.GF[fslot(15, fs, N2, v - 5, pt)] = s;
    }
  }
}

// ----------------------------------------------------------------- face stage
// Interior faces whose sides have sizes {NL, NH}, NL <= NH.  Face record
// (L, R, d, low_is_R): L's +d face is R's -d face; the area vector S points
// from L to R and is evaluated once per face point from L's map.
// Block: fpb faces x NH^2 threads (one face point each).  The stage runs in
// three phases: face_gather (the inputs of the face point, interpolated from
// the low side of a mixed face), face_fn, face_scatter (the results to the
// face slots of both sides, L2-projected to the low side of a mixed face).
// The gather and scatter depend on (NL, NH), face_fn does not, so the fused
// kernel holds one copy of face_fn after its switch over the tile kinds.

// State of one interior face point between the phases.
template <class T> struct FacePt {
  using B = base_t<T>;
  T q[2][5];   // q of both sides at the point
  T g[5][3];   // sum of both sides' gradient traces (Navier-Stokes)
  B S[3], cL, cR;
  int oL, oR;  // first face slot of the face on L and on R
  int lf, pt;  // face of the tile, point of the face
  bool act, lowL, lowR;
};

template <int NL, int NH, class T, bool NS>
__device__ __forceinline__ void face_gather(const ResArgs<T>& a, const int4* __restrict__ faces, int nf, int fpb,
                                            int blk, unsigned char* smem, FacePt<T>& P) {
  using B = base_t<T>;
  constexpr int NH2 = NH * NH, NL2 = NL * NL;
  constexpr bool MIX = NL < NH;
  constexpr int NV = NS ? 20 : 5;
  T* slow = reinterpret_cast<T*>(smem);  // [fpb][NV][NL2] low-side traces
  const OpsTab<B>& O = ops<B>();
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
  if (MIX) {  // stage the low side's own-point traces
    for (int it = tid; it < fpb * NV * NL2; it += blockDim.x) {
      const int l2 = it / (NV * NL2), rem = it - l2 * NV * NL2;
      const int vv = rem / NL2, p2 = rem - vv * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      slow[it] = vv < 5 ? a.QF[fslot(5, fs, NL2, vv, p2)] : a.GF[fslot(15, fs, NL2, vv - 5, p2)];
    }
    __syncthreads();
  }
  if (!P.act) return;
  const int pt = P.pt, A = pt % NH, Bq = pt / NH;
  // q of both sides and the SUM of their gradient traces (all that the BR2
  // common gradient needs), each side read at the face point
  if (NS) {
#pragma unroll
    for (int vc = 0; vc < 15; ++vc) P.g[vc / 3][vc % 3] = T(B(0));
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool low = s ? P.lowR : P.lowL;
    if (low) {
      const T* src = slow + P.lf * NV * NL2;
#pragma unroll
      for (int vv = 0; vv < NV; ++vv) {
        T acc = T(B(0));
#pragma unroll
        for (int b = 0; b < NL; ++b) {
          T row = T(B(0));
#pragma unroll
          for (int aa = 0; aa < NL; ++aa) row = fmab(O.I[NL - 2][NH - 2][A][aa], src[vv * NL2 + aa + NL * b], row);
          acc = fmab(O.I[NL - 2][NH - 2][Bq][b], row, acc);
        }
        if (vv < 5) P.q[s][vv] = acc;
        else P.g[(vv - 5) / 3][(vv - 5) % 3] += acc;
      }
    } else {
      const long fs = s ? F.oR : F.oL;
#pragma unroll
      for (int v = 0; v < 5; ++v) P.q[s][v] = a.QF[fslot(5, fs, NH2, v, pt)];
      if (NS) {
#pragma unroll
        for (int vc = 0; vc < 15; ++vc) P.g[vc / 3][vc % 3] += a.GF[fslot(15, fs, NH2, vc, pt)];
      }
    }
  }
  // geometry at the face point, kept at the high side's slot
  const long og = P.lowL ? F.oR : F.oL;
  P.S[0] = a.fgeo[fslot(5, og, NH2, 0, pt)];
  P.S[1] = a.fgeo[fslot(5, og, NH2, 1, pt)];
  P.S[2] = a.fgeo[fslot(5, og, NH2, 2, pt)];
  P.cL = P.cR = B(0);
  if (NS) {
    P.cL = a.fgeo[fslot(5, og, NH2, 3, pt)];
    P.cR = a.fgeo[fslot(5, og, NH2, 4, pt)];
  }
}

// FS_OUT false: the jumps alone (fS unused, no common flux written).
template <int NL, int NH, class T, bool FS_OUT = true>
__device__ __forceinline__ void face_scatter(const ResArgs<T>& a, const int4* __restrict__ faces, int nf, int fpb,
                                             int blk, unsigned char* smem, const FacePt<T>& P, const T fS[5],
                                             int nv_low) {
  using B = base_t<T>;
  constexpr int NH2 = NH * NH, NL2 = NL * NL;
  constexpr bool MIX = NL < NH;
  T* sout = reinterpret_cast<T*>(smem) + (MIX ? fpb * nv_low * NL2 : 0);  // [fpb][10][NH2] low-side results
  const int pt = P.pt;
  if (P.act) {
    T jL[5], jR[5];
    face_jumps<T, B>(P.q[0], P.q[1], jL, jR);
    if (!P.lowL) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        if (FS_OUT) a.FS[fslot(5, P.oL, NH2, v, pt)] = fS[v];
        a.DQ[fslot(5, P.oL, NH2, v, pt)] = jL[v];
      }
    }
    if (!P.lowR) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        if (FS_OUT) a.FS[fslot(5, P.oR, NH2, v, pt)] = fS[v];
        a.DQ[fslot(5, P.oR, NH2, v, pt)] = jR[v];
      }
    }
    if (MIX) {
      T* dst = sout + P.lf * 10 * NH2;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        dst[v * NH2 + pt] = fS[v];
        dst[(5 + v) * NH2 + pt] = sel(P.lowL, jL[v], jR[v]);
      }
    }
  }
  if (MIX) {
    const OpsTab<B>& O = ops<B>();
    __syncthreads();
    for (int it = threadIdx.x; it < fpb * NL2; it += blockDim.x) {
      const int l2 = it / NL2, p2 = it - l2 * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      const int aa = p2 % NL, bb = p2 / NL;
      const T* src = sout + l2 * 10 * NH2;
      for (int vv = 0; vv < 10; ++vv) {
        T acc = T(B(0));
#pragma unroll
        for (int Bq = 0; Bq < NH; ++Bq) {
          T row = T(B(0));
#pragma unroll
          for (int A = 0; A < NH; ++A) row = fmab(O.P[NL - 2][NH - 2][aa][A], src[vv * NH2 + A + NH * Bq], row);
          acc = fmab(O.P[NL - 2][NH - 2][bb][Bq], row, acc);
        }
        if (vv >= 5) a.DQ[fslot(5, fs, NL2, vv - 5, p2)] = acc;
        else if (FS_OUT) a.FS[fslot(5, fs, NL2, vv, p2)] = acc;
      }
    }
  }
}

template <int NL, int NH, class T, bool NS, int FLUX = -1>
__device__ __forceinline__ void face_body(const ResArgs<T>& a, const int4* __restrict__ faces, int nf, int fpb,
                                          int blk, unsigned char* smem) {
  using B = base_t<T>;
  FacePt<T> P;
  face_gather<NL, NH, T, NS>(a, faces, nf, fpb, blk, smem, P);
  T fS[5];
  if (P.act) face_fn<NS, T, B, FLUX>(P.q[0], P.q[1], P.g, P.S, P.cL, P.cR, a.gas, a.flux, fS);
  face_scatter<NL, NH, T>(a, faces, nf, fpb, blk, smem, P, fS, NS ? 20 : 5);
}

// Boundary faces of elements of size N: record (e, f, bc, 0).  One thread per
// face point.
template <int N, class T, bool NS, int FLUX = -1>
__device__ __forceinline__ void bface_body(const ResArgs<T>& a, const int4* __restrict__ faces, int nf, int blk) {
  using B = base_t<T>;
  constexpr int N2 = N * N;
  const int gid = blk * blockDim.x + threadIdx.x;
  if (gid >= nf * N2) return;
  const int fi = gid / N2, pt = gid - fi * N2;
  const int4 F = faces[fi];
  const int bc = F.z, side = F.y & 1;
  const long fs = F.w;
  T q[5], g[5][3];
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = a.QF[fslot(5, fs, N2, v, pt)];
  if (NS) {
#pragma unroll
    for (int vc = 0; vc < 15; ++vc) g[vc / 3][vc % 3] = a.GF[fslot(15, fs, N2, vc, pt)];
  }
  const B S[3] = {a.fgeo[fslot(5, fs, N2, 0, pt)], a.fgeo[fslot(5, fs, N2, 1, pt)], a.fgeo[fslot(5, fs, N2, 2, pt)]};
  const B cf = a.fgeo[fslot(5, fs, N2, 3, pt)];
  T fS[5], jmp[5];
  bface_fn<NS, T, B, FLUX>(q, g, S, cf, bc, side, a.gas, a.flux, fS, jmp);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.FS[fslot(5, fs, N2, v, pt)] = fS[v];
    a.DQ[fslot(5, fs, N2, v, pt)] = jmp[v];
  }
}

// ------------------------------------------------- face-point geometry
// The face stages read their geometry per face point instead of evaluating
// two trilinear maps there, which keeps 48 map coefficients out of the face
// kernels' registers.  Computed once per mesh with the same formulas:
// interior face point (grid of the high side, stored at that side's slot):
// S from L's map at r_d = +1 and the BR2 lifting coefficients
// cL = g_R'(+1)/J_L = n_L^2/(2 J_L) > 0, cR = g_L'(-1)/J_R = -n_R^2/(2 J_R);
// boundary face point: S and c = +-n^2/(2 J) (+ on the +xi^d face).
// Values (fslot, nv 5): S_x, S_y, S_z, cL (or c), cR.
template <class B>
__global__ void k_face_geo(const B* __restrict__ geo, const int4* __restrict__ faces, int nf, int nl, int nh,
                           B* __restrict__ fg) {
  const int nh2 = nh * nh;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nf * nh2) return;
  const int fi = (int)(gid / nh2), pt = (int)(gid - (long)fi * nh2);
  const FaceRec F = face_rec(faces[fi]);
  const bool lowR = nl < nh && F.low_is_R, lowL = nl < nh && !F.low_is_R;
  const OpsTab<B>& O = ops<B>();
  const B ta = O.x[nh][pt % nh], tb = O.x[nh][pt / nh];
  B S[3], JL, SR[3], JR;
  face_geom<B>(geo + 24L * F.L, F.d, B(1), ta, tb, S, JL);
  face_geom<B>(geo + 24L * F.R, F.d, B(-1), ta, tb, SR, JR);
  const int nL = lowL ? nl : nh, nR = lowR ? nl : nh;
  const long fs = lowL ? F.oR : F.oL;
  fg[fslot(5, fs, nh2, 0, pt)] = S[0];
  fg[fslot(5, fs, nh2, 1, pt)] = S[1];
  fg[fslot(5, fs, nh2, 2, pt)] = S[2];
  fg[fslot(5, fs, nh2, 3, pt)] = B(0.5) * B(nL * nL) / JL;
  fg[fslot(5, fs, nh2, 4, pt)] = -B(0.5) * B(nR * nR) / JR;
}
template <class B>
__global__ void k_bface_geo(const B* __restrict__ geo, const int4* __restrict__ faces, int nf, int n,
                            B* __restrict__ fg) {
  const int n2 = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nf * n2) return;
  const int fi = (int)(gid / n2), pt = (int)(gid - (long)fi * n2);
  const int4 F = faces[fi];
  const int e = F.x, f = F.y, d = f >> 1, side = f & 1;
  const OpsTab<B>& O = ops<B>();
  B S[3], J;
  face_geom<B>(geo + 24L * e, d, side ? B(1) : B(-1), O.x[n][pt % n], O.x[n][pt / n], S, J);
  const long fs = F.w;
  fg[fslot(5, fs, n2, 0, pt)] = S[0];
  fg[fslot(5, fs, n2, 1, pt)] = S[1];
  fg[fslot(5, fs, n2, 2, pt)] = S[2];
  fg[fslot(5, fs, n2, 3, pt)] = (side ? B(0.5) : B(-0.5)) * B(n2) / J;
  fg[fslot(5, fs, n2, 4, pt)] = B(0);
}

// ------------------------------------------------- viscous face correction
// Navier-Stokes interior faces in two passes: the inviscid pass is face_body
// with the Euler flag (common solution, jumps, f_inv . S), this pass
// subtracts the viscous common flux (eq. com_grad_q and the viscous part of
// f_com . S) from the face slots it wrote.  Each pass needs about half the
// registers of the one-pass face function, so both run two waves per SIMD.
// The low side of a mixed face receives the L2 projection of the viscous flux
// (the projection is linear, so the two passes together give the projection
// of the full flux).  LDS: [fpb][20][NL2] low-side q and gradient traces,
// [fpb][4][NH2] viscous flux at the high side's points.
template <int NL, int NH, class T>
__device__ __forceinline__ void face_visc_body(const ResArgs<T>& a, const int4* __restrict__ faces, int nf, int fpb,
                                               int blk, unsigned char* smem) {
  using B = base_t<T>;
  constexpr int NH2 = NH * NH, NL2 = NL * NL;
  constexpr bool MIX = NL < NH;
  T* slow = reinterpret_cast<T*>(smem);           // [fpb][20][NL2]
  T* sout = slow + (MIX ? fpb * 20 * NL2 : 0);     // [fpb][4][NH2]
  const OpsTab<B>& O = ops<B>();
  const int tid = threadIdx.x;
  const int lf = tid / NH2, pt = tid - lf * NH2;
  const int fi = blk * fpb + lf;
  const bool act = lf < fpb && fi < nf;
  const FaceRec F = face_rec(act ? faces[fi] : make_int4(0, 0, 0, 0));
  const bool lowR = MIX && F.low_is_R;
  const bool lowL = MIX && !F.low_is_R;
  if (MIX) {
    for (int it = tid; it < fpb * 20 * NL2; it += blockDim.x) {
      const int l2 = it / (20 * NL2), rem = it - l2 * 20 * NL2;
      const int vv = rem / NL2, p2 = rem - vv * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      slow[it] = vv < 5 ? a.QF[fslot(5, fs, NL2, vv, p2)] : a.GF[fslot(15, fs, NL2, vv - 5, p2)];
    }
    __syncthreads();
  }
  const int A = pt % NH, Bq = pt / NH;
  T fv[4];
  if (act) {
    T q[2][5], g[5][3];
#pragma unroll
    for (int vc = 0; vc < 15; ++vc) g[vc / 3][vc % 3] = T(B(0));
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const bool low = s ? lowR : lowL;
      if (low) {
        const T* src = slow + lf * 20 * NL2;
#pragma unroll
        for (int vv = 0; vv < 20; ++vv) {
          T acc = T(B(0));
#pragma unroll
          for (int b = 0; b < NL; ++b) {
            T row = T(B(0));
#pragma unroll
            for (int aa = 0; aa < NL; ++aa) row = fmab(O.I[NL - 2][NH - 2][A][aa], src[vv * NL2 + aa + NL * b], row);
            acc = fmab(O.I[NL - 2][NH - 2][Bq][b], row, acc);
          }
          if (vv < 5) q[s][vv] = acc;
          else g[(vv - 5) / 3][(vv - 5) % 3] += acc;
        }
      } else {
        const long fs = s ? F.oR : F.oL;
#pragma unroll
        for (int v = 0; v < 5; ++v) q[s][v] = a.QF[fslot(5, fs, NH2, v, pt)];
#pragma unroll
        for (int vc = 0; vc < 15; ++vc) g[vc / 3][vc % 3] += a.GF[fslot(15, fs, NH2, vc, pt)];
      }
    }
    const long og = lowL ? F.oR : F.oL;
    const B S[3] = {a.fgeo[fslot(5, og, NH2, 0, pt)], a.fgeo[fslot(5, og, NH2, 1, pt)],
                    a.fgeo[fslot(5, og, NH2, 2, pt)]};
    const B cL = a.fgeo[fslot(5, og, NH2, 3, pt)];
    const B cR = a.fgeo[fslot(5, og, NH2, 4, pt)];
    // common solution and the BR2 common gradient from the jumps
    // q_com - q^- = (q^+ - q^-)/2, q_com - q^+ = -(q^+ - q^-)/2
    T qc[5], Gc[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      qc[v] = B(0.5) * (q[0][v] + q[1][v]);
      const T jl = qc[v] - q[0][v], jr = qc[v] - q[1][v];
      const T lift = cL * jl + cR * jr;
#pragma unroll
      for (int c = 0; c < 3; ++c) Gc[v][c] = B(0.5) * (g[v][c] + S[c] * lift);
    }
    T tau[3][3], e[3];
    viscous_terms<T, B>(qc, Gc, a.gas, tau, e);
#pragma unroll
    for (int c = 0; c < 3; ++c) fv[c] = tau[c][0] * S[0] + tau[c][1] * S[1] + tau[c][2] * S[2];
    fv[3] = e[0] * S[0] + e[1] * S[1] + e[2] * S[2];
    if (!lowL) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const long o = fslot(5, F.oL, NH2, 1 + c, pt);
        a.FS[o] = a.FS[o] - fv[c];
      }
    }
    if (!lowR) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const long o = fslot(5, F.oR, NH2, 1 + c, pt);
        a.FS[o] = a.FS[o] - fv[c];
      }
    }
    if (MIX) {
      T* dst = sout + lf * 4 * NH2;
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[c * NH2 + pt] = fv[c];
    }
  }
  if (MIX) {
    __syncthreads();
    for (int it = tid; it < fpb * NL2; it += blockDim.x) {
      const int l2 = it / NL2, p2 = it - l2 * NL2;
      const int f2 = blk * fpb + l2;
      if (f2 >= nf) continue;
      const FaceRec G2 = face_rec(faces[f2]);
      const long fs = G2.low_is_R ? G2.oR : G2.oL;
      const int aa = p2 % NL, bb = p2 / NL;
      const T* src = sout + l2 * 4 * NH2;
      for (int c = 0; c < 4; ++c) {
        T acc = T(B(0));
#pragma unroll
        for (int Bq2 = 0; Bq2 < NH; ++Bq2) {
          T row = T(B(0));
#pragma unroll
          for (int A2 = 0; A2 < NH; ++A2) row = fmab(O.P[NL - 2][NH - 2][aa][A2], src[c * NH2 + A2 + NH * Bq2], row);
          acc = fmab(O.P[NL - 2][NH - 2][bb][Bq2], row, acc);
        }
        const long o = fslot(5, fs, NL2, 1 + c, p2);
        a.FS[o] = a.FS[o] - acc;
      }
    }
  }
}

// ------------------------------------------------------------------ div stage
// Block: epb elements x N^3 threads.  LDS per element: a region X of 5 N^3
// (q, then one direction of the contravariant flux at a time) and a region Y
// of 30 N^2 (the solution jumps of the 6 faces, then the flux jumps
// f_com . S - f_loc).
template <int N, class T, bool NS>
__device__ __forceinline__ void div_body(const ResArgs<T>& a, const int4* __restrict__ elems, int nel, int epb,
                                         int blk, unsigned char* smem) {
  using B = base_t<T>;
  constexpr int N2 = N * N, N3 = N2 * N;
  T* sX = reinterpret_cast<T*>(smem);  // [epb][5][N3]
  T* sY = sX + epb * 5 * N3;           // [epb][6][5][N2]
  const OpsTab<B>& O = ops<B>();
  const int tid = threadIdx.x;
  const int le = tid / N3, k = tid - le * N3;
  const int slot = blk * epb + le;
  const bool act = le < epb && slot < nel;
  const int4 ER = act ? elems[slot] : make_int4(0, 0, 0, 0);
  const int e = ER.x;
  const long off = act ? (long)ER.y + k : 0;
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = IO<T>::load(a.U, a.V, (long)v * a.nsp + off);
  }
  if (NS) {
    for (int it = tid; it < epb * 30 * N2; it += blockDim.x) {
      // (element, face, variable, point): Y has the element's slot block layout
      const int l2 = it / (30 * N2), rem = it - l2 * 30 * N2;
      const int s2 = blk * epb + l2;
      if (s2 >= nel) continue;
      sY[it] = a.DQ[5L * elems[s2].z + rem];
    }
  }
  __syncthreads();
  const int i0 = k % N, i1 = (k / N) % N, i2 = k / N2;
  const int id[3] = {i0, i1, i2};
  B Ja[3][3], J = B(1);
  T Ft[3][5];
  if (act) {
    tri_metrics<B>(a.geo + 24L * e, O.x[N][i0], O.x[N][i1], O.x[N][i2], Ja, J);
    const T* qs = sX + le * 5 * N3;
    T q[5], Gq[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = qs[v * N3 + k];
    // (written so that a NaN density or pressure is flagged as well)
    if (!(val(q[0]) > B(0)) || !(val(pressure<T, B>(q, a.gas)) > B(0))) *a.flag = 1;
    if (NS) {
      const T* jm = sY + le * 30 * N2;
      const B iJ = B(1) / J;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        T d0 = T(B(0)), d1 = T(B(0)), d2 = T(B(0));
#pragma unroll
        for (int m = 0; m < N; ++m) {
          d0 = fmab(O.D[N][i0][m], qs[v * N3 + m + N * (i1 + N * i2)], d0);
          d1 = fmab(O.D[N][i1][m], qs[v * N3 + i0 + N * (m + N * i2)], d1);
          d2 = fmab(O.D[N][i2][m], qs[v * N3 + i0 + N * (i1 + N * m)], d2);
        }
        // corrections from the solution jumps of the two faces of each direction
        d0 = fmab(O.gL[N][i0], jm[(0 * 5 + v) * N2 + i1 + N * i2], d0);
        d0 = fmab(O.gR[N][i0], jm[(1 * 5 + v) * N2 + i1 + N * i2], d0);
        d1 = fmab(O.gL[N][i1], jm[(2 * 5 + v) * N2 + i0 + N * i2], d1);
        d1 = fmab(O.gR[N][i1], jm[(3 * 5 + v) * N2 + i0 + N * i2], d1);
        d2 = fmab(O.gL[N][i2], jm[(4 * 5 + v) * N2 + i0 + N * i1], d2);
        d2 = fmab(O.gR[N][i2], jm[(5 * 5 + v) * N2 + i0 + N * i1], d2);
#pragma unroll
        for (int c = 0; c < 3; ++c) Gq[v][c] = (Ja[0][c] * d0 + Ja[1][c] * d1 + Ja[2][c] * d2) * iJ;
      }
    }
    volume_flux<T, B, NS>(q, Gq, Ja, a.gas, Ft);
  }
  T acc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) acc[v] = T(B(0));
  // face items (element, variable, side, point) of one direction: at most
  // epb 10 N^2 <= blockDim.x 10 / N of them, FIT per thread
  constexpr int FIT = (10 + N - 1) / N;
  const int items = epb * 10 * N2;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // the common fluxes f_com . S of the two faces of direction d, loaded
    // before the barrier so that the loads overlap the contraction below
    T fsr[FIT];
#pragma unroll
    for (int q = 0; q < FIT; ++q) {
      const int it = tid + q * (int)blockDim.x;
      fsr[q] = T(B(0));
      if (it < items) {
        const int l2 = it / (10 * N2), rem = it - l2 * 10 * N2;
        const int s2 = blk * epb + l2;
        if (s2 < nel) fsr[q] = a.FS[5L * elems[s2].z + 10 * d * N2 + rem];
      }
    }
    __syncthreads();  // X (q or the previous direction) and Y are no longer read
    if (act) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sX[(le * 5 + v) * N3 + k] = Ft[d][v];
    }
    __syncthreads();
    if (act) {
      const T* X = sX + le * 5 * N3;
      const int kd = id[d];
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int m = 0; m < N; ++m) {
          const int kk = d == 0 ? m + N * (i1 + N * i2) : (d == 1 ? i0 + N * (m + N * i2) : i0 + N * (i1 + N * m));
          acc[v] = fmab(O.D[N][kd][m], X[v * N3 + kk], acc[v]);
        }
    }
    // flux jumps f_com . S - f_loc on the two faces of direction d
    // (element, side, variable, point): the two faces are one contiguous block
#pragma unroll
    for (int q = 0; q < FIT; ++q) {
      const int it = tid + q * (int)blockDim.x;
      if (it >= items) continue;
      const int l2 = it / (10 * N2), rem = it - l2 * 10 * N2;
      const int side = rem / (5 * N2), vp2 = rem - side * 5 * N2;
      const int v = vp2 / N2, p2 = vp2 - v * N2, f = 2 * d + side;
      const int s2 = blk * epb + l2;
      if (s2 >= nel) continue;
      const B* lf = side ? O.lp[N] : O.lm[N];
      const T* X = sX + (l2 * 5 + v) * N3;
      T floc = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) floc = fmab(lf[m], X[line_pt<N>(d, p2 % N, p2 / N, m)], floc);
      sY[(l2 * 30 + f * 5 + v) * N2 + p2] = fsr[q] - floc;
    }
    // (only for block shapes with more than FIT items per thread, which the
    // launchers do not make)
    for (int it = tid + FIT * (int)blockDim.x; it < items; it += blockDim.x) {
      const int l2 = it / (10 * N2), rem = it - l2 * 10 * N2;
      const int side = rem / (5 * N2), vp2 = rem - side * 5 * N2;
      const int v = vp2 / N2, p2 = vp2 - v * N2, f = 2 * d + side;
      const int s2 = blk * epb + l2;
      if (s2 >= nel) continue;
      const B* lf = side ? O.lp[N] : O.lm[N];
      const T* X = sX + (l2 * 5 + v) * N3;
      T floc = T(B(0));
#pragma unroll
      for (int m = 0; m < N; ++m) floc = fmab(lf[m], X[line_pt<N>(d, p2 % N, p2 / N, m)], floc);
      sY[(l2 * 30 + f * 5 + v) * N2 + p2] = a.FS[5L * elems[s2].z + 10 * d * N2 + rem] - floc;
    }
    __syncthreads();
    if (act) {
      const T* jm = sY + le * 30 * N2;
      const int kd = id[d];
      const int fp = d == 0 ? i1 + N * i2 : (d == 1 ? i0 + N * i2 : i0 + N * i1);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        acc[v] = fmab(O.gL[N][kd], jm[((2 * d) * 5 + v) * N2 + fp], acc[v]);
        acc[v] = fmab(O.gR[N][kd], jm[((2 * d + 1) * 5 + v) * N2 + fp], acc[v]);
      }
    }
  }
  if (act) {
    const B mJ = B(-1) / J;
    const B alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T res = acc[v] * mJ;
      const B r = IO<T>::out(res);
      const long idx = (long)v * a.nsp + off;
      a.out[idx] = a.in2 ? alpha * a.in2[idx] + a.beta * r : a.beta * r;
      if (a.out_val) a.out_val[idx] = IO<T>::value(res);
    }
  }
}

// ------------------------------------------------------ per-bucket kernels
template <int N, class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_trace(ResArgs<T> a, const int4* __restrict__ elems, int nel, int epb) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  trace_body<N, T, NS>(a, elems, nel, epb, blockIdx.x, smem);
}
template <int NL, int NH, class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_face(ResArgs<T> a, const int4* __restrict__ faces, int nf, int fpb) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  face_body<NL, NH, T, NS>(a, faces, nf, fpb, blockIdx.x, smem);
}
template <int NL, int NH, class T>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_face_visc(ResArgs<T> a, const int4* __restrict__ faces, int nf,
                                                               int fpb) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  face_visc_body<NL, NH, T>(a, faces, nf, fpb, blockIdx.x, smem);
}
template <int N, class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_bface(ResArgs<T> a, const int4* __restrict__ faces, int nf) {
  if (a.skip && *a.skip) return;
  bface_body<N, T, NS>(a, faces, nf, blockIdx.x);
}
template <int N, class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_div(ResArgs<T> a, const int4* __restrict__ elems, int nel, int epb) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  div_body<N, T, NS>(a, elems, nel, epb, blockIdx.x, smem);
}

// ------------------------------------------------- degree-bucketed launches
// Element lists hold records (e, first solution point, first face slot, 0).
// One launch per stage over every degree bucket.  tiles[blockIdx.x] =
// (code, first, count, per): code = n for element tiles, 8 nl + nh for
// interior-face tiles, 64 + n for boundary-face tiles; `first` indexes the
// concatenated element (face) list; count <= per items of one block.  The
// host orders the tiles by decreasing work (the heavy degrees first), so the
// hardware dispatcher hands out the long tiles before the short ones.
#define FRX_ECASE(BODY, N) \
  case N: BODY<N, T, NS>(a, elems + t.y, t.z, t.w, 0, smem); break;

template <class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(StageWaves<T, 0>::value))) k_trace_fused(ResArgs<T> a, const int4* __restrict__ elems,
                                                     const int4* __restrict__ tiles) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_ECASE(trace_body, 2)
    FRX_ECASE(trace_body, 3)
    FRX_ECASE(trace_body, 4)
    FRX_ECASE(trace_body, 5)
    FRX_ECASE(trace_body, 6)
    default: break;
  }
}

template <class T, bool NS>
__global__ void __launch_bounds__(FRX_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(StageWaves<T, 2>::value))) k_div_fused(ResArgs<T> a, const int4* __restrict__ elems,
                                                   const int4* __restrict__ tiles) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_ECASE(div_body, 2)
    FRX_ECASE(div_body, 3)
    FRX_ECASE(div_body, 4)
    FRX_ECASE(div_body, 5)
    FRX_ECASE(div_body, 6)
    default: break;
  }
}
#undef FRX_ECASE

// Interior-face tiles of the face stage (the plan puts them first), with the
// Riemann solver fixed at compile time; boundary-face tiles go to
// k_bface_fused, so that the wall and far-field code does not set the
// register count of the interior faces.
#define FRX_FLIST(X)                                            \
  X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(3, 3) X(3, 4) X(3, 5) \
  X(3, 6) X(4, 4) X(4, 5) X(4, 6) X(5, 5) X(5, 6) X(6, 6)
#define FRX_GCASE(NL, NH) \
  case 8 * NL + NH: face_gather<NL, NH, T, NS>(a, faces + t.y, t.z, t.w, 0, smem, P); break;
#define FRX_SCASE(NL, NH) \
  case 8 * NL + NH: face_scatter<NL, NH, T>(a, faces + t.y, t.z, t.w, 0, smem, P, fS, NS ? 20 : 5); break;

// Register budget from FRX_STAGE_WAVES: the float64-dual Navier-Stokes face
// needs about 270 registers per lane, one wave per SIMD with nothing to
// overlap its loads; held to two waves (256) it spills about 26 registers to
// scratch and runs about a fifth faster.
template <class T, bool NS, int FLUX>
__global__ void __launch_bounds__(FRX_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(StageWaves<T, 1>::value))) k_face_fused(ResArgs<T> a, const int4* __restrict__ faces,
                                                    const int4* __restrict__ tiles) {
  using B = base_t<T>;
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  FacePt<T> P;
  switch (t.x) {
    FRX_FLIST(FRX_GCASE)
    default: return;
  }
  T fS[5];
  if (P.act) face_fn<NS, T, B, FLUX>(P.q[0], P.q[1], P.g, P.S, P.cL, P.cR, a.gas, a.flux, fS);
  switch (t.x) {
    FRX_FLIST(FRX_SCASE)
    default: break;
  }
}
#undef FRX_GCASE
#undef FRX_SCASE

// The solution jumps q_com - q alone at the interior faces' own face points
// (eq. com_q; the low side of a mixed face receives their L2 projection), for
// the forward recomputation of the adjoint: its reverse stages read the
// forward traces and these jumps, not the common fluxes.  The q traces are
// gathered as for Euler; same tiles and LDS as k_face_fused.
#define FRX_GCASE(NL, NH) \
  case 8 * NL + NH: face_gather<NL, NH, T, false>(a, faces + t.y, t.z, t.w, 0, smem, P); break;
#define FRX_SCASE(NL, NH) \
  case 8 * NL + NH: face_scatter<NL, NH, T, false>(a, faces + t.y, t.z, t.w, 0, smem, P, fS, 5); break;
template <class T>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_face_jumps_fused(ResArgs<T> a, const int4* __restrict__ faces,
                                                                    const int4* __restrict__ tiles) {
  using B = base_t<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  FacePt<T> P;
  switch (t.x) {
    FRX_FLIST(FRX_GCASE)
    default: return;
  }
  const T fS[5] = {T(B(0)), T(B(0)), T(B(0)), T(B(0)), T(B(0))};
  switch (t.x) {
    FRX_FLIST(FRX_SCASE)
    default: break;
  }
}
#undef FRX_GCASE
#undef FRX_SCASE

// Two-pass face stage of Navier-Stokes (interior-face tiles only, which the
// plan puts first): PASS 0 the inviscid pass, PASS 1 the viscous correction.
#define FRX_SCASE(NL, NH)                                                        \
  case 8 * NL + NH:                                                             \
    if constexpr (PASS == 0) face_body<NL, NH, T, false, FLUX>(a, faces + t.y, t.z, t.w, 0, smem); \
    else face_visc_body<NL, NH, T>(a, faces + t.y, t.z, t.w, 0, smem);           \
    break;

template <class T, int PASS, int FLUX>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_face_split_fused(ResArgs<T> a, const int4* __restrict__ faces,
                                                                      const int4* __restrict__ tiles) {
  if (a.skip && *a.skip) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_FLIST(FRX_SCASE)
    default: break;
  }
}
#undef FRX_SCASE
#undef FRX_FLIST

// Boundary-face tiles of the face stage (the plan puts them last).
#define FRX_BCASE(N) \
  case 64 + N: bface_body<N, T, NS, FLUX>(a, faces + t.y, t.z, 0); break;
template <class T, bool NS, int FLUX>
__global__ void __launch_bounds__(FRX_MAX_THREADS) k_bface_fused(ResArgs<T> a, const int4* __restrict__ faces,
                                                                 const int4* __restrict__ tiles) {
  if (a.skip && *a.skip) return;
  const int4 t = tiles[blockIdx.x];
  switch (t.x) {
    FRX_BCASE(2) FRX_BCASE(3) FRX_BCASE(4) FRX_BCASE(5) FRX_BCASE(6)
    default: break;
  }
}
#undef FRX_BCASE

}  // namespace frx
