// Launchers of the three residual stages for one scalar type T; each kernel
// translation unit includes this file once with its own T.
#pragma once
#include "frx_host.hpp"
#include "frx_residual.hpp"

namespace frx {

template <class B> __host__ inline const B* geo_of(const MeshDev& M);
template <> __host__ inline const double* geo_of<double>(const MeshDev& M) { return M.geo_d; }
template <> __host__ inline const float* geo_of<float>(const MeshDev& M) { return M.geo_f; }
template <class B> __host__ inline const B* fgeo_of(const MeshDev& M);
template <> __host__ inline const double* fgeo_of<double>(const MeshDev& M) { return M.fgeo_d; }
template <> __host__ inline const float* fgeo_of<float>(const MeshDev& M) { return M.fgeo_f; }
template <class B> __host__ inline const Gas<B>& gas_of(const MeshDev& M);
template <> __host__ inline const Gas<double>& gas_of<double>(const MeshDev& M) { return M.gas_d; }
template <> __host__ inline const Gas<float>& gas_of<float>(const MeshDev& M) { return M.gas_f; }

inline int round64(int t) { return (t + 63) / 64 * 64; }

// Every residual kernel is compiled with __launch_bounds__(FRX_MAX_THREADS);
// a wider block is refused on the host instead of being launched.
inline bool block_ok(int threads) { return threads >= 1 && threads <= FRX_MAX_THREADS; }

// LDS scalars per element of the trace stage (see trace_in_rounds)
inline int trace_vals_host(int n, bool ns, size_t sb) { return trace_lds_vals(ns, n, (int)sb); }
template <class T> size_t trace_lds(int n, int epb, bool ns) {
  return (size_t)epb * trace_vals_host(n, ns, sizeof(T)) * n * n * n * sizeof(T);
}
template <class T> size_t div_lds(int n, int epb) { return (size_t)epb * (5 * n * n * n + 30 * n * n) * sizeof(T); }
template <class T> size_t face_lds(int nl, int nh, bool ns, int fpb) {
  return nl < nh ? (size_t)fpb * ((ns ? 20 : 5) * nl * nl + 10 * nh * nh) * sizeof(T) : 0;
}

template <int N, class T, bool NS>
hipError_t run_trace(const ResArgs<T>& a, const ElemBucket& b, int epb, hipStream_t s) {
  const int grid = (b.count + epb - 1) / epb;
  if (!block_ok(round64(epb * N * N * N))) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_trace<N, T, NS>), dim3(grid), dim3(round64(epb * N * N * N)), trace_lds<T>(N, epb, NS), s, a,
                     b.recs, b.count, epb);
  return hipGetLastError();
}
template <int N, class T, bool NS>
hipError_t run_div(const ResArgs<T>& a, const ElemBucket& b, int epb, hipStream_t s) {
  const int grid = (b.count + epb - 1) / epb;
  if (!block_ok(round64(epb * N * N * N))) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_div<N, T, NS>), dim3(grid), dim3(round64(epb * N * N * N)), div_lds<T>(N, epb), s, a, b.recs,
                     b.count, epb);
  return hipGetLastError();
}
template <int NL, int NH, class T, bool NS>
hipError_t run_face(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  const int grid = (b.count + fpb - 1) / fpb;
  if (!block_ok(round64(fpb * NH * NH))) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_face<NL, NH, T, NS>), dim3(grid), dim3(round64(fpb * NH * NH)), face_lds<T>(NL, NH, NS, fpb),
                     s, a, b.faces, b.count, fpb);
  return hipGetLastError();
}
template <int NL, int NH, class T>
hipError_t run_face_visc(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  const int grid = (b.count + fpb - 1) / fpb;
  if (!block_ok(round64(fpb * NH * NH))) return hipErrorInvalidConfiguration;
  const size_t lds = NL < NH ? (size_t)fpb * (20 * NL * NL + 4 * NH * NH) * sizeof(T) : 0;
  hipLaunchKernelGGL((k_face_visc<NL, NH, T>), dim3(grid), dim3(round64(fpb * NH * NH)), lds, s, a, b.faces, b.count,
                     fpb);
  return hipGetLastError();
}
template <int N, class T, bool NS>
hipError_t run_bface(const ResArgs<T>& a, const BFaceBucket& b, hipStream_t s) {
  const int tot = b.count * N * N;
  hipLaunchKernelGGL((k_bface<N, T, NS>), dim3((tot + 255) / 256), dim3(256), 0, s, a, b.faces, b.count);
  return hipGetLastError();
}

#define FRX_SWITCH_N(n, CALL) \
  switch (n) {                \
    case 2: return CALL(2);   \
    case 3: return CALL(3);   \
    case 4: return CALL(4);   \
    case 5: return CALL(5);   \
    case 6: return CALL(6);   \
    default: return hipErrorInvalidValue; \
  }

template <class T, bool NS>
hipError_t trace_n(const ResArgs<T>& a, const ElemBucket& b, int epb, hipStream_t s) {
#define FRX_C(N) run_trace<N, T, NS>(a, b, epb, s)
  FRX_SWITCH_N(b.n, FRX_C)
#undef FRX_C
}
template <class T, bool NS>
hipError_t div_n(const ResArgs<T>& a, const ElemBucket& b, int epb, hipStream_t s) {
#define FRX_C(N) run_div<N, T, NS>(a, b, epb, s)
  FRX_SWITCH_N(b.n, FRX_C)
#undef FRX_C
}
template <class T, bool NS>
hipError_t bface_n(const ResArgs<T>& a, const BFaceBucket& b, hipStream_t s) {
#define FRX_C(N) run_bface<N, T, NS>(a, b, s)
  FRX_SWITCH_N(b.n, FRX_C)
#undef FRX_C
}
template <class T, bool NS, int NL>
hipError_t face_nh(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  switch (b.nh) {
    case 2: if constexpr (NL <= 2) return run_face<NL, 2, T, NS>(a, b, fpb, s); break;
    case 3: if constexpr (NL <= 3) return run_face<NL, 3, T, NS>(a, b, fpb, s); break;
    case 4: if constexpr (NL <= 4) return run_face<NL, 4, T, NS>(a, b, fpb, s); break;
    case 5: if constexpr (NL <= 5) return run_face<NL, 5, T, NS>(a, b, fpb, s); break;
    case 6: return run_face<NL, 6, T, NS>(a, b, fpb, s);
    default: break;
  }
  return hipErrorInvalidValue;
}
template <class T, bool NS>
hipError_t face_n(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  switch (b.nl) {
    case 2: return face_nh<T, NS, 2>(a, b, fpb, s);
    case 3: return face_nh<T, NS, 3>(a, b, fpb, s);
    case 4: return face_nh<T, NS, 4>(a, b, fpb, s);
    case 5: return face_nh<T, NS, 5>(a, b, fpb, s);
    case 6: return face_nh<T, NS, 6>(a, b, fpb, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T, int NL>
hipError_t face_visc_nh(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  switch (b.nh) {
    case 2: if constexpr (NL <= 2) return run_face_visc<NL, 2, T>(a, b, fpb, s); break;
    case 3: if constexpr (NL <= 3) return run_face_visc<NL, 3, T>(a, b, fpb, s); break;
    case 4: if constexpr (NL <= 4) return run_face_visc<NL, 4, T>(a, b, fpb, s); break;
    case 5: if constexpr (NL <= 5) return run_face_visc<NL, 5, T>(a, b, fpb, s); break;
    case 6: return run_face_visc<NL, 6, T>(a, b, fpb, s);
    default: break;
  }
  return hipErrorInvalidValue;
}
template <class T>
hipError_t face_visc_n(const ResArgs<T>& a, const FaceBucket& b, int fpb, hipStream_t s) {
  switch (b.nl) {
    case 2: return face_visc_nh<T, 2>(a, b, fpb, s);
    case 3: return face_visc_nh<T, 3>(a, b, fpb, s);
    case 4: return face_visc_nh<T, 4>(a, b, fpb, s);
    case 5: return face_visc_nh<T, 5>(a, b, fpb, s);
    case 6: return face_visc_nh<T, 6>(a, b, fpb, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T, bool NS>
hipError_t residual_stages(const ResArgs<T>& a, const MeshDev& M, int sk, hipStream_t s) {
  hipError_t e;
  ProfHook* P = M.prof;
  for (const ElemBucket& b : M.eb) {
    if (!b.count) continue;
    if (P) P->begin("k_trace", b.n, b.n, b.count, s);
    if ((e = trace_n<T, NS>(a, b, b.epb_trace[sk], s)) != hipSuccess) return e;
    if (P) P->end(s);
  }
  const bool split = NS && M.split_faces[0][sk];
  for (const FaceBucket& b : M.fb) {
    if (!b.count) continue;
    if (P) P->begin("k_face", b.nl, b.nh, b.count, s);
    if (split) {
      if ((e = face_n<T, false>(a, b, b.fpb[sk], s)) != hipSuccess) return e;
      if ((e = face_visc_n<T>(a, b, b.fpb[sk], s)) != hipSuccess) return e;
    } else if ((e = face_n<T, NS>(a, b, b.fpb[sk], s)) != hipSuccess) {
      return e;
    }
    if (P) P->end(s);
  }
  for (const BFaceBucket& b : M.bb) {
    if (!b.count) continue;
    if (P) P->begin("k_bface", b.n, b.n, b.count, s);
    if ((e = bface_n<T, NS>(a, b, s)) != hipSuccess) return e;
    if (P) P->end(s);
  }
  for (const ElemBucket& b : M.eb) {
    if (!b.count) continue;
    if (P) P->begin("k_div", b.n, b.n, b.count, s);
    if ((e = div_n<T, NS>(a, b, b.epb_div[sk], s)) != hipSuccess) return e;
    if (P) P->end(s);
  }
  return hipSuccess;
}

// Face stage of the fused plan: interior-face tiles (one or two passes), then
// the boundary-face tiles in a launch of their own.
template <class T, bool NS, int FLUX>
hipError_t face_stage_fused(const ResArgs<T>& a, const MeshDev& M, const FusedPlan& P, bool two_pass, hipStream_t s,
                            const int4* faces = nullptr) {
  hipError_t e;
  if (!faces) faces = M.all_faces;
  if (P.n_interior > 0) {
    if (two_pass) {
      hipLaunchKernelGGL((k_face_split_fused<T, 0, FLUX>), dim3(P.n_interior), dim3(256), P.lds[1], s, a, faces,
                         P.tiles[1]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL((k_face_split_fused<T, 1, FLUX>), dim3(P.n_interior), dim3(256), P.lds[1], s, a, faces,
                         P.tiles[1]);
    } else {
      hipLaunchKernelGGL((k_face_fused<T, NS, FLUX>), dim3(P.n_interior), dim3(256), P.lds[1], s, a, faces,
                         P.tiles[1]);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (P.count[1] > P.n_interior) {
    hipLaunchKernelGGL((k_bface_fused<T, NS, FLUX>), dim3(P.count[1] - P.n_interior), dim3(256), 0, s, a, faces,
                       P.tiles[1] + P.n_interior);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class T, bool NS>
hipError_t residual_fused(const ResArgs<T>& a, const MeshDev& M, int sk, hipStream_t s,
                          const FusedSubset* sub = nullptr, const FusedSubset* tsub = nullptr) {
  const FusedPlan& P = tsub ? tsub->plan[sk] : M.plan[sk];  // trace stage
  const FusedPlan& Q = sub ? sub->plan[sk] : M.plan[sk];    // face and divergence stages
  const int4* elems0 = tsub ? tsub->elems : M.all_elems;
  const int4* faces = sub ? sub->faces : M.all_faces;
  const int4* elems2 = sub ? sub->elems : M.all_elems;
  ProfHook* H = M.prof;
  const char* names[3] = {"k_trace_fused", "k_face_fused", "k_div_fused"};
  hipError_t e;
  for (int st = 0; st < 3; ++st) {
    const FusedPlan& X = st == 0 ? P : Q;
    if (!X.count[st]) continue;
    if (H) H->begin(names[st], 0, 0, X.count[st], s);
    if (st == 0)
      hipLaunchKernelGGL((k_trace_fused<T, NS>), dim3(P.count[0]), dim3(256), P.lds[0], s, a, elems0, P.tiles[0]);
    else if (st == 1) {
      const bool two_pass = NS && M.split_faces[1][sk];
      e = M.flux == 1 ? face_stage_fused<T, NS, 1>(a, M, Q, two_pass, s, faces)
                      : face_stage_fused<T, NS, 0>(a, M, Q, two_pass, s, faces);
      if (e != hipSuccess) return e;
    } else
      hipLaunchKernelGGL((k_div_fused<T, NS>), dim3(Q.count[2]), dim3(256), Q.lds[2], s, a, elems2, Q.tiles[2]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (H) H->end(s);
  }
  return hipSuccess;
}

template <class T>
hipError_t launch_residual_T(const MeshDev& M, const ResCall<base_t<T>>& c, int sk, hipStream_t s,
                             const FusedSubset* sub = nullptr, const FusedSubset* tsub = nullptr) {
  using B = base_t<T>;
  ResArgs<T> a;
  a.U = c.U;
  a.V = c.V;
  a.out = c.out;
  a.out_val = c.out_val;
  a.in2 = c.in2;
  a.alpha_dev = c.alpha_dev;
  a.alpha = c.alpha;
  a.beta = c.beta;
  a.nsp = M.nsp;
  a.nfp = M.nfp;
  a.flux = M.flux;
  a.sp_off = M.sp_off;
  a.fp_off = M.fp_off;
  a.geo = geo_of<B>(M);
  a.fgeo = fgeo_of<B>(M);
  T* fb = reinterpret_cast<T*>(M.facebuf);
  a.QF = fb;
  a.GF = fb + 5L * M.nfp;
  a.DQ = fb + 20L * M.nfp;
  a.FS = fb + 25L * M.nfp;
  a.gas = gas_of<B>(M);
  a.flag = M.flag;
  a.skip = c.skip;
  if (M.fused)
    return M.physics == 1 ? residual_fused<T, true>(a, M, sk, s, sub, tsub)
                          : residual_fused<T, false>(a, M, sk, s, sub, tsub);
  return M.physics == 1 ? residual_stages<T, true>(a, M, sk, s) : residual_stages<T, false>(a, M, sk, s);
}

}  // namespace frx
