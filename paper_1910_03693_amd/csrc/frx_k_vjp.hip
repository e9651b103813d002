// Adjoint (vector-Jacobian product) kernels and their launcher.
#include "frx_launch.hpp"
#include "frx_vjp.hpp"

namespace frx {

hipError_t upload_tables_vjp(const OpsTab<double>& d, const OpsTab<float>& f) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ops_d), &d, sizeof(d));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_ops_f), &f, sizeof(f));
}

namespace {

int epb_for(int n, size_t per_elem_bytes) {
  const int n3 = n * n * n;
  int e = n3 >= 128 ? 1 : 128 / n3;
  while (e > 1 && (size_t)e * per_elem_bytes > 48 * 1024) --e;
  return e;
}

template <int N, bool NS>
hipError_t elem_rev(const VjpArgs& va, const ElemBucket& b, bool trace, hipStream_t s) {
  const int n3 = N * N * N;
  const size_t per = (size_t)(5 * n3 + (trace ? 0 : 30 * N * N)) * sizeof(double);
  const int epb = epb_for(N, per);
  const int grid = (b.count + epb - 1) / epb;
  if (trace)
    hipLaunchKernelGGL((k_trace_rev<N, NS>), dim3(grid), dim3(round64(epb * n3)), epb * per, s, va, b.elems, b.count,
                       epb);
  else
    hipLaunchKernelGGL((k_div_rev<N, NS>), dim3(grid), dim3(round64(epb * n3)), epb * per, s, va, b.elems, b.count,
                       epb);
  return hipGetLastError();
}

template <int NL, int NH, bool NS>
hipError_t face_rev(const VjpArgs& va, const FaceBucket& b, hipStream_t s) {
  constexpr int NV = NS ? 20 : 5;
  const size_t per = NL < NH ? (size_t)(NV * NL * NL + 10 * NL * NL + NV * NH * NH) * sizeof(double) : 0;
  int fpb = std::max(1, 128 / (NH * NH));
  while (fpb > 1 && (size_t)fpb * per > 48 * 1024) --fpb;
  const int grid = (b.count + fpb - 1) / fpb;
  hipLaunchKernelGGL((k_face_rev<NL, NH, NS>), dim3(grid), dim3(round64(fpb * NH * NH)), fpb * per, s, va, b.faces,
                     b.count, fpb);
  return hipGetLastError();
}

template <int N, bool NS>
hipError_t bface_rev(const VjpArgs& va, const BFaceBucket& b, hipStream_t s) {
  const int tot = b.count * N * N;
  hipLaunchKernelGGL((k_bface_rev<N, NS>), dim3((tot + 255) / 256), dim3(256), 0, s, va, b.faces, b.count);
  return hipGetLastError();
}

template <bool NS>
hipError_t elem_rev_n(const VjpArgs& va, const ElemBucket& b, bool trace, hipStream_t s) {
#define FRX_C(N) elem_rev<N, NS>(va, b, trace, s)
  FRX_SWITCH_N(b.n, FRX_C)
#undef FRX_C
}
template <bool NS>
hipError_t bface_rev_n(const VjpArgs& va, const BFaceBucket& b, hipStream_t s) {
#define FRX_C(N) bface_rev<N, NS>(va, b, s)
  FRX_SWITCH_N(b.n, FRX_C)
#undef FRX_C
}
template <bool NS, int NL>
hipError_t face_rev_nh(const VjpArgs& va, const FaceBucket& b, hipStream_t s) {
  switch (b.nh) {
    case 2: if constexpr (NL <= 2) return face_rev<NL, 2, NS>(va, b, s); break;
    case 3: if constexpr (NL <= 3) return face_rev<NL, 3, NS>(va, b, s); break;
    case 4: if constexpr (NL <= 4) return face_rev<NL, 4, NS>(va, b, s); break;
    case 5: if constexpr (NL <= 5) return face_rev<NL, 5, NS>(va, b, s); break;
    case 6: return face_rev<NL, 6, NS>(va, b, s);
    default: break;
  }
  return hipErrorInvalidValue;
}
template <bool NS>
hipError_t face_rev_n(const VjpArgs& va, const FaceBucket& b, hipStream_t s) {
  switch (b.nl) {
    case 2: return face_rev_nh<NS, 2>(va, b, s);
    case 3: return face_rev_nh<NS, 3>(va, b, s);
    case 4: return face_rev_nh<NS, 4>(va, b, s);
    case 5: return face_rev_nh<NS, 5>(va, b, s);
    case 6: return face_rev_nh<NS, 6>(va, b, s);
    default: return hipErrorInvalidValue;
  }
}

// The fused path: forward traces with the fused forward kernel of the float64
// plan, and for Navier-Stokes the solution jumps (the interior faces' jumps
// alone, the boundary faces' full face function), then one launch per reverse
// stage.  The reverse stages read the forward traces, and the jumps for the
// corrected gradient; the common fluxes are recomputed by face_rev.
template <bool NS>
hipError_t vjp_fused(const ResArgs<double>& fa, const VjpArgs& va, const MeshDev& M, hipStream_t s) {
  const FusedPlan& P = M.plan[SK_F64];
  const FusedPlan& V = M.vplan;
  hipError_t e;
  if (P.count[0]) {
    hipLaunchKernelGGL((k_trace_fused<double, NS>), dim3(P.count[0]), dim3(256), P.lds[0], s, fa, M.all_elems,
                       P.tiles[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (NS && P.n_interior > 0) {
    hipLaunchKernelGGL((k_face_jumps_fused<double>), dim3(P.n_interior), dim3(256), P.lds[1], s, fa, M.all_faces,
                       P.tiles[1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (NS && P.count[1] > P.n_interior) {
    if (M.flux == 1)
      hipLaunchKernelGGL((k_bface_fused<double, NS, 1>), dim3(P.count[1] - P.n_interior), dim3(256), 0, s, fa,
                         M.all_faces, P.tiles[1] + P.n_interior);
    else
      hipLaunchKernelGGL((k_bface_fused<double, NS, 0>), dim3(P.count[1] - P.n_interior), dim3(256), 0, s, fa,
                         M.all_faces, P.tiles[1] + P.n_interior);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (V.count[2]) {
    hipLaunchKernelGGL((k_elem_rev_fused<NS, false>), dim3(V.count[2]), dim3(256), V.lds[2], s, va,
                       (const int*)M.all_ids, V.tiles[2]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (V.n_interior > 0) {
    if (M.flux == 1)
      hipLaunchKernelGGL((k_face_rev_fused<NS, 1>), dim3(V.n_interior), dim3(256), V.lds[1], s, va, M.all_faces,
                         V.tiles[1]);
    else
      hipLaunchKernelGGL((k_face_rev_fused<NS, 0>), dim3(V.n_interior), dim3(256), V.lds[1], s, va, M.all_faces,
                         V.tiles[1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (V.count[1] > V.n_interior) {
    hipLaunchKernelGGL((k_bface_rev_fused<NS>), dim3(V.count[1] - V.n_interior), dim3(256), 0, s, va, M.all_faces,
                       V.tiles[1] + V.n_interior);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (V.count[0]) {
    hipLaunchKernelGGL((k_elem_rev_fused<NS, true>), dim3(V.count[0]), dim3(256), V.lds[0], s, va,
                       (const int*)M.all_ids, V.tiles[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool NS>
hipError_t vjp_stages(const ResArgs<double>& fa, const VjpArgs& va, const MeshDev& M, hipStream_t s) {
  if (M.fused) return vjp_fused<NS>(fa, va, M, s);
  hipError_t e;
  // forward face intermediates
  for (const ElemBucket& b : M.eb)
    if (b.count && (e = trace_n<double, NS>(fa, b, b.epb_trace[SK_F64], s)) != hipSuccess) return e;
  for (const FaceBucket& b : M.fb)
    if (b.count && (e = face_n<double, NS>(fa, b, b.fpb[SK_F64], s)) != hipSuccess) return e;
  for (const BFaceBucket& b : M.bb)
    if (b.count && (e = bface_n<double, NS>(fa, b, s)) != hipSuccess) return e;
  // reverse sweep
  for (const ElemBucket& b : M.eb)
    if (b.count && (e = elem_rev_n<NS>(va, b, false, s)) != hipSuccess) return e;
  for (const FaceBucket& b : M.fb)
    if (b.count && (e = face_rev_n<NS>(va, b, s)) != hipSuccess) return e;
  for (const BFaceBucket& b : M.bb)
    if (b.count && (e = bface_rev_n<NS>(va, b, s)) != hipSuccess) return e;
  for (const ElemBucket& b : M.eb)
    if (b.count && (e = elem_rev_n<NS>(va, b, true, s)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace

hipError_t launch_vjp(const MeshDev& M, const double* U, const double* w, double* out, hipStream_t s) {
  ResArgs<double> fa;
  fa.U = U;
  fa.V = nullptr;
  fa.out = nullptr;
  fa.out_val = nullptr;
  fa.in2 = nullptr;
  fa.alpha_dev = nullptr;
  fa.alpha = 0.0;
  fa.beta = 1.0;
  fa.nsp = M.nsp;
  fa.nfp = M.nfp;
  fa.flux = M.flux;
  fa.sp_off = M.sp_off;
  fa.fp_off = M.fp_off;
  fa.geo = M.geo_d;
  fa.fgeo = M.fgeo_d;
  double* fb = reinterpret_cast<double*>(M.facebuf);
  fa.QF = fb;
  fa.GF = fb + 5L * M.nfp;
  fa.DQ = fb + 20L * M.nfp;
  fa.FS = fb + 25L * M.nfp;
  fa.gas = M.gas_d;
  fa.flag = M.flag;
  fa.skip = nullptr;
  VjpArgs va;
  va.U = U;
  va.W = w;
  va.out = out;
  va.nsp = M.nsp;
  va.nfp = M.nfp;
  va.flux = M.flux;
  va.sp_off = M.sp_off;
  va.fp_off = M.fp_off;
  va.geo = M.geo_d;
  va.fgeo = M.fgeo_d;
  va.QF = fa.QF;
  va.GF = fa.GF;
  va.DQ = fa.DQ;
  va.FS = fa.FS;
  va.gas = M.gas_d;
  return M.physics == 1 ? vjp_stages<true>(fa, va, M, s) : vjp_stages<false>(fa, va, M, s);
}

}  // namespace frx
