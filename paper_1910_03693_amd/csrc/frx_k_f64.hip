// Residual kernels instantiated for the scalar double.
#include "frx_launch.hpp"
#include "frx_indicator.hpp"

namespace frx {

hipError_t upload_tables_f64(const OpsTab<double>& d, const OpsTab<float>& f) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ops_d), &d, sizeof(d));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_ops_f), &f, sizeof(f));
}

hipError_t launch_residual_f64(const MeshDev& M, const ResCall<double>& c, hipStream_t s) {
  return launch_residual_T<double>(M, c, SK_F64, s);
}

hipError_t launch_face_geometry(const MeshDev& M, hipStream_t s) {
  for (const FaceBucket& b : M.fb) {
    if (!b.count) continue;
    const long tot = (long)b.count * b.nh * b.nh;
    const dim3 grid((unsigned)((tot + 255) / 256));
    hipLaunchKernelGGL(k_face_geo<double>, grid, dim3(256), 0, s, M.geo_d, b.faces, b.count, b.nl, b.nh, M.fgeo_d);
    hipLaunchKernelGGL(k_face_geo<float>, grid, dim3(256), 0, s, M.geo_f, b.faces, b.count, b.nl, b.nh, M.fgeo_f);
  }
  for (const BFaceBucket& b : M.bb) {
    if (!b.count) continue;
    const long tot = (long)b.count * b.n * b.n;
    const dim3 grid((unsigned)((tot + 255) / 256));
    hipLaunchKernelGGL(k_bface_geo<double>, grid, dim3(256), 0, s, M.geo_d, b.faces, b.count, b.n, M.fgeo_d);
    hipLaunchKernelGGL(k_bface_geo<float>, grid, dim3(256), 0, s, M.geo_f, b.faces, b.count, b.n, M.fgeo_f);
  }
  return hipGetLastError();
}

hipError_t launch_indicator(const MeshDev& M, const double* U, int var, double* eta, double* eta_max,
                            hipStream_t s) {
  for (const ElemBucket& b : M.eb) {
    if (!b.count) continue;
    const int n = b.n, n3 = n * n * n;
    const int epb = n3 >= 256 ? 1 : 256 / n3;
    const int grid = (b.count + epb - 1) / epb;
    const size_t lds = (size_t)epb * 4 * n3 * sizeof(double);
    const dim3 blk(round64(epb * n3));
    switch (n) {
      case 2: hipLaunchKernelGGL(k_indicator<2>, dim3(grid), blk, lds, s, U, M.nsp, var, M.sp_off, M.geo_d, b.elems, b.count, epb, eta); break;
      case 3: hipLaunchKernelGGL(k_indicator<3>, dim3(grid), blk, lds, s, U, M.nsp, var, M.sp_off, M.geo_d, b.elems, b.count, epb, eta); break;
      case 4: hipLaunchKernelGGL(k_indicator<4>, dim3(grid), blk, lds, s, U, M.nsp, var, M.sp_off, M.geo_d, b.elems, b.count, epb, eta); break;
      case 5: hipLaunchKernelGGL(k_indicator<5>, dim3(grid), blk, lds, s, U, M.nsp, var, M.sp_off, M.geo_d, b.elems, b.count, epb, eta); break;
      case 6: hipLaunchKernelGGL(k_indicator<6>, dim3(grid), blk, lds, s, U, M.nsp, var, M.sp_off, M.geo_d, b.elems, b.count, epb, eta); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_max, dim3(1), dim3(256), 0, s, eta, M.E, eta_max);
  return hipGetLastError();
}
hipError_t launch_select_degrees(const MeshDev& M, const double* U, int var, double nu_max, double nu_min, int p_min,
                                 int p_max, int by_degree, int8_t* p_new, hipStream_t s) {
  double* eta = M.eta_w;
  double* eta_max = M.eta_w + M.E;  // [0]: over all elements; [n]: over the elements of size n
  hipError_t e = launch_indicator(M, U, var, eta, eta_max, s);
  if (e != hipSuccess) return e;
  if (by_degree) {
    hipLaunchKernelGGL(k_max_by_degree, dim3(1), dim3(256), 0, s, (const double*)eta, (const int8_t*)M.p_dev, M.E,
                       eta_max + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int grid = (M.E + 255) / 256;
  int8_t* a = M.psel;
  int8_t* b = M.psel + M.E;
  // (k_max_by_degree writes eta_max[1 + n'] for n' = 0..6; k_select reads eta_max[p + 1])
  hipLaunchKernelGGL(k_select, dim3(grid), dim3(256), 0, s, (const double*)eta,
                     (const double*)(by_degree ? eta_max + 1 : eta_max), by_degree, (const int8_t*)M.p_dev, M.E,
                     nu_max, nu_min, p_min, p_max, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int it = 0; it < p_max - p_min; ++it) {
    hipLaunchKernelGGL(k_limit, dim3(grid), dim3(256), 0, s, (const int8_t*)a, (const int*)M.nbr, M.E, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(a, b);
  }
  return hipMemcpyAsync(p_new, a, M.E, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_filter(const MeshDev& M, const double* U, double* Uout, double alpha, int p_from, hipStream_t s) {
  for (const ElemBucket& b : M.eb) {
    if (!b.count || b.n - 1 < p_from) continue;
    const dim3 grid(b.count), blk(round64(b.n * b.n * b.n));
    switch (b.n) {
      case 2: hipLaunchKernelGGL(k_filter<2>, grid, blk, 0, s, U, M.nsp, (const int4*)b.recs, alpha, Uout); break;
      case 3: hipLaunchKernelGGL(k_filter<3>, grid, blk, 0, s, U, M.nsp, (const int4*)b.recs, alpha, Uout); break;
      case 4: hipLaunchKernelGGL(k_filter<4>, grid, blk, 0, s, U, M.nsp, (const int4*)b.recs, alpha, Uout); break;
      case 5: hipLaunchKernelGGL(k_filter<5>, grid, blk, 0, s, U, M.nsp, (const int4*)b.recs, alpha, Uout); break;
      case 6: hipLaunchKernelGGL(k_filter<6>, grid, blk, 0, s, U, M.nsp, (const int4*)b.recs, alpha, Uout); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_project(const MeshDev& Ms, const double* Us, const MeshDev& Md, double* Ud, hipStream_t s) {
  hipLaunchKernelGGL(k_project, dim3(Ms.E), dim3(256), 0, s, Us, Ms.nsp, (const int*)Ms.sp_off,
                     (const int8_t*)Ms.p_dev, Ud, Md.nsp, (const int*)Md.sp_off, (const int8_t*)Md.p_dev);
  return hipGetLastError();
}

}  // namespace frx
