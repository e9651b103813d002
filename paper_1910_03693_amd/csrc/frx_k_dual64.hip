// Residual kernels instantiated for the scalar Dual<double>.
#include "frx_launch.hpp"


namespace frx {

hipError_t upload_tables_dual64(const OpsTab<double>& d, const OpsTab<float>& f) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ops_d), &d, sizeof(d));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_ops_f), &f, sizeof(f));
}

hipError_t launch_residual_dual64(const MeshDev& M, const ResCall<double>& c, hipStream_t s, const FusedSubset* sub,
                                  const FusedSubset* tsub) {
  return launch_residual_T<Dual<double>>(M, c, SK_DUAL64, s, sub, tsub);
}
}  // namespace frx
