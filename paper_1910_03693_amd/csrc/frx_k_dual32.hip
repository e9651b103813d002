// Residual kernels instantiated for the scalar Dual<float>.
#include "frx_launch.hpp"


namespace frx {

hipError_t upload_tables_dual32(const OpsTab<double>& d, const OpsTab<float>& f) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ops_d), &d, sizeof(d));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_ops_f), &f, sizeof(f));
}

hipError_t launch_residual_dual32(const MeshDev& M, const ResCall<float>& c, hipStream_t s, const FusedSubset* sub,
                                  const FusedSubset* tsub) {
  return launch_residual_T<Dual<float>>(M, c, SK_DUAL32, s, sub, tsub);
}
}  // namespace frx
