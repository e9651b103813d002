// Host-side description of a mesh resident on the device and the launchers of
// the kernel translation units (one per scalar type of the residual).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "frx_device.hpp"

namespace frx {

enum ScalarKind { SK_F64 = 0, SK_DUAL64 = 1, SK_DUAL32 = 2, SK_COUNT = 3 };

struct ElemBucket {
  int n = 0;        // p + 1
  int count = 0;
  int* elems = nullptr;  // device, ascending element ids of this degree
  int4* recs = nullptr;  // device, the same elements as (e, first solution point, first face slot, 0)
  int epb_trace[SK_COUNT] = {0, 0, 0};
  int epb_div[SK_COUNT] = {0, 0, 0};
};

struct FaceBucket {
  int nl = 0, nh = 0;
  int count = 0;
  int4* faces = nullptr;  // device (L, R, d, low_is_R)
  int fpb[SK_COUNT] = {0, 0, 0};
};

struct BFaceBucket {
  int n = 0;
  int count = 0;
  int4* faces = nullptr;  // device (e, f, bc, 0)
};

// Optional per-launch timing: every residual-stage launch is bracketed by two
// events on its stream.
struct ProfHook {
  struct Rec {
    const char* stage;
    int nl, nh;
    long units;  // elements or faces of the launch
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  void begin(const char* stage, int nl, int nh, long units, hipStream_t s) {
    Rec r{stage, nl, nh, units, nullptr, nullptr};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end(hipStream_t s) { (void)hipEventRecord(recs.back().b, s); }
};

// Tile tables of the degree-bucketed (fused) launches, per scalar kind.
struct FusedPlan {
  int4* tiles[3] = {nullptr, nullptr, nullptr};  // trace, face, div
  int count[3] = {0, 0, 0};
  size_t lds[3] = {0, 0, 0};
  int n_interior = 0;  // face stage: interior-face tiles come first, boundary-face tiles after them
};

struct MeshDev {
  int E = 0;
  int nsp = 0, nfp = 0;
  int physics = 0, flux = 0;
  int* sp_off = nullptr;
  int* fp_off = nullptr;
  double* geo_d = nullptr;
  float* geo_f = nullptr;
  double* fgeo_d = nullptr;  // [5][nfp] face-point geometry (see k_face_geo), float64
  float* fgeo_f = nullptr;   // the same from the float32 map
  std::vector<ElemBucket> eb;
  std::vector<FaceBucket> fb;
  std::vector<BFaceBucket> bb;
  void* facebuf = nullptr;  // 30 * nfp scalars of the widest scalar type
  int* flag = nullptr;
  int8_t* p_dev = nullptr;        // [E] degrees
  int* nbr = nullptr;             // [E][6] neighbours (negative: boundary)
  double* eta_w = nullptr;        // [E + 8] indicator workspace of the degree selection (eta, maxima)
  int8_t* psel = nullptr;         // [2 E] degree-selection ping-pong buffers
  ProfHook* prof = nullptr;
  bool fused = false;             // one launch per stage over all buckets
  // Navier-Stokes face stage in two passes (inviscid, then viscous correction),
  // per launch mode [per-bucket, fused] and scalar kind; chosen by fr_autotune
  bool split_faces[2][SK_COUNT] = {{false, false, false}, {false, false, false}};
  int4* all_elems = nullptr;      // concatenated bucket element records
  int4* all_faces = nullptr;      // concatenated interior + boundary face lists
  FusedPlan plan[SK_COUNT];
  // adjoint: tiles of the reverse stages [trace_rev, face_rev, div_rev] over
  // the element ids in all_ids (the order of all_elems)
  FusedPlan vplan;
  int* all_ids = nullptr;
  Gas<double> gas_d;
  Gas<float> gas_f;
};

// out = alpha * in2 + beta * result (in2 may be null); alpha_dev overrides alpha
template <class B> struct ResCall {
  const B* U = nullptr;
  const B* V = nullptr;
  B* out = nullptr;
  B* out_val = nullptr;  // duals: also write the value part (the residual)
  const B* in2 = nullptr;
  const B* alpha_dev = nullptr;
  B alpha = B(0), beta = B(1);
  const int* skip = nullptr;  // device flag: skip all work when nonzero
};

// The stages of the fused launch restricted to a subset of the elements:
// the divergence over them, the face stage over the faces with a side among
// them (their residual rows need no other face), the trace stage over them.
struct FusedSubset {
  const int4* elems = nullptr;  // records of the subset's elements, by degree bucket
  const int4* faces = nullptr;  // interior faces with a side in the subset, then its boundary faces
  FusedPlan plan[SK_COUNT];     // tiles of the three stages per scalar kind
};

// residual (SK_F64) or residual-and-tangent (duals) on a stream.  Fused
// launch mode only: with a subset `sub` R and Jv are written for its elements
// only; with a trace subset `tsub` the trace stage runs over its elements
// only, and the face slots of every other element must already hold its
// traces (of the same U and v) from an earlier pass.
hipError_t launch_residual_f64(const MeshDev& M, const ResCall<double>& c, hipStream_t s);
hipError_t launch_residual_dual64(const MeshDev& M, const ResCall<double>& c, hipStream_t s,
                                  const FusedSubset* sub = nullptr, const FusedSubset* tsub = nullptr);
hipError_t launch_residual_dual32(const MeshDev& M, const ResCall<float>& c, hipStream_t s,
                                  const FusedSubset* sub = nullptr, const FusedSubset* tsub = nullptr);

// operator tables into each translation unit's constant memory
hipError_t upload_tables_f64(const OpsTab<double>& d, const OpsTab<float>& f);
hipError_t upload_tables_dual64(const OpsTab<double>& d, const OpsTab<float>& f);
hipError_t upload_tables_dual32(const OpsTab<double>& d, const OpsTab<float>& f);

// default launch shapes for the residual kernels of one scalar kind
void default_shapes(MeshDev& M, int sk);
size_t scalar_bytes(int sk);

}  // namespace frx

namespace frx {
hipError_t upload_tables_vjp(const OpsTab<double>& d, const OpsTab<float>& f);
hipError_t launch_vjp(const MeshDev& M, const double* U, const double* w, double* out, hipStream_t s);
hipError_t launch_indicator(const MeshDev& M, const double* U, int var, double* eta, double* eta_max,
                            hipStream_t s);
hipError_t launch_select_degrees(const MeshDev& M, const double* U, int var, double nu_max, double nu_min, int p_min,
                                 int p_max, int by_degree, int8_t* p_new, hipStream_t s);
hipError_t launch_project(const MeshDev& Ms, const double* Us, const MeshDev& Md, double* Ud, hipStream_t s);
// nodal polynomial filter of the elements of degree >= p_from (Uout may be U)
hipError_t launch_filter(const MeshDev& M, const double* U, double* Uout, double alpha, int p_from, hipStream_t s);
// fills M.fgeo_d and M.fgeo_f from the trilinear maps (once per mesh)
hipError_t launch_face_geometry(const MeshDev& M, hipStream_t s);
}  // namespace frx
